// Backward, part 1 (Supplement Algorithm A1, part 2): re-find, from the saved
// visibility buffer, every fragment the backward needs -- the winner of each
// pixel with a colour gradient, and, where the pixel carries a score weight,
// every fragment in front of it (Eq. (9)).
//
// Persistent workgroups take screen tiles from a counter and walk the tile's
// depth-sorted triangle list with the forward's exact coverage test, in the
// forward's order, stopping where the rest of the list lies behind every
// active pixel's winner. Each wave compacts its candidates in LDS and appends
// them, 64 at a time, to a flat fragment list (one counter bump per batch).
// No MLP work happens here: the list is decoded by the decode kernel, whose
// registers then hold only the MLP state, and whose waves are always full.
#include "raster_common.hpp"

namespace soup {

template <int NW>
struct ReplayQueue {
    uint32_t pix[NW][128];
    uint32_t tri[NW][128];     // triangle | winner << 31
    float b1[NW][128];
    float b2[NW][128];
    float beta[3][NW][128];
};

template <int TS>
__global__ __launch_bounds__(TileCfg<TS>::NT) void replay_kernel(ReplayArgs a) {
    using Cfg = TileCfg<TS>;
    constexpr int NT = Cfg::NT, PPT = Cfg::PPT, NW = Cfg::NW;
    __shared__ ChunkLds<NT> ch;
    __shared__ ReplayQueue<NW> q;
    __shared__ uint64_t s_wmax[NW];
    __shared__ int s_wact[NW];
    __shared__ int64_t s_tile;

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const RasterArgs& r = a.r;

    for (;;) {
        if (tid == 0) s_tile = static_cast<int64_t>(atomicAdd(r.work, 1u));
        __syncthreads();
        const int64_t tile = uniform_i64(s_tile);
        __syncthreads();
        if (tile >= r.n_tiles) break;

        const int v = view_of_tile(r.views, r.V, tile);
        const ViewDesc& vd = r.views[v];
        const int W = vd.W, H = vd.H;
        const int64_t tl = tile - vd.tile_base;
        const int tx0 = static_cast<int>(tl % vd.tiles_x) * TS;
        const int ty0 = static_cast<int>(tl / vd.tiles_x) * TS;
        const TriRec* __restrict__ recs = uniform_ptr(r.recs + vd.rec_base);

        // per-pixel state: saved winner key; which fragments the pixel needs
        uint64_t kc[PPT];
        bool act[PPT], front[PPT];
        uint32_t pix[PPT];
        uint64_t wmax = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int pl = tid + k * NT;
            const int gx = tx0 + px_of<TS>(pl), gy = ty0 + py_of<TS>(pl);
            act[k] = false;
            front[k] = false;
            kc[k] = 0;
            pix[k] = 0;
            if (gx < W && gy < H) {
                const int64_t p = vd.pix_base + static_cast<int64_t>(gy) * W + gx;
                pix[k] = static_cast<uint32_t>(p);
                kc[k] = a.vis[p];
                if (a.all_front) {
                    act[k] = true;
                    front[k] = true;
                } else {
                    const float gl = (a.grad_logp && r.o.mode == 0) ? a.grad_logp[p] : 0.0f;
                    act[k] = gl != 0.0f || a.grad_color[3 * p] != 0.0f || a.grad_color[3 * p + 1] != 0.0f ||
                             a.grad_color[3 * p + 2] != 0.0f;
                    front[k] = gl != 0.0f;
                }
            }
            if (act[k]) wmax = kc[k] > wmax ? kc[k] : wmax;
        }
        bool any_act = false;
#pragma unroll
        for (int k = 0; k < PPT; ++k) any_act |= act[k];
        any_act = __ballot(any_act) != 0;
        wmax = wave_max_u64(wmax);

        // append the first n queue entries to the fragment list
        auto flush = [&](int n) __attribute__((always_inline)) {
            __threadfence_block();
            uint64_t base = 0;
            if (lane == 0) base = atomicAdd(a.frag_count, static_cast<unsigned long long>(n));
            base = static_cast<uint64_t>(uniform_i64(static_cast<int64_t>(__shfl(base, 0, 64))));
            const uint64_t slot = base + lane;
            if (lane < n && slot < a.frag_cap) {
                FragRec* f = a.frags + slot;
                f->a = make_uint4(q.pix[w][lane], q.tri[w][lane], __float_as_uint(q.b1[w][lane]),
                                  __float_as_uint(q.b2[w][lane]));
                f->b = make_uint4(__float_as_uint(q.beta[0][w][lane]), __float_as_uint(q.beta[1][w][lane]),
                                  __float_as_uint(q.beta[2][w][lane]), static_cast<uint32_t>(v));
            }
        };

        const int64_t beg = r.tile_start[tile], end = r.tile_start[tile + 1];
        int qn = 0;
        for (int64_t c0 = beg; c0 < end; c0 += NT) {
            const int n = static_cast<int>(min<int64_t>(NT, end - c0));
            if (lane == 0) {
                s_wmax[w] = any_act ? wmax : 0ull;
                s_wact[w] = any_act ? 1 : 0;
            }
            __syncthreads();
            uint64_t bmax = 0;
            int bact = 0;
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                bmax = s_wmax[i] > bmax ? s_wmax[i] : bmax;
                bact |= s_wact[i];
            }
            // stop when no pixel needs fragments, or when the rest of the list
            // lies behind every active pixel's winner
            if (!bact || remaining_min(r.entries, beg, c0, end) > bmax) break;
            if (tid < n) {
                const uint64_t e = r.entries[c0 + tid];
                load_slot<NT, TS>(ch, tid, e, recs[static_cast<uint32_t>(e)], tx0, ty0);
            }
            __syncthreads();
            if (any_act) {
                for (int j = 0; j < n; ++j) {
                    const uint64_t zk = (static_cast<uint64_t>(ch.zmin[j]) << 32) | ch.tri[j];
                    if (zk > wmax) break;
                    const uint32_t box =
                        static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(ch.box[j])));
#pragma unroll
                    for (int k = 0; k < PPT; ++k) {
                        if (!box_hits_block<TS>(box, w + k * NW)) continue;   // uniform: the wave's 8x8 block
                        const int pl = tid + k * NT;
                        Frag f;
                        bool cand = false, win = false;
                        float b1 = 0.f, b2 = 0.f;
                        if (act[k] && zk <= kc[k] && cover(ch, j, px_of<TS>(pl), py_of<TS>(pl), f) && f.key <= kc[k]) {
                            win = f.key == kc[k];
                            cand = win || front[k];
                            if (cand) persp_b(ch, j, f, b1, b2);
                        }
                        const uint64_t mk = __ballot(cand);
                        if (cand) {
                            const int pos = qn + __popcll(mk & lanemask_lt());
                            q.pix[w][pos] = pix[k];
                            q.tri[w][pos] = ch.tri[j] | (win ? 0x80000000u : 0u);
                            q.b1[w][pos] = b1;
                            q.b2[w][pos] = b2;
                            q.beta[0][w][pos] = f.beta[0];
                            q.beta[1][w][pos] = f.beta[1];
                            q.beta[2][w][pos] = f.beta[2];
                        }
                        qn += __popcll(mk);
                        if (qn >= 64) {
                            flush(64);
                            __threadfence_block();
                            if (lane < qn - 64) {
                                q.pix[w][lane] = q.pix[w][64 + lane];
                                q.tri[w][lane] = q.tri[w][64 + lane];
                                q.b1[w][lane] = q.b1[w][64 + lane];
                                q.b2[w][lane] = q.b2[w][64 + lane];
#pragma unroll
                                for (int i = 0; i < 3; ++i) q.beta[i][w][lane] = q.beta[i][w][64 + lane];
                            }
                            qn -= 64;
                            __threadfence_block();
                        }
                    }
                }
                if (qn > 0) {
                    flush(qn);
                    qn = 0;
                    __threadfence_block();
                }
            }
        }
        __syncthreads();
    }
}

void launch_replay(const ReplayArgs& a, int tile, hipStream_t s) {
    if (a.r.n_tiles <= 0) return;
    if (tile == 8)
        hipLaunchKernelGGL(replay_kernel<8>, dim3(a.n_blocks), dim3(TileCfg<8>::NT), 0, s, a);
    else if (tile == 32)
        hipLaunchKernelGGL(replay_kernel<32>, dim3(a.n_blocks), dim3(TileCfg<32>::NT), 0, s, a);
    else
        hipLaunchKernelGGL(replay_kernel<16>, dim3(a.n_blocks), dim3(TileCfg<16>::NT), 0, s, a);
}

}  // namespace soup
