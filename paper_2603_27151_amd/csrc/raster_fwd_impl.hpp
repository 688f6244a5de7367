#pragma once
// Forward raster: stochastic opacity masking with a 64-bit depth|triangle
// visibility buffer (Eq. (5); Supplement Algorithm A1, part 1).
//
// Persistent workgroups take screen tiles from a counter. A tile's triangle list (sorted by the
// lower bound of their depth) is staged through LDS in chunks; every lane
// tests its pixel(s) against each staged triangle with exact edge functions.
// A fragment whose key is below the pixel's current best key is a candidate:
// candidates are compacted per wave (ballot + prefix count) into an LDS queue
// and decoded 64 at a time, one per lane, so the expensive texture + MLP
// decode always runs on full waves. A decoded fragment that passes its draw
// lowers the pixel's key with an LDS 64-bit atomicMin; the lane holding the
// pixel's minimum then stores its colour. Triangles whose depth bound is
// already behind every pixel of a wave are skipped, and the tile stops once
// the remaining list is behind every pixel: front-to-back early-out without
// sorting fragments.
#include "raster_common.hpp"

namespace soup {

template <int NW>
struct FwdQueue {
    uint64_t key[NW][128];
    float beta[3][NW][128];   // screen barycentrics
    uint32_t info[NW][128];   // tile pixel | chunk slot << 10
};

template <int TS, class S>
__global__ __launch_bounds__(TileCfg<TS>::NT) void raster_fwd_kernel(RasterArgs a) {
    using Cfg = TileCfg<TS>;
    constexpr int NT = Cfg::NT, PPT = Cfg::PPT, NW = Cfg::NW;
    __shared__ ChunkLds<NT> ch;
    __shared__ FwdQueue<NW> q;
    __shared__ uint64_t s_key[TS * TS];
    __shared__ float s_rgb[TS * TS * 3];
    __shared__ uint64_t s_wmax[NW];
    __shared__ int64_t s_tile;

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int G = a.G;
    // optional log of every decoded fragment: this wave's region, private cursor
    const uint64_t log_base = (static_cast<uint64_t>(blockIdx.x) * NW + w) * a.log_region;
    uint32_t log_cursor = 0;   // wave-uniform

    for (;;) {   // persistent: tiles from a counter
    if (tid == 0) s_tile = static_cast<int64_t>(atomicAdd(a.work, 1u));
    __syncthreads();
    const int64_t tile = uniform_i64(s_tile);
    __syncthreads();
    if (tile >= a.n_tiles) break;
    const int v = view_of_tile(a.views, a.V, tile);
    const ViewDesc& vd = a.views[v];
    const int W = vd.W, H = vd.H;
    const int64_t tl = tile - vd.tile_base;
    const int tx0 = static_cast<int>(tl % vd.tiles_x) * TS;
    const int ty0 = static_cast<int>(tl / vd.tiles_x) * TS;
    const SceneDesc sc = a.scenes[vd.scene];
    gfloat* __restrict__ feats = as_global(uniform_ptr(sc.feats));
    const float* mlp_p = uniform_ptr(sc.mlp);
    const TriRec* __restrict__ recs = uniform_ptr(a.recs + vd.rec_base);

    uint64_t kc[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pl = tid + k * NT;
        const int gx = tx0 + px_of<TS>(pl), gy = ty0 + py_of<TS>(pl);
        kc[k] = (gx < W && gy < H) ? kBgKey : 0ull;   // pixels outside the view never take fragments
        s_key[pl] = kc[k];
    }
    uint64_t wmax = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) wmax = kc[k] > wmax ? kc[k] : wmax;
    wmax = wave_max_u64(wmax);

    // decode a batch of n queued candidates of this wave, one per lane
    auto run_batch = [&](int n) __attribute__((always_inline)) {
        __threadfence_block();
        const bool act = lane < n;
        uint64_t key = 0;
        int pl = 0;
        bool pass = false;
        float o[4] = {0.f, 0.f, 0.f, 0.f};
        if (act) {
            key = q.key[w][lane];
            const uint32_t info = q.info[w][lane];
            pl = static_cast<int>(info & 1023u);
            const int j = static_cast<int>(info >> 10);
            float b1, b2;
            persp_from_t(q.beta[0][w][lane] * ch.iw[0][j], q.beta[1][w][lane] * ch.iw[1][j],
                         q.beta[2][w][lane] * ch.iw[2][j], b1, b2);
            const uint32_t tri = static_cast<uint32_t>(key);
            const Cell c = cell_of(b1, b2, G);
            float x[S::C];
            fetch_feature<S::C>(feats, tri, G, c, x);
            // an opaque copy of the weight pointer per batch: the compiler may
            // not hoist the weights' scalar loads out of the traversal loops
            mlp_logits<S>(as_const(opaque_ptr(mlp_p)), x, o);
            if (a.o.mode == 0) {
                const float alpha = sigmoid_c(o[3]);
                const uint32_t pidx = static_cast<uint32_t>((ty0 + py_of<TS>(pl)) * W + tx0 + px_of<TS>(pl));
                pass = uniform24(a.o.seed, pidx, tri, vd.view_id, a.o.step) < alpha;
            } else {
                pass = o[3] > 0.0f;
            }
            if (pass) atomicMin(reinterpret_cast<unsigned long long*>(&s_key[pl]), static_cast<unsigned long long>(key));
            if (a.log_frag) {
                const uint32_t at = log_cursor + static_cast<uint32_t>(lane);
                if (at < a.log_region) {
                    const int64_t pg = vd.pix_base + static_cast<int64_t>(ty0 + py_of<TS>(pl)) * W + tx0 + px_of<TS>(pl);
                    a.log_frag[log_base + at] =
                        make_uint4(static_cast<uint32_t>(pg), tri, __float_as_uint(b1), __float_as_uint(b2));
                    a.log_aux[log_base + at] = make_uint2(static_cast<uint32_t>(key >> 32), static_cast<uint32_t>(v));
                }
            }
        }
        if (a.log_frag) log_cursor += static_cast<uint32_t>(n);
        __threadfence_block();
        if (pass && s_key[pl] == key) {
            s_rgb[3 * pl + 0] = sigmoid_c(o[0]);
            s_rgb[3 * pl + 1] = sigmoid_c(o[1]);
            s_rgb[3 * pl + 2] = sigmoid_c(o[2]);
        }
        if (a.counter && lane == 0) atomicAdd(a.counter, static_cast<unsigned long long>(n));
        __threadfence_block();
    };
    auto refresh = [&]() __attribute__((always_inline)) {
        uint64_t m = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            kc[k] = s_key[tid + k * NT];
            m = kc[k] > m ? kc[k] : m;
        }
        wmax = wave_max_u64(m);
    };

    const int64_t beg = a.tile_start[tile], end = a.tile_start[tile + 1];
    int qn = 0;
    for (int64_t c0 = beg; c0 < end; c0 += NT) {
        const int n = static_cast<int>(min<int64_t>(NT, end - c0));
        if (lane == 0) s_wmax[w] = wmax;
        __syncthreads();
        uint64_t bmax = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) bmax = s_wmax[i] > bmax ? s_wmax[i] : bmax;
        if (remaining_min(a.entries, beg, c0, end) >= bmax) break;
        if (tid < n) {
            const uint64_t e = a.entries[c0 + tid];
            load_slot<NT, TS>(ch, tid, e, recs[static_cast<uint32_t>(e)], tx0, ty0);
        }
        __syncthreads();
        for (int j = 0; j < n; ++j) {
            const uint64_t zk = (static_cast<uint64_t>(ch.zmin[j]) << 32) | ch.tri[j];
            if (zk >= wmax) break;   // sorted: nothing further can beat any pixel of this wave
            const uint32_t box = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(ch.box[j])));
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!box_hits_block<TS>(box, w + k * NW)) continue;   // uniform: the wave's 8x8 block
                const int pl = tid + k * NT;
                double e[3];
                const bool in = (zk < kc[k]) & edge_inside(ch, j, px_of<TS>(pl), py_of<TS>(pl), e);
                if (__ballot(in) == 0) continue;   // uniform: no pixel of the wave is covered
                Frag f;
                frag_of(ch, j, e, f);
                const bool cand = in & (f.key < kc[k]);
                const uint64_t m = __ballot(cand);
                if (cand) {
                    const int pos = qn + __popcll(m & lanemask_lt());
                    q.key[w][pos] = f.key;
#pragma unroll
                    for (int i = 0; i < 3; ++i) q.beta[i][w][pos] = f.beta[i];
                    q.info[w][pos] = static_cast<uint32_t>(pl) | (static_cast<uint32_t>(j) << 10);
                }
                qn += __popcll(m);
                if (qn >= 64) {
                    run_batch(64);
                    if (lane < qn - 64) {
                        q.key[w][lane] = q.key[w][64 + lane];
#pragma unroll
                        for (int i = 0; i < 3; ++i) q.beta[i][w][lane] = q.beta[i][w][64 + lane];
                        q.info[w][lane] = q.info[w][64 + lane];
                    }
                    qn -= 64;
                    refresh();
                }
            }
        }
        if (qn > 0) {
            run_batch(qn);
            qn = 0;
            refresh();
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pl = tid + k * NT;
        const int gx = tx0 + px_of<TS>(pl), gy = ty0 + py_of<TS>(pl);
        if (gx >= W || gy >= H) continue;
        const uint64_t key = s_key[pl];
        const int64_t off = static_cast<int64_t>(gy) * W + gx;
        float* col = vd.color_out ? vd.color_out + 3 * off : a.color + 3 * (vd.pix_base + off);
        if (vd.vis_out) vd.vis_out[off] = key;
        else if (a.vis) a.vis[vd.pix_base + off] = key;
        if (key == kBgKey) {
            col[0] = a.o.bg[0];
            col[1] = a.o.bg[1];
            col[2] = a.o.bg[2];
        } else {
            col[0] = s_rgb[3 * pl + 0];
            col[1] = s_rgb[3 * pl + 1];
            col[2] = s_rgb[3 * pl + 2];
        }
    }
    }   // tiles
    if (a.log_counts && lane == 0) a.log_counts[blockIdx.x * NW + w] = log_cursor;
}

template <int TS, class S>
static void launch_fwd_t(const RasterArgs& a, hipStream_t s) {
    if (a.n_tiles <= 0 || a.n_blocks <= 0) return;
    hipLaunchKernelGGL((raster_fwd_kernel<TS, S>), dim3(static_cast<unsigned>(a.n_blocks)), dim3(TileCfg<TS>::NT), 0,
                       s, a);
}


}  // namespace soup
