// Backward, part 1 (Supplement Algorithm A1, part 2): re-find, from the saved
// visibility buffer, every fragment the backward needs -- the winner of each
// pixel with a colour gradient, and, where the pixel carries a score weight,
// every fragment in front of it (Eq. (9)).
//
// Persistent workgroups take screen tiles from a counter and walk the tile's
// depth-sorted triangle list with the forward's exact coverage test, in the
// forward's order, stopping where the rest of the list lies behind every
// active pixel's winner. Each wave compacts its candidates in LDS and appends
// them, 64 at a time, to its own region of the fragment list with a private
// cursor (no shared counter). No MLP work happens here: the list is decoded
// by the decode kernel, whose registers then hold only the MLP state, and
// whose waves are always full.
#include "raster_common.hpp"

namespace soup {

template <int NW>
struct ReplayQueue {
    uint32_t pix[NW][128];
    uint32_t tri[NW][128];     // triangle | winner << 31
    float t[3][NW][128];       // beta_i / w_i
    float gl[NW][128];         // the pixel's score weight
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
    const uint64_t region_base = (static_cast<uint64_t>(blockIdx.x) * NW + w) * a.region;
    uint32_t cursor = 0;   // wave-uniform

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
        float gp[PPT][6];   // g_L, g_C, edge weights (x, y) of the pixel
        uint64_t wmax = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int pl = tid + k * NT;
            const int gx = tx0 + px_of<TS>(pl), gy = ty0 + py_of<TS>(pl);
            act[k] = false;
            front[k] = false;
            kc[k] = 0;
            pix[k] = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i) gp[k][i] = 0.0f;
            if (gx < W && gy < H) {
                const int64_t p = vd.pix_base + static_cast<int64_t>(gy) * W + gx;
                pix[k] = static_cast<uint32_t>(p);
                kc[k] = a.vis[p];
                if (a.all_front) {
                    act[k] = true;
                    front[k] = true;
                } else {
                    gp[k][0] = (a.grad_logp && r.o.mode == 0) ? a.grad_logp[p] : 0.0f;
#pragma unroll
                    for (int i = 0; i < 3; ++i) gp[k][1 + i] = a.grad_color[3 * p + i];
                    if (a.edge_w && kc[k] != kBgKey) {   // written for covered pixels only
                        const float2 e = a.edge_w[p];
                        gp[k][4] = e.x;
                        gp[k][5] = e.y;
                    }
                    act[k] = gp[k][0] != 0.0f || gp[k][1] != 0.0f || gp[k][2] != 0.0f || gp[k][3] != 0.0f ||
                             gp[k][4] != 0.0f || gp[k][5] != 0.0f;
                    front[k] = gp[k][0] != 0.0f;
                }
            }
            if (act[k]) wmax = kc[k] > wmax ? kc[k] : wmax;
        }
        bool any_act = false;
#pragma unroll
        for (int k = 0; k < PPT; ++k) any_act |= act[k];
        any_act = __ballot(any_act) != 0;
        wmax = wave_max_u64(wmax);

        // append the first n queue entries to this wave's region
        auto flush = [&](int n) __attribute__((always_inline)) {
            __threadfence_block();
            const uint32_t at = cursor + static_cast<uint32_t>(lane);
            if (lane < n && at < a.region) {
                float b1, b2;   // the perspective division, on full batches
                persp_from_t(q.t[0][w][lane], q.t[1][w][lane], q.t[2][w][lane], b1, b2);
                FragRec* f = a.frags + region_base + at;
                f->p0 = make_uint2(q.pix[w][lane], q.tri[w][lane]);
                f->p1 = make_uint2(__float_as_uint(b1), __float_as_uint(b2));
                f->x = make_uint2(__float_as_uint(q.gl[w][lane]), static_cast<uint32_t>(v));
            }
            // fragments per triangle, counting only those stored (one atomic
            // per run of equal triangles)
            if (a.tri_count) {
                const bool stored = lane < n && at < a.region;
                const uint32_t tk = stored ? (q.tri[w][lane] & 0x7FFFFFFFu) : 0xFFFFFFFFu;
                const uint32_t tp = __shfl_up(tk, 1, 64);
                const bool head = lane == 0 || tp != tk;
                const uint64_t heads = __ballot(head);
                if (head && stored) {
                    const uint64_t above = lane == 63 ? 0ull : (heads & (~0ull << (lane + 1)));
                    const int endl = above ? __builtin_ctzll(above) : 64;   // the run ends at the next head
                    atomicAdd(&a.tri_count[tk], endl - lane);
                }
            }
            cursor += static_cast<uint32_t>(n);
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
                        double e[3];
                        const bool in =
                            act[k] & (zk <= kc[k]) & edge_inside(ch, j, px_of<TS>(pl), py_of<TS>(pl), e);
                        if (__ballot(in) == 0) continue;   // uniform: no pixel of the wave is covered
                        Frag f;
                        frag_of(ch, j, e, f);
                        const bool le = in & (f.key <= kc[k]);
                        const bool win = le & (f.key == kc[k]);
                        const bool cand = win | (le & front[k]);
                        const uint64_t mk = __ballot(cand);
                        if (cand) {
                            const int pos = qn + __popcll(mk & lanemask_lt());
                            q.pix[w][pos] = pix[k];
                            q.tri[w][pos] = ch.tri[j] | (win ? 0x80000000u : 0u);
#pragma unroll
                            for (int i = 0; i < 3; ++i) q.t[i][w][pos] = f.beta[i] * ch.iw[i][j];
                            q.gl[w][pos] = gp[k][0];
                        }
                        qn += __popcll(mk);
                        if (qn >= 64) {
                            flush(64);
                            __threadfence_block();
                            if (lane < qn - 64) {
                                q.pix[w][lane] = q.pix[w][64 + lane];
                                q.tri[w][lane] = q.tri[w][64 + lane];
#pragma unroll
                                for (int i = 0; i < 3; ++i) q.t[i][w][lane] = q.t[i][w][64 + lane];
                                q.gl[w][lane] = q.gl[w][64 + lane];
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
    if (lane == 0) a.counts[blockIdx.x * NW + w] = cursor;
}

// One workgroup of 1024 threads, n <= kMaxRegions: each thread scans four
// consecutive regions, then the per-thread sums are scanned in LDS.
__global__ __launch_bounds__(1024) void region_scan_kernel(const uint32_t* __restrict__ counts, int n,
                                                           uint32_t region, uint32_t* __restrict__ boff,
                                                           unsigned long long* __restrict__ summary,
                                                           unsigned int* __restrict__ sticky) {
    constexpr int kPer = kMaxRegions / 1024;
    __shared__ uint32_t s_sum[1024];
    __shared__ unsigned long long s_tot[1024];
    __shared__ uint32_t s_max[1024];
    const int t = threadIdx.x;
    uint32_t nb[kPer];
    uint32_t local = 0, mx = 0;
    unsigned long long tot = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int r = t * kPer + i;
        const uint32_t c = r < n ? counts[r] : 0u;
        const uint32_t cl = c < region ? c : region;
        nb[i] = (cl + 63u) / 64u;
        local += nb[i];
        tot += c;
        mx = c > mx ? c : mx;
    }
    s_sum[t] = local;
    s_tot[t] = tot;
    s_max[t] = mx;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread batch counts
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = t >= d ? s_sum[t - d] : 0u;
        __syncthreads();
        s_sum[t] += v;
        __syncthreads();
    }
    uint32_t run = s_sum[t] - local;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int r = t * kPer + i;
        if (r < n) boff[r] = run;
        run += nb[i];
    }
    if (t == 1023) boff[n] = s_sum[1023];
    for (int d = 512; d > 0; d >>= 1) {
        if (t < d) {
            s_tot[t] += s_tot[t + d];
            s_max[t] = s_max[t + d] > s_max[t] ? s_max[t + d] : s_max[t];
        }
        __syncthreads();
    }
    if (t == 0) {
        summary[0] = s_tot[0];
        summary[1] = s_sum[1023];
        summary[2] = s_max[0];
        if (sticky && s_max[0] > region) atomicOr(sticky, kOverflowFragments);
    }
}

void launch_region_scan(const uint32_t* counts, int n, uint32_t region, uint32_t* boff,
                        unsigned long long* summary, unsigned int* sticky, hipStream_t s) {
    hipLaunchKernelGGL(region_scan_kernel, dim3(1), dim3(1024), 0, s, counts, n, region, boff, summary, sticky);
}

// Persistent waves take batches of the region list (as the logp decode
// does). Triangle t's winners go to sorted[tri_off[t] + k] and its other
// fragments to sorted[tri_off[t + 1] - 1 - k], k from a per-triangle pair of
// fill counters (one 64-bit atomic per run of equal triangles among
// consecutive lanes).
__global__ __launch_bounds__(256) void place_kernel(PlaceArgs a) {
    __shared__ uint32_t s_boff[kMaxRegions + 1];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i <= a.n_regions; i += blockDim.x) s_boff[i] = a.boff[i];
    __syncthreads();
    const uint32_t n_batch = s_boff[a.n_regions];
    const uint32_t n_waves = gridDim.x * 4;
    for (uint32_t bi = blockIdx.x * 4 + w; bi < n_batch; bi += n_waves) {
        int lo = 0, hi = a.n_regions - 1;   // region: last w with boff[w] <= bi
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_boff[mid] <= bi) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t cr = a.counts[lo];
        const uint32_t in_region = (bi - s_boff[lo]) * 64u + static_cast<uint32_t>(lane);
        const bool on = in_region < (cr < a.region ? cr : a.region);
        FragRec fr = {make_uint2(0u, 0u), make_uint2(0u, 0u), make_uint2(0u, 0u)};
        if (on) fr = a.frags[static_cast<uint64_t>(lo) * a.region + in_region];
        const uint32_t tri = on ? (fr.p0.y & 0x7FFFFFFFu) : 0xFFFFFFFFu;
        const bool win = on && (fr.p0.y >> 31);
        const uint32_t tprev = __shfl_up(tri, 1, 64);
        const bool head = lane == 0 || tprev != tri;
        const uint64_t heads = __ballot(head);
        const uint64_t wins = __ballot(win);
        const uint64_t upto = lane == 63 ? heads : (heads & ((2ull << lane) - 1));
        const int hl = 63 - __builtin_clzll(upto);   // lane 0 is always a head: this lane's run starts at hl
        const uint64_t above = lane == 63 ? 0ull : (heads & (~0ull << (lane + 1)));
        const int endl = above ? __builtin_ctzll(above) : 64;
        // the run [hl, end): winners before this lane, winners in the whole run
        const uint64_t run_lo = (hl == 0 ? ~0ull : (~0ull << hl));
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        const int w_before = __popcll(wins & run_lo & below);
        unsigned long long base = 0;
        if (head && on) {
            const uint64_t run = run_lo & (endl == 64 ? ~0ull : ((1ull << endl) - 1));
            const unsigned long long nw = static_cast<unsigned long long>(__popcll(wins & run));
            const unsigned long long nf = static_cast<unsigned long long>(endl - lane) - nw;
            base = atomicAdd(&a.tri_fill[tri], nw | (nf << 32));
        }
        const unsigned long long hb = __shfl(base, hl, 64);
        if (on) {
            const int64_t dst = win ? a.tri_off[tri] + static_cast<int64_t>(hb & 0xFFFFFFFFull) + w_before
                                    : a.tri_off[tri + 1] - 1 - static_cast<int64_t>(hb >> 32) - ((lane - hl) - w_before);
            a.sorted[dst] = fr;
            if (a.frag_gates) {   // 8-byte units of the padded gate record
                const uint64_t src = static_cast<uint64_t>(lo) * a.region + in_region;
                const int g2 = gate_stride(a.gate_words) / 2;
                const uint2* gs = reinterpret_cast<const uint2*>(a.frag_gates) + src * g2;
                uint2* gd = reinterpret_cast<uint2*>(a.sorted_gates) + static_cast<uint64_t>(dst) * g2;
                for (int w = 0; w < g2; ++w) gd[w] = gs[w];
            }
        }
    }
}

void launch_place(const PlaceArgs& a, hipStream_t s) {
    if (a.n_blocks <= 0) return;
    hipLaunchKernelGGL(place_kernel, dim3(a.n_blocks), dim3(256), 0, s, a);
}

// Persistent waves take batches of the forward's log (region by region, as
// the place kernel does) and keep the fragments the backward needs: the
// pixel's winner (key == the saved key), and every fragment in front of it
// (key < the saved key) when the pixel carries a score weight. Kept
// fragments are compacted per batch and appended to the wave's output
// region; per-triangle counts as in the replay.
__global__ __launch_bounds__(256) void collect_kernel(CollectArgs a) {
    __shared__ uint32_t s_boff[kMaxRegions + 1];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i <= a.log_regions; i += blockDim.x) s_boff[i] = a.log_boff[i];
    __syncthreads();
    const uint32_t n_batch = s_boff[a.log_regions];
    const uint32_t n_waves = gridDim.x * 4;
    const uint32_t wid = blockIdx.x * 4 + w;
    const uint64_t out_base = static_cast<uint64_t>(wid) * a.region;
    uint32_t cursor = 0;   // wave-uniform
    for (uint32_t bi = wid; bi < n_batch; bi += n_waves) {
        int lo = 0, hi = a.log_regions - 1;   // region: last w with boff[w] <= bi
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_boff[mid] <= bi) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t cr = a.log_counts[lo];
        const uint32_t in_region = (bi - s_boff[lo]) * 64u + static_cast<uint32_t>(lane);
        const bool on = in_region < (cr < a.log_region ? cr : a.log_region);
        bool keep = false, win = false;
        FragRec fr = {make_uint2(0u, 0u), make_uint2(0u, 0u), make_uint2(0u, 0u)};
        if (on) {
            const uint64_t at = static_cast<uint64_t>(lo) * a.log_region + in_region;
            const uint4 e = a.log_frag[at];
            const int aw2 = aux_words(a.gate_words) / 2;
            const uint2 x = a.log_aux[at * aw2];
            const uint64_t key = (static_cast<uint64_t>(x.x) << 32) | e.y;
            const uint64_t kstar = a.vis[e.x];
            win = key == kstar;
            const bool front = key < kstar;
            // every winner (its colour gradient and edge weights are read by the
            // decode; a winner without any adds zeros), and the fragments in front
            // of it where the pixel carries a score weight
            const float gl = (!a.all_front && a.grad_logp) ? a.grad_logp[e.x] : 0.0f;
            keep = win || (front && (a.all_front || gl != 0.0f));
            fr.p0 = make_uint2(e.x, e.y | (win ? 0x80000000u : 0u));
            fr.p1 = make_uint2(e.z, e.w);
            fr.x = make_uint2(__float_as_uint(gl), x.y);
        }
        const uint64_t km = __ballot(keep);
        const uint32_t pos = cursor + static_cast<uint32_t>(__popcll(km & lanemask_lt()));
        if (keep && pos < a.region) {
            a.frags[out_base + pos] = fr;
            if (a.frag_gates) {   // the aux record's gates (words 2.., zero-padded to even) as 8-byte units
                const uint64_t at = static_cast<uint64_t>(lo) * a.log_region + in_region;
                const int g2 = gate_stride(a.gate_words) / 2;
                const uint2* g = a.log_aux + at * (aux_words(a.gate_words) / 2) + 1;
                uint2* gd = reinterpret_cast<uint2*>(a.frag_gates) + (out_base + pos) * g2;
                for (int w = 0; w < g2; ++w) gd[w] = g[w];
            }
        }
        // fragments per triangle, counting only those stored (one atomic per
        // run of equal triangles among consecutive lanes)
        if (a.tri_count) {
            const bool stored = keep && pos < a.region;
            const uint32_t tk = stored ? (fr.p0.y & 0x7FFFFFFFu) : 0xFFFFFFFFu;
            const uint32_t tp = __shfl_up(tk, 1, 64);
            const bool head = lane == 0 || tp != tk;
            const uint64_t heads = __ballot(head);
            if (head && stored) {
                const uint64_t above = lane == 63 ? 0ull : (heads & (~0ull << (lane + 1)));
                const int endl = above ? __builtin_ctzll(above) : 64;
                atomicAdd(&a.tri_count[tk], endl - lane);
            }
        }
        cursor += static_cast<uint32_t>(__popcll(km));
    }
    if (lane == 0) a.counts[wid] = cursor;
}

void launch_collect(const CollectArgs& a, hipStream_t s) {
    if (a.n_blocks <= 0) return;
    hipLaunchKernelGGL(collect_kernel, dim3(a.n_blocks), dim3(256), 0, s, a);
}

int replay_waves_per_block(int tile) { return TileCfg<8>::NW * (tile == 8) + TileCfg<16>::NW * (tile != 8); }

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
