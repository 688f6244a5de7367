#pragma once
// Backward raster (Supplement Algorithm A1, part 2; Eq. (8), (9)) and the
// edge term of Section 3.2, recomputing fragments from the saved visibility
// buffer.
//
// raster_bwd: persistent workgroups take screen tiles from a counter. For a
//   tile, every fragment whose key is <= the pixel's saved winner key is
//   re-found by the same exact coverage test as the forward (the winner
//   itself and every fragment in front of it), compacted per wave into an LDS
//   queue and processed 64 per wave:
//     - recompute the bilinear feature and the MLP (float32, as the forward);
//     - logit gradients: winner -> colour path g_C sigma'(o_rgb) and score
//       g_L (1 - alpha); fragment in front -> score -g_L alpha (Eq. (9)
//       through the sigmoid);
//     - back-propagate through the MLP; the weight gradient sum_f delta_f a_f^T
//       is accumulated in registers: each lane owns 4x4 blocks of every weight
//       matrix and reads the batch's activations and deltas transposed from
//       LDS; each wave writes its sums once, at the end, to its own row of a
//       partial-sum buffer (no atomics; rows are reduced in a fixed order);
//     - feature gradients scatter to the four texels (float atomics);
//     - for the winner, the texture-position gradient goes back through the
//       perspective-correct and screen barycentrics to the screen positions
//       and 1/w of the triangle's vertices (per-record accumulators).
//   A logp variant of the same kernel sums log(1 - alpha) over the front set
//   and log(alpha) of the winner per pixel (log p(f*) of Eq. (6)).
// edge: one thread per pixel, pairs (x, x+1) and (y, y+1): w = 1/2 (g_a+g_b).
//   (C_a - C_b) goes to the nearer pixel's triangle as moments sum w,
//   sum w dx, sum w dy about its vertex 0, per direction (the barycentric
//   weight is affine in the pixel position, so these moments carry it
//   exactly).
// vertex_chain: one thread per triangle, loop over views: moments -> screen
//   gradients of the vertices, then screen/1-w -> clip -> world through the
//   view-projection, summed over views in a fixed order.
#include "raster_common.hpp"

namespace soup {

constexpr int kStageRows = 16;   // fragments staged per transpose pass

template <class S>
struct StageCfg {
    static constexpr int kMax2(int a, int b) { return a > b ? a : b; }
    static constexpr int kWidth = kMax2(kMax2(S::C + S::H, 2 * S::H), S::H + 4);
};

typedef float f4v __attribute__((ext_vector_type(4)));

// Accumulators of one layer's weight gradient dW[DOUT][DIN] += sum_f d_f a_f^T
// on the matrix cores: the contraction runs over fragments, four per
// v_mfma_f32_16x16x4f32 (A[m][k] = d[f_k][m], B[k][n] = a[f_k][n]); dW is
// tiled in 16x16 blocks held in registers (4 per lane per block), padded
// with zeros where DIN or DOUT is below 16. Lane j < DOUT owns db_j.
template <int DIN, int DOUT>
struct LayerAcc {
    static constexpr int BI = (DIN + 15) / 16;
    static constexpr int BO = (DOUT + 15) / 16;
    static constexpr int NB = BI * BO;
    static_assert(DOUT <= 64, "bias ownership assumes DOUT <= 64");
    f4v w[NB];
    float b;
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int i = 0; i < NB; ++i) w[i] = f4v{0.f, 0.f, 0.f, 0.f};
        b = 0.0f;
    }
    // kStageRows (16) staged fragments: in[r][DIN] and d[r][DOUT] in LDS
    __device__ __forceinline__ void accumulate(const float* __restrict__ in, const float* __restrict__ d, int lane) {
        const int col = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < kStageRows / 4; ++kk) {
            const int r = 4 * kk + kq;
            float av[BO], bv[BI];
#pragma unroll
            for (int bo = 0; bo < BO; ++bo) {
                const int m = 16 * bo + col;
                av[bo] = m < DOUT ? d[r * DOUT + m] : 0.0f;
            }
#pragma unroll
            for (int bi = 0; bi < BI; ++bi) {
                const int n = 16 * bi + col;
                bv[bi] = n < DIN ? in[r * DIN + n] : 0.0f;
            }
#pragma unroll
            for (int bo = 0; bo < BO; ++bo)
#pragma unroll
                for (int bi = 0; bi < BI; ++bi)
                    w[bo * BI + bi] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bo], bv[bi], w[bo * BI + bi], 0, 0, 0);
        }
        if (lane < DOUT) {
#pragma unroll
            for (int r = 0; r < kStageRows; ++r) b += d[r * DOUT + lane];
        }
    }
    // D of a 16x16 block: lane l holds column l % 16, rows 4 (l / 16) + i
    __device__ __forceinline__ void store(float* __restrict__ row, int w_off, int b_off, int lane) const {
#pragma unroll
        for (int bo = 0; bo < BO; ++bo)
#pragma unroll
            for (int bi = 0; bi < BI; ++bi)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = 16 * bo + 4 * (lane >> 4) + i, n = 16 * bi + (lane & 15);
                    if (m < DOUT && n < DIN) row[w_off + m * DIN + n] = w[bo * BI + bi][i];
                }
        if (lane < DOUT) row[b_off + lane] = b;
    }
};

// Stage the activations (in) and deltas (dl) of the wave's 64 fragments
// through LDS, kStageRows at a time, and accumulate them on the matrix cores.
template <int DIN, int DOUT>
__device__ __forceinline__ void stage_accumulate(LayerAcc<DIN, DOUT>& la, float* __restrict__ st,
                                                 const float (&in)[DIN], const float (&dl)[DOUT], int lane) {
#pragma unroll
    for (int half = 0; half < 64; half += kStageRows) {
        if (lane >= half && lane < half + kStageRows) {
            float* row = st + (lane - half) * DIN;
#pragma unroll
            for (int k = 0; k < DIN; k += 4) *reinterpret_cast<float4*>(row + k) = make_float4(in[k], in[k + 1], in[k + 2], in[k + 3]);
            float* drow = st + kStageRows * DIN + (lane - half) * DOUT;
#pragma unroll
            for (int k = 0; k < DOUT; k += 4)
                *reinterpret_cast<float4*>(drow + k) = make_float4(dl[k], dl[k + 1], dl[k + 2], dl[k + 3]);
        }
        __threadfence_block();
        la.accumulate(st, st + kStageRows * DIN, lane);
        __threadfence_block();
    }
}

template <class S>
struct MlpGrad {
    LayerAcc<S::C, S::H> l0;
    LayerAcc<S::H, S::H> mid[S::NH > 1 ? S::NH - 1 : 1];
    LayerAcc<S::H, 4> out;
};

template <int NW>
struct BwdQueue {
    uint32_t info[NW][128];   // pixel | slot << 10 | winner << 31
    float b1[NW][128];
    float b2[NW][128];
    float beta[3][NW][128];   // screen barycentrics found by the coverage test
};

template <int TS, class S, bool LOGP>
__global__ __launch_bounds__(TileCfg<TS>::NT) void raster_bwd_kernel(BwdArgs a) {
    using Cfg = TileCfg<TS>;
    constexpr int NT = Cfg::NT, PPT = Cfg::PPT, NW = Cfg::NW;
    constexpr int SW = StageCfg<S>::kWidth;
    __shared__ ChunkLds<NT> ch;
    __shared__ BwdQueue<NW> q;
    __shared__ uint64_t s_key[TS * TS];
    __shared__ float s_gc[TS * TS * 3];
    __shared__ float s_gl[TS * TS];
    __shared__ __align__(16) float s_stage[LOGP ? 1 : NW][LOGP ? 4 : kStageRows * SW];
    __shared__ uint64_t s_wmax[NW];
    __shared__ int s_wact[NW];
    __shared__ int64_t s_tile;

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const RasterArgs& r = a.r;
    const int G = r.G;

    MlpGrad<S> acc;
    if (!LOGP) {
        acc.l0.zero();
        if constexpr (S::NH == 2) acc.mid[0].zero();
        acc.out.zero();
    }

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
        const SceneDesc sc = r.scenes[vd.scene];
        gfloat* __restrict__ feats = as_global(uniform_ptr(sc.feats));
        cfloat* __restrict__ mlp = as_const(uniform_ptr(sc.mlp));
        const TriRec* __restrict__ recs = uniform_ptr(r.recs + vd.rec_base);

        // per-pixel state: saved winner key, upstream gradients
        uint64_t kc[PPT];
        bool act[PPT], front[PPT];
        uint64_t wmax = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int pl = tid + k * NT;
            const int gx = tx0 + px_of<TS>(pl), gy = ty0 + py_of<TS>(pl);
            act[k] = false;
            front[k] = false;
            kc[k] = 0;
            float g0 = 0.f, g1 = 0.f, g2 = 0.f, gl = 0.f;
            if (gx < W && gy < H) {
                const int64_t p = vd.pix_base + static_cast<int64_t>(gy) * W + gx;
                kc[k] = a.vis[p];
                if (LOGP) {
                    act[k] = true;
                    front[k] = true;
                } else {
                    g0 = a.grad_color[3 * p];
                    g1 = a.grad_color[3 * p + 1];
                    g2 = a.grad_color[3 * p + 2];
                    gl = (a.grad_logp && r.o.mode == 0) ? a.grad_logp[p] : 0.0f;
                    act[k] = g0 != 0.0f || g1 != 0.0f || g2 != 0.0f || gl != 0.0f;
                    front[k] = gl != 0.0f;
                }
            }
            s_key[pl] = kc[k];
            s_gc[3 * pl] = g0;
            s_gc[3 * pl + 1] = g1;
            s_gc[3 * pl + 2] = g2;
            s_gl[pl] = gl;
            if (act[k]) wmax = kc[k] > wmax ? kc[k] : wmax;
        }
        bool any_act = false;
#pragma unroll
        for (int k = 0; k < PPT; ++k) any_act |= act[k];
        any_act = __ballot(any_act) != 0;
        wmax = wave_max_u64(wmax);

        auto run_batch = [&](int n) __attribute__((always_inline)) {
            __threadfence_block();
            const bool on = lane < n;
            uint32_t info = on ? q.info[w][lane] : 0u;
            const int pl = info & 1023u;
            const int j = (info >> 10) & 255u;
            const bool win = (info >> 31) & 1u;
            const float b1 = on ? q.b1[w][lane] : 0.f, b2 = on ? q.b2[w][lane] : 0.f;
            const uint32_t tri = on ? ch.tri[j] : 0u;
            const Cell c = cell_of(b1, b2, G);
            float x[S::C];
            MlpAct<S> m;
            if (on) {
                fetch_feature<S::C>(feats, tri, G, c, x);
            } else {
#pragma unroll
                for (int k = 0; k < S::C; ++k) x[k] = 0.0f;
            }
            mlp_forward<S>(mlp, x, m);
            const float alpha = sigmoid_c(m.o[3]);
            if (r.counter && lane == 0) atomicAdd(r.counter, static_cast<unsigned long long>(n));
            if (LOGP) {
                if (on && r.o.mode == 0) atomicAdd(&s_gl[pl], win ? logf(alpha) : log1pf(-alpha));
                return;
            }
            float d[4] = {0.f, 0.f, 0.f, 0.f};
            if (on) {
                const float gl = s_gl[pl];
                if (win) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const float s = sigmoid_c(m.o[k]);
                        d[k] = s_gc[3 * pl + k] * s * (1.0f - s);
                    }
                    d[3] = gl * (1.0f - alpha);
                } else {
                    d[3] = -gl * alpha;
                }
            }
            // --- MLP backward, output layer first ---
            float* st = s_stage[w];
            float dh[S::H];
#pragma unroll
            for (int k = 0; k < S::H; ++k) {
                cfloat* Wk = mlp + S::w_off(S::NH) + k;
                float s = 0.0f;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) s = __builtin_fmaf(Wk[jj * S::H], d[jj], s);
                dh[k] = m.h[S::NH - 1][k] > 0.0f ? s : 0.0f;
            }
            stage_accumulate<S::H, 4>(acc.out, st, m.h[S::NH - 1], d, lane);
            // hidden layer 1 -> 0 (the compiled shapes have one or two hidden layers)
            static_assert(S::NH == 1 || S::NH == 2, "one or two hidden layers");
            if constexpr (S::NH == 2) {
                float dprev[S::H];
#pragma unroll
                for (int k = 0; k < S::H; ++k) {
                    float s = 0.0f;
#pragma unroll
                    for (int jj = 0; jj < S::H; ++jj) s = __builtin_fmaf(mlp[S::w_off(1) + jj * S::H + k], dh[jj], s);
                    dprev[k] = m.h[0][k] > 0.0f ? s : 0.0f;
                }
                stage_accumulate<S::H, S::H>(acc.mid[0], st, m.h[0], dh, lane);
#pragma unroll
                for (int k = 0; k < S::H; ++k) dh[k] = dprev[k];
            }
            float dx[S::C];
#pragma unroll
            for (int k = 0; k < S::C; ++k) {
                float s = 0.0f;
#pragma unroll
                for (int jj = 0; jj < S::H; ++jj) s = __builtin_fmaf(mlp[S::w_off(0) + jj * S::C + k], dh[jj], s);
                dx[k] = s;
            }
            stage_accumulate<S::C, S::H>(acc.l0, st, x, dh, lane);
            // --- one record per fragment: texture cell, position, feature gradient
            //     and, for the winner, its world-space vertex gradient ---
            float gw[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (on && win) {
                const size_t t00 = ((static_cast<size_t>(tri) * G + c.iy) * G + c.ix) * S::C;
                const size_t t10 = t00 + S::C, t01 = t00 + static_cast<size_t>(G) * S::C, t11 = t01 + S::C;
                // texture position -> barycentrics -> vertex screen positions and 1/w
                float dfx = 0.f, dfy = 0.f;
#pragma unroll
                for (int k = 0; k < S::C; ++k) {
                    const float T00 = feats[t00 + k], T10 = feats[t10 + k], T01 = feats[t01 + k], T11 = feats[t11 + k];
                    dfx = __builtin_fmaf(dx[k], (1.0f - c.fy) * (T10 - T00) + c.fy * (T11 - T01), dfx);
                    dfy = __builtin_fmaf(dx[k], (1.0f - c.fx) * (T01 - T00) + c.fx * (T11 - T10), dfy);
                }
                const float gm1 = static_cast<float>(G - 1);
                const int lx = px_of<TS>(pl), ly = py_of<TS>(pl);
                const float fb[3] = {q.beta[0][w][lane], q.beta[1][w][lane], q.beta[2][w][lane]};
                float tt[3], S3 = 0.f;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    tt[i] = fb[i] * ch.iw[i][j];
                    S3 += tt[i];
                }
                const float inv_s = 1.0f / S3;
                const float bb[3] = {tt[0] * inv_s, tt[1] * inv_s, tt[2] * inv_s};
                const float db[3] = {0.0f, dfx * gm1, dfy * gm1};
                const float dot = db[1] * bb[1] + db[2] * bb[2];
                float dbeta[3], diw[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const float dt = (db[i] - dot) * inv_s;
                    dbeta[i] = dt * ch.iw[i][j];
                    diw[i] = dt * fb[i];
                }
                // geometry in pixel units from exact integer differences
                const int32_t PX = kSnap * (tx0 + lx) + kSnap / 2, PY = kSnap * (ty0 + ly) + kSnap / 2;
                int32_t Xv[3], Yv[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    Xv[i] = ch.X[i][j];
                    Yv[i] = ch.Y[i][j];
                }
                const int64_t Ai = static_cast<int64_t>(Xv[1] - Xv[0]) * (Yv[2] - Yv[0]) -
                                   static_cast<int64_t>(Yv[1] - Yv[0]) * (Xv[2] - Xv[0]);
                const float inv_area = 65536.0f / static_cast<float>(Ai);
                const float inv256 = 1.0f / 256.0f;
                float gsx[3] = {0.f, 0.f, 0.f}, gsy[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int p = i == 2 ? 0 : i + 1, qq = i == 0 ? 2 : (i == 1 ? 0 : 1);
                    // beta_i = e_i / area with e_i = edge(v_p, v_q, pixel centre)
                    const float bi = fb[i];
#pragma unroll
                    for (int jv = 0; jv < 3; ++jv) {
                        const int jp = jv == 2 ? 0 : jv + 1, jq = jv == 0 ? 2 : (jv == 1 ? 0 : 1);
                        const float dax = static_cast<float>(Yv[jp] - Yv[jq]) * inv256;
                        const float day = static_cast<float>(Xv[jq] - Xv[jp]) * inv256;
                        float dex = 0.f, dey = 0.f;
                        if (jv == p) {
                            dex = static_cast<float>(Yv[qq] - PY) * inv256;
                            dey = static_cast<float>(PX - Xv[qq]) * inv256;
                        } else if (jv == qq) {
                            dex = static_cast<float>(PY - Yv[p]) * inv256;
                            dey = static_cast<float>(Xv[p] - PX) * inv256;
                        }
                        gsx[jv] += dbeta[i] * (dex - bi * dax) * inv_area;
                        gsy[jv] += dbeta[i] * (dey - bi * day) * inv_area;
                    }
                }
                // screen position and 1/w -> clip -> world through the view-projection
                const float hw = 0.5f * static_cast<float>(W), hh = 0.5f * static_cast<float>(H);
#pragma unroll
                for (int jv = 0; jv < 3; ++jv) {
                    const float iwv = ch.iw[jv][j];
                    const float sx = static_cast<float>(Xv[jv]) * inv256, sy = static_cast<float>(Yv[jv]) * inv256;
                    const float gc0 = gsx[jv] * hw * iwv;
                    const float gc1 = -gsy[jv] * hh * iwv;
                    const float gc3 = (-gsx[jv] * (sx - hw) + gsy[jv] * (hh - sy)) * iwv - diw[jv] * iwv * iwv;
#pragma unroll
                    for (int k = 0; k < 3; ++k) gw[3 * jv + k] = vd.M[k] * gc0 + vd.M[4 + k] * gc1 + vd.M[12 + k] * gc3;
                }
            }
            // slot: one counter bump per batch, records contiguous in lane order
            uint64_t base = 0;
            if (lane == 0) base = atomicAdd(a.rec_count, static_cast<unsigned long long>(n));
            base = static_cast<uint64_t>(uniform_i64(static_cast<int64_t>(__shfl(base, 0, 64))));
            const uint64_t slot = base + lane;
            if (on && slot < a.rec_cap) {
                float* rec = a.records + slot * kRecStride<S::C>;
                rec[0] = __uint_as_float(tri);
                rec[1] = __uint_as_float(static_cast<uint32_t>(c.ix) | (static_cast<uint32_t>(c.iy) << 8) |
                                         (win ? 0x80000000u : 0u));
                rec[2] = c.fx;
                rec[3] = c.fy;
#pragma unroll
                for (int k = 0; k < S::C; k += 4)
                    *reinterpret_cast<float4*>(rec + 4 + k) = make_float4(dx[k], dx[k + 1], dx[k + 2], dx[k + 3]);
                if (win) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) rec[4 + S::C + k] = gw[k];
                }
                a.rec_tri[slot] = tri;
            }
            // per-triangle record counts, one atomic per run of equal triangles
            const uint32_t tprev = __shfl_up(tri, 1, 64);
            const bool head = on && (lane == 0 || tprev != tri);
            const uint64_t heads = __ballot(head);
            if (head) {
                const uint64_t above = lane == 63 ? 0ull : (heads & (~0ull << (lane + 1)));
                const int endl = above ? __builtin_ctzll(above) : n;
                atomicAdd(&a.tri_count[tri], endl - lane);
            }
        };

        const int64_t beg = r.tile_start[tile], end = r.tile_start[tile + 1];
        int qn = 0;
        if (LOGP) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) s_gl[tid + k * NT] = 0.0f;
        }
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
                            q.info[w][pos] = static_cast<uint32_t>(pl) | (static_cast<uint32_t>(j) << 10) |
                                             (win ? 0x80000000u : 0u);
                            q.b1[w][pos] = b1;
                            q.b2[w][pos] = b2;
                            q.beta[0][w][pos] = f.beta[0];
                            q.beta[1][w][pos] = f.beta[1];
                            q.beta[2][w][pos] = f.beta[2];
                        }
                        qn += __popcll(mk);
                        if (qn >= 64) {
                            run_batch(64);
                            __threadfence_block();
                            if (lane < qn - 64) {
                                q.info[w][lane] = q.info[w][64 + lane];
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
                    run_batch(qn);
                    qn = 0;
                    __threadfence_block();
                }
            }
        }
        __syncthreads();
        if (LOGP) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int pl = tid + k * NT;
                const int gx = tx0 + px_of<TS>(pl), gy = ty0 + py_of<TS>(pl);
                if (gx < W && gy < H) a.logp[vd.pix_base + static_cast<int64_t>(gy) * W + gx] = s_gl[pl];
            }
            __syncthreads();
        }
    }
    if (!LOGP) {
        float* row = a.mlp_partial + (static_cast<size_t>(blockIdx.x) * NW + w) * S::kParams;
        acc.l0.store(row, S::w_off(0), S::b_off(0), lane);
        if constexpr (S::NH == 2) acc.mid[0].store(row, S::w_off(1), S::b_off(1), lane);
        acc.out.store(row, S::w_off(S::NH), S::b_off(S::NH), lane);
    }
}

template <int TS, class S>
static void launch_bwd_t(const BwdArgs& a, bool logp, hipStream_t s) {
    if (a.r.n_tiles <= 0) return;
    if (logp)
        hipLaunchKernelGGL((raster_bwd_kernel<TS, S, true>), dim3(a.n_blocks), dim3(TileCfg<TS>::NT), 0, s, a);
    else
        hipLaunchKernelGGL((raster_bwd_kernel<TS, S, false>), dim3(a.n_blocks), dim3(TileCfg<TS>::NT), 0, s, a);
}


}  // namespace soup
