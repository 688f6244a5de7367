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

// Register accumulators of one layer's weight (4x4 blocks) and bias gradients.
template <int DIN, int DOUT>
struct LayerAcc {
    static constexpr int NBK = DIN / 4;
    static constexpr int NB = (DOUT / 4) * NBK;
    static constexpr int PER = (NB + 63) / 64;
    static constexpr int PB = (DOUT + 63) / 64;
    float w[PER][16];
    float b[PB];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int p = 0; p < PER; ++p)
#pragma unroll
            for (int i = 0; i < 16; ++i) w[p][i] = 0.0f;
#pragma unroll
        for (int p = 0; p < PB; ++p) b[p] = 0.0f;
    }
    // rows [0, nrows) of the stage: in[r][DIN] then d[r][DOUT]
    __device__ __forceinline__ void accumulate(const float* __restrict__ in, const float* __restrict__ d, int nrows, int lane) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int blk = lane + 64 * p;
            if (blk < NB) {
                const int bj = blk / NBK, bk = blk % NBK;
                for (int r = 0; r < nrows; ++r) {
                    const float4 dv = *reinterpret_cast<const float4*>(d + r * DOUT + 4 * bj);
                    const float4 iv = *reinterpret_cast<const float4*>(in + r * DIN + 4 * bk);
                    const float dd[4] = {dv.x, dv.y, dv.z, dv.w};
                    const float ii[4] = {iv.x, iv.y, iv.z, iv.w};
#pragma unroll
                    for (int x = 0; x < 4; ++x)
#pragma unroll
                        for (int y = 0; y < 4; ++y) w[p][4 * x + y] = __builtin_fmaf(dd[x], ii[y], w[p][4 * x + y]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int j = lane + 64 * p;
            if (j < DOUT)
                for (int r = 0; r < nrows; ++r) b[p] += d[r * DOUT + j];
        }
    }
    __device__ __forceinline__ void store(float* __restrict__ row, int w_off, int b_off, int lane) const {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int blk = lane + 64 * p;
            if (blk < NB) {
                const int bj = blk / NBK, bk = blk % NBK;
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) row[w_off + (4 * bj + x) * DIN + 4 * bk + y] = w[p][4 * x + y];
            }
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int j = lane + 64 * p;
            if (j < DOUT) row[b_off + j] = b[p];
        }
    }
};

// Stage the activations (in) and deltas (dl) of the wave's 64 fragments
// through LDS, kStageRows at a time, and let every lane accumulate its blocks.
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
        la.accumulate(st, st + kStageRows * DIN, kStageRows, lane);
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
            const int gx = tx0 + pl % TS, gy = ty0 + pl / TS;
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
            if (!on) return;
            // --- bilinear scatter to the four texels ---
            const float w00 = (1.0f - c.fx) * (1.0f - c.fy), w10 = c.fx * (1.0f - c.fy);
            const float w01 = (1.0f - c.fx) * c.fy, w11 = c.fx * c.fy;
            const size_t t00 = ((static_cast<size_t>(tri) * G + c.iy) * G + c.ix) * S::C;
            const size_t t10 = t00 + S::C, t01 = t00 + static_cast<size_t>(G) * S::C, t11 = t01 + S::C;
            float* gf = a.grad_feats;
#pragma unroll
            for (int k = 0; k < S::C; ++k) {
                if (dx[k] == 0.0f) continue;
                atomicAdd(gf + t00 + k, w00 * dx[k]);
                atomicAdd(gf + t10 + k, w10 * dx[k]);
                atomicAdd(gf + t01 + k, w01 * dx[k]);
                atomicAdd(gf + t11 + k, w11 * dx[k]);
            }
            if (!win) return;
            // --- winner: texture position -> barycentrics -> vertex screen positions ---
            float dfx = 0.f, dfy = 0.f;
#pragma unroll
            for (int k = 0; k < S::C; ++k) {
                const float T00 = feats[t00 + k], T10 = feats[t10 + k], T01 = feats[t01 + k], T11 = feats[t11 + k];
                dfx = __builtin_fmaf(dx[k], (1.0f - c.fy) * (T10 - T00) + c.fy * (T11 - T01), dfx);
                dfy = __builtin_fmaf(dx[k], (1.0f - c.fx) * (T01 - T00) + c.fx * (T11 - T10), dfy);
            }
            const float gm1 = static_cast<float>(G - 1);
            const int lx = pl % TS, ly = pl / TS;
            Frag f;
            cover(ch, j, lx, ly, f);
            float tt[3], S3 = 0.f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                tt[i] = f.beta[i] * ch.iw[i][j];
                S3 += tt[i];
            }
            const float bb[3] = {tt[0] / S3, tt[1] / S3, tt[2] / S3};
            const float db[3] = {0.0f, dfx * gm1, dfy * gm1};
            const float dot = db[1] * bb[1] + db[2] * bb[2];
            float dbeta[3], diw[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float dt = (db[i] - dot) / S3;
                dbeta[i] = dt * ch.iw[i][j];
                diw[i] = dt * f.beta[i];
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
            const float area = static_cast<float>(Ai) * (1.0f / 65536.0f);
            const float inv256 = 1.0f / 256.0f;
            float gsx[3] = {0.f, 0.f, 0.f}, gsy[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int p = i == 2 ? 0 : i + 1, qq = i == 0 ? 2 : (i == 1 ? 0 : 1);
                // beta_i = e_i / area, e_i = edge(v_p, v_q, pixel)
                const float bi = f.beta[i];
#pragma unroll
                for (int jv = 0; jv < 3; ++jv) {
                    const int jp = jv == 2 ? 0 : jv + 1, jq = jv == 0 ? 2 : (jv == 1 ? 0 : 1);
                    float dax = static_cast<float>(Yv[jp] - Yv[jq]) * inv256;
                    float day = static_cast<float>(Xv[jq] - Xv[jp]) * inv256;
                    float dex = 0.f, dey = 0.f;
                    if (jv == p) {
                        dex = static_cast<float>(Yv[qq] - PY) * inv256;
                        dey = static_cast<float>(PX - Xv[qq]) * inv256;
                    } else if (jv == qq) {
                        dex = static_cast<float>(PY - Yv[p]) * inv256;
                        dey = static_cast<float>(Xv[p] - PX) * inv256;
                    }
                    gsx[jv] += dbeta[i] * (dex - bi * dax) / area;
                    gsy[jv] += dbeta[i] * (dey - bi * day) / area;
                }
            }
            float* va = a.vacc + static_cast<size_t>(vd.rec_base + tri) * kVacc;
#pragma unroll
            for (int jv = 0; jv < 3; ++jv) {
                atomicAdd(va + 3 * jv + 0, gsx[jv]);
                atomicAdd(va + 3 * jv + 1, gsy[jv]);
                atomicAdd(va + 3 * jv + 2, diw[jv]);
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
#pragma unroll
                    for (int k = 0; k < PPT; ++k) {
                        const int pl = tid + k * NT;
                        Frag f;
                        bool cand = false, win = false;
                        float b1 = 0.f, b2 = 0.f;
                        if (act[k] && zk <= kc[k] && cover(ch, j, pl % TS, pl / TS, f) && f.key <= kc[k]) {
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
                        }
                        qn += __popcll(mk);
                        if (qn >= 64) {
                            run_batch(64);
                            __threadfence_block();
                            if (lane < qn - 64) {
                                q.info[w][lane] = q.info[w][64 + lane];
                                q.b1[w][lane] = q.b1[w][64 + lane];
                                q.b2[w][lane] = q.b2[w][64 + lane];
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
                const int gx = tx0 + pl % TS, gy = ty0 + pl / TS;
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

template <class S>
static void launch_bwd_s(const BwdArgs& a, int tile, bool logp, hipStream_t s) {
    switch (tile) {
        case 8: launch_bwd_t<8, S>(a, logp, s); break;
        case 32: launch_bwd_t<32, S>(a, logp, s); break;
        default: launch_bwd_t<16, S>(a, logp, s); break;
    }
}

void launch_raster_bwd(const BwdArgs& a, int tile, MlpKind k, bool logp, hipStream_t s) {
    switch (k) {
        case MlpKind::k8_16_1: launch_bwd_s<MlpShape<8, 16, 1>>(a, tile, logp, s); break;
        case MlpKind::k16_32_2: launch_bwd_s<MlpShape<16, 32, 2>>(a, tile, logp, s); break;
        case MlpKind::k32_64_2: launch_bwd_s<MlpShape<32, 64, 2>>(a, tile, logp, s); break;
        default: break;
    }
}

// ---------------------------------------------------------------------------
// edge term
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void edge_kernel(const ViewDesc* __restrict__ views, int V, int64_t P, Opts o,
                                                   const uint64_t* __restrict__ vis,
                                                   const float* __restrict__ color,
                                                   const float* __restrict__ gcol,
                                                   const TriRec* __restrict__ recs, float* __restrict__ vacc) {
    const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (p >= P) return;
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].pix_base <= p) lo = mid;
        else hi = mid - 1;
    }
    const ViewDesc& vd = views[lo];
    const int64_t local = p - vd.pix_base;
    const int x = static_cast<int>(local % vd.W), y = static_cast<int>(local / vd.W);
    const uint64_t ka = vis[p];
    const float ca[3] = {color[3 * p], color[3 * p + 1], color[3 * p + 2]};
    const float ga[3] = {gcol[3 * p], gcol[3 * p + 1], gcol[3 * p + 2]};
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const int xb = x + (dir == 0), yb = y + (dir == 1);
        if (xb >= vd.W || yb >= vd.H) continue;
        const int64_t q = p + (dir == 0 ? 1 : vd.W);
        const uint64_t kb = vis[q];
        if (ka == kBgKey && kb == kBgKey) continue;
        if (o.edge_pairs == 1 && ka != kBgKey && kb != kBgKey &&
            static_cast<uint32_t>(ka) == static_cast<uint32_t>(kb))
            continue;
        float wgt = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) wgt += 0.5f * (ga[c] + gcol[3 * q + c]) * (ca[c] - color[3 * q + c]);
        if (wgt == 0.0f) continue;
        const bool oa = ka < kb;
        const uint32_t tri = static_cast<uint32_t>(oa ? ka : kb);
        const int xo = oa ? x : xb, yo = oa ? y : yb;
        const int64_t rec = vd.rec_base + tri;
        const int32_t X0 = recs[rec].X[0], Y0 = recs[rec].Y[0];
        const float dx = static_cast<float>(kSnap * xo + kSnap / 2 - X0) * (1.0f / 256.0f);
        const float dy = static_cast<float>(kSnap * yo + kSnap / 2 - Y0) * (1.0f / 256.0f);
        float* va = vacc + static_cast<size_t>(rec) * kVacc + 9 + 3 * dir;
        atomicAdd(va + 0, wgt);
        atomicAdd(va + 1, wgt * dx);
        atomicAdd(va + 2, wgt * dy);
    }
}

void launch_edge(const ViewDesc* views, int V, int64_t P, const Opts& o, const uint64_t* vis, const float* color,
                 const float* grad_color, const TriRec* recs, float* vacc, hipStream_t s) {
    if (P <= 0 || o.edge_pairs == 2) return;
    hipLaunchKernelGGL(edge_kernel, dim3(static_cast<unsigned>((P + 255) / 256)), dim3(256), 0, s, views, V, P, o, vis,
                       color, grad_color, recs, vacc);
}

// ---------------------------------------------------------------------------
// vertex chain: screen-space accumulators -> world-space vertex gradients
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void vertex_chain_kernel(const ViewDesc* __restrict__ views, int V,
                                                           const SceneDesc* __restrict__ scenes, int T,
                                                           const TriRec* __restrict__ recs,
                                                           const float* __restrict__ vacc,
                                                           float* __restrict__ grad_verts, bool accumulate) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const float* vt = scenes[0].verts + static_cast<size_t>(t) * 9;
    float g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = 0.0f;
    for (int v = 0; v < V; ++v) {
        const ViewDesc& vd = views[v];
        const int64_t rec = vd.rec_base + t;
        const TriRec R = recs[rec];
        if (R.x0 > R.x1) continue;
        const float* a = vacc + static_cast<size_t>(rec) * kVacc;
        float gs[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) gs[i][k] = a[3 * i + k];
        // edge moments about vertex 0 -> screen gradients (beta affine in the pixel)
        const float m[2][3] = {{a[9], a[10], a[11]}, {a[12], a[13], a[14]}};
        if (m[0][0] != 0.f || m[0][1] != 0.f || m[0][2] != 0.f || m[1][0] != 0.f || m[1][1] != 0.f ||
            m[1][2] != 0.f) {
            const int64_t Ai = static_cast<int64_t>(R.X[1] - R.X[0]) * (R.Y[2] - R.Y[0]) -
                               static_cast<int64_t>(R.Y[1] - R.Y[0]) * (R.X[2] - R.X[0]);
            const float area = static_cast<float>(Ai) * (1.0f / 65536.0f);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int p = i == 2 ? 0 : i + 1, q = i == 0 ? 2 : (i == 1 ? 0 : 1);
                const float dbx = -static_cast<float>(R.Y[q] - R.Y[p]) * (1.0f / 256.0f) / area;
                const float dby = static_cast<float>(R.X[q] - R.X[p]) * (1.0f / 256.0f) / area;
                const float b0 = i == 0 ? 1.0f : 0.0f;
#pragma unroll
                for (int dir = 0; dir < 2; ++dir) gs[i][dir] += m[dir][0] * b0 + m[dir][1] * dbx + m[dir][2] * dby;
            }
        }
        const float hw = 0.5f * static_cast<float>(vd.W), hh = 0.5f * static_cast<float>(vd.H);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (gs[i][0] == 0.f && gs[i][1] == 0.f && gs[i][2] == 0.f) continue;
            float c[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                c[j] = vd.M[4 * j + 3] + vd.M[4 * j] * vt[3 * i] + vd.M[4 * j + 1] * vt[3 * i + 1] +
                       vd.M[4 * j + 2] * vt[3 * i + 2];
            const float iw = 1.0f / c[3];
            const float gc0 = gs[i][0] * hw * iw;
            const float gc1 = -gs[i][1] * hh * iw;
            const float gc3 = (-gs[i][0] * hw * c[0] + gs[i][1] * hh * c[1]) * iw * iw - gs[i][2] * iw * iw;
#pragma unroll
            for (int k = 0; k < 3; ++k) g[3 * i + k] += vd.M[k] * gc0 + vd.M[4 + k] * gc1 + vd.M[12 + k] * gc3;
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        float* o = grad_verts + static_cast<size_t>(t) * 9 + i;
        *o = accumulate ? *o + g[i] : g[i];
    }
}

void launch_vertex_chain(const ViewDesc* views, int V, const SceneDesc* scenes, int T, const TriRec* recs,
                         const float* vacc, float* grad_verts, bool accumulate, hipStream_t s) {
    if (T <= 0) return;
    hipLaunchKernelGGL(vertex_chain_kernel, dim3((T + 255) / 256), dim3(256), 0, s, views, V, scenes, T, recs, vacc,
                       grad_verts, accumulate);
}

// ---------------------------------------------------------------------------
// MLP gradient: fixed-order reduction of the per-wave partial sums
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partial, int n_rows, int n_params,
                                                         float* __restrict__ out, bool accumulate) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_params) return;
    double s = accumulate ? static_cast<double>(out[p]) : 0.0;
    for (int r = 0; r < n_rows; ++r) s += partial[static_cast<size_t>(r) * n_params + p];
    out[p] = static_cast<float>(s);
}

void launch_mlp_reduce(const float* partial, int n_rows, int n_params, float* out, bool accumulate, hipStream_t s) {
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((n_params + 255) / 256), dim3(256), 0, s, partial, n_rows, n_params,
                       out, accumulate);
}

// ---------------------------------------------------------------------------
// L2 loss and contract self-tests
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void loss_l2_kernel(const float* __restrict__ color, const float* __restrict__ target,
                                                      int64_t P, float* __restrict__ gc, float* __restrict__ gl,
                                                      float* __restrict__ loss) {
    __shared__ float red[4];
    const float inv = 1.0f / (3.0f * static_cast<float>(P));
    float part = 0.0f;
    for (int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; p < P;
         p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        float s = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = color[3 * p + c] - target[3 * p + c];
            gc[3 * p + c] = 2.0f * d * inv;
            s = __builtin_fmaf(d, d, s);
        }
        gl[p] = s * inv;
        part += s * inv;
    }
    if (loss) {
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) part += __shfl_xor(part, d, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(loss, red[0] + red[1] + red[2] + red[3]);
    }
}

void launch_loss_l2(const float* color, const float* target, int64_t P, float* gc, float* gl, float* loss,
                    hipStream_t s) {
    if (P <= 0) return;
    if (loss) launch_fill_f32(loss, 1, 0.0f, s);
    int64_t g = (P + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(loss_l2_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, color, target, P, gc, gl, loss);
}

__global__ void selftest_sigmoid_kernel(const float* __restrict__ x, float* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        y[i] = sigmoid_c(x[i]);
}

__global__ void selftest_uniform_kernel(uint64_t seed, const uint32_t* __restrict__ pixel,
                                        const uint32_t* __restrict__ tri, uint32_t view_id, uint32_t step,
                                        float* __restrict__ u, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        u[i] = uniform24(seed, pixel[i], tri[i], view_id, step);
}

void launch_selftest_sigmoid(const float* x, float* y, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(selftest_sigmoid_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, x, y, n);
}

void launch_selftest_uniform(uint64_t seed, const uint32_t* pixel, const uint32_t* tri, uint32_t view_id,
                             uint32_t step, float* u, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(selftest_uniform_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, seed, pixel, tri,
                       view_id, step, u, n);
}

}  // namespace soup
