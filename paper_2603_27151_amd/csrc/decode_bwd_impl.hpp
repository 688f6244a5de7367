#pragma once
// Backward, part 2 (Supplement Algorithm A1, part 2; Eq. (8), (9)): decode of
// the fragment list written by the replay kernel.
//
// The backward walks the fragment list sorted by triangle: every wave takes a
// contiguous range of 64-fragment batches. For each batch:
//   - recompute the bilinear feature and the MLP (float32, as the forward);
//   - logit gradients: winner -> colour path g_C sigma'(o_rgb) and score
//     g_L (1 - alpha); fragment in front -> score -g_L alpha (Eq. (9) through
//     the sigmoid);
//   - back-propagate through the MLP; the weight gradient sum_f delta_f a_f^T
//     runs on the matrix cores over the batch (activations and deltas staged
//     through LDS); each wave writes its sums once, at the end, to its own row
//     of a partial-sum buffer (rows are reduced later in a fixed order);
//   - for the winner, the gradient of its triangle's world-space vertices
//     from its colour logits only (the score term moves no vertex, Section
//     3.2): the feature gradient of the colour logits (a second data backward
//     where the winner also carries a score weight) dotted with the texture's
//     derivative along the cell position, then through the perspective-
//     correct and screen barycentrics, the screen positions and 1/w, and the
//     view-projection; the edge term of Section 3.2 (the pixel's edge weights
//     times its screen barycentrics) joins it in screen space;
//   - the feature gradient (bilinear weights of the four texels) and the
//     vertex gradient are summed into the wave's LDS copy of the current
//     triangle's G x G x C grid; when the triangle changes, the grid goes to
//     HBM once (a plain store when the wave holds all of the triangle's
//     fragments, float atomics for a triangle split between waves).
// A logp variant walks the unsorted fragment list region by region (batch b
// lies in the region w with boff[w] <= b < boff[w + 1], found by a binary
// search over the offsets staged in LDS) and sums log(1 - alpha) over the
// front set and log(alpha) of the winner per pixel (log p(f*) of Eq. (6)).
#include "decode_mfma.hpp"

namespace soup {

constexpr int kStageRows = 16;   // fragments staged per transpose pass
// floats after a wave's gradient grid: the current triangle's nine vertex
// gradient sums, as doubles
constexpr int kGridTail = 32;

// 1/x in double: the hardware estimate refined by two Newton steps (about one
// ulp; the backward needs no correctly rounded quotient)
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// The sigmoid of the backward's recompute, from the hardware exp2 and
// reciprocal (a few ulp; only the forward's mask decision is bit-exact)
__device__ __forceinline__ float sigmoid_fast(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

template <class S>
struct StageCfg {
    static constexpr int kMax2(int a, int b) { return a > b ? a : b; }
    // the widest pair of staged rows (in, d), each row padded by kRowPad floats
    static constexpr int kWidth = kMax2(kMax2(S::C + S::H, 2 * S::H), S::H + 4) + 2 * kRowPad;
};

// Accumulators of one layer's weight gradient dW[DOUT][DIN] += sum_f d_f a_f^T
// on the matrix cores: the contraction runs over fragments, four per
// v_mfma_f32_16x16x4f32 (A[m][k] = d[f_k][m], B[k][n] = a[f_k][n]); dW is
// tiled in 16x16 blocks held in registers (4 per lane per block), padded
// with zeros where DIN or DOUT is below 16. The bias gradient sum_f d_f is
// kept per lane in the unit-major layout of d (units 16 bo + 4 grp + i of the
// lane's fragments; for the output layer, OUTL, output grp in element 0) and
// summed over the lanes of a lane group at the end.
template <int DIN, int DOUT, bool OUTL = false>
struct LayerAcc {
    static constexpr int BI = (DIN + 15) / 16;
    static constexpr int BO = (DOUT + 15) / 16;
    static constexpr int NB = BI * BO;
    static_assert(!OUTL || DOUT == 4, "the output layer has four outputs, one per lane group");
    f4v w[NB];
    f4v bs[BO];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int i = 0; i < NB; ++i) w[i] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < BO; ++i) bs[i] = f4v{0.f, 0.f, 0.f, 0.f};
    }
    __device__ __forceinline__ void add_bias(const f4v (&d)[BO]) {
        if (OUTL) {
            bs[0][0] += d[0][0];
        } else {
#pragma unroll
            for (int i = 0; i < BO; ++i) bs[i] += d[i];
        }
    }
    // kStageRows (16) staged fragments: in[r][DIN] and d[r][DOUT] in LDS, rows
    // padded by kRowPad; every step's operands are read before the first product
    __device__ __forceinline__ void accumulate(const float* __restrict__ in, const float* __restrict__ d, int lane) {
        constexpr int KS = kStageRows / 4;
        const int col = lane & 15, kq = lane >> 4;
        float av[KS][BO], bv[KS][BI];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int r = 4 * kk + kq;
#pragma unroll
            for (int bo = 0; bo < BO; ++bo) {
                const int m = 16 * bo + col;
                av[kk][bo] = m < DOUT ? d[r * (DOUT + kRowPad) + m] : 0.0f;
            }
#pragma unroll
            for (int bi = 0; bi < BI; ++bi) {
                const int n = 16 * bi + col;
                bv[kk][bi] = n < DIN ? in[r * (DIN + kRowPad) + n] : 0.0f;
            }
        }
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
#pragma unroll
            for (int bo = 0; bo < BO; ++bo)
#pragma unroll
                for (int bi = 0; bi < BI; ++bi)
                    w[bo * BI + bi] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk][bo], bv[kk][bi], w[bo * BI + bi], 0, 0, 0);
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
        // bias: sum over the 16 lanes (fragments) of each lane group
#pragma unroll
        for (int bo = 0; bo < BO; ++bo) {
            f4v v = bs[bo];
#pragma unroll
            for (int sh = 1; sh < 16; sh <<= 1)
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] += __shfl_xor(v[i], sh, 64);
            if ((lane & 15) == 0) {
                if (OUTL) {
                    row[b_off + (lane >> 4)] = v[0];
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int m = 16 * bo + 4 * (lane >> 4) + i;
                        if (m < DOUT) row[b_off + m] = v[i];
                    }
                }
            }
        }
    }
};

// The output layer's weight gradient dW[4][DIN] += sum_f d_f a_f^T on
// v_mfma_f32_4x4x1f32: block b (lanes 4b .. 4b + 3) accumulates the 4 x 4
// tile of units 4 (b % 8) .. + 3 over the fragments of half b / 8 of the 16
// staged rows, one fragment per product (A = the fragment's four output
// deltas, B = its four units); the two halves are added at the end. The
// bias gradient as in LayerAcc (output grp in element 0 of lane group grp).
template <int DIN>
struct OutAcc {
    static_assert(DIN == 32, "the tiles cover 32 input units");
    f4v w;
    f4v bs[1];
    __device__ __forceinline__ void zero() {
        w = f4v{0.f, 0.f, 0.f, 0.f};
        bs[0] = f4v{0.f, 0.f, 0.f, 0.f};
    }
    __device__ __forceinline__ void add_bias(const f4v (&d)[1]) { bs[0][0] += d[0][0]; }
    __device__ __forceinline__ void accumulate(const float* __restrict__ in, const float* __restrict__ d, int lane) {
        const int x = lane & 3, t = (lane >> 2) & 7, half = lane >> 5;
        float av[8], bv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int f = 8 * half + k;
            av[k] = d[f * (4 + kRowPad) + x];
            bv[k] = in[f * (DIN + kRowPad) + 4 * t + x];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) w = mfma4x4(av[k], bv[k], w);
    }
    __device__ __forceinline__ void store(float* __restrict__ row, int w_off, int b_off, int lane) const {
        // lanes 0..31 (the first half) add the second half's tiles
        f4v s;
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] = pair32f(w[i], w[i]);
        if (lane < 32) {
            const int t = lane >> 2, j = lane & 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) row[w_off + i * DIN + 4 * t + j] = s[i];
        }
        f4v v = bs[0];
#pragma unroll
        for (int sh = 1; sh < 16; sh <<= 1) v[0] += __shfl_xor(v[0], sh, 64);
        if ((lane & 15) == 0) row[b_off + (lane >> 4)] = v[0];
    }
};

template <class S, bool OUT4 = (S::H == 32)>
struct OutAccOf {
    using type = LayerAcc<S::H, 4, true>;
};
template <class S>
struct OutAccOf<S, true> {
    using type = OutAcc<S::H>;
};

template <class S>
struct MlpGrad {
    LayerAcc<S::C, S::H> l0;
    LayerAcc<S::H, S::H> mid[S::NH > 1 ? S::NH - 1 : 1];
    typename OutAccOf<S>::type out;
};

template <class S, bool LOGP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void decode_bwd_kernel(DecodeArgs a) {
    constexpr int NW = 4;
    constexpr int SW = StageCfg<S>::kWidth;
    __shared__ __align__(16) float s_stage[LOGP ? 1 : NW][LOGP ? 4 : kStageRows * SW];
    __shared__ uint32_t s_boff[LOGP ? kMaxRegions + 1 : 1];
    __shared__ MfmaWeights<S> s_w;     // the MLP in the matrix cores' operand order (backward only)
    // the batch's feature gradients, rows of C padded by kRowPad (not for C = 32: that
    // shape's LDS is full)
    constexpr int DXS = S::C + (S::C >= 32 ? 0 : kRowPad);
    __shared__ __align__(16) float s_dx[LOGP ? 1 : NW][LOGP ? 4 : 64 * DXS];
    extern __shared__ __align__(16) float s_dyn[];   // [NW][G*G*C + kGridTail]: per-wave gradient grid of the current triangle

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int G = a.G;
    const int n_grid = G * G * S::C;
    gfloat* __restrict__ feats = as_global(uniform_ptr(a.feats));

    MlpGrad<S> acc;
    if (!LOGP) {
        acc.l0.zero();
        if constexpr (S::NH == 2) acc.mid[0].zero();
        acc.out.zero();
    }
    if (!LOGP) {
        s_w.load(a.mlp, tid, blockDim.x);
        __syncthreads();
    }
    const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * NW;
    const uint64_t wid = static_cast<uint64_t>(blockIdx.x) * NW + w;
    uint64_t b_begin, b_end, b_step;
    int64_t E = 0, f0 = 0, f1 = 0;   // sorted list: fragments, this wave's range
    float* grid = s_dyn + static_cast<size_t>(w) * (n_grid + kGridTail);
    double* vgrid = reinterpret_cast<double*>(grid + n_grid);   // the nine vertex sums (n_grid is even)
    int cur = -1;                    // triangle held in grid (wave-uniform)
    if (LOGP) {
        for (int i = tid; i <= a.n_regions; i += blockDim.x) s_boff[i] = a.boff[i];
        __syncthreads();
        b_begin = wid;
        b_end = s_boff[a.n_regions];
        b_step = n_waves;
    } else {
        E = a.tri_off[a.T];
        const uint64_t nb = (static_cast<uint64_t>(E) + 63) / 64;
        const uint64_t per = (nb + n_waves - 1) / n_waves;
        b_begin = wid * per;
        b_end = b_begin + per < nb ? b_begin + per : nb;
        b_step = 1;
        f0 = static_cast<int64_t>(b_begin) * 64;
        f1 = static_cast<int64_t>(b_end) * 64 < E ? static_cast<int64_t>(b_end) * 64 : E;
        for (int k = lane; k < n_grid + kGridTail; k += 64) grid[k] = 0.0f;
    }
    // sorted list: the next batch's records, loaded one batch ahead, and the
    // per-pixel data of its winners (colour gradient, edge weights), loaded
    // once those records are in (after the current batch's MLP)
    uint4 na = make_uint4(0u, 0u, 0u, 0u);   // (pixel, triangle | winner, b1, b2)
    uint2 nx = make_uint2(0u, 0u);           // (score weight, view)
    float ng0 = 0.f, ng1 = 0.f, ng2 = 0.f, nex = 0.f, ney = 0.f;
    bool nvalid = false;
    constexpr int GW = GateWords<S>::kWords;
    // the forward's ReLU gates of every sorted fragment (from its log, or from
    // fragment_gates_kernel for a replayed list): the host always provides them
    const bool use_gates = !LOGP;
    uint32_t ngate[GW];
#pragma unroll
    for (int k = 0; k < GW; ++k) ngate[k] = 0u;
    auto prefetch = [&](uint64_t bi) __attribute__((always_inline)) {
        const int64_t fi = static_cast<int64_t>(bi) * 64 + lane;
        nvalid = bi < b_end && fi < E;
        if (nvalid) {
            const FragRec fr = a.sorted[fi];
            na = make_uint4(fr.p0.x, fr.p0.y, fr.p1.x, fr.p1.y);
            nx = fr.x;
            if (use_gates) {
#pragma unroll
                for (int k = 0; k < GW; k += 2) {   // 8-byte units of the padded gate record
                    const uint2 g = reinterpret_cast<const uint2*>(a.sorted_gates)[fi * (gate_stride(GW) / 2) + k / 2];
                    ngate[k] = g.x;
                    if (k + 1 < GW) ngate[k + 1] = g.y;
                }
            }
        }
    };
    auto pixfetch = [&]() __attribute__((always_inline)) {
        ng0 = ng1 = ng2 = nex = ney = 0.0f;
        if (nvalid && (na.y >> 31)) {
            const size_t p = na.x;
            ng0 = a.grad_color[3 * p];
            ng1 = a.grad_color[3 * p + 1];
            ng2 = a.grad_color[3 * p + 2];
            if (a.edge_w) {
                const float2 e = a.edge_w[p];
                nex = e.x;
                ney = e.y;
            }
        }
    };
    if (!LOGP) {
        prefetch(b_begin);
        pixfetch();
    }
    // the grid of triangle t goes to HBM and is cleared (whole wave)
    auto flush = [&](int t) __attribute__((always_inline)) {
        wave_fence();
        const bool owned = a.tri_off[t] >= f0 && a.tri_off[t + 1] <= f1;
        float* gf = a.grad_feats + static_cast<size_t>(t) * n_grid;
        for (int k = lane; k < n_grid; k += 64) {
            const float v = grid[k];
            grid[k] = 0.0f;
            if (owned) gf[k] = a.accumulate ? gf[k] + v : v;
            else if (v != 0.0f) atomicAdd(&gf[k], v);
        }
        if (lane < 9) {
            const float v = static_cast<float>(vgrid[lane]);
            vgrid[lane] = 0.0;
            float* gv = a.grad_verts + static_cast<size_t>(t) * 9 + lane;
            if (owned) *gv = a.accumulate ? *gv + v : v;
            else if (v != 0.0f) atomicAdd(gv, v);
        }
        wave_fence();
    };
    for (uint64_t bi = b_begin; bi < b_end; bi += b_step) {
        bool on;
        uint4 fa = make_uint4(0u, 0u, 0u, 0u), fb4 = make_uint4(0u, 0u, 0u, 0u), fc4 = make_uint4(0u, 0u, 0u, 0u);
        uint32_t gt[GW];   // this lane's fragment: the forward's ReLU gates
#pragma unroll
        for (int k = 0; k < GW; ++k) gt[k] = ngate[k];
        if (LOGP) {
            int lo = 0, hi = a.n_regions - 1;   // region: last w with boff[w] <= bi
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_boff[mid] <= bi) lo = mid;
                else hi = mid - 1;
            }
            const uint32_t cr = a.counts[lo];
            const uint32_t in_region = (static_cast<uint32_t>(bi) - s_boff[lo]) * 64u + static_cast<uint32_t>(lane);
            on = in_region < (cr < a.region ? cr : a.region);
            if (on) {
                const FragRec fr = a.frags[static_cast<uint64_t>(lo) * a.region + in_region];
                fa = make_uint4(fr.p0.x, fr.p0.y, fr.p1.x, fr.p1.y);
            }
        } else {
            on = static_cast<int64_t>(bi) * 64 + lane < E;
            if (on) {
                fa = na;
                fb4 = make_uint4(nx.x, __float_as_uint(ng0), __float_as_uint(ng1), __float_as_uint(ng2));
                fc4 = make_uint4(__float_as_uint(nex), __float_as_uint(ney), nx.y, 0u);
            }
            prefetch(bi + 1);
        }
        const uint32_t pix = fa.x;
        const uint32_t tri = fa.y & 0x7FFFFFFFu;
        const bool win = on && (fa.y >> 31);
        const float b1 = __uint_as_float(fa.z), b2 = __uint_as_float(fa.w);
        const Cell c = cell_of(b1, b2, G);
        const uint64_t on_mask = __ballot(on);
        if (a.counter && lane == 0) atomicAdd(a.counter, static_cast<unsigned long long>(__popcll(on_mask)));
        if (LOGP) {
            float x[S::C];
            MlpAct<S> m;
            if (on) {
                fetch_feature<S::C>(feats, tri, G, c, x);
            } else {
#pragma unroll
                for (int k = 0; k < S::C; ++k) x[k] = 0.0f;
            }
            // an opaque copy of the weight pointer per batch: the compiler may
            // not hoist the weights' scalar loads out of the batch loop
            mlp_forward<S>(as_const(opaque_ptr(a.mlp)), x, m);
            const float alpha = sigmoid_c(m.o[3]);
            if (on) atomicAdd(&a.logp[pix], win ? logf(alpha) : log1pf(-alpha));
            continue;
        }
        float* st = s_stage[w];
        const uint32_t cellw = static_cast<uint32_t>(c.ix) | (static_cast<uint32_t>(c.iy) << 16);
        // the fragment's triangle and winner bit, 0x7FFFFFFF for an empty lane
        // (no triangle has that index: T is below 2^31)
        const uint32_t fkey = on ? fa.y : 0x7FFFFFFFu;
        float my_dfx = 0.0f, my_dfy = 0.0f;   // this lane's fragment: d loss / d (fx, fy), colour logits
        {   // ---- the batch's MLP on the matrix cores, one 16-fragment block at a time ----
            constexpr int CB = MfmaWeights<S>::CB, HB = MfmaWeights<S>::HB;
            const int col = lane & 15, grp = lane >> 4;
            const MfmaWeights<S>& Wt = s_w;
            // The four corners of block nb's texels are loaded one block ahead:
            // they are in flight while the previous block runs on the matrix
            // cores. Lane (col, grp) takes channels 16 cb + 4 grp .. + 3 of
            // fragment 16 nb + col.
            float4 qv[CB][4];
            float qw[4];
            float qfx = 0.0f, qfy = 0.0f;   // the block fragment's position in its texture cell
            auto gather = [&](int nb) __attribute__((always_inline)) {
                const uint32_t key_n = row_bcast(fkey, nb);
                const uint32_t tri_n = key_n & 0x7FFFFFFFu;
                const bool on_n = tri_n != 0x7FFFFFFFu;
                const uint32_t cw = row_bcast(cellw, nb);
                const float fx = row_bcast(c.fx, nb), fy = row_bcast(c.fy, nb);
                qfx = fx;
                qfy = fy;
                // an empty lane's weights are zero, so that its input is zero
                const float ox = on_n ? 1.0f - fx : 0.0f, oy = 1.0f - fy;
                qw[0] = ox * oy;
                qw[1] = on_n ? fx * oy : 0.0f;
                qw[2] = ox * fy;
                qw[3] = on_n ? fx * fy : 0.0f;
                // unconditional loads (an empty lane reads texel 0 of triangle
                // 0 and its input is zeroed), so that the wait before their use
                // can leave the next block's loads in flight
                const size_t t00 =
                    on_n ? ((static_cast<size_t>(tri_n) * G + (cw >> 16)) * G + (cw & 0xFFFFu)) * S::C : 0;
                const size_t toff[4] = {0, S::C, static_cast<size_t>(G) * S::C, static_cast<size_t>(G + 1) * S::C};
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int ch = 16 * cb + 4 * grp < S::C ? 16 * cb + 4 * grp : 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) qv[cb][q] = *reinterpret_cast<gfloat4*>(feats + t00 + toff[q] + ch);
                }
            };
            gather(0);
            // While a wave runs its chains of products it issues ahead of the other
            // wave of its SIMD, whose LDS and VALU work then fills the gaps between
            // them: priority 2 for the MLP, 1 for the grid adds, the default for the
            // vertex chain and the record loads (decode 2.95 -> 2.91 ms).
            __builtin_amdgcn_s_setprio(2);
            for (int nb = 0; nb < 4; ++nb) {   // fragment 16 nb + col (lane 16 nb + col holds its record)
                // inputs, unit-major: channels 16 cb + 4 grp .. + 3 (an empty lane's
                // weights are zero; channels past C meet zero weights in layer 0)
                f4v xin[CB];
                // d feature / d fx and d feature / d fy at the fragment's texture
                // position (bilinear), the directions in which a winner's vertices
                // move its texture sample (an empty lane's are multiplied by a
                // zero feature gradient)
                f4v tgx[CB], tgy[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const float4 q00 = qv[cb][0], q10 = qv[cb][1], q01 = qv[cb][2], q11 = qv[cb][3];
                    const float ax = 1.0f - qfy, ay = 1.0f - qfx;
                    const float a00[4] = {q00.x, q00.y, q00.z, q00.w}, a10[4] = {q10.x, q10.y, q10.z, q10.w};
                    const float a01[4] = {q01.x, q01.y, q01.z, q01.w}, a11[4] = {q11.x, q11.y, q11.z, q11.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        xin[cb][i] = __builtin_fmaf(qw[3], a11[i], __builtin_fmaf(qw[2], a01[i],
                                                    __builtin_fmaf(qw[1], a10[i], qw[0] * a00[i])));
                        tgx[cb][i] = __builtin_fmaf(ax, a10[i] - a00[i], qfy * (a11[i] - a01[i]));
                        tgy[cb][i] = __builtin_fmaf(ay, a01[i] - a00[i], qfx * (a11[i] - a10[i]));
                    }
                }
                if (nb < 3) gather(nb + 1);
                // the block fragment's gates of this lane's units 16 ob + 4 grp + i
                uint32_t gate0[HB], gate1[HB];
#pragma unroll
                for (int ob = 0; ob < HB; ++ob) {
                    gate0[ob] = 0u;
                    gate1[ob] = 0u;
                }
                if (use_gates) {
#pragma unroll
                    for (int ob = 0; ob < HB; ++ob) {
                        constexpr int kH = S::H;
                        const int b0 = 16 * ob, b1 = kH + 16 * ob;   // first unit of the block, layers 0 and 1
                        const uint32_t w0 = row_bcast(gt[b0 >> 5], nb);
                        gate0[ob] = (w0 >> ((b0 & 31) + 4 * grp)) & 0xFu;
                        if constexpr (S::NH == 2) {
                            const uint32_t w1 = row_bcast(gt[b1 >> 5], nb);
                            gate1[ob] = (w1 >> ((b1 & 31) + 4 * grp)) & 0xFu;
                        }
                    }
                }
                // forward
                f4v h0[HB];
                mfma_layer_gated<HB, CB>(Wt.l0, Wt.b0, xin, h0, lane, use_gates, gate0);
                f4v h1[S::NH == 2 ? HB : 1];
                if constexpr (S::NH == 2) mfma_layer_gated<HB, HB>(Wt.l1, Wt.b1, h0, h1, lane, use_gates, gate1);
                const f4v (&hl)[HB] = *reinterpret_cast<const f4v (*)[HB]>(S::NH == 2 ? &h1[0] : &h0[0]);
                // output layer and the logit gradients (Eq. (9) through the sigmoid for the score term)
                float dO;   // lane group j: output j of the fragment
                // an empty fragment has zero colour gradient and score weight, so its dO is zero
                const bool win_n = (row_bcast(fkey, nb) >> 31) != 0;
                const float gl_n = row_bcast(__uint_as_float(fb4.x), nb);
                {
                    // lane group g: outputs 0..3 summed over its own units 16 ib + 4 g + s
                    f4v pr = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ib = 0; ib < HB; ++ib) {
                        const f4v wv = Wt.lo[ib][lane];
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4) pr = mfma4x4(wv[s4], hl[ib][s4], pr);
                    }
                    // the four lane groups' parts summed, output g to lane group g
                    const float og = pair16f(pair32f(pr[0], pr[2]), pair32f(pr[1], pr[3])) + Wt.bo[lane];
                    const float g0 = row_bcast(__uint_as_float(fb4.y), nb), g1 = row_bcast(__uint_as_float(fb4.z), nb),
                                g2 = row_bcast(__uint_as_float(fb4.w), nb);
                    const float sg = sigmoid_fast(og);
                    float d;
                    if (grp == 3) d = win_n ? gl_n * (1.0f - sg) : -gl_n * sg;
                    else d = win_n ? (grp == 0 ? g0 : (grp == 1 ? g1 : g2)) * sg * (1.0f - sg) : 0.0f;
                    dO = d;
                }
                // A winner's vertices move with the feature gradient of its colour
                // logits only: the score logit reaches texture and MLP but no vertex
                // (Section 3.2). Where a winner of the block carries a score weight,
                // the colour logits get a data backward of their own; otherwise the
                // full one below is the same thing.
                const bool split = __ballot(win_n && gl_n != 0.0f) != 0;
                const float dOc = grp == 3 ? 0.0f : dO;
                float pfx = 0.0f, pfy = 0.0f;   // this lane's channels of d logits / d (fx, fy)
                // output-layer weight gradient (rows = this block's fragments)
                stage_rows<HB>(st, S::H, hl, lane);
                st[kStageRows * (S::H + kRowPad) + col * (4 + kRowPad) + grp] = dO;
                wave_fence();
                acc.out.accumulate(st, st + kStageRows * (S::H + kRowPad), lane);
                {
                    const f4v db[1] = {f4v{dO, 0.f, 0.f, 0.f}};
                    acc.out.add_bias(db);
                }
                wave_fence();
                // back through the output layer: K = the four outputs, one step
                // (with split, the colour logits' backward runs beside it)
                f4v dl[HB], dlc[HB];
#pragma unroll
                for (int ob = 0; ob < HB; ++ob) {
                    const float wl = Wt.loT[ob][lane];
                    f4v v = mfma4(wl, dO, f4v{0.f, 0.f, 0.f, 0.f});
                    f4v vc = split ? mfma4(wl, dOc, f4v{0.f, 0.f, 0.f, 0.f}) : f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        v[i] = hl[ob][i] > 0.0f ? v[i] : 0.0f;
                        vc[i] = hl[ob][i] > 0.0f ? vc[i] : 0.0f;
                    }
                    dl[ob] = v;
                    dlc[ob] = vc;
                }
                f4v dh0[HB], dh0c[HB];
                if constexpr (S::NH == 2) {
                    // hidden layer 1 weight gradient, then back to layer 0
                    stage_rows<HB>(st, S::H, h0, lane);
                    stage_rows<HB>(st + kStageRows * (S::H + kRowPad), S::H, dl, lane);
                    wave_fence();
                    acc.mid[0].accumulate(st, st + kStageRows * (S::H + kRowPad), lane);
                    acc.mid[0].add_bias(dl);
                    wave_fence();
                    if (split) mfma_back2<HB, HB, true>(Wt.l1T, dl, dlc, h0, dh0, dh0c, lane);
                    else mfma_back<HB, HB, true>(Wt.l1T, dl, h0, dh0, lane);
                } else {
#pragma unroll
                    for (int ob = 0; ob < HB; ++ob) {
                        dh0[ob] = dl[ob];
                        dh0c[ob] = dlc[ob];
                    }
                }
                // first-layer weight gradient
                stage_rows<CB>(st, S::C, xin, lane);
                stage_rows<HB>(st + kStageRows * (S::C + kRowPad), S::H, dh0, lane);
                wave_fence();
                acc.l0.accumulate(st, st + kStageRows * (S::C + kRowPad), lane);
                acc.l0.add_bias(dh0);
                wave_fence();
                // feature gradients into the rows [fragment][C] kept past the stage's working rows;
                // the winners' vertices move with those of the colour logits alone
                f4v dxv[CB], dxc[CB];
                if (split) {
                    mfma_back2<CB, HB, false>(Wt.l0T, dh0, dh0c, nullptr, dxv, dxc, lane);
                } else {
                    mfma_back<CB, HB, false>(Wt.l0T, dh0, nullptr, dxv, lane);
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) dxc[cb] = dxv[cb];
                }
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int ch = 16 * cb + 4 * grp;
                    if (ch < S::C)
                        *reinterpret_cast<float4*>(s_dx[w] + (16 * nb + col) * DXS + ch) =
                            make_float4(dxv[cb][0], dxv[cb][1], dxv[cb][2], dxv[cb][3]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        pfx = __builtin_fmaf(dxc[cb][i], tgx[cb][i], pfx);
                        pfy = __builtin_fmaf(dxc[cb][i], tgy[cb][i], pfy);
                    }
                }
                // sum over the four lane groups' channels; lane 16 nb + col keeps
                // the values of its own fragment
                pfx = rows_sum(pfx);
                pfy = rows_sum(pfy);
                if (grp == nb) {
                    my_dfx = pfx;
                    my_dfy = pfy;
                }
            }
            wave_fence();
        }
        __builtin_amdgcn_s_setprio(0);
        pixfetch();   // the next batch's winners
        // --- the winner's world-space vertex gradient, in double precision ---
        // The chain is evaluated at the snapped vertex positions and the pixel
        // centre from exact integers, with the clip coordinates recomputed in
        // the setup's float32 order; its sums cancel, and float32 left errors
        // of about 1e-4 of a vertex's total.
        double gw[9] = {0., 0., 0., 0., 0., 0., 0., 0., 0.};
        if (win) {
            const ViewDesc& vd = a.views[fc4.z];
            const TriRec& tr = a.recs[vd.rec_base + tri];
            const int W = vd.W, H = vd.H;
            // the pixel within its view (below 2^32: a view has at most 16384^2 pixels)
            const uint32_t local = pix - static_cast<uint32_t>(vd.pix_base);
            const int py = static_cast<int>(local / static_cast<uint32_t>(W));
            const int px = static_cast<int>(local - static_cast<uint32_t>(py) * static_cast<uint32_t>(W));
            // texture position -> barycentrics -> vertex screen positions and 1/w
            const double gm1 = static_cast<double>(G - 1);
            double iwv[3];
            int32_t Xv[3], Yv[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                iwv[i] = tr.iw[i];
                Xv[i] = tr.X[i];
                Yv[i] = tr.Y[i];
            }
            const int32_t PX = kSnap * px + kSnap / 2, PY = kSnap * py + kSnap / 2;
            // screen barycentrics beta_i = E_i / A: E_i the orientation-normalised
            // integer edge function of edge i at the pixel centre, A their sum.
            // Every factor is an integer below 2^26 and every E_i below 2^52, so
            // the products and the fused sums are exact in double.
            double fb[3];
            {
                const double sgn = tr.rA < 0.0f ? -1.0 : 1.0;
                double Ei[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int ea = i == 2 ? 0 : i + 1, eb = i == 0 ? 2 : (i == 1 ? 0 : 1);
                    const double ex = static_cast<double>(Xv[eb] - Xv[ea]), ey = static_cast<double>(Yv[eb] - Yv[ea]);
                    Ei[i] = sgn * __builtin_fma(ex, static_cast<double>(PY - Yv[ea]),
                                                -(ey * static_cast<double>(PX - Xv[ea])));
                }
                const double inv_a = rcp64((Ei[0] + Ei[1]) + Ei[2]);
#pragma unroll
                for (int i = 0; i < 3; ++i) fb[i] = Ei[i] * inv_a;
            }
            const double tt[3] = {fb[0] * iwv[0], fb[1] * iwv[1], fb[2] * iwv[2]};
            const double inv_s = rcp64((tt[0] + tt[1]) + tt[2]);
            const double bb[3] = {tt[0] * inv_s, tt[1] * inv_s, tt[2] * inv_s};
            const double db[3] = {0.0, static_cast<double>(my_dfx) * gm1, static_cast<double>(my_dfy) * gm1};
            const double dot = db[1] * bb[1] + db[2] * bb[2];
            double dbeta[3], diw[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double dt = (db[i] - dot) * inv_s;
                dbeta[i] = dt * iwv[i];
                diw[i] = dt * fb[i];
            }
            const double Ai = __builtin_fma(static_cast<double>(Xv[1] - Xv[0]), static_cast<double>(Yv[2] - Yv[0]),
                                            -(static_cast<double>(Yv[1] - Yv[0]) * static_cast<double>(Xv[2] - Xv[0])));
            const double inv_area = 65536.0 * rcp64(Ai);   // 1 / (signed 2 x area in px^2)
            const double inv256 = 1.0 / 256.0;
            // beta_i = e_i / area, e_i = edge(v_p(i), v_q(i), pixel centre) with edge i
            // joining vertices p(i) = i + 1 and q(i) = i + 2 (mod 3). Vertex jv moves
            // e_i only for the two edges it belongs to (i = jv + 2 as p, i = jv + 1 as
            // q), and the area as a whole; so d beta . dbeta / d(vertex jv) is
            // (sum over those two edges of dbeta_i de_i - d area . sb) / area with
            // sb = sum_i dbeta_i beta_i.
            double sb = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) sb = __builtin_fma(dbeta[i], fb[i], sb);
            double gsx[3], gsy[3];
#pragma unroll
            for (int jv = 0; jv < 3; ++jv) {
                const int jp = jv == 2 ? 0 : jv + 1, jq = jv == 0 ? 2 : (jv == 1 ? 0 : 1);
                const double dax = static_cast<double>(Yv[jp] - Yv[jq]) * inv256;
                const double day = static_cast<double>(Xv[jq] - Xv[jp]) * inv256;
                // edge ip has jv as its first vertex (its other one is jp), edge iq as its second (other: jq)
                const int ip = jv == 0 ? 2 : jv - 1, iq = jv == 2 ? 0 : jv + 1;
                const double ex_p = static_cast<double>(Yv[jp] - PY) * inv256, ey_p = static_cast<double>(PX - Xv[jp]) * inv256;
                const double ex_q = static_cast<double>(PY - Yv[jq]) * inv256, ey_q = static_cast<double>(Xv[jq] - PX) * inv256;
                gsx[jv] = (__builtin_fma(dbeta[ip], ex_p, dbeta[iq] * ex_q) - dax * sb) * inv_area;
                gsy[jv] = (__builtin_fma(dbeta[ip], ey_p, dbeta[iq] * ey_q) - day * sb) * inv_area;
            }
            // edge term (Section 3.2): the boundaries this pixel occludes move
            // with its surface point, w beta_i e on the screen position of vertex i
            const double ex = __uint_as_float(fc4.x), ey = __uint_as_float(fc4.y);
#pragma unroll
            for (int jv = 0; jv < 3; ++jv) {
                gsx[jv] += ex * fb[jv];
                gsy[jv] += ey * fb[jv];
            }
            // screen position (s = W/2 (c_x / c_w) + W/2, H/2 - H/2 (c_y / c_w)) and 1/w
            // -> clip -> world through the view-projection
            const double hw = 0.5 * W, hh = 0.5 * H;
            const float* vp = a.verts + static_cast<size_t>(tri) * 9;
#pragma unroll
            for (int jv = 0; jv < 3; ++jv) {
                const float x = vp[3 * jv], y = vp[3 * jv + 1], z = vp[3 * jv + 2];
                float cc[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {   // the setup's transform (row z unused)
                    float acc = vd.M[j * 4 + 3];
                    acc = __builtin_fmaf(vd.M[j * 4 + 0], x, acc);
                    acc = __builtin_fmaf(vd.M[j * 4 + 1], y, acc);
                    acc = __builtin_fmaf(vd.M[j * 4 + 2], z, acc);
                    cc[j] = acc;
                }
                const double cx = cc[0], cy = cc[1], iw = rcp64(static_cast<double>(cc[3]));
                const double gc0 = gsx[jv] * hw * iw;
                const double gc1 = -gsy[jv] * hh * iw;
                const double gc3 = (-gsx[jv] * hw * cx + gsy[jv] * hh * cy - diw[jv]) * (iw * iw);
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    gw[3 * jv + k] = static_cast<double>(vd.M[k]) * gc0 + static_cast<double>(vd.M[4 + k]) * gc1 +
                                     static_cast<double>(vd.M[12 + k]) * gc3;
            }
        }
        __builtin_amdgcn_s_setprio(1);
        // --- sum into the wave's grid, one run of equal triangles at a time ---
        // The feature gradients are staged (row = fragment) and added one
        // fragment per step with the wave's lanes spread over (corner,
        // channel), so that no two lanes of an LDS add share an address;
        // the winners' vertex gradients are summed over the run by a wave
        // reduction.
        constexpr int LPF = 4 * S::C;                  // (corner, channel) pairs of one fragment
        constexpr int FPS = LPF >= 64 ? 1 : 64 / LPF;  // fragments per step
        constexpr int PPF = LPF >= 64 ? LPF / 64 : 1;  // steps per fragment
        // One fragment per step: each lane's fragment leaves its four corner
        // weights (corner q = 2 dy + dx) in the stage, free once the MLP is
        // done, and keeps its cell's first texel; the steps then need no
        // per-fragment weight or address arithmetic beyond one add.
        int cbase = 0;
        if constexpr (FPS == 1) {
            const float x1 = c.fx, y1 = c.fy, x0 = 1.0f - c.fx, y0 = 1.0f - c.fy;
            *reinterpret_cast<float4*>(st + 4 * lane) = make_float4(x0 * y0, x1 * y0, x0 * y1, x1 * y1);
            cbase = (c.iy * G + c.ix) * S::C;
        }
        wave_fence();
        const uint32_t tkey = on ? tri : 0xFFFFFFFFu;
        const uint32_t tprev = __shfl_up(tkey, 1, 64);
        uint64_t heads = __ballot(lane == 0 || tprev != tkey);
        while (heads) {
            const int h = __builtin_ctzll(heads);
            heads &= heads - 1;
            const int t = __builtin_amdgcn_readlane(static_cast<int>(tkey), h);
            if (t < 0) break;   // the sentinel run: empty lanes at the batch's end
            if (t != cur) {
                if (cur >= 0) flush(cur);
                cur = t;
            }
            const int end = heads ? __builtin_ctzll(heads) : 64;
            const bool in_run = lane >= h && lane < end;
            if (__ballot(in_run && win)) {   // the run's winners: vertex gradient summed over the wave
                double v[9], q[3];
#pragma unroll
                for (int k = 0; k < 9; ++k) v[k] = in_run ? gw[k] : 0.0;   // gw is zero for fragments in front
                wave_sum9(v, q);
                if ((lane & 15) == 0) {   // row g's first lane: components c, c + 2 (and 4 in row 0)
                    const int g = lane >> 4, c0 = (g & 1) + 5 * (g >> 1);
                    vgrid[c0] += q[0];
                    vgrid[c0 + 2] += q[1];
                    if (g == 0) vgrid[4] += q[2];
                }
            }
            constexpr int UF = 4;                          // steps in flight: their staged reads go first
            if constexpr (FPS == 1) {
                // lane (corner q, channel k) of step pp: weight st[4 f + q],
                // gradient s_dx[f][k], texel q of the fragment's cell
                float* gl[PPF];
                const float* wl[PPF];
                const float* dl[PPF];
#pragma unroll
                for (int pp = 0; pp < PPF; ++pp) {
                    const int idx = pp * 64 + lane;
                    const int q = idx / S::C, k = idx % S::C;
                    gl[pp] = grid + ((q >> 1) * G + (q & 1)) * S::C + k;
                    wl[pp] = st + q;
                    dl[pp] = s_dx[w] + k;
                }
                auto add = [&](int f, const float (&wv)[PPF], const float (&dv)[PPF]) __attribute__((always_inline)) {
                    const int cb = __builtin_amdgcn_readlane(cbase, f);
#pragma unroll
                    for (int pp = 0; pp < PPF; ++pp) {
                        float* gp = gl[pp] + cb;   // one fragment: 64 distinct addresses
                        *gp = __builtin_fmaf(wv[pp], dv[pp], *gp);
                    }
                };
                int f = h;
                for (; f + UF <= end; f += UF) {
                    float wv[UF][PPF], dv[UF][PPF];
#pragma unroll
                    for (int u = 0; u < UF; ++u)
#pragma unroll
                        for (int pp = 0; pp < PPF; ++pp) {
                            wv[u][pp] = wl[pp][4 * (f + u)];
                            dv[u][pp] = dl[pp][(f + u) * DXS];
                        }
#pragma unroll
                    for (int u = 0; u < UF; ++u) add(f + u, wv[u], dv[u]);
                }
                for (; f < end; ++f) {
                    float wv[PPF], dv[PPF];
#pragma unroll
                    for (int pp = 0; pp < PPF; ++pp) {
                        wv[pp] = wl[pp][4 * f];
                        dv[pp] = dl[pp][f * DXS];
                    }
                    add(f, wv, dv);
                }
            } else {
                for (int f0 = h; f0 < end; f0 += FPS * UF) {
                    int fs[UF];
                    bool ok[UF];
                    float dv[UF];
#pragma unroll
                    for (int u = 0; u < UF; ++u) {
                        const int f = f0 + u * FPS + lane / LPF;
                        ok[u] = f < end;
                        fs[u] = ok[u] ? f : h;                     // lanes past the run repeat h with weight 0
                        dv[u] = s_dx[w][fs[u] * DXS + lane % LPF % S::C];
                    }
#pragma unroll
                    for (int u = 0; u < UF; ++u) {
                        const uint32_t cw = static_cast<uint32_t>(__shfl(static_cast<int>(cellw), fs[u], 64));
                        const float fx = __shfl(c.fx, fs[u], 64);
                        const float fy = __shfl(c.fy, fs[u], 64);
                        const int ix = static_cast<int>(cw & 0xFFFFu), iy = static_cast<int>(cw >> 16);
                        const int q = lane % LPF / S::C, k = lane % LPF % S::C;   // corner, channel
                        const int dxq = q & 1, dyq = q >> 1;
                        const float wq = (dxq ? fx : 1.0f - fx) * (dyq ? fy : 1.0f - fy);
                        // two fragments per step may share a texel
                        atomicAdd(&grid[((iy + dyq) * G + ix + dxq) * S::C + k], ok[u] ? wq * dv[u] : 0.0f);
                    }
                }
            }
            wave_fence();
        }
    }
    if (!LOGP && cur >= 0) flush(cur);
    if (!LOGP) {
        float* row = a.mlp_partial + (static_cast<size_t>(blockIdx.x) * NW + w) * S::kParams;
        acc.l0.store(row, S::w_off(0), S::b_off(0), lane);
        if constexpr (S::NH == 2) acc.mid[0].store(row, S::w_off(1), S::b_off(1), lane);
        acc.out.store(row, S::w_off(S::NH), S::b_off(S::NH), lane);
    }
}

// The forward's ReLU gates of every fragment of a replayed list (a backward
// without the forward's log): each lane decodes its fragment with the
// forward's float32 arithmetic (the contract's texture fetch and MLP, from the
// same barycentrics) and keeps the gates in gates_out, at the fragment's slot
// of the region list. Waves take batches as the logp decode does.
template <class S>
__global__ __launch_bounds__(256) void fragment_gates_kernel(DecodeArgs a, uint32_t* __restrict__ gates_out) {
    constexpr int NW = 4, GW = GateWords<S>::kWords;
    __shared__ uint32_t s_boff[kMaxRegions + 1];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i <= a.n_regions; i += blockDim.x) s_boff[i] = a.boff[i];
    __syncthreads();
    gfloat* __restrict__ feats = as_global(uniform_ptr(a.feats));
    const uint32_t n_batch = s_boff[a.n_regions];
    const uint32_t n_waves = gridDim.x * NW;
    for (uint32_t bi = blockIdx.x * NW + w; bi < n_batch; bi += n_waves) {
        int lo = 0, hi = a.n_regions - 1;   // region: last w with boff[w] <= bi
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_boff[mid] <= bi) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t cr = a.counts[lo];
        const uint32_t in_region = (bi - s_boff[lo]) * 64u + static_cast<uint32_t>(lane);
        if (in_region >= (cr < a.region ? cr : a.region)) continue;
        const uint64_t at = static_cast<uint64_t>(lo) * a.region + in_region;
        const FragRec fr = a.frags[at];
        const Cell c = cell_of(__uint_as_float(fr.p1.x), __uint_as_float(fr.p1.y), a.G);
        float x[S::C];
        fetch_feature<S::C>(feats, fr.p0.y & 0x7FFFFFFFu, a.G, c, x);
        float o[4];
        uint32_t g[GW];
        mlp_logits_gates<S>(as_const(opaque_ptr(a.mlp)), x, o, g);
#pragma unroll
        for (int k = 0; k < GW; k += 2)   // the padded gate record, 8 bytes at a time
            reinterpret_cast<uint2*>(gates_out)[at * (gate_stride(GW) / 2) + k / 2] =
                make_uint2(g[k], k + 1 < GW ? g[k + 1] : 0u);
    }
}

template <class S>
static void launch_fragment_gates_s(const DecodeArgs& a, uint32_t* gates_out, hipStream_t s) {
    hipLaunchKernelGGL(fragment_gates_kernel<S>, dim3(a.n_blocks), dim3(256), 0, s, a, gates_out);
}

// Bytes of LDS one workgroup of the decode needs (static + dynamic), or 0 when
// the runtime cannot say.
template <class S>
static size_t decode_bwd_lds_s(int G, bool logp) {
    hipFuncAttributes fa;
    const hipError_t e = logp ? hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(decode_bwd_kernel<S, true>))
                              : hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(decode_bwd_kernel<S, false>));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const size_t dyn = logp ? 0 : static_cast<size_t>(4) * (static_cast<size_t>(G) * G * S::C + kGridTail) * sizeof(float);
    return fa.sharedSizeBytes + dyn;
}

template <class S>
static void launch_decode_bwd_s(const DecodeArgs& a, bool logp, hipStream_t s) {
    if (logp) {
        hipLaunchKernelGGL((decode_bwd_kernel<S, true>), dim3(a.n_blocks), dim3(256), 0, s, a);
    } else {
        const size_t lds = static_cast<size_t>(4) * (static_cast<size_t>(a.G) * a.G * S::C + kGridTail) * sizeof(float);
        hipLaunchKernelGGL((decode_bwd_kernel<S, false>), dim3(a.n_blocks), dim3(256), lds, s, a);
    }
}

}  // namespace soup
