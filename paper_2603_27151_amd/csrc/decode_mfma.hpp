#pragma once
// The backward's MLP over a 64-fragment batch on the matrix cores
// (v_mfma_f32_16x16x4f32): recompute, data backward and weight gradient.
//
// Operand layout of the instruction (lane l, col = l & 15, grp = l >> 4): the
// lane supplies A[col][grp] and B[grp][col] (K = 4 runs over the four lane
// groups) and holds D[4 grp + i][col], i = 0..3.
//
// Activations are kept unit-major: an f4v act[ub][nb] holds units
// 16 ub + 4 grp + i of fragment 16 nb + col. A layer out = W in runs as
// D = W act with the contraction over input units split in steps of four,
// step s of input block ib taking unit 16 ib + 4 grp + s in lane group grp;
// the B operand of step s is then register s of the previous layer's D, so
// layers chain without moving data between lanes, and the A operand is the
// weight W[16 ob + col][16 ib + 4 grp + s] (pre-arranged in LDS, four steps
// per 16-byte read). The output layer (four outputs) runs on
// v_mfma_f32_4x4x1f32, sixteen independent 4x4 blocks of four lanes each
// (lane 4b + j supplies A[j][0] and B[0][j] of block b and holds D[i][j] in
// register i): block b's lanes share one lane group, so its B operand is the
// hidden units 16 ib + 4 grp + s of four fragments and its A operand the four
// outputs' weights of those units; the four lane groups' partial sums are
// then summed across rows with row swaps so that lane group j ends with
// output j of every fragment, which is exactly the B operand of the first
// backward product (K = the 4 outputs).
// Weight gradients contract over fragments, the other index; activations and
// deltas are staged through LDS as rows, 16 fragments at a time.
//
// The backward needs no bit-exact forward (only the forward's mask decision
// is fixed by the contract), so the recompute may sum in the matrix cores'
// order.
#include "raster_common.hpp"

namespace soup {

typedef float f4v __attribute__((ext_vector_type(4)));

// Staged rows in LDS are padded by this many floats: the 16 rows a wave writes
// at once then start on different banks (unpadded rows of 16 or 32 floats all
// began on the same four).
constexpr int kRowPad = 4;

__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma4x4(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// ---- cross-lane moves on the vector ALU ----
// A wave's 64 lanes are four rows of 16. gfx950's row swaps exchange rows
// between two registers in one VALU instruction, where a general shuffle
// (ds_bpermute) would go through the LDS pipe and wait for it:
//   swap16(a, b) -> (a.r0, b.r0, a.r2, b.r2), (a.r1, b.r1, a.r3, b.r3)
//   swap32(a, b) -> (a.r0, a.r1, b.r0, b.r1), (a.r2, a.r3, b.r2, b.r3)
// (rX = row X; the lane within the row is kept).
struct U2 {
    uint32_t a, b;
};
__device__ __forceinline__ U2 swap16(uint32_t a, uint32_t b) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    return {static_cast<uint32_t>(r[0]), static_cast<uint32_t>(r[1])};
}
__device__ __forceinline__ U2 swap32(uint32_t a, uint32_t b) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    return {static_cast<uint32_t>(r[0]), static_cast<uint32_t>(r[1])};
}

// Row n of x in every row: lane (row g, column c) receives lane 16 n + c.
// Two swaps; the first is shared by every n (the compiler merges it).
__device__ __forceinline__ uint32_t row_bcast(uint32_t x, int n) {
    const U2 h = swap16(x, x);                   // (x0, x0, x2, x2), (x1, x1, x3, x3)
    const uint32_t y = (n & 1) ? h.b : h.a;
    const U2 q = swap32(y, y);                   // (y0, y0, y0, y0), (y2, y2, y2, y2)
    return (n & 2) ? q.b : q.a;
}
__device__ __forceinline__ float row_bcast(float x, int n) {
    return __uint_as_float(row_bcast(__float_as_uint(x), n));
}

// Sum over the four rows, in every row: (x0 + x1) + (x2 + x3) per column.
__device__ __forceinline__ float rows_sum(float x) {
    const U2 h = swap16(__float_as_uint(x), __float_as_uint(x));
    const float y = __uint_as_float(h.a) + __uint_as_float(h.b);
    const U2 q = swap32(__float_as_uint(y), __float_as_uint(y));
    return __uint_as_float(q.a) + __uint_as_float(q.b);
}

// a over rows {0, 1} + {2, 3} in rows 0 and 1, b likewise in rows 2 and 3.
__device__ __forceinline__ float pair32f(float a, float b) {
    const U2 r = swap32(__float_as_uint(a), __float_as_uint(b));
    return __uint_as_float(r.a) + __uint_as_float(r.b);
}
// a over rows 0 + 1 in row 0 and 2 + 3 in row 2; b likewise in rows 1 and 3.
__device__ __forceinline__ float pair16f(float a, float b) {
    const U2 r = swap16(__float_as_uint(a), __float_as_uint(b));
    return __uint_as_float(r.a) + __uint_as_float(r.b);
}

// Doubles through the 32-bit moves, one half at a time.
__device__ __forceinline__ uint32_t dlo(double v) { return static_cast<uint32_t>(__double_as_longlong(v)); }
__device__ __forceinline__ uint32_t dhi(double v) { return static_cast<uint32_t>(__double_as_longlong(v) >> 32); }
__device__ __forceinline__ double djoin(uint32_t lo, uint32_t hi) {
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// a over rows {0, 1} + {2, 3} in rows 0 and 1, b likewise in rows 2 and 3.
__device__ __forceinline__ double pair32(double a, double b) {
    const U2 l = swap32(dlo(a), dlo(b)), h = swap32(dhi(a), dhi(b));
    return djoin(l.a, h.a) + djoin(l.b, h.b);
}
// a over rows 0 + 1 in row 0 and 2 + 3 in row 2; b likewise in rows 1 and 3.
__device__ __forceinline__ double pair16(double a, double b) {
    const U2 l = swap16(dlo(a), dlo(b)), h = swap16(dhi(a), dhi(b));
    return djoin(l.a, h.a) + djoin(l.b, h.b);
}

// Lane l + x of the lane's row by a DPP pattern, for both halves.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(dlo(v)), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(dhi(v)), CTRL, 0xF, 0xF, false);
    return djoin(static_cast<uint32_t>(lo), static_cast<uint32_t>(hi));
}
// Sum over the 16 lanes of each row, in every lane of the row: partners at
// distance 1 and 2 within quads, then the half-row and row mirrors (lane i
// with 7 - i, then with 15 - i).
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);   // row_half_mirror
    v += dpp_d<0x140>(v);   // row_mirror
    return v;
}

// Nine per-lane doubles summed over the wave as a transposed reduction
// (each exchange carries two components): on return, lane 16 g of row g
// holds the sums of components c = (g & 1) + 5 (g >> 1) in q[0] and c + 2 in
// q[1], and row 0 that of component 4 in q[2].
__device__ __forceinline__ void wave_sum9(const double (&v)[9], double (&q)[3]) {
    double r[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) r[k] = pair32(v[k], k + 5 < 9 ? v[k + 5] : 0.0);   // rows 0-1: k, rows 2-3: k + 5
    q[0] = pair16(r[0], r[1]);   // rows: 0, 1, 5, 6
    q[1] = pair16(r[2], r[3]);   // rows: 2, 3, 7, 8
    q[2] = pair16(r[4], 0.0);    // row 0: 4
#pragma unroll
    for (int j = 0; j < 3; ++j) q[j] = row16_sum(q[j]);
}

// Weights and biases of one MLP in the A-operand arrangement, per lane.
template <class S>
struct MfmaWeights {
    static constexpr int CB = (S::C + 15) / 16;   // channel blocks
    static constexpr int HB = S::H / 16;          // hidden-unit blocks
    static constexpr int MB = S::NH == 2 ? HB : 1;
    f4v l0[HB][CB][64];      // W0[16 ob + col][16 ib + 4 grp + s]
    f4v l1[MB][MB][64];      // W1[16 ob + col][16 ib + 4 grp + s]
    f4v lo[HB][64];          // W_out[lane & 3][16 ib + 4 grp + s]: A operand of the 4x4x1 output products
    float loT[HB][64];       // W_out[grp][16 ob + col]
    f4v l1T[MB][MB][64];     // W1[16 ib + 4 grp + s][16 ob + col]
    f4v l0T[CB][HB][64];     // W0[16 ib + 4 grp + s][16 cb + col]
    f4v b0[HB][64];          // b0[16 ob + 4 grp + i]
    f4v b1[MB][64];          // b1[16 ob + 4 grp + i]
    float bo[64];            // b_out[grp]

    // Cooperative fill by the whole workgroup from the flat parameter array.
    __device__ void load(const float* __restrict__ p, int tid, int nt) {
        const float* W0 = p + S::w_off(0);
        const float* B0 = p + S::b_off(0);
        const float* WO = p + S::w_off(S::NH);
        const float* BO = p + S::b_off(S::NH);
        for (int e = tid; e < HB * CB * 64; e += nt) {
            const int l = e & 63, ib = (e >> 6) % CB, ob = (e >> 6) / CB, col = l & 15, grp = l >> 4;
            f4v v, t;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 16 * ib + 4 * grp + s;
                v[s] = k < S::C ? W0[(16 * ob + col) * S::C + k] : 0.0f;
            }
            l0[ob][ib][l] = v;
            // transposed: output block = channel block ib (as cb), input block = ob (as unit block)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int u = 16 * ob + 4 * grp + s, ch = 16 * ib + col;
                t[s] = ch < S::C ? W0[u * S::C + ch] : 0.0f;
            }
            l0T[ib][ob][l] = t;
        }
        for (int e = tid; e < HB * 64; e += nt) {
            const int l = e & 63, b = e >> 6, col = l & 15, grp = l >> 4;
            f4v v, bb;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 16 * b + 4 * grp + s;
                v[s] = WO[(l & 3) * S::H + k];
                bb[s] = B0[16 * b + 4 * grp + s];
            }
            lo[b][l] = v;
            b0[b][l] = bb;
            loT[b][l] = WO[grp * S::H + 16 * b + col];
        }
        if constexpr (S::NH == 2) {
            const float* W1 = p + S::w_off(1);
            const float* B1 = p + S::b_off(1);
            for (int e = tid; e < HB * HB * 64; e += nt) {
                const int l = e & 63, ib = (e >> 6) % HB, ob = (e >> 6) / HB, col = l & 15, grp = l >> 4;
                f4v v, t;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    v[s] = W1[(16 * ob + col) * S::H + 16 * ib + 4 * grp + s];
                    t[s] = W1[(16 * ib + 4 * grp + s) * S::H + 16 * ob + col];
                }
                l1[ob][ib][l] = v;
                l1T[ob][ib][l] = t;
            }
            for (int e = tid; e < HB * 64; e += nt) {
                const int l = e & 63, b = e >> 6, grp = l >> 4;
                f4v bb;
#pragma unroll
                for (int s = 0; s < 4; ++s) bb[s] = B1[16 * b + 4 * grp + s];
                b1[b][l] = bb;
            }
        }
        for (int e = tid; e < 64; e += nt) bo[e] = BO[e >> 4];
    }
};

// One 16-fragment block: out[ob] = act(bias + W in), IB input blocks, OB
// output blocks.
template <int OB, int IB, bool RELU>
__device__ __forceinline__ void mfma_layer(const f4v (*w)[IB][64], const f4v (*bias)[64], const f4v (&in)[IB],
                                           f4v (&out)[OB], int lane) {
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
        f4v acc = bias[ob][lane];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
            const f4v wv = w[ob][ib][lane];
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma4(wv[s], in[ib][s], acc);
        }
        if (RELU) {
#pragma unroll
            for (int i = 0; i < 4; ++i)   // max(x, 0) on the bit pattern: one integer max, no canonicalisation
                acc[i] = __int_as_float(max(__float_as_int(acc[i]), 0));
        }
        out[ob] = acc;
    }
}

// mfma_layer with the ReLU gate of unit 16 ob + 4 grp + i taken from bit i of
// gate[ob] when use_gates (the forward's decision, logged by its bit-exact
// decode), else from the sign of the recomputed value. The recompute sums in
// the matrix cores' order, so a pre-activation within rounding of zero may
// land on the other side of the kink than in the forward; the logged gate
// keeps the forward's side. An open gate keeps at least FLT_MIN, so that the
// "> 0" tests of the backward see it.
template <int OB, int IB>
__device__ __forceinline__ void mfma_layer_gated(const f4v (*w)[IB][64], const f4v (*bias)[64], const f4v (&in)[IB],
                                                 f4v (&out)[OB], int lane, bool use_gates, const uint32_t (&gate)[OB]) {
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
        f4v acc = bias[ob][lane];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
            const f4v wv = w[ob][ib][lane];
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma4(wv[s], in[ib][s], acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (use_gates) {   // bit i of the gate as an all-ones or all-zeros mask
                const int m = static_cast<int>(gate[ob] << (31 - i)) >> 31;
                acc[i] = __int_as_float(__float_as_int(__builtin_fmaxf(acc[i], 0x1p-126f)) & m);
            } else {
                acc[i] = acc[i] > 0.0f ? acc[i] : 0.0f;
            }
        }
        out[ob] = acc;
    }
}

// One 16-fragment block: d_in[ob] = (W^T d_out), masked by act > 0 when MASK.
template <int OB, int IB, bool MASK>
__device__ __forceinline__ void mfma_back(const f4v (*wT)[IB][64], const f4v (&d_out)[IB], const f4v* mask,
                                          f4v (&d_in)[OB], int lane) {
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
        f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
            const f4v wv = wT[ob][ib][lane];
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma4(wv[s], d_out[ib][s], acc);
        }
        if (MASK) {
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = mask[ob][i] > 0.0f ? acc[i] : 0.0f;
        }
        d_in[ob] = acc;
    }
}

// Two data backwards through the same layer at once (each weight operand read
// once, two independent product chains): d_in1 = W^T d_out1, d_in2 = W^T d_out2,
// both masked by act > 0 when MASK.
template <int OB, int IB, bool MASK>
__device__ __forceinline__ void mfma_back2(const f4v (*wT)[IB][64], const f4v (&d_out1)[IB], const f4v (&d_out2)[IB],
                                           const f4v* mask, f4v (&d_in1)[OB], f4v (&d_in2)[OB], int lane) {
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
        f4v acc1 = {0.f, 0.f, 0.f, 0.f}, acc2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
            const f4v wv = wT[ob][ib][lane];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc1 = mfma4(wv[s], d_out1[ib][s], acc1);
                acc2 = mfma4(wv[s], d_out2[ib][s], acc2);
            }
        }
        if (MASK) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                acc1[i] = mask[ob][i] > 0.0f ? acc1[i] : 0.0f;
                acc2[i] = mask[ob][i] > 0.0f ? acc2[i] : 0.0f;
            }
        }
        d_in1[ob] = acc1;
        d_in2[ob] = acc2;
    }
}

// The 16 rows of one fragment block into an LDS stage laid out [row][D + kRowPad]
// (D = n_units): lane (grp, col) writes its four units of row col.
template <int NBLK>
__device__ __forceinline__ void stage_rows(float* __restrict__ st, int D, const f4v (&v)[NBLK], int lane) {
    const int col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
        const int u = 16 * b + 4 * grp;
        if (u < D) *reinterpret_cast<float4*>(st + col * (D + kRowPad) + u) = make_float4(v[b][0], v[b][1], v[b][2], v[b][3]);
    }
}

}  // namespace soup
