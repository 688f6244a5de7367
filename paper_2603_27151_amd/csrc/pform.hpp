// Paper form of the step (Section 3.3, the learnable multi-resolution
// triangle texture and neural deferred shading; Supplement B.3, the shading
// MLP and the RGBA skip blend; Supplement B.6, 561 grid points at R = 5).
//
// Texture: per triangle the level-R mesh-colour grid, n = 2^R segments per
// edge, grid vertex (i, j) (i + j <= n) at barycentrics (i / n, j / n),
// stored row-major (row j holds the n + 1 - j vertices i = 0..n-j) with eight
// channels of 32 bytes: seven colour features, then the opacity, all already
// through the sigmoid. A fragment's values are those of the micro-triangle
// containing its perspective-correct barycentrics, interpolated linearly.
// Opacity stays outside the MLP: the mask needs one channel at three grid
// vertices per fragment. Only the winner of each pixel is shaded: its seven
// features and the nine degree-2 real spherical harmonics of the pixel's view
// direction feed a 16 -> 16 -> 16 -> 3 MLP (ReLU, sigmoid outputs), and the
// colour is A RGB + (1 - A) MLP with features 0..3 read as RGBA.
//
// Everything up to the mask decision and the deferred colour follows the
// float32 contract (explicit fused multiply-adds in a fixed order, correctly
// rounded division and square root, the contract's exp), so both reproduce
// an independent evaluation in the same order bit for bit.
#pragma once

#include "raster_common.hpp"

namespace soup {

constexpr int kPCh = 8;           // channels per grid vertex
constexpr int kPFeat = 7;         // colour features
constexpr int kPIn = 16, kPHid = 16, kPOut = 3;
constexpr int kPW0 = 0, kPB0 = kPW0 + kPHid * kPIn;
constexpr int kPW1 = kPB0 + kPHid, kPB1 = kPW1 + kPHid * kPHid;
constexpr int kPW2 = kPB1 + kPHid, kPB2 = kPW2 + kPOut * kPHid;
constexpr int kPParams = kPB2 + kPOut;   // 595
constexpr int kPMaxR = 7;         // finest level compiled for: 8385 grid vertices per triangle

// The forward raster's policy for this form (the workloads' MLP shapes carry
// kPaper = false).
struct PaperTex {
    static constexpr bool kPaper = true;
    static constexpr int C = kPCh, H = 0, NH = 0;
};

__host__ __device__ constexpr int mc_count(int R) { return ((1 << R) + 1) * ((1 << R) + 2) / 2; }

__device__ __forceinline__ int mc_index(int n, int i, int j) { return j * (n + 1) - (j * (j - 1)) / 2 + i; }

struct Micro {
    int idx[3];      // grid vertices (storage indices)
    float w[3];      // their weights
    float fu, fv;    // position inside the cell (i, j)
    bool inv;        // the inverted micro-triangle of the cell
};

// The micro-triangle containing (b1, b2) on the level with n segments per
// edge: u = b1 n, v = b2 n (exact, n a power of two), i = floor(u) in
// [0, n-1], j = floor(v) in [0, n-1-i], fu = u - i, fv = v - j; the inverted
// micro-triangle (i+1, j+1), (i+1, j), (i, j+1) when fu + fv > 1 and it
// exists, with weights (fu + fv - 1, 1 - fv, 1 - fu), else the upright one
// (i, j), (i+1, j), (i, j+1) with weights ((1 - fu) - fv, fu, fv).
__device__ __forceinline__ Micro micro_of(int n, float b1, float b2) {
    const float u = b1 * static_cast<float>(n), v = b2 * static_cast<float>(n);
    int i = static_cast<int>(__builtin_floorf(u));
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    int j = static_cast<int>(__builtin_floorf(v));
    j = j < 0 ? 0 : (j > n - 1 - i ? n - 1 - i : j);
    Micro m;
    m.fu = u - static_cast<float>(i);
    m.fv = v - static_cast<float>(j);
    const float s = m.fu + m.fv;
    m.inv = s > 1.0f && i + j <= n - 2;
    const int r0 = mc_index(n, i, j), r1 = mc_index(n, i, j + 1);   // rows j and j + 1 at column i
    if (m.inv) {
        m.idx[0] = r1 + 1;
        m.idx[1] = r0 + 1;
        m.idx[2] = r1;
        m.w[0] = s - 1.0f;
        m.w[1] = 1.0f - m.fv;
        m.w[2] = 1.0f - m.fu;
    } else {
        m.idx[0] = r0;
        m.idx[1] = r0 + 1;
        m.idx[2] = r1;
        m.w[0] = (1.0f - m.fu) - m.fv;
        m.w[1] = m.fu;
        m.w[2] = m.fv;
    }
    return m;
}

__device__ __forceinline__ float mc_mix(const Micro& m, float t0, float t1, float t2) {
    return __builtin_fmaf(m.w[2], t2, __builtin_fmaf(m.w[1], t1, m.w[0] * t0));
}

// Opacity of a fragment of triangle `tri` at (b1, b2): channel 7 of the
// micro-triangle's three grid vertices.
__device__ __forceinline__ float mc_alpha(gfloat* __restrict__ tex, uint32_t tri, int R, float b1, float b2) {
    const int n = 1 << R;
    const Micro m = micro_of(n, b1, b2);
    gfloat* t = tex + static_cast<size_t>(tri) * mc_count(R) * kPCh + (kPCh - 1);
    return mc_mix(m, t[m.idx[0] * kPCh], t[m.idx[1] * kPCh], t[m.idx[2] * kPCh]);
}

// Unit view direction through the centre of pixel (x, y): the pixel's
// normalised device coordinates at depth -1 and +1 through Minv (the inverse
// view-projection, row-major; each row bias first, then x, y, z by FMA),
// divided by w, the difference normalised.
__device__ __forceinline__ void view_dir(const float* __restrict__ Mi, int W, int H, int x, int y, float (&d)[3]) {
    const float nx = (2.0f * static_cast<float>(x) + 1.0f) / static_cast<float>(W) - 1.0f;
    const float ny = 1.0f - (2.0f * static_cast<float>(y) + 1.0f) / static_cast<float>(H);
    float p[2][4];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float nz = e == 0 ? -1.0f : 1.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float a = Mi[r * 4 + 3];
            a = __builtin_fmaf(Mi[r * 4 + 0], nx, a);
            a = __builtin_fmaf(Mi[r * 4 + 1], ny, a);
            a = __builtin_fmaf(Mi[r * 4 + 2], nz, a);
            p[e][r] = a;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = p[1][k] / p[1][3] - p[0][k] / p[0][3];
    const float len = __builtin_sqrtf(__builtin_fmaf(d[2], d[2], __builtin_fmaf(d[1], d[1], d[0] * d[0])));
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = d[k] / len;
}

// The nine real spherical harmonics of degree <= 2 of a unit vector
// (orthonormal on the sphere, no Condon-Shortley sign), in the order
// Y00; Y1 (y, z, x); Y2 (xy, yz, 2z^2 - x^2 - y^2, xz, x^2 - y^2).
__device__ __forceinline__ void sh2(const float (&d)[3], float* out) {
    const float x = d[0], y = d[1], z = d[2];
    const float c0 = 0.28209479177387814f, c1 = 0.48860251190291992f;
    const float c2 = 1.0925484305920792f, c3 = 0.31539156525252005f, c4 = 0.54627421529603959f;
    out[0] = c0;
    out[1] = c1 * y;
    out[2] = c1 * z;
    out[3] = c1 * x;
    out[4] = c2 * (x * y);
    out[5] = c2 * (y * z);
    out[6] = c3 * __builtin_fmaf(2.0f * z, z, -__builtin_fmaf(x, x, y * y));
    out[7] = c2 * (x * z);
    out[8] = c4 * __builtin_fmaf(x, x, -(y * y));
}

}  // namespace soup
