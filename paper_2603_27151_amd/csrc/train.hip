// The training step around the rasterizer (Section 3.4 "Loss function";
// Supplement "Hyperparameters").
//
//  * ssim_stats_kernel: per pixel and channel, the local statistics of the
//    SSIM map under an 11 x 11 Gaussian window (zero outside the image):
//    the three factors through which S depends on the window sums,
//        G1 = dS/dmu_x - 2 mu_x dS/dsigma_x^2 - mu_y dS/dsigma_xy,
//        G2 = dS/dsigma_x^2,   G3 = dS/dsigma_xy,
//    so that dS(q)/dx_p = w(p - q) (G1(q) + 2 x_p G2(q) + y_p G3(q)). It also
//    writes each pixel's share of the loss (the score term's weight) and adds
//    the loss into a scalar.
//  * ssim_grad_kernel: dL/dC = lambda sign(C - T) / (3P) minus
//    (1 - lambda) / (3P) times the window sums of G1, G2, G3 around p.
//    One thread per pixel of a 32 x 8 tile; the window is applied as two
//    11-tap passes over an LDS copy of the tile and its halo, columns first
//    (the halo's 42 columns for the tile's 8 rows, two rows per thread from
//    their 12 shared input rows), then rows (the tile's 32 columns).
//  * adam_kernel: Adam (vec = 1) or VectorAdam (vec = 3: one second moment
//    per 3-vector from its squared norm), one thread per vector.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace soup {

namespace {

constexpr float kC1 = 0.0001f;  // 0.01^2
constexpr float kC2 = 0.0009f;  // 0.03^2
// The window statistics are formed from values shifted by this constant
// (colours and targets live in [0, 1]): variances and covariances do not
// change under a shift, and sigma^2 = E[x^2] - mu^2 then cancels far fewer
// digits in float32 (E[(x - 1/2)^2] <= 1/4 against E[x^2] <= 1). Padding
// outside the image is the shifted zero, -1/2; the means are shifted back.
constexpr float kShift = 0.5f;

// Both SSIM passes work on 32 x 8 pixel tiles, one thread per pixel. The
// tile plus its 5-pixel halo is staged in LDS (zeros outside the image: the
// zero padding of the definition) and filtered along columns for the tile's
// rows over the halo's columns (a thread takes two output rows of one
// column, whose windows share 10 of their 12 input rows), then along rows:
// 22 taps per map instead of 121. Columns first: for a tile wider than
// tall the first pass covers 42 x 8 positions instead of 18 x 32.
constexpr int kTW = 32, kTH = 8;
constexpr int kHW = kTW + 2 * kSsimR, kHH = kTH + 2 * kSsimR;
static_assert(kTH % 2 == 0, "the column pass takes output rows in pairs");

__global__ void __launch_bounds__(256) ssim_stats_kernel(const float* __restrict__ color,
                                                         const float* __restrict__ target, int W, int H, float lam,
                                                         float inv_n, SsimWindow win, float* __restrict__ stats,
                                                         float* __restrict__ grad_logp, float* __restrict__ loss) {
    __shared__ float in[kHH][kHW][6];   // colour rgb, target rgb
    __shared__ float vs[kTH][15][kHW];  // column sums: x, y, x^2, y^2, xy per channel
    __shared__ float part[4];
    const int tx0 = blockIdx.x * kTW, ty0 = blockIdx.y * kTH;
    for (int i = threadIdx.x; i < kHH * kHW; i += blockDim.x) {
        const int r = i / kHW, cc = i % kHW;
        const int gx = tx0 + cc - kSsimR, gy = ty0 + r - kSsimR;
        const bool ok = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const int64_t q = ok ? static_cast<int64_t>(gy) * W + gx : 0;
        for (int c = 0; c < 3; ++c) {
            in[r][cc][c] = (ok ? color[q * 3 + c] : 0.0f) - kShift;
            in[r][cc][3 + c] = (ok ? target[q * 3 + c] : 0.0f) - kShift;
        }
    }
    __syncthreads();
    // columns: output rows 2 pr and 2 pr + 1 of halo column cc, from input
    // rows 2 pr .. 2 pr + 11 (row 2 pr + k is tap k of the first, k - 1 of the second)
    for (int i = threadIdx.x; i < kHW * (kTH / 2); i += blockDim.x) {
        const int cc = i % kHW, pr = i / kHW;
        float a0[15], a1[15];
        for (int j = 0; j < 15; ++j) {
            a0[j] = 0.0f;
            a1[j] = 0.0f;
        }
        for (int k = 0; k <= 2 * kSsimR + 1; ++k) {
            const float* px = in[2 * pr + k][cc];
            float v[15];
            for (int c = 0; c < 3; ++c) {
                const float a = px[c], b = px[3 + c];
                v[c] = a;
                v[3 + c] = b;
                v[6 + c] = a * a;
                v[9 + c] = b * b;
                v[12 + c] = a * b;
            }
            if (k <= 2 * kSsimR) {
                const float w = win.g[k];
                for (int j = 0; j < 15; ++j) a0[j] += w * v[j];
            }
            if (k >= 1) {
                const float w = win.g[k - 1];
                for (int j = 0; j < 15; ++j) a1[j] += w * v[j];
            }
        }
        for (int j = 0; j < 15; ++j) {
            vs[2 * pr][j][cc] = a0[j];
            vs[2 * pr + 1][j][cc] = a1[j];
        }
    }
    __syncthreads();
    const int lx = threadIdx.x % kTW, ly = threadIdx.x / kTW;
    const int x = tx0 + lx, y = ty0 + ly;
    float share = 0.0f;
    if (x < W && y < H) {
        float sm[15];
        for (int j = 0; j < 15; ++j) sm[j] = 0.0f;
        for (int k = 0; k <= 2 * kSsimR; ++k) {
            const float w = win.g[k];
            for (int j = 0; j < 15; ++j) sm[j] += w * vs[ly][j][lx + k];
        }
        const int64_t p = static_cast<int64_t>(y) * W + x;
        float* st = stats + p * 12;
        for (int c = 0; c < 3; ++c) {
            const float sx = sm[c], sy = sm[3 + c];   // shifted means
            const float vx = sm[6 + c] - sx * sx, vy = sm[9 + c] - sy * sy, cxy = sm[12 + c] - sx * sy;
            const float mx = sx + kShift, my = sy + kShift;
            const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * cxy + kC2;
            const float B1 = mx * mx + my * my + kC1, B2 = vx + vy + kC2;
            const float S = (A1 * A2) / (B1 * B2);
            const float dS_dmx = 2.0f * my * A2 / (B1 * B2) - S * 2.0f * mx / B1;
            const float dS_dvx = -S / B2;
            const float dS_dcxy = 2.0f * A1 / (B1 * B2);
            // G1 in shifted coordinates: the gradient pass pairs it with shifted values
            st[c] = dS_dmx - 2.0f * sx * dS_dvx - sy * dS_dcxy;
            st[3 + c] = dS_dvx;
            st[6 + c] = dS_dcxy;
            const float d = color[p * 3 + c] - target[p * 3 + c];
            share += lam * fabsf(d) + (1.0f - lam) * (1.0f - S);
        }
        share *= inv_n;
        grad_logp[p] = share;
    }
    // the loss: a wave sum, then one atomic per workgroup
    for (int o = 32; o > 0; o >>= 1) share += __shfl_xor(share, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = share;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, part[0] + part[1] + part[2] + part[3]);
}

__global__ void __launch_bounds__(256) ssim_grad_kernel(const float* __restrict__ color,
                                                        const float* __restrict__ target, int W, int H, float lam,
                                                        float inv_n, SsimWindow win, const float* __restrict__ stats,
                                                        float* __restrict__ grad_color) {
    __shared__ float in[kHH][kHW][9];   // G1, G2, G3 per channel (zero outside the image)
    __shared__ float vs[kTH][9][kHW];   // their column sums
    const int tx0 = blockIdx.x * kTW, ty0 = blockIdx.y * kTH;
    for (int i = threadIdx.x; i < kHH * kHW; i += blockDim.x) {
        const int r = i / kHW, cc = i % kHW;
        const int gx = tx0 + cc - kSsimR, gy = ty0 + r - kSsimR;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
            // a record is G1[3] G2[3] G3[3] and three unused floats: three 16-byte loads
            const float4* st = reinterpret_cast<const float4*>(stats + (static_cast<int64_t>(gy) * W + gx) * 12);
            const float4 r0 = st[0], r1 = st[1], r2 = st[2];
            in[r][cc][0] = r0.x;
            in[r][cc][1] = r0.y;
            in[r][cc][2] = r0.z;
            in[r][cc][3] = r0.w;
            in[r][cc][4] = r1.x;
            in[r][cc][5] = r1.y;
            in[r][cc][6] = r1.z;
            in[r][cc][7] = r1.w;
            in[r][cc][8] = r2.x;
        } else {
            for (int j = 0; j < 9; ++j) in[r][cc][j] = 0.0f;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHW * (kTH / 2); i += blockDim.x) {   // columns, two output rows each
        const int cc = i % kHW, pr = i / kHW;
        float a0[9], a1[9];
        for (int j = 0; j < 9; ++j) {
            a0[j] = 0.0f;
            a1[j] = 0.0f;
        }
        for (int k = 0; k <= 2 * kSsimR + 1; ++k) {
            const float* px = in[2 * pr + k][cc];
            if (k <= 2 * kSsimR) {
                const float w = win.g[k];
                for (int j = 0; j < 9; ++j) a0[j] += w * px[j];
            }
            if (k >= 1) {
                const float w = win.g[k - 1];
                for (int j = 0; j < 9; ++j) a1[j] += w * px[j];
            }
        }
        for (int j = 0; j < 9; ++j) {
            vs[2 * pr][j][cc] = a0[j];
            vs[2 * pr + 1][j][cc] = a1[j];
        }
    }
    __syncthreads();
    const int lx = threadIdx.x % kTW, ly = threadIdx.x / kTW;
    const int x = tx0 + lx, y = ty0 + ly;
    if (x >= W || y >= H) return;
    float sm[9];
    for (int j = 0; j < 9; ++j) sm[j] = 0.0f;
    for (int k = 0; k <= 2 * kSsimR; ++k) {
        const float w = win.g[k];
        for (int j = 0; j < 9; ++j) sm[j] += w * vs[ly][j][lx + k];
    }
    const int64_t p = static_cast<int64_t>(y) * W + x;
    for (int c = 0; c < 3; ++c) {
        const float a = color[p * 3 + c], b = target[p * 3 + c];
        const float d = a - b;
        const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
        const float dssim = sm[c] + 2.0f * (a - kShift) * sm[3 + c] + (b - kShift) * sm[6 + c];
        grad_color[p * 3 + c] = inv_n * (lam * sgn - (1.0f - lam) * dssim);
    }
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t nvec, int vec,
                                                   float lr, float b1, float omb1, float b2, float omb2, float eps,
                                                   float bc1, float bc2) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nvec;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        float g2 = 0.0f;
        for (int k = 0; k < vec; ++k) {
            const float gk = g[i * vec + k];
            g2 += gk * gk;
        }
        const float vi = b2 * v[i] + omb2 * g2;
        v[i] = vi;
        const float den = sqrtf(vi / bc2) + eps;
        for (int k = 0; k < vec; ++k) {
            const int64_t j = i * vec + k;
            const float mj = b1 * m[j] + omb1 * g[j];
            m[j] = mj;
            p[j] -= lr * (mj / bc1) / den;
        }
    }
}

// Adam on 16-byte groups of four parameters (vec = 1, n a multiple of 4,
// every array 16-byte aligned): the same arithmetic per element, with
// 16-byte loads and stores.
__global__ void __launch_bounds__(256) adam4_kernel(float4* __restrict__ p, const float4* __restrict__ g,
                                                    float4* __restrict__ m, float4* __restrict__ v, int64_t n4,
                                                    float lr, float b1, float omb1, float b2, float omb2, float eps,
                                                    float bc1, float bc2) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float4 gi = g[i];
        float4 mi = m[i], vi = v[i], pi = p[i];
        float* pm = &mi.x;
        float* pv = &vi.x;
        float* pp = &pi.x;
        const float* pg = &gi.x;
        for (int k = 0; k < 4; ++k) {
            pv[k] = b2 * pv[k] + omb2 * (pg[k] * pg[k]);
            pm[k] = b1 * pm[k] + omb1 * pg[k];
            pp[k] -= lr * (pm[k] / bc1) / (sqrtf(pv[k] / bc2) + eps);
        }
        m[i] = mi;
        v[i] = vi;
        p[i] = pi;
    }
}

}  // namespace

void launch_loss_l1_ssim(const float* color, const float* target, int W, int H, float lam, float inv_n,
                         const SsimWindow& win, float* stats, float* grad_color, float* grad_logp, float* loss,
                         hipStream_t s) {
    const int64_t np = static_cast<int64_t>(W) * H;
    if (np <= 0) return;
    const dim3 g(static_cast<unsigned>((W + kTW - 1) / kTW), static_cast<unsigned>((H + kTH - 1) / kTH));
    hipLaunchKernelGGL(ssim_stats_kernel, g, dim3(kTW * kTH), 0, s, color, target, W, H, lam, inv_n, win, stats,
                       grad_logp, loss);
    hipLaunchKernelGGL(ssim_grad_kernel, g, dim3(kTW * kTH), 0, s, color, target, W, H, lam, inv_n, win, stats,
                       grad_color);
}

void launch_adam(float* p, const float* g, float* m, float* v, int64_t nvec, int vec, float lr, float b1, float omb1,
                 float b2, float omb2, float eps, float bc1, float bc2, hipStream_t s) {
    if (nvec <= 0) return;
    const uintptr_t align = reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(g) |
                            reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v);
    if (vec == 1 && nvec % 4 == 0 && (align & 15) == 0) {
        const int64_t n4 = nvec / 4;
        int64_t blocks = (n4 + 255) / 256;
        if (blocks > 16384) blocks = 16384;
        hipLaunchKernelGGL(adam4_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                           reinterpret_cast<float4*>(p), reinterpret_cast<const float4*>(g),
                           reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), n4, lr, b1, omb1, b2, omb2,
                           eps, bc1, bc2);
        return;
    }
    int64_t blocks = (nvec + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(adam_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, g, m, v, nvec, vec, lr,
                       b1, omb1, b2, omb2, eps, bc1, bc2);
}

}  // namespace soup
