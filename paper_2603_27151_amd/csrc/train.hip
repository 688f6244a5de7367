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
//    One thread per pixel; the 11 x 11 taps come through the L1 and L2
//    caches (a view's image is read 121 times per pass, from cache).
//  * adam_kernel: Adam (vec = 1) or VectorAdam (vec = 3: one second moment
//    per 3-vector from its squared norm), one thread per vector.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace soup {

namespace {

constexpr float kC1 = 0.0001f;  // 0.01^2
constexpr float kC2 = 0.0009f;  // 0.03^2

__global__ void __launch_bounds__(256) ssim_stats_kernel(const float* __restrict__ color,
                                                         const float* __restrict__ target, int W, int H, float lam,
                                                         float inv_n, SsimWindow win, float* __restrict__ stats,
                                                         float* __restrict__ grad_logp, float* __restrict__ loss) {
    __shared__ float part[4];
    const int64_t np = static_cast<int64_t>(W) * H;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    float share = 0.0f;
    if (p < np) {
        const int x = static_cast<int>(p % W), y = static_cast<int>(p / W);
        float sx[3] = {0, 0, 0}, sy[3] = {0, 0, 0}, sxx[3] = {0, 0, 0}, syy[3] = {0, 0, 0}, sxy[3] = {0, 0, 0};
        for (int dy = -kSsimR; dy <= kSsimR; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= H) continue;
            for (int dx = -kSsimR; dx <= kSsimR; ++dx) {
                const int xx = x + dx;
                if (xx < 0 || xx >= W) continue;
                const float w = win.g[dy + kSsimR] * win.g[dx + kSsimR];
                const int64_t q = static_cast<int64_t>(yy) * W + xx;
                for (int c = 0; c < 3; ++c) {
                    const float a = color[q * 3 + c], b = target[q * 3 + c];
                    sx[c] += w * a;
                    sy[c] += w * b;
                    sxx[c] += w * (a * a);
                    syy[c] += w * (b * b);
                    sxy[c] += w * (a * b);
                }
            }
        }
        float* st = stats + p * 12;
        for (int c = 0; c < 3; ++c) {
            const float mx = sx[c], my = sy[c];
            const float vx = sxx[c] - mx * mx, vy = syy[c] - my * my, cxy = sxy[c] - mx * my;
            const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * cxy + kC2;
            const float B1 = mx * mx + my * my + kC1, B2 = vx + vy + kC2;
            const float S = (A1 * A2) / (B1 * B2);
            const float dS_dmx = 2.0f * my * A2 / (B1 * B2) - S * 2.0f * mx / B1;
            const float dS_dvx = -S / B2;
            const float dS_dcxy = 2.0f * A1 / (B1 * B2);
            st[c] = dS_dmx - 2.0f * mx * dS_dvx - my * dS_dcxy;
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
    const int64_t np = static_cast<int64_t>(W) * H;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int x = static_cast<int>(p % W), y = static_cast<int>(p / W);
    float s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0}, s3[3] = {0, 0, 0};
    for (int dy = -kSsimR; dy <= kSsimR; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= H) continue;
        for (int dx = -kSsimR; dx <= kSsimR; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= W) continue;
            const float w = win.g[dy + kSsimR] * win.g[dx + kSsimR];
            // a pixel's record is G1[3] G2[3] G3[3] and three unused floats: three 16-byte loads
            const float4* st = reinterpret_cast<const float4*>(stats + (static_cast<int64_t>(yy) * W + xx) * 12);
            const float4 r0 = st[0], r1 = st[1], r2 = st[2];
            s1[0] += w * r0.x;
            s1[1] += w * r0.y;
            s1[2] += w * r0.z;
            s2[0] += w * r0.w;
            s2[1] += w * r1.x;
            s2[2] += w * r1.y;
            s3[0] += w * r1.z;
            s3[1] += w * r1.w;
            s3[2] += w * r2.x;
        }
    }
    for (int c = 0; c < 3; ++c) {
        const float a = color[p * 3 + c], b = target[p * 3 + c];
        const float d = a - b;
        const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
        const float dssim = s1[c] + 2.0f * a * s2[c] + b * s3[c];
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

}  // namespace

void launch_loss_l1_ssim(const float* color, const float* target, int W, int H, float lam, float inv_n,
                         const SsimWindow& win, float* stats, float* grad_color, float* grad_logp, float* loss,
                         hipStream_t s) {
    const int64_t np = static_cast<int64_t>(W) * H;
    if (np <= 0) return;
    const unsigned g = static_cast<unsigned>((np + 255) / 256);
    hipLaunchKernelGGL(ssim_stats_kernel, dim3(g), dim3(256), 0, s, color, target, W, H, lam, inv_n, win, stats,
                       grad_logp, loss);
    hipLaunchKernelGGL(ssim_grad_kernel, dim3(g), dim3(256), 0, s, color, target, W, H, lam, inv_n, win, stats,
                       grad_color);
}

void launch_adam(float* p, const float* g, float* m, float* v, int64_t nvec, int vec, float lr, float b1, float omb1,
                 float b2, float omb2, float eps, float bc1, float bc2, hipStream_t s) {
    if (nvec <= 0) return;
    int64_t blocks = (nvec + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(adam_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, g, m, v, nvec, vec, lr,
                       b1, omb1, b2, omb2, eps, bc1, bc2);
}

}  // namespace soup
