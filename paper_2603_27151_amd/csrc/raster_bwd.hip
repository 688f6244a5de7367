// Per-pixel edge weights, MLP-gradient reduction, loss and contract self-test
// kernels; dispatch of the backward fragment decode over the compiled MLP
// shapes (the kernel is in decode_bwd_impl.hpp, instantiated once per shape in
// dbwd_*.hip).
#include "raster_common.hpp"

namespace soup {

void launch_decode_bwd_k8_16_1(const DecodeArgs& a, bool logp, hipStream_t s);
void launch_decode_bwd_k16_32_2(const DecodeArgs& a, bool logp, hipStream_t s);
void launch_decode_bwd_k32_64_2(const DecodeArgs& a, bool logp, hipStream_t s);

size_t decode_bwd_lds_k8_16_1(int G, bool logp);
size_t decode_bwd_lds_k16_32_2(int G, bool logp);
size_t decode_bwd_lds_k32_64_2(int G, bool logp);

size_t decode_bwd_lds(MlpKind k, int G, bool logp) {
    switch (k) {
        case MlpKind::k8_16_1: return decode_bwd_lds_k8_16_1(G, logp);
        case MlpKind::k16_32_2: return decode_bwd_lds_k16_32_2(G, logp);
        case MlpKind::k32_64_2: return decode_bwd_lds_k32_64_2(G, logp);
        default: return 0;
    }
}

void launch_fragment_gates_k8_16_1(const DecodeArgs& a, uint32_t* gates_out, hipStream_t s);
void launch_fragment_gates_k16_32_2(const DecodeArgs& a, uint32_t* gates_out, hipStream_t s);
void launch_fragment_gates_k32_64_2(const DecodeArgs& a, uint32_t* gates_out, hipStream_t s);

void launch_fragment_gates(const DecodeArgs& a, MlpKind k, uint32_t* gates_out, hipStream_t s) {
    if (a.n_blocks <= 0) return;
    switch (k) {
        case MlpKind::k8_16_1: launch_fragment_gates_k8_16_1(a, gates_out, s); break;
        case MlpKind::k16_32_2: launch_fragment_gates_k16_32_2(a, gates_out, s); break;
        case MlpKind::k32_64_2: launch_fragment_gates_k32_64_2(a, gates_out, s); break;
        default: break;
    }
}

void launch_decode_bwd(const DecodeArgs& a, MlpKind k, bool logp, hipStream_t s) {
    if (a.n_blocks <= 0) return;
    switch (k) {
        case MlpKind::k8_16_1: launch_decode_bwd_k8_16_1(a, logp, s); break;
        case MlpKind::k16_32_2: launch_decode_bwd_k16_32_2(a, logp, s); break;
        case MlpKind::k32_64_2: launch_decode_bwd_k32_64_2(a, logp, s); break;
        default: break;
    }
}

// ---------------------------------------------------------------------------
// edge term (Section 3.2), per pixel
// ---------------------------------------------------------------------------

// For each pixel p and direction e (x, then y): the sum of the pair weights
// w = 1/2 (g_a + g_b) . (C_a - C_b) of the two adjacent pairs (p - e, p) and
// (p, p + e) in which p is the occluder (the smaller key). The backward
// decode adds w beta_i(p) e to the screen position of vertex i of p's winner
// triangle, so that the edge term joins the winner's own vertex chain.
__global__ __launch_bounds__(256) void edge_weight_kernel(const ViewDesc* __restrict__ views, int V, int64_t P,
                                                          Opts o, const uint64_t* __restrict__ vis,
                                                          const float* __restrict__ color,
                                                          const float* __restrict__ gcol, float2* __restrict__ ew) {
    // Workgroups are dealt to the eight XCDs in turn; block b takes pixel block
    // (b % 8) * per + b / 8, so that each XCD walks one contiguous eighth of the
    // pixels and the rows above and below a block are read through its own L2.
    const uint32_t per = gridDim.x / kXcds;
    const uint32_t pb = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    // the view of the workgroup's first pixel (a wave-uniform search), then per lane
    // the few steps past it when the workgroup straddles views
    const int64_t p0 = pb * static_cast<int64_t>(blockDim.x);
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].pix_base <= p0) lo = mid;
        else hi = mid - 1;
    }
    const int64_t p = p0 + threadIdx.x;
    if (p >= P) return;
    while (lo + 1 < V && views[lo + 1].pix_base <= p) ++lo;
    const ViewDesc& vd = views[lo];
    const uint32_t Wv = static_cast<uint32_t>(vd.W);
    const uint32_t local = static_cast<uint32_t>(p - vd.pix_base);   // below W * H <= 2^28
    const int y = static_cast<int>(local / Wv), x = static_cast<int>(local - static_cast<uint32_t>(y) * Wv);
    const uint64_t kp = vis[p];
    float e[2] = {0.0f, 0.0f};
    if (kp != kBgKey) {   // a background pixel never occludes
        const float cp[3] = {color[3 * p], color[3 * p + 1], color[3 * p + 2]};
        const float gp[3] = {gcol[3 * p], gcol[3 * p + 1], gcol[3 * p + 2]};
#pragma unroll
        for (int dir = 0; dir < 2; ++dir) {
            const int64_t step = dir == 0 ? 1 : vd.W;
            const bool has_prev = dir == 0 ? x > 0 : y > 0;
            const bool has_next = dir == 0 ? x + 1 < vd.W : y + 1 < vd.H;
#pragma unroll
            for (int side = 0; side < 2; ++side) {   // 0: pair (p - e, p); 1: pair (p, p + e)
                if (side == 0 ? !has_prev : !has_next) continue;
                const int64_t q = side == 0 ? p - step : p + step;
                const uint64_t kq = vis[q];
                // p must be the occluder: the smaller key, a tie going to the pair's second pixel
                if (side == 0 ? kq < kp : !(kp < kq)) continue;
                if (o.edge_pairs == 1 && kq != kBgKey && static_cast<uint32_t>(kq) == static_cast<uint32_t>(kp))
                    continue;
                float w = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float ca = side == 0 ? color[3 * q + c] : cp[c];
                    const float cb = side == 0 ? cp[c] : color[3 * q + c];
                    w += 0.5f * (gp[c] + gcol[3 * q + c]) * (ca - cb);
                }
                e[dir] += w;
            }
        }
    }
    if (kp != kBgKey) ew[p] = make_float2(e[0], e[1]);   // read for covered pixels only
}

void launch_edge_weights(const ViewDesc* views, int V, int64_t P, const Opts& o, const uint64_t* vis,
                         const float* color, const float* grad_color, float2* ew, hipStream_t s) {
    if (P <= 0) return;
    // a multiple of the XCD count, so that the block remapping is a bijection
    // (blocks past the last pixel return at once)
    const int64_t nb = ((P + 255) / 256 + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(edge_weight_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, views, V, P, o, vis,
                       color, grad_color, ew);
}

// ---------------------------------------------------------------------------
// MLP gradient: fixed-order reduction of the per-wave partial sums
// ---------------------------------------------------------------------------

constexpr int kMlpRowsPerBlock = 64;

// Level 1: block (param chunk, row chunk) sums kMlpRowsPerBlock rows in order.
__global__ __launch_bounds__(256) void mlp_reduce1_kernel(const float* __restrict__ partial, int n_rows, int n_params,
                                                          double* __restrict__ mid) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_params) return;
    const int r0 = blockIdx.y * kMlpRowsPerBlock, r1 = min(n_rows, r0 + kMlpRowsPerBlock);
    double s = 0.0;
    for (int r = r0; r < r1; ++r) s += partial[static_cast<size_t>(r) * n_params + p];
    mid[static_cast<size_t>(blockIdx.y) * n_params + p] = s;
}

// Level 2: sum the row chunks in order.
__global__ __launch_bounds__(256) void mlp_reduce2_kernel(const double* __restrict__ mid, int n_mid, int n_params,
                                                          float* __restrict__ out, bool accumulate) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_params) return;
    double s = accumulate ? static_cast<double>(out[p]) : 0.0;
    for (int r = 0; r < n_mid; ++r) s += mid[static_cast<size_t>(r) * n_params + p];
    out[p] = static_cast<float>(s);
}

int mlp_reduce_mid_rows(int n_rows) { return (n_rows + kMlpRowsPerBlock - 1) / kMlpRowsPerBlock; }

void launch_mlp_reduce(const float* partial, int n_rows, int n_params, double* mid, float* out, bool accumulate,
                       hipStream_t s) {
    const int n_mid = mlp_reduce_mid_rows(n_rows);
    const unsigned gp = static_cast<unsigned>((n_params + 255) / 256);
    hipLaunchKernelGGL(mlp_reduce1_kernel, dim3(gp, n_mid), dim3(256), 0, s, partial, n_rows, n_params, mid);
    hipLaunchKernelGGL(mlp_reduce2_kernel, dim3(gp), dim3(256), 0, s, mid, n_mid, n_params, out, accumulate);
}

// ---------------------------------------------------------------------------
// L2 loss and contract self-tests
// ---------------------------------------------------------------------------

// Per pixel: d = colour - target, g_C = 2 d / (3P), g_L = |d|^2 / (3P) (its
// share of the mean), loss += g_L. Four pixels (48 bytes of each input) per
// thread and step with 16-byte loads and stores when every array is 16-byte
// aligned; the pixels past the last group of four (and unaligned arrays) one
// at a time.
__global__ __launch_bounds__(256) void loss_l2_kernel(const float* __restrict__ color, const float* __restrict__ target,
                                                      int64_t P, float* __restrict__ gc, float* __restrict__ gl,
                                                      float* __restrict__ loss, int vec4) {
    __shared__ float red[4];
    const float inv = 1.0f / (3.0f * static_cast<float>(P));
    float part = 0.0f;
    const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t P4 = vec4 ? P / 4 : 0;
    for (int64_t q = tid; q < P4; q += stride) {
        const float4* c4 = reinterpret_cast<const float4*>(color) + 3 * q;
        const float4* t4 = reinterpret_cast<const float4*>(target) + 3 * q;
        const float4 a0 = c4[0], a1 = c4[1], a2 = c4[2];
        const float4 b0 = t4[0], b1 = t4[1], b2 = t4[2];
        const float cv[12] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w, a2.x, a2.y, a2.z, a2.w};
        const float tv[12] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w, b2.x, b2.y, b2.z, b2.w};
        float g[12], l[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float sq = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float d = cv[3 * k + c] - tv[3 * k + c];
                g[3 * k + c] = 2.0f * d * inv;
                sq = __builtin_fmaf(d, d, sq);
            }
            l[k] = sq * inv;
            part += sq * inv;
        }
        float4* g4 = reinterpret_cast<float4*>(gc) + 3 * q;
        g4[0] = make_float4(g[0], g[1], g[2], g[3]);
        g4[1] = make_float4(g[4], g[5], g[6], g[7]);
        g4[2] = make_float4(g[8], g[9], g[10], g[11]);
        reinterpret_cast<float4*>(gl)[q] = make_float4(l[0], l[1], l[2], l[3]);
    }
    for (int64_t p = 4 * P4 + tid; p < P; p += stride) {
        float sq = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = color[3 * p + c] - target[3 * p + c];
            gc[3 * p + c] = 2.0f * d * inv;
            sq = __builtin_fmaf(d, d, sq);
        }
        gl[p] = sq * inv;
        part += sq * inv;
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
    const uintptr_t al = reinterpret_cast<uintptr_t>(color) | reinterpret_cast<uintptr_t>(target) |
                         reinterpret_cast<uintptr_t>(gc) | reinterpret_cast<uintptr_t>(gl);
    const int vec4 = (al & 15) == 0 ? 1 : 0;
    int64_t g = ((vec4 ? (P + 3) / 4 : P) + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(loss_l2_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, color, target, P, gc, gl, loss,
                       vec4);
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
