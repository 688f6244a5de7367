// Gradient reduction, edge term, vertex chain, MLP-gradient reduction, loss and
// contract self-test kernels; dispatch of the backward fragment decode over
// the compiled MLP shapes (the kernel is in decode_bwd_impl.hpp, instantiated
// once per shape in dbwd_*.hip).
#include "raster_common.hpp"

namespace soup {

void launch_decode_bwd_k8_16_1(const DecodeArgs& a, bool logp, hipStream_t s);
void launch_decode_bwd_k16_32_2(const DecodeArgs& a, bool logp, hipStream_t s);
void launch_decode_bwd_k32_64_2(const DecodeArgs& a, bool logp, hipStream_t s);

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
// edge term
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wave_incl_sum(float v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const float u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

__global__ __launch_bounds__(256) void edge_kernel(const ViewDesc* __restrict__ views, int V, int64_t P, Opts o,
                                                   const uint64_t* __restrict__ vis,
                                                   const float* __restrict__ color,
                                                   const float* __restrict__ gcol,
                                                   const TriRec* __restrict__ recs, float* __restrict__ vacc) {
    const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool inb = p < P;
    int lo = 0, hi = V - 1;
    const int64_t pc = inb ? p : P - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].pix_base <= pc) lo = mid;
        else hi = mid - 1;
    }
    const ViewDesc& vd = views[lo];
    const int64_t local = pc - vd.pix_base;
    const int x = static_cast<int>(local % vd.W), y = static_cast<int>(local / vd.W);
    const uint64_t ka = vis[pc];
    const float ca[3] = {color[3 * pc], color[3 * pc + 1], color[3 * pc + 2]};
    const float ga[3] = {gcol[3 * pc], gcol[3 * pc + 1], gcol[3 * pc + 2]};
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        // this lane's pair (a, b = a + e): weight, occluder record and the occluder pixel
        int64_t key = -1;
        float wgt = 0.0f;
        int xo = 0, yo = 0;
        const int xb = x + (dir == 0), yb = y + (dir == 1);
        if (inb && xb < vd.W && yb < vd.H) {
            const int64_t q = pc + (dir == 0 ? 1 : vd.W);
            const uint64_t kb = vis[q];
            const bool skip = (ka == kBgKey && kb == kBgKey) ||
                              (o.edge_pairs == 1 && ka != kBgKey && kb != kBgKey &&
                               static_cast<uint32_t>(ka) == static_cast<uint32_t>(kb));
            if (!skip) {
#pragma unroll
                for (int c = 0; c < 3; ++c) wgt += 0.5f * (ga[c] + gcol[3 * q + c]) * (ca[c] - color[3 * q + c]);
                if (wgt != 0.0f) {
                    const bool oa = ka < kb;
                    key = vd.rec_base + static_cast<uint32_t>(oa ? ka : kb);
                    xo = oa ? x : xb;
                    yo = oa ? y : yb;
                }
            }
        }
        // runs of consecutive lanes with the same occluder record: sums by
        // prefix sums, one atomic per moment per run (issued by the run head)
        // every lane takes part in the shuffles (no short-circuit around them)
        const int64_t kprev = __shfl_up(key, 1, 64);
        const int64_t knext = __shfl_down(key, 1, 64);
        const bool head = key >= 0 && (lane == 0 || kprev != key);
        const bool tail = key >= 0 && (lane == 63 || knext != key);
        const uint64_t heads = __ballot(head);
        const uint64_t ends = __ballot(tail);
        const uint64_t upto = lane == 63 ? heads : (heads & ((2ull << lane) - 1));
        const int hl = upto ? 63 - __builtin_clzll(upto) : 0;
        const int hx = __shfl(xo, hl, 64), hy = __shfl(yo, hl, 64);
        const float v0 = wgt;
        const float v1 = key >= 0 ? wgt * static_cast<float>(xo - hx) : 0.0f;
        const float v2 = key >= 0 ? wgt * static_cast<float>(yo - hy) : 0.0f;
        const float s0 = wave_incl_sum(v0), s1 = wave_incl_sum(v1), s2 = wave_incl_sum(v2);
        // run [hl, end]: sum = S(end) - S(hl - 1); the run's end lane issues it
        const float p0 = __shfl(s0, hl > 0 ? hl - 1 : 0, 64), p1 = __shfl(s1, hl > 0 ? hl - 1 : 0, 64),
                    p2 = __shfl(s2, hl > 0 ? hl - 1 : 0, 64);
        if (key >= 0 && ((ends >> lane) & 1ull)) {
            const float r0 = s0 - (hl > 0 ? p0 : 0.0f);
            const float r1 = s1 - (hl > 0 ? p1 : 0.0f);
            const float r2 = s2 - (hl > 0 ? p2 : 0.0f);
            // moments about vertex 0 of the occluding triangle
            const int32_t X0 = recs[key].X[0], Y0 = recs[key].Y[0];
            const float ox = static_cast<float>(kSnap * hx + kSnap / 2 - X0) * (1.0f / 256.0f);
            const float oy = static_cast<float>(kSnap * hy + kSnap / 2 - Y0) * (1.0f / 256.0f);
            float* va = vacc + static_cast<size_t>(key) * kVacc + 9 + 3 * dir;
            atomicAdd(va + 0, r0);
            atomicAdd(va + 1, r1 + ox * r0);
            atomicAdd(va + 2, r2 + oy * r0);
        }
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
                                                           float* __restrict__ grad_verts) {
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
        float gs[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
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
    for (int i = 0; i < 9; ++i) grad_verts[static_cast<size_t>(t) * 9 + i] += g[i];
}

void launch_vertex_chain(const ViewDesc* views, int V, const SceneDesc* scenes, int T, const TriRec* recs,
                         const float* vacc, float* grad_verts, hipStream_t s) {
    if (T <= 0) return;
    hipLaunchKernelGGL(vertex_chain_kernel, dim3((T + 255) / 256), dim3(256), 0, s, views, V, scenes, T, recs, vacc,
                       grad_verts);
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
