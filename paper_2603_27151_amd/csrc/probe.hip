// Measured ceilings of the machine, for the rooflines the kernels are measured
// against: a streaming copy and a streaming read of HBM, float atomics to
// scattered global addresses, the vector ALU's float32 FMA rate (non-packed,
// as the library is built) and the matrix cores' float32 rate
// (v_mfma_f32_16x16x4f32). Each kernel does a known amount of work that its
// caller times; each leaves a result that a test can check exactly, so that
// none of the work can be dropped by the compiler.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace soup {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

// dst[i] = src[i] over n 16-byte elements, four per thread and step, with
// non-temporal loads and stores (the fastest of the variants measured: 64
// workgroups per CU, four or eight elements in flight, with and without the
// non-temporal hint, and one contiguous chunk per workgroup; it also beats
// hipMemcpy device to device).
__global__ __launch_bounds__(256) void probe_copy_kernel(const f4v* __restrict__ src, f4v* __restrict__ dst,
                                                         int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        f4v v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * stride]);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * stride]);
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// partial[block] = the sum of every float of the block's share of src.
__global__ __launch_bounds__(256) void probe_read_kernel(const f4v* __restrict__ src, int64_t n,
                                                         float* __restrict__ partial) {
    __shared__ float red[4];
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const f4v a = __builtin_nontemporal_load(&src[i]), b = __builtin_nontemporal_load(&src[i + stride]);
        const f4v c = __builtin_nontemporal_load(&src[i + 2 * stride]), d = __builtin_nontemporal_load(&src[i + 3 * stride]);
        s0 += (a.x + a.y) + (a.z + a.w);
        s1 += (b.x + b.y) + (b.z + b.w);
        s2 += (c.x + c.y) + (c.z + c.w);
        s3 += (d.x + d.y) + (d.z + d.w);
    }
    for (; i < n; i += stride) {
        const f4v a = src[i];
        s0 += (a.x + a.y) + (a.z + a.w);
    }
    float s = (s0 + s1) + (s2 + s3);
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// n_ops float atomic adds of 1 to slots spread by a multiplicative hash
// (op k goes to slot (k * 2654435761) mod n_slots): neighbouring lanes hit
// unrelated cache lines, as the scattered gradient adds of a per-pixel
// backward do.
__global__ __launch_bounds__(256) void probe_atomic_kernel(float* __restrict__ slots, int64_t n_slots, int64_t n_ops) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n_ops; k += stride) {
        const uint64_t h = (static_cast<uint64_t>(k) * 2654435761ull) % static_cast<uint64_t>(n_slots);
        atomicAdd(&slots[h], 1.0f);
    }
}

// Eight independent chains per thread of acc = acc * m + c, iters steps each;
// out[thread] = the sum of the chains (with m = 1, c = 1 and the chains
// starting at 0 .. 7: 8 iters + 28, exact below 2^24).
__global__ __launch_bounds__(256) void probe_fma_kernel(float* __restrict__ out, int iters, float m, float c) {
    float a0 = 0.f, a1 = 1.f, a2 = 2.f, a3 = 3.f, a4 = 4.f, a5 = 5.f, a6 = 6.f, a7 = 7.f;
    for (int it = 0; it < iters; ++it) {
        a0 = __builtin_fmaf(a0, m, c);
        a1 = __builtin_fmaf(a1, m, c);
        a2 = __builtin_fmaf(a2, m, c);
        a3 = __builtin_fmaf(a3, m, c);
        a4 = __builtin_fmaf(a4, m, c);
        a5 = __builtin_fmaf(a5, m, c);
        a6 = __builtin_fmaf(a6, m, c);
        a7 = __builtin_fmaf(a7, m, c);
    }
    out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

// Per wave, four independent accumulations of v_mfma_f32_16x16x4f32 with
// A = a and B = b in every lane, iters products each: every element of an
// accumulator ends at 4 a b iters (exact for small integers). out[wave * 64 +
// lane] = the sum of the lane's sixteen accumulator values.
__global__ __launch_bounds__(256) void probe_mfma_kernel(float* __restrict__ out, int iters, float a, float b) {
    f4v c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0, c2 = c0, c3 = c0;
    for (int it = 0; it < iters; ++it) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) s += ((c0[i] + c1[i]) + (c2[i] + c3[i]));
    out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

int grid_for(int64_t n, int64_t cap) {
    int64_t g = (n + 255) / 256;
    if (g > cap) g = cap;
    return static_cast<int>(g < 1 ? 1 : g);
}

}  // namespace

void launch_probe_copy(const float4* src, float4* dst, int64_t n, int num_cus, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(probe_copy_kernel, dim3(grid_for(n, static_cast<int64_t>(num_cus) * 64)), dim3(256), 0, s,
                       reinterpret_cast<const f4v*>(src), reinterpret_cast<f4v*>(dst), n);
}

void launch_probe_read(const float4* src, int64_t n, float* partial, int64_t n_partial, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(probe_read_kernel, dim3(grid_for(n, n_partial)), dim3(256), 0, s, reinterpret_cast<const f4v*>(src),
                       n, partial);
}

void launch_probe_atomic(float* slots, int64_t n_slots, int64_t n_ops, int num_cus, hipStream_t s) {
    if (n_ops <= 0 || n_slots <= 0) return;
    hipLaunchKernelGGL(probe_atomic_kernel, dim3(grid_for(n_ops, static_cast<int64_t>(num_cus) * 32)), dim3(256), 0, s,
                       slots, n_slots, n_ops);
}

void launch_probe_fma(float* out, int64_t n_threads, int iters, hipStream_t s) {
    if (n_threads <= 0) return;
    hipLaunchKernelGGL(probe_fma_kernel, dim3(static_cast<unsigned>(n_threads / 256)), dim3(256), 0, s, out, iters,
                       1.0f, 1.0f);
}

void launch_probe_mfma(float* out, int64_t n_threads, int iters, hipStream_t s) {
    if (n_threads <= 0) return;
    hipLaunchKernelGGL(probe_mfma_kernel, dim3(static_cast<unsigned>(n_threads / 256)), dim3(256), 0, s, out, iters,
                       1.0f, 1.0f);
}

}  // namespace soup
