// Adaptive control of primitives (Section 3.4, "Adaptive control of
// primitives"; Supplement B, resampling of a random initialisation).
//
//  * coverage_kernel: pixels won per triangle, from the visibility keys
//    (8 bytes read per pixel). Device-scope atomics set its pace, and
//    stochastic masking interleaves the winners of neighbouring pixels (runs
//    of equal winners average under two pixels), so each wave loads 256
//    consecutive keys and issues one atomic per distinct triangle among
//    them, with the count of its pixels.
//  * edge_length_kernel: per triangle, the longest screen-space length of
//    each edge over up to kEdgeViews views, in units of the view's height.
//    One thread per triangle; the views travel as a kernel argument. Float64
//    so that the cull and bounding-box decisions are the exact ones of the
//    definition (products of float32 values are exact in float64; sums are
//    taken left to right).
//  * apply_kernel: the new soup. One workgroup per source triangle (grid
//    stride): kept triangles are copied, split ones write their two halves.
//    A half's texel (ix, iy) maps to parent grid coordinates that are
//    multiples of 1/2, so the resampling weights are 0, 1/2 or 1 exactly.
//  * plan_host: the split/prune decisions, host code on host arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "internal.hpp"

namespace soup {

namespace {

constexpr int kCoverUnroll = 4;  // 64-key chunks per wave and iteration, loaded together

__global__ void __launch_bounds__(256) coverage_kernel(const uint64_t* __restrict__ vis, int64_t n, uint32_t T,
                                                       uint32_t* __restrict__ counts) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x * kCoverUnroll;
    // w0 is the wave's first key: every lane of a wave runs the same iterations
    for (int64_t w0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + (threadIdx.x & ~63)) * kCoverUnroll; w0 < n;
         w0 += stride) {
        uint64_t k[kCoverUnroll];
        for (int u = 0; u < kCoverUnroll; ++u) {
            const int64_t i = w0 + u * 64 + lane;
            k[u] = i < n ? vis[i] : kBgKey;
        }
        uint32_t id[kCoverUnroll];
        uint64_t pending[kCoverUnroll];
        for (int u = 0; u < kCoverUnroll; ++u) {
            const uint32_t t = static_cast<uint32_t>(k[u]);
            id[u] = (k[u] != kBgKey && t < T) ? t : 0xFFFFFFFFu;
            pending[u] = __ballot(id[u] != 0xFFFFFFFFu);
        }
        // one atomic per distinct triangle among the wave's keys: the first
        // pending lane names a triangle, every lane holding it is counted
        // and retired (each pass retires at least that lane)
        for (int u0 = 0; u0 < kCoverUnroll; ++u0) {
            while (pending[u0]) {
                const int leader = __builtin_ctzll(pending[u0]);
                const uint32_t lid = __builtin_amdgcn_readlane(id[u0], leader);
                uint32_t total = 0;
                for (int u = u0; u < kCoverUnroll; ++u) {
                    const uint64_t same = __ballot(id[u] == lid);
                    total += static_cast<uint32_t>(__builtin_popcountll(same));
                    pending[u] &= ~same;
                }
                if (lane == leader) atomicAdd(&counts[lid], total);
            }
        }
    }
}

__global__ void __launch_bounds__(256) edge_length_kernel(const float* __restrict__ verts, int32_t T, EdgeViews ev,
                                                          double near_w, int first, float* __restrict__ rel) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double p[3][3];
    for (int i = 0; i < 3; ++i)
        for (int d = 0; d < 3; ++d) p[i][d] = static_cast<double>(verts[static_cast<int64_t>(t) * 9 + i * 3 + d]);
    double best[3];
    for (int k = 0; k < 3; ++k) best[k] = first ? 0.0 : static_cast<double>(rel[static_cast<int64_t>(t) * 3 + k]);
    for (int v = 0; v < ev.n; ++v) {
        const float* M = ev.m[v];
        const double W = ev.w[v], H = ev.h[v];
        double sx[3], sy[3];
        bool culled = false;
        for (int i = 0; i < 3; ++i) {
            double c[4];
            for (int r = 0; r < 4; ++r) {
                double acc = static_cast<double>(M[r * 4 + 0]) * p[i][0];
                acc = acc + static_cast<double>(M[r * 4 + 1]) * p[i][1];
                acc = acc + static_cast<double>(M[r * 4 + 2]) * p[i][2];
                acc = acc + static_cast<double>(M[r * 4 + 3]);
                c[r] = acc;
            }
            culled = culled || c[3] < near_w;
            sx[i] = W / 2 * (c[0] / c[3] + 1.0);
            sy[i] = H / 2 * (1.0 - c[1] / c[3]);
        }
        if (culled) continue;
        const double x0 = fmin(fmin(sx[0], sx[1]), sx[2]), x1 = fmax(fmax(sx[0], sx[1]), sx[2]);
        const double y0 = fmin(fmin(sy[0], sy[1]), sy[2]), y1 = fmax(fmax(sy[0], sy[1]), sy[2]);
        if (x1 < 0.0 || x0 > W || y1 < 0.0 || y0 > H) continue;
        for (int k = 0; k < 3; ++k) {
            const int j = k == 2 ? 0 : k + 1;
            const double dx = sx[j] - sx[k], dy = sy[j] - sy[k];
            best[k] = fmax(best[k], sqrt(dx * dx + dy * dy) / H);
        }
    }
    for (int k = 0; k < 3; ++k) rel[static_cast<int64_t>(t) * 3 + k] = static_cast<float>(best[k]);
}

// Twice the parent barycentric weight of vertex i at vertex slot j of half
// `half` of a triangle split on edge k (0, 1 or 2).
__device__ __forceinline__ int twice_parent_bary(int k, int half, int j, int i) {
    const int a = k, b = k == 2 ? 0 : k + 1;
    const int rep = half == 0 ? b : a;  // the slot that takes the midpoint
    if (j == rep) return (i == a || i == b) ? 1 : 0;
    return i == j ? 2 : 0;
}

__global__ void __launch_bounds__(256) apply_kernel(const float* __restrict__ verts, const float* __restrict__ feats,
                                                    const int32_t* __restrict__ actions,
                                                    const int32_t* __restrict__ offsets, int32_t T, int32_t G,
                                                    int32_t C, int32_t n_new, float* __restrict__ vout,
                                                    float* __restrict__ fout) {
    const int64_t per = static_cast<int64_t>(G) * G * C;
    for (int t = blockIdx.x; t < T; t += gridDim.x) {
        const int a = actions[t];
        const int o = offsets[t];
        const int kids = a == kActKeep ? 1 : (a >= kActSplit0 && a < kActSplit0 + 3 ? 2 : 0);
        if (kids == 0 || o < 0 || o > n_new - kids) continue;  // removed, or not a plan's entry
        const float* vp = verts + static_cast<int64_t>(t) * 9;
        const float* fp = feats + static_cast<int64_t>(t) * per;
        if (kids == 1) {
            if (threadIdx.x < 9) vout[static_cast<int64_t>(o) * 9 + threadIdx.x] = vp[threadIdx.x];
            float* fo = fout + static_cast<int64_t>(o) * per;
            if ((per & 3) == 0) {  // 16-byte rows: the caller's buffers are at least 16-byte aligned
                const float4* s4 = reinterpret_cast<const float4*>(fp);
                float4* d4 = reinterpret_cast<float4*>(fo);
                for (int64_t i = threadIdx.x; i < per / 4; i += blockDim.x) d4[i] = s4[i];
            } else {
                for (int64_t i = threadIdx.x; i < per; i += blockDim.x) fo[i] = fp[i];
            }
            continue;
        }
        const int k = a - kActSplit0;
        for (int half = 0; half < 2; ++half) {
            const int64_t oo = static_cast<int64_t>(o) + half;
            if (threadIdx.x < 9) {
                const int j = threadIdx.x / 3, d = threadIdx.x % 3;
                const int ka = k, kb = k == 2 ? 0 : k + 1;
                const int rep = half == 0 ? kb : ka;
                // the midpoint: the float sum rounds once, the halving is exact
                vout[oo * 9 + threadIdx.x] = j == rep ? (vp[ka * 3 + d] + vp[kb * 3 + d]) * 0.5f : vp[j * 3 + d];
            }
            float* fo = fout + oo * per;
            for (int64_t i = threadIdx.x; i < per; i += blockDim.x) {
                const int c = static_cast<int>(i % C);
                const int tx = static_cast<int>(i / C);
                const int ix = tx % G, iy = tx / G;
                // (G-1) x the half's barycentrics of the texel: (G-1-ix-iy, ix, iy);
                // 2 (G-1) x the parent's: U2, V2 (integers)
                const int bw[3] = {G - 1 - ix - iy, ix, iy};
                int U2 = 0, V2 = 0;
                for (int j = 0; j < 3; ++j) {
                    U2 += bw[j] * twice_parent_bary(k, half, j, 1);
                    V2 += bw[j] * twice_parent_bary(k, half, j, 2);
                }
                U2 = min(max(U2, 0), 2 * (G - 1));
                V2 = min(max(V2, 0), 2 * (G - 1));
                const int cx = min(U2 >> 1, G - 2), cy = min(V2 >> 1, G - 2);
                const float fx = 0.5f * static_cast<float>(U2 - 2 * cx), fy = 0.5f * static_cast<float>(V2 - 2 * cy);
                const float* q = fp + (static_cast<int64_t>(cy) * G + cx) * C + c;
                const float t00 = q[0], t10 = q[C], t01 = q[static_cast<int64_t>(G) * C],
                            t11 = q[static_cast<int64_t>(G) * C + C];
                fo[i] = (1.0f - fx) * (1.0f - fy) * t00 + fx * (1.0f - fy) * t10 + (1.0f - fx) * fy * t01 +
                        fx * fy * t11;
            }
        }
    }
}

}  // namespace

void launch_coverage(const uint64_t* vis, int64_t n, int32_t T, uint32_t* counts, int num_cus, hipStream_t s) {
    if (n <= 0 || T <= 0) return;
    int64_t g = (n + 256 * kCoverUnroll - 1) / (256 * kCoverUnroll);
    const int64_t cap = static_cast<int64_t>(num_cus) * 16;
    if (g > cap) g = cap;
    hipLaunchKernelGGL(coverage_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, vis, n,
                       static_cast<uint32_t>(T), counts);
}

void launch_edge_lengths(const float* verts, int32_t T, const EdgeViews& ev, float near_w, bool first, float* rel,
                         hipStream_t s) {
    if (T <= 0) return;
    hipLaunchKernelGGL(edge_length_kernel, dim3(static_cast<unsigned>((T + 255) / 256)), dim3(256), 0, s, verts, T, ev,
                       static_cast<double>(near_w), first ? 1 : 0, rel);
}

void launch_apply(const float* verts, const float* feats, const int32_t* actions, const int32_t* offsets, int32_t T,
                  int32_t G, int32_t C, int32_t n_new, float* vout, float* fout, hipStream_t s) {
    if (T <= 0 || n_new <= 0) return;
    const int g = std::min<int32_t>(T, 16384);
    hipLaunchKernelGGL(apply_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, verts, feats, actions, offsets, T,
                       G, C, n_new, vout, fout);
}

int32_t plan_host(const uint32_t* counts, const float* rel, int32_t T, float split_frac, int32_t target,
                  bool prune_zero, bool fill, int32_t* actions, int32_t* offsets) {
    std::vector<int> longest(T);
    std::vector<char> split(T), removed(T, 0);
    for (int t = 0; t < T; ++t) {
        int k = 0;
        if (rel[t * 3 + 1] > rel[t * 3 + k]) k = 1;
        if (rel[t * 3 + 2] > rel[t * 3 + k]) k = 2;
        longest[t] = k;
        split[t] = rel[t * 3 + k] > split_frac;
        if (prune_zero && counts[t] == 0) {
            removed[t] = 1;
            split[t] = 0;
        }
    }
    int64_t n = 0;
    for (int t = 0; t < T; ++t)
        if (!removed[t]) n += split[t] ? 2 : 1;
    if (n > target) {
        // lowest coverage first; a stable sort keeps equal counts in index order
        std::vector<int> order(T);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return counts[x] < counts[y]; });
        for (int t : order) {
            if (n <= target) break;
            if (removed[t]) continue;
            n -= split[t] ? 2 : 1;
            removed[t] = 1;
            split[t] = 0;
        }
    }
    if (fill && n < target) {
        std::vector<int> cand;
        for (int t = 0; t < T; ++t)
            if (!removed[t] && !split[t]) cand.push_back(t);
        std::stable_sort(cand.begin(), cand.end(),
                         [&](int x, int y) { return rel[x * 3 + longest[x]] > rel[y * 3 + longest[y]]; });
        for (int t : cand) {
            if (n >= target) break;
            split[t] = 1;
            ++n;
        }
    }
    int32_t o = 0;
    for (int t = 0; t < T; ++t) {
        offsets[t] = o;
        if (removed[t]) {
            actions[t] = kActRemove;
        } else if (split[t]) {
            actions[t] = kActSplit0 + longest[t];
            o += 2;
        } else {
            actions[t] = kActKeep;
            o += 1;
        }
    }
    return o;
}

}  // namespace soup
