// Triangle setup and screen-tile binning.
//
// setup:   per (view, triangle): projection, culling, snapping to 1/256 px,
//          bounding box, a lower bound of the depth of any of its fragments;
//          counts its (tile, triangle) pairs per tile (through an LDS
//          histogram per chunk of triangles when the view's tiles fit).
// scan:    exclusive scan of the per-tile counts -> per-tile list offsets.
// scatter: per (view, triangle): writes (zmin << 32 | tri) into the list of
//          every tile its bounding box touches.
// sort:    sorts each tile's list ascending (a wave sorts a short list
//          bitonic in registers; a workgroup sorts a long one bitonic in LDS,
//          in blocks of kSortBlock entries), so that the raster can walk
//          triangles front to back and stop early.
#include "internal.hpp"

namespace soup {

// One workgroup bins a chunk of `chunk` triangles of one view. When the chunk
// is large (kBinChunk) and the view has at most kHistBins tiles, its (tile,
// triangle) pairs are counted in an LDS histogram, and only the chunk's non-zero tile counts go to the global
// counters (one returning atomic per tile touched: the chunk's first slot in
// that tile's list); otherwise every pair is counted with a global atomic.
__global__ __launch_bounds__(256) void setup_kernel(const ViewDesc* __restrict__ views,
                                                    const SceneDesc* __restrict__ scenes, Opts o, int tile, int chunk,
                                                    TriRec* __restrict__ recs, int32_t* __restrict__ tile_count,
                                                    int32_t* __restrict__ chunk_base, int64_t n_tiles,
                                                    unsigned long long* __restrict__ visible) {
    __shared__ int32_t hist[kHistBins];
    const ViewDesc& vd = views[blockIdx.y];
    const int t_beg = blockIdx.x * chunk;
    if (t_beg >= vd.T) return;
    const int t_end = min(t_beg + chunk, vd.T);
    const int nb = vd.tiles_x * vd.tiles_y;
    const bool local = chunk >= kBinChunk && nb <= kHistBins;
    if (local) {
        for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0;
        __syncthreads();
    }
    const SceneDesc sc = scenes[vd.scene];
    const float* M = vd.M;
    const float hw = 0.5f * static_cast<float>(vd.W), hh = 0.5f * static_cast<float>(vd.H);
    for (int t = t_beg + static_cast<int>(threadIdx.x); t < t_end; t += blockDim.x) {
        TriRec r;
        bool ok = true;
        const float* p = sc.verts + static_cast<size_t>(t) * 9;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
            float c[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float a = M[j * 4 + 3];
                a = __builtin_fmaf(M[j * 4 + 0], x, a);
                a = __builtin_fmaf(M[j * 4 + 1], y, a);
                a = __builtin_fmaf(M[j * 4 + 2], z, a);
                c[j] = a;
            }
            ok = ok && (c[3] >= o.near_w) && __builtin_isfinite(c[0]) && __builtin_isfinite(c[1]) &&
                 __builtin_isfinite(c[2]) && __builtin_isfinite(c[3]);
            const float iw = 1.0f / c[3];
            const float sx = __builtin_fmaf(c[0] * iw, hw, hw);
            const float sy = __builtin_fmaf(-(c[1] * iw), hh, hh);
            const float z01 = __builtin_fmaf(c[2] * iw, 0.5f, 0.5f);
            const float fx = sx * 256.0f, fy = sy * 256.0f;
            ok = ok && (__builtin_fabsf(fx) <= kGuard) && (__builtin_fabsf(fy) <= kGuard) && __builtin_isfinite(z01);
            r.X[i] = ok ? static_cast<int32_t>(__builtin_rintf(fx)) : 0;
            r.Y[i] = ok ? static_cast<int32_t>(__builtin_rintf(fy)) : 0;
            r.z01[i] = z01;
            r.iw[i] = iw;
        }
        const int64_t A = static_cast<int64_t>(r.X[1] - r.X[0]) * (r.Y[2] - r.Y[0]) -
                          static_cast<int64_t>(r.Y[1] - r.Y[0]) * (r.X[2] - r.X[0]);
        ok = ok && A != 0;
        const int32_t mnx = min(r.X[0], min(r.X[1], r.X[2])), mxx = max(r.X[0], max(r.X[1], r.X[2]));
        const int32_t mny = min(r.Y[0], min(r.Y[1], r.Y[2])), mxy = max(r.Y[0], max(r.Y[1], r.Y[2]));
        // pixel x is a candidate when mnx <= 256 x + 128 <= mxx
        const int32_t x0 = max((mnx + 127) >> 8, 0), x1 = min((mxx - 128) >> 8, vd.W - 1);
        const int32_t y0 = max((mny + 127) >> 8, 0), y1 = min((mxy - 128) >> 8, vd.H - 1);
        ok = ok && x0 <= x1 && y0 <= y1;
        if (ok) {
            const int64_t aA = A < 0 ? -A : A;
            float rA = 1.0f / static_cast<float>(aA);
            r.rA = A < 0 ? -rA : rA;
            float zm = fminf(r.z01[0], fminf(r.z01[1], r.z01[2]));
            if (!(zm > 0.0f)) zm = 0.0f;
            if (zm > 1.0f) zm = 1.0f;
            const uint32_t zb = __float_as_uint(zm);
            r.zmin = zb > kZminMargin ? zb - kZminMargin : 0u;
            r.x0 = static_cast<int16_t>(x0);
            r.x1 = static_cast<int16_t>(x1);
            r.y0 = static_cast<int16_t>(y0);
            r.y1 = static_cast<int16_t>(y1);
            const int tx0 = x0 / tile, tx1 = x1 / tile, ty0 = y0 / tile, ty1 = y1 / tile;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    const int b = ty * vd.tiles_x + tx;
                    if (local) atomicAdd(&hist[b], 1);
                    else atomicAdd(&tile_count[vd.tile_base + b], 1);
                }
        } else {
            r.rA = 0.0f;
            r.zmin = 0xFFFFFFFFu;
            r.x0 = 1;
            r.x1 = 0;
            r.y0 = 1;
            r.y1 = 0;
        }
        recs[vd.rec_base + t] = r;
        if (visible) {
            const uint64_t m = __ballot(ok);
            if (lane_id() == __builtin_ctzll(__ballot(1)) && m)
                atomicAdd(visible, static_cast<unsigned long long>(__popcll(m)));
        }
    }
    if (local) {
        __syncthreads();
        int32_t* base = chunk_base + static_cast<int64_t>(blockIdx.x) * n_tiles + vd.tile_base;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            const int n = hist[b];
            if (n) base[b] = atomicAdd(&tile_count[vd.tile_base + b], n);
        }
    }
}

// Writes (zmin << 32 | tri) into the list of every tile a triangle's bounding
// box touches, over the same chunks as the setup. A view binned in LDS takes
// its positions from an LDS cursor per tile, started at the tile's list offset
// plus the chunk's first slot; other views take them from a global atomic.
__global__ __launch_bounds__(256) void scatter_kernel(const ViewDesc* __restrict__ views, int tile, int chunk,
                                                      const TriRec* __restrict__ recs,
                                                      const int64_t* __restrict__ tile_start, int64_t n_tiles,
                                                      const int32_t* __restrict__ chunk_base,
                                                      int32_t* __restrict__ tile_fill,
                                                      uint64_t* __restrict__ entries) {
    __shared__ unsigned long long cur[kHistBins];
    const ViewDesc& vd = views[blockIdx.y];
    const int t_beg = blockIdx.x * chunk;
    if (t_beg >= vd.T) return;
    const int64_t total = tile_start[n_tiles];
    if (total == 0) return;   // no entries, or lists emptied by the static capacity check
    const int t_end = min(t_beg + chunk, vd.T);
    const int nb = vd.tiles_x * vd.tiles_y;
    const bool local = chunk >= kBinChunk && nb <= kHistBins;
    if (local) {
        // bins this chunk does not touch hold stale offsets and are never used
        const int32_t* base = chunk_base + static_cast<int64_t>(blockIdx.x) * n_tiles + vd.tile_base;
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            cur[b] = static_cast<unsigned long long>(tile_start[vd.tile_base + b] + base[b]);
        __syncthreads();
    }
    for (int t = t_beg + static_cast<int>(threadIdx.x); t < t_end; t += blockDim.x) {
        const TriRec r = recs[vd.rec_base + t];
        if (r.x0 > r.x1) continue;
        const uint64_t e = (static_cast<uint64_t>(r.zmin) << 32) | static_cast<uint32_t>(t);
        const int tx0 = r.x0 / tile, tx1 = r.x1 / tile, ty0 = r.y0 / tile, ty1 = r.y1 / tile;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                const int b = ty * vd.tiles_x + tx;
                int64_t at;
                if (local) {
                    at = static_cast<int64_t>(atomicAdd(&cur[b], 1ull));
                } else {
                    const int64_t g = vd.tile_base + b;
                    at = tile_start[g] + atomicAdd(&tile_fill[g], 1);
                }
                if (at < total) entries[at] = e;   // always true: the lists hold exactly these entries
            }
    }
}

// Bitonic sort of a short list by one wave, held in registers: entry e =
// 64 r + lane is register r of its lane (R = entries per lane, n <= 64 R; the
// slots past n hold the largest key and stay at the end). A compare-exchange
// at distance j pairs e with e ^ j: between lanes for j < 64, between two
// registers of one lane for j >= 64. Entry e keeps the smaller key when it is
// the lower of its pair in an ascending run (e & k == 0) or the upper of its
// pair in a descending one.
template <int R>
__device__ __forceinline__ void wave_bitonic_sort(uint64_t* __restrict__ list, int n) {
    const int lane = lane_id();
    constexpr int N = 64 * R;
    uint64_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = 64 * r + lane < n ? list[64 * r + lane] : kBgKey;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                const int jr = j >> 6;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r & jr) continue;   // the pair (r, r + jr), seen from its lower register
                    const int e = 64 * r + lane;
                    const uint64_t a = v[r], b = v[r | jr];
                    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
                    const bool up = (e & k) == 0;
                    v[r] = up ? lo : hi;
                    v[r | jr] = up ? hi : lo;
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int e = 64 * r + lane;
                    const uint64_t b = static_cast<uint64_t>(__shfl_xor(static_cast<long long>(v[r]), j, 64));
                    const bool keep_min = ((e & j) == 0) == ((e & k) == 0);
                    const uint64_t a = v[r];
                    v[r] = keep_min ? (a < b ? a : b) : (a < b ? b : a);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (64 * r + lane < n) list[64 * r + lane] = v[r];
}

constexpr int kWaveSortMax = 256;   // longest list sorted by one wave

// Workgroup b owns tiles b + i * gridDim.x, i = 0..3 (strided, so that the
// long lists of a crowded screen region spread over many workgroups). A list
// of at most kWaveSortMax entries is sorted by the wave of its tile;
// longer lists are then sorted by the whole workgroup, bitonic in LDS, in
// blocks of kSortBlock.
__global__ __launch_bounds__(256) void sort_kernel(const int64_t* __restrict__ tile_start, int64_t n_tiles,
                                                   uint64_t* __restrict__ entries) {
    __shared__ uint64_t s[kSortBlock];
    const int w = threadIdx.x >> 6;
    const int64_t stride = gridDim.x;
    {
        const int64_t tile = blockIdx.x + w * stride;
        if (tile < n_tiles) {
            const int64_t beg = tile_start[tile];
            const int n = static_cast<int>(min<int64_t>(tile_start[tile + 1] - beg, kWaveSortMax + 1));
            if (n > 1 && n <= 64) wave_bitonic_sort<1>(entries + beg, n);
            else if (n > 64 && n <= 128) wave_bitonic_sort<2>(entries + beg, n);
            else if (n > 128 && n <= kWaveSortMax) wave_bitonic_sort<4>(entries + beg, n);
        }
    }
    for (int i = 0; i < 4; ++i) {
        const int64_t tile = blockIdx.x + i * stride;
        if (tile >= n_tiles) break;
        const int64_t beg = tile_start[tile], end = tile_start[tile + 1];
        if (end - beg <= kWaveSortMax) continue;
        for (int64_t b0 = beg; b0 < end; b0 += kSortBlock) {
            const int n = static_cast<int>(min<int64_t>(kSortBlock, end - b0));
            int N = 1;
            while (N < n) N <<= 1;
            __syncthreads();
            for (int j = threadIdx.x; j < N; j += blockDim.x) s[j] = j < n ? entries[b0 + j] : kBgKey;
            __syncthreads();
            for (int k = 2; k <= N; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    // one compare-exchange per thread and step: pair t has its lower
                    // element at t with a zero bit inserted at j's position
                    for (int t = threadIdx.x; t < (N >> 1); t += blockDim.x) {
                        const int x = 2 * t - (t & (j - 1)), xj = x + j;
                        const uint64_t a = s[x], c = s[xj];
                        const bool up = (x & k) == 0;
                        if ((a > c) == up) {
                            s[x] = c;
                            s[xj] = a;
                        }
                    }
                    __syncthreads();
                }
            }
            for (int j = threadIdx.x; j < n; j += blockDim.x) entries[b0 + j] = s[j];
        }
    }
}

// ---------------------------------------------------------------------------
// exclusive scan int32 -> int64 (three passes over blocks of 1024)
// ---------------------------------------------------------------------------

constexpr int kScanBlock = 1024;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t u = __shfl_up(v, d, 64);
        if (lane_id() >= d) v += u;
    }
    return v;
}

// Exclusive scan over the 256 threads of a block; returns the block total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t& total) {
    __shared__ int64_t wsum[4];
    const int w = threadIdx.x >> 6;
    const int64_t inc = wave_incl_scan(v);
    if (lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    int64_t off = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < w) off += wsum[i];
        total += wsum[i];
    }
    __syncthreads();
    return off + inc - v;
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const int32_t* __restrict__ in, int64_t n,
                                                          int64_t* __restrict__ bsum) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock;
    int64_t v = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + threadIdx.x * 4 + k;
        if (i < n) v += in[i];
    }
    int64_t total;
    block_excl_scan(v, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void scan_bsum_kernel(int64_t* __restrict__ bsum, int64_t nb) {
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < nb ? bsum[i] : 0;
        int64_t total;
        const int64_t ex = block_excl_scan(v, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void scan_apply_kernel(const int32_t* __restrict__ in, int64_t n,
                                                         const int64_t* __restrict__ bsum,
                                                         int64_t* __restrict__ out) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock;
    int64_t vals[4];
    int64_t v = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + threadIdx.x * 4 + k;
        vals[k] = i < n ? in[i] : 0;
        v += vals[k];
    }
    int64_t total;
    int64_t ex = block_excl_scan(v, total) + bsum[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + threadIdx.x * 4 + k;
        if (i < n) out[i] = ex;
        ex += vals[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) out[n] = ex;
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void fill_f32_kernel(float* __restrict__ p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

static unsigned grid_for(int64_t n, int bs = 256) {
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return static_cast<unsigned>(g);
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}

void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}

// Large chunks when they still give every CU two workgroups, else one triangle per thread.
int bin_chunk_size(int V, int maxT, int num_cus) {
    const int64_t wgs = static_cast<int64_t>(V) * bin_chunks(maxT, kBinChunk);
    return wgs >= 2 * static_cast<int64_t>(num_cus) ? kBinChunk : 256;
}

void launch_setup(const ViewDesc* views, int V, int maxT, int chunk, const SceneDesc* scenes, const Opts& o,
                  int tile, TriRec* recs, int32_t* tile_count, int32_t* chunk_base, int64_t n_tiles,
                  unsigned long long* visible, hipStream_t s) {
    if (maxT <= 0) return;
    dim3 grid(bin_chunks(maxT, chunk), V);
    hipLaunchKernelGGL(setup_kernel, grid, dim3(256), 0, s, views, scenes, o, tile, chunk, recs, tile_count,
                       chunk_base, n_tiles, visible);
}

void launch_scan(const int32_t* in, int64_t n, int64_t* bsum, int64_t* out, hipStream_t s) {
    if (n <= 0) {   // empty input: the single offset is 0
        launch_fill_i32(reinterpret_cast<int32_t*>(out), 2, 0, s);
        return;
    }
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, in, n, bsum);
    hipLaunchKernelGGL(scan_bsum_kernel, dim3(1), dim3(256), 0, s, bsum, nb);
    hipLaunchKernelGGL(scan_apply_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, in, n, bsum, out);
}

void launch_scatter(const ViewDesc* views, int V, int maxT, int chunk, int tile, const TriRec* recs,
                    const int64_t* tile_start, int64_t n_tiles, const int32_t* chunk_base, int32_t* tile_fill,
                    uint64_t* entries, hipStream_t s) {
    if (maxT <= 0) return;
    dim3 grid(bin_chunks(maxT, chunk), V);
    hipLaunchKernelGGL(scatter_kernel, grid, dim3(256), 0, s, views, tile, chunk, recs, tile_start, n_tiles,
                       chunk_base, tile_fill, entries);
}

// Static-capacity mode: when the lists need more than `cap` entries, flag the
// overflow (sticky bit 1) and empty every tile list, so that no kernel of
// the call touches entries beyond the capacity.
__global__ void clip_check_kernel(const int64_t* __restrict__ tile_start, int64_t n_tiles, int64_t cap,
                                  unsigned int* __restrict__ local, unsigned int* __restrict__ sticky) {
    const bool over = tile_start[n_tiles] > cap;
    *local = over ? 1u : 0u;
    if (over) atomicOr(sticky, 1u);
}

__global__ void clip_apply_kernel(int64_t* __restrict__ tile_start, int64_t n_tiles,
                                  const unsigned int* __restrict__ local) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i <= n_tiles && *local) tile_start[i] = 0;
}

void launch_clip(int64_t* tile_start, int64_t n_tiles, int64_t cap, unsigned int* local, unsigned int* sticky,
                 hipStream_t s) {
    hipLaunchKernelGGL(clip_check_kernel, dim3(1), dim3(1), 0, s, tile_start, n_tiles, cap, local, sticky);
    hipLaunchKernelGGL(clip_apply_kernel, dim3(static_cast<unsigned>((n_tiles + 256) / 256)), dim3(256), 0, s,
                       tile_start, n_tiles, local);
}

void launch_sort(const int64_t* tile_start, int64_t n_tiles, uint64_t* entries, hipStream_t s) {
    if (n_tiles <= 0) return;
    hipLaunchKernelGGL(sort_kernel, dim3(static_cast<unsigned>((n_tiles + 3) / 4)), dim3(256), 0, s, tile_start,
                       n_tiles, entries);
}

}  // namespace soup
