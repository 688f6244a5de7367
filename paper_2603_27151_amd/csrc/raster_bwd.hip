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
// gradient records -> per-triangle lists -> per-triangle reduction
// ---------------------------------------------------------------------------

// Counting-sort placement of record indices into per-triangle lists; runs of
// equal triangles in a wave take one atomic.
__global__ __launch_bounds__(256) void bucket_kernel(const uint32_t* __restrict__ rec_tri,
                                                     const unsigned long long* __restrict__ n_batch,
                                                     const int64_t* __restrict__ tri_off,
                                                     int32_t* __restrict__ tri_fill, uint32_t* __restrict__ idx) {
    const int64_t n = static_cast<int64_t>(*n_batch) * 64;
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint32_t tri = i < n ? rec_tri[i] : 0xFFFFFFFFu;
    const bool on = tri != 0xFFFFFFFFu;   // empty record lanes carry the sentinel
    const uint32_t tprev = __shfl_up(tri, 1, 64);
    const bool head = lane == 0 || tprev != tri;   // a sentinel lane ends a run
    const uint64_t heads = __ballot(head);   // outside any branch: a ballot sees only the lanes that execute it
    int base = 0;
    if (head && on) {
        const uint64_t above = lane == 63 ? 0ull : (heads & (~0ull << (lane + 1)));
        const int endl = above ? __builtin_ctzll(above) : 64;
        base = atomicAdd(&tri_fill[tri], endl - lane);
    }
    const uint64_t upto = lane == 63 ? heads : (heads & ((2ull << lane) - 1));
    const int hl = upto ? 63 - __builtin_clzll(upto) : 0;
    const int hb = __shfl(base, hl, 64);
    if (on) idx[tri_off[tri] + hb + (lane - hl)] = static_cast<uint32_t>(i);
}

// Records per reduction chunk: 64 per thread of a 256-thread workgroup.
template <int C>
constexpr int64_t kChunkRecs = 64 * (256 / C);

// Chunks per triangle (at least one, so that untouched triangles still get
// their zero gradient written). A triangle split over several chunks is summed
// with global atomics, so its outputs are cleared here first unless the call
// accumulates.
template <int C>
__global__ __launch_bounds__(256) void reduce_prep_kernel(const int64_t* __restrict__ tri_off, int T, int n_feat,
                                                          int32_t* __restrict__ chunk_n,
                                                          float* __restrict__ grad_feats,
                                                          float* __restrict__ grad_verts, bool accumulate) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int64_t cnt = tri_off[t + 1] - tri_off[t];
    const int32_t nch = cnt <= kChunkRecs<C> ? 1 : static_cast<int32_t>((cnt + kChunkRecs<C> - 1) / kChunkRecs<C>);
    chunk_n[t] = nch;
    if (nch > 1 && !accumulate) {
        float* gf = grad_feats + static_cast<size_t>(t) * n_feat;
        for (int k = 0; k < n_feat; ++k) gf[k] = 0.0f;
        for (int k = 0; k < 9; ++k) grad_verts[static_cast<size_t>(t) * 9 + k] = 0.0f;
    }
}

// One workgroup per chunk of at most kChunkRecs records of one triangle: sums
// the records' feature gradients into the G x G x C grid in LDS (bilinear
// weights of each record's cell position) and its winners' vertex gradients.
// Thread (seg, c) walks a contiguous segment of the chunk for channel c;
// consecutive records mostly share a cell (they come from the same tile), so
// the four corner sums stay in registers for a run of equal cells and reach
// LDS once per run. A triangle of one chunk stores its sums; the chunks of a
// larger triangle add theirs with global atomics, so that no workgroup walks
// more than a chunk however many pixels one triangle covers.
// chunk_tri[c] = the triangle that owns chunk c.
__global__ __launch_bounds__(256) void chunk_map_kernel(const int64_t* __restrict__ chunk_off, int T,
                                                        int32_t* __restrict__ chunk_tri) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    for (int64_t c = chunk_off[t]; c < chunk_off[t + 1]; ++c) chunk_tri[c] = t;
}

template <int C>
__global__ __launch_bounds__(256) void reduce_kernel(const float* __restrict__ records, int G, int T,
                                                     const int64_t* __restrict__ tri_off,
                                                     const int64_t* __restrict__ chunk_off,
                                                     const int32_t* __restrict__ chunk_tri,
                                                     const uint32_t* __restrict__ idx, float* __restrict__ grad_feats,
                                                     float* __restrict__ grad_verts, bool accumulate) {
    extern __shared__ float s_acc[];      // [G*G*C + 16]
    const int64_t b = blockIdx.x;
    if (b >= chunk_off[T]) return;        // the grid is sized by an upper bound of the chunk count
    const int t = chunk_tri[b];
    const int64_t ci = b - chunk_off[t];
    const bool whole = chunk_off[t + 1] - chunk_off[t] == 1;
    const int n_feat = G * G * C;
    float* s_gv = s_acc + n_feat;
    for (int k = threadIdx.x; k < n_feat + 16; k += blockDim.x) s_acc[k] = 0.0f;
    __syncthreads();
    const int64_t beg = tri_off[t] + ci * kChunkRecs<C>;
    const int64_t end = min(tri_off[t + 1], beg + kChunkRecs<C>);
    constexpr int NSEG = 256 / C;
    const int c = threadIdx.x % C, seg = threadIdx.x / C;
    const int64_t per = (end - beg + NSEG - 1) / NSEG;
    const int64_t i0 = beg + seg * per, i1 = min(end, i0 + per);
    float a00 = 0.f, a10 = 0.f, a01 = 0.f, a11 = 0.f;
    int cur = -1;
    auto flush = [&]() {
        if (cur < 0) return;
        const int ix = cur & 255, iy = cur >> 8;
        const int t00 = (iy * G + ix) * C + c;
        atomicAdd(&s_acc[t00], a00);
        atomicAdd(&s_acc[t00 + C], a10);
        atomicAdd(&s_acc[t00 + G * C], a01);
        atomicAdd(&s_acc[t00 + G * C + C], a11);
        a00 = a10 = a01 = a11 = 0.f;
    };
    constexpr int U = 4;   // records in flight per thread
    for (int64_t i = i0; i < i1; i += U) {
        uint32_t cells[U];
        float fxs[U], fys[U], ds[U];
        const float* recs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) recs[u] = i + u < i1 ? records + static_cast<size_t>(idx[i + u]) * kRecStride<C> : nullptr;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!recs[u]) continue;
            cells[u] = __float_as_uint(recs[u][1]);
            fxs[u] = recs[u][2];
            fys[u] = recs[u][3];
            ds[u] = recs[u][4 + c];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!recs[u]) continue;
            const int key = static_cast<int>(cells[u] & 0xFFFFu);
            const float fx = fxs[u], fy = fys[u], d = ds[u];
            if (key != cur) {
                flush();
                cur = key;
            }
            a00 = __builtin_fmaf((1.0f - fx) * (1.0f - fy), d, a00);
            a10 = __builtin_fmaf(fx * (1.0f - fy), d, a10);
            a01 = __builtin_fmaf((1.0f - fx) * fy, d, a01);
            a11 = __builtin_fmaf(fx * fy, d, a11);
            if (cells[u] >> 31)
                for (int k = c; k < 9; k += C) atomicAdd(&s_gv[k], recs[u][4 + C + k]);
        }
    }
    flush();
    __syncthreads();
    float* gf = grad_feats + static_cast<size_t>(t) * n_feat;
    float* gv = grad_verts + static_cast<size_t>(t) * 9;
    if (whole) {
        for (int k = threadIdx.x; k < n_feat; k += blockDim.x) gf[k] = accumulate ? gf[k] + s_acc[k] : s_acc[k];
        if (threadIdx.x < 9) gv[threadIdx.x] = accumulate ? gv[threadIdx.x] + s_gv[threadIdx.x] : s_gv[threadIdx.x];
    } else {
        for (int k = threadIdx.x; k < n_feat; k += blockDim.x)
            if (s_acc[k] != 0.0f) atomicAdd(&gf[k], s_acc[k]);
        if (threadIdx.x < 9 && s_gv[threadIdx.x] != 0.0f) atomicAdd(&gv[threadIdx.x], s_gv[threadIdx.x]);
    }
}

void launch_bucket(const uint32_t* rec_tri, const unsigned long long* n_batch, int64_t bound,
                   const int64_t* tri_off, int32_t* tri_fill, uint32_t* idx, hipStream_t s) {
    if (bound <= 0) return;
    hipLaunchKernelGGL(bucket_kernel, dim3(static_cast<unsigned>((bound + 255) / 256)), dim3(256), 0, s, rec_tri,
                       n_batch, tri_off, tri_fill, idx);
}

template <int C>
static void launch_reduce_c(const float* records, int G, int T, int64_t n_rec, const int64_t* tri_off,
                            int32_t* chunk_n, int64_t* chunk_bsum, int64_t* chunk_off, int32_t* chunk_tri,
                            const uint32_t* idx, float* grad_feats, float* grad_verts, bool accumulate,
                            hipStream_t s) {
    const int n_feat = G * G * C;
    hipLaunchKernelGGL(reduce_prep_kernel<C>, dim3((T + 255) / 256), dim3(256), 0, s, tri_off, T, n_feat, chunk_n,
                       grad_feats, grad_verts, accumulate);
    launch_scan(chunk_n, T, chunk_bsum, chunk_off, s);
    hipLaunchKernelGGL(chunk_map_kernel, dim3((T + 255) / 256), dim3(256), 0, s, chunk_off, T, chunk_tri);
    const int64_t blocks = reduce_chunk_bound(C, T, n_rec);
    const size_t lds = (static_cast<size_t>(n_feat) + 16) * sizeof(float);
    hipLaunchKernelGGL(reduce_kernel<C>, dim3(static_cast<unsigned>(blocks)), dim3(256), lds, s, records, G, T,
                       tri_off, chunk_off, chunk_tri, idx, grad_feats, grad_verts, accumulate);
}

int64_t reduce_chunk_bound(int C, int T, int64_t n_rec) {
    const int64_t K = 64 * (256 / C);
    return T + n_rec / K + 1;   // >= sum over t of max(1, ceil(n_t / K))
}

void launch_reduce(const float* records, int C, int G, int T, int64_t n_rec, const int64_t* tri_off,
                   int32_t* chunk_n, int64_t* chunk_bsum, int64_t* chunk_off, int32_t* chunk_tri,
                   const uint32_t* idx, float* grad_feats, float* grad_verts, bool accumulate, hipStream_t s) {
    if (T <= 0) return;
    switch (C) {
        case 8:
            launch_reduce_c<8>(records, G, T, n_rec, tri_off, chunk_n, chunk_bsum, chunk_off, chunk_tri, idx,
                               grad_feats, grad_verts, accumulate, s);
            break;
        case 16:
            launch_reduce_c<16>(records, G, T, n_rec, tri_off, chunk_n, chunk_bsum, chunk_off, chunk_tri, idx,
                                grad_feats, grad_verts, accumulate, s);
            break;
        case 32:
            launch_reduce_c<32>(records, G, T, n_rec, tri_off, chunk_n, chunk_bsum, chunk_off, chunk_tri, idx,
                                grad_feats, grad_verts, accumulate, s);
            break;
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
