#pragma once
// Forward raster: stochastic opacity masking with a 64-bit depth|triangle
// visibility buffer (Eq. (5); Supplement Algorithm A1, part 1).
//
// One wave is one workgroup and owns one 8x8 pixel block of a screen tile at a
// time, taken from a counter (persistent), so no barrier ever waits for
// another wave. It walks the tile's triangle list (sorted by a lower bound of
// their depth) in three steps:
//  - scan, lanes over list entries: an entry whose bounding box touches the
//    block and whose depth bound can beat a pixel is appended (in list order)
//    to a queue of waiting entries;
//  - coverage, lanes over 64 waiting triangles: each computes its triangle's
//    exact 64-pixel coverage mask of the block from its float64 edge
//    functions (every value an exact integer); covering triangles leave their
//    edge and vertex data in the wave's LDS;
//  - fragments, lanes over pixels: the covering triangles are visited in list
//    order; each covered pixel computes its fragment's key, and a fragment
//    whose key is below the pixel's current best is a candidate, compacted
//    (ballot + prefix count) into an LDS queue.
// The queue is decoded 64 candidates at a time, one per lane, so the
// expensive texture + MLP decode always runs on full waves. A decoded
// fragment that passes its draw lowers the pixel's key with an LDS 64-bit
// atomicMin; the lane holding the pixel's minimum then stores its colour.
// Entries whose depth bound is already behind every pixel of the block are
// skipped, and the walk stops once the rest of the list is behind every
// pixel: front-to-back early-out without sorting fragments. The result does
// not depend on the visiting order (the draws are fixed by Philox), only the
// amount of work does.
#include "raster_common.hpp"

namespace soup {

// LDS of one wave.
struct FwdWaveLds {
    // triangles of the current 64-entry slice that cover a pixel of the block
    double e0[3][64];    // orientation-normalised edge functions at the block's first pixel centre
    double ea[3][64];    // ... step per pixel in x
    double eb[3][64];    // ... step per pixel in y
    float z[3][64];      // vertex depths
    float iw[3][64];     // 1 / w at the vertices
    float ra[64];        // 1 / |2 x area|
    // list entries waiting for the coverage phase (in list order)
    uint64_t pend[128];
    // candidate queue
    uint64_t qkey[128];
    float qt[3][128];    // beta_i / w_i
    uint32_t qpl[128];   // pixel of the block
    // the block's pixels
    uint64_t key[64];
    float rgb[3][64];
};

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), l));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

template <int TS, class S>
__global__ __launch_bounds__(64) void raster_fwd_kernel(RasterArgs a) {
    constexpr int BX = TS / 8, BPT = BX * BX;   // 8x8 blocks per tile
    __shared__ FwdWaveLds L;
    const int lane = threadIdx.x;
    const int pu = lane & 7, pv = lane >> 3;    // the lane's pixel in the block
    const int G = a.G;
    const uint64_t n_items = static_cast<uint64_t>(a.n_tiles) * BPT;
    // optional log of every decoded fragment: this wave's region, private cursor
    const uint64_t log_base = static_cast<uint64_t>(blockIdx.x) * a.log_region;
    uint32_t log_cursor = 0;   // wave-uniform

    for (;;) {   // persistent: blocks from a counter
    uint32_t taken = 0;
    if (lane == 0) taken = atomicAdd(a.work, 1u);
    const uint64_t item = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(taken)));
    if (item >= n_items) break;
    const int64_t tile = static_cast<int64_t>(item / BPT);
    const int blk = static_cast<int>(item % BPT);
    const int v = view_of_tile(a.views, a.V, tile);
    const ViewDesc& vd = a.views[v];
    const int W = vd.W, H = vd.H;
    const int64_t tl = tile - vd.tile_base;
    const int bx = static_cast<int>(tl % vd.tiles_x) * TS + (blk % BX) * 8;
    const int by = static_cast<int>(tl / vd.tiles_x) * TS + (blk / BX) * 8;
    if (bx >= W || by >= H) continue;   // a block of a ragged tile that lies outside the view
    const SceneDesc sc = a.scenes[vd.scene];
    gfloat* __restrict__ feats = as_global(uniform_ptr(sc.feats));
    const float* mlp_p = uniform_ptr(sc.mlp);
    const TriRec* __restrict__ recs = uniform_ptr(a.recs + vd.rec_base);

    const bool inview = bx + pu < W && by + pv < H;
    uint64_t kc = inview ? kBgKey : 0ull;   // pixels outside the view never take fragments
    L.key[lane] = kc;
    uint64_t wmax = wave_max_u64(kc);

    // decode a batch of n queued candidates, one per lane
    auto run_batch = [&](int n) __attribute__((always_inline)) {
        __syncthreads();
        const bool act = lane < n;
        uint64_t key = 0;
        int pl = 0;
        bool pass = false;
        float o[4] = {0.f, 0.f, 0.f, 0.f};
        if (act) {
            key = L.qkey[lane];
            pl = static_cast<int>(L.qpl[lane]);
            float b1, b2;
            persp_from_t(L.qt[0][lane], L.qt[1][lane], L.qt[2][lane], b1, b2);
            const uint32_t tri = static_cast<uint32_t>(key);
            const Cell c = cell_of(b1, b2, G);
            float x[S::C];
            fetch_feature<S::C>(feats, tri, G, c, x);
            // an opaque copy of the weight pointer per batch: the compiler may
            // not hoist the weights' scalar loads out of the traversal loops
            mlp_logits<S>(as_const(opaque_ptr(mlp_p)), x, o);
            const int gy = by + (pl >> 3), gx = bx + (pl & 7);
            if (a.o.mode == 0) {
                const float alpha = sigmoid_c(o[3]);
                const uint32_t pidx = static_cast<uint32_t>(gy * W + gx);
                pass = uniform24(a.o.seed, pidx, tri, vd.view_id, a.o.step) < alpha;
            } else {
                pass = o[3] > 0.0f;
            }
            if (pass) atomicMin(reinterpret_cast<unsigned long long*>(&L.key[pl]), static_cast<unsigned long long>(key));
            if (a.log_frag) {
                const uint32_t at = log_cursor + static_cast<uint32_t>(lane);
                if (at < a.log_region) {
                    const int64_t pg = vd.pix_base + static_cast<int64_t>(gy) * W + gx;
                    a.log_frag[log_base + at] =
                        make_uint4(static_cast<uint32_t>(pg), tri, __float_as_uint(b1), __float_as_uint(b2));
                    a.log_aux[log_base + at] = make_uint2(static_cast<uint32_t>(key >> 32), static_cast<uint32_t>(v));
                }
            }
        }
        if (a.log_frag) log_cursor += static_cast<uint32_t>(n);
        __syncthreads();
        if (pass && L.key[pl] == key) {
            L.rgb[0][pl] = sigmoid_c(o[0]);
            L.rgb[1][pl] = sigmoid_c(o[1]);
            L.rgb[2][pl] = sigmoid_c(o[2]);
        }
        if (a.counter && lane == 0) atomicAdd(a.counter, static_cast<unsigned long long>(n));
        __syncthreads();
        kc = L.key[lane];
        wmax = wave_max_u64(kc);
    };

    // snapped position of the block's first pixel centre
    const int64_t PX0 = static_cast<int64_t>(kSnap) * bx + kSnap / 2;
    const int64_t PY0 = static_cast<int64_t>(kSnap) * by + kSnap / 2;
    const int64_t beg = a.tile_start[tile], end = a.tile_start[tile + 1];
    const double fx = static_cast<double>(pu), fy = static_cast<double>(pv);
    int64_t c0 = beg;         // next list entry to scan
    bool listed = false;      // the scan has reached the end of the list or its early-out
    int pn = 0;               // entries waiting for the coverage phase (L.pend)
    int qn = 0;               // queued candidates
    uint64_t hit = 0;         // slice slots that cover a pixel and are not visited yet
    uint64_t ent = kBgKey;    // this lane's slice entry
    uint32_t mlo = 0, mhi = 0;   // ... and its coverage of block pixels 0..31, 32..63
    // One loop, uniform control flow: decode when 64 candidates wait (or at the
    // end), else visit the next covering slot, else run coverage on the next 64
    // waiting entries, else scan the next 64 list entries.
    for (;;) {
        if (qn >= 64 || (hit == 0 && pn == 0 && listed)) {
            if (qn == 0) break;
            const int n = qn < 64 ? qn : 64;
            run_batch(n);
            if (lane < qn - n) {
                L.qkey[lane] = L.qkey[n + lane];
#pragma unroll
                for (int i = 0; i < 3; ++i) L.qt[i][lane] = L.qt[i][n + lane];
                L.qpl[lane] = L.qpl[n + lane];
            }
            qn -= n;
            __syncthreads();
            continue;
        }
        if (hit) {
            // ---- fragments of one covering triangle: lane = pixel ----
            const int j = __builtin_ctzll(hit);
            hit &= hit - 1;
            const uint64_t zk = readlane_u64(ent, j);
            // the depth bound no longer beats any pixel of the block (a list longer than a sort
            // block is sorted only block by block, so later slots are tested one by one)
            if (zk >= wmax) continue;
            // lanes 0..31 test their bit in mlo of slot j, lanes 32..63 in mhi
            const uint32_t mj_lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(mlo), j));
            const uint32_t mj_hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(mhi), j));
            const bool cov = (((lane < 32 ? mj_lo >> lane : mj_hi >> (lane - 32)) & 1u) != 0u) & (zk < kc);
            bool cand = false;
            Frag f;
            if (cov) {
                double e[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) e[i] = __builtin_fma(fx, L.ea[i][j], __builtin_fma(fy, L.eb[i][j], L.e0[i][j]));
                const float ra = L.ra[j];
#pragma unroll
                for (int i = 0; i < 3; ++i) f.beta[i] = static_cast<float>(e[i]) * ra;
                float z = __builtin_fmaf(f.beta[2], L.z[2][j], __builtin_fmaf(f.beta[1], L.z[1][j], f.beta[0] * L.z[0][j]));
                if (!(z > 0.0f)) z = 0.0f;
                if (z > 1.0f) z = 1.0f;
                f.key = (static_cast<uint64_t>(__float_as_uint(z)) << 32) | static_cast<uint32_t>(zk);
                cand = f.key < kc;
            }
            const uint64_t m = __ballot(cand);
            if (cand) {
                const int pos = qn + __popcll(m & lanemask_lt());
                L.qkey[pos] = f.key;
#pragma unroll
                for (int i = 0; i < 3; ++i) L.qt[i][pos] = f.beta[i] * L.iw[i][j];
                L.qpl[pos] = static_cast<uint32_t>(lane);
            }
            qn += __popcll(m);
            continue;
        }
        if (pn >= 64 || (listed && pn > 0)) {
            // ---- coverage of up to 64 waiting entries: lane = triangle ----
            const int n = pn < 64 ? pn : 64;
            ent = lane < n ? L.pend[lane] : kBgKey;
            mlo = 0;
            mhi = 0;
            if (ent < wmax) {   // still able to beat a pixel of the block (pads are kBgKey)
                guint4* rp = as_global(reinterpret_cast<const uint4*>(recs + static_cast<uint32_t>(ent)));
                const uint4 q0 = rp[0], q1 = rp[1], q2 = rp[2], q3 = rp[3];
                const int32_t X[3] = {static_cast<int32_t>(q0.x), static_cast<int32_t>(q0.y), static_cast<int32_t>(q0.z)};
                const int32_t Y[3] = {static_cast<int32_t>(q0.w), static_cast<int32_t>(q1.x), static_cast<int32_t>(q1.y)};
                const float rA = __uint_as_float(q3.x);
                const int sgn = rA < 0.0f ? -1 : 1;
                double e0[3], ea[3], eb[3], thr[3];
#pragma unroll
                for (int e = 0; e < 3; ++e) {   // edge e joins vertices e+1 and e+2
                    const int va = e == 2 ? 0 : e + 1;
                    const int vb = e == 0 ? 2 : (e == 1 ? 0 : 1);
                    const int32_t dx = X[vb] - X[va], dy = Y[vb] - Y[va];
                    const int64_t E0 =
                        static_cast<int64_t>(dx) * (PY0 - Y[va]) - static_cast<int64_t>(dy) * (PX0 - X[va]);
                    e0[e] = static_cast<double>(sgn * E0);
                    ea[e] = static_cast<double>(-static_cast<int64_t>(sgn) * kSnap * dy);
                    eb[e] = static_cast<double>(static_cast<int64_t>(sgn) * kSnap * dx);
                    // an edge owns the centres exactly on it when it is a top or left edge:
                    // E > 0, or E == 0 on an owning edge, is E > -1/2 for integer E
                    const int32_t ndx = sgn * dx, ndy = sgn * dy;
                    thr[e] = (ndy < 0 || (ndy == 0 && ndx > 0)) ? -0.5 : 0.0;
                }
#pragma unroll
                for (int pv2 = 0; pv2 < 8; ++pv2) {
                    double c[3];
#pragma unroll
                    for (int e = 0; e < 3; ++e) c[e] = __builtin_fma(static_cast<double>(pv2), eb[e], e0[e]);
                    uint32_t row = 0;
#pragma unroll
                    for (int pu2 = 0; pu2 < 8; ++pu2) {
                        bool in = true;
#pragma unroll
                        for (int e = 0; e < 3; ++e)
                            in = in & (__builtin_fma(static_cast<double>(pu2), ea[e], c[e]) > thr[e]);
                        row |= in ? (1u << pu2) : 0u;
                    }
                    if (pv2 < 4) mlo |= row << (8 * pv2);
                    else mhi |= row << (8 * (pv2 - 4));
                }
                if ((mlo | mhi) != 0) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        L.e0[e][lane] = e0[e];
                        L.ea[e][lane] = ea[e];
                        L.eb[e][lane] = eb[e];
                    }
                    L.z[0][lane] = __uint_as_float(q1.z);
                    L.z[1][lane] = __uint_as_float(q1.w);
                    L.z[2][lane] = __uint_as_float(q2.x);
                    L.iw[0][lane] = __uint_as_float(q2.y);
                    L.iw[1][lane] = __uint_as_float(q2.z);
                    L.iw[2][lane] = __uint_as_float(q2.w);
                    L.ra[lane] = __builtin_fabsf(rA);
                }
            }
            hit = __ballot((mlo | mhi) != 0);
            __syncthreads();
            if (lane < pn - n) L.pend[lane] = L.pend[n + lane];
            pn -= n;
            __syncthreads();
            continue;
        }
        // ---- scan the next 64 list entries: keep those that can cover the block ----
        if (c0 >= end || remaining_min(a.entries, beg, c0, end) >= wmax) {
            listed = true;
            continue;
        }
        const uint64_t e = c0 + lane < end ? a.entries[c0 + lane] : kBgKey;
        bool keep = false;
        if (e < wmax) {   // its depth bound can beat some pixel of the block
            const uint4 q3 = as_global(reinterpret_cast<const uint4*>(recs + static_cast<uint32_t>(e)))[3];
            const int x0 = static_cast<int16_t>(q3.z & 0xFFFFu), y0 = static_cast<int16_t>(q3.z >> 16);
            const int x1 = static_cast<int16_t>(q3.w & 0xFFFFu), y1 = static_cast<int16_t>(q3.w >> 16);
            keep = !(x1 < bx || x0 > bx + 7 || y1 < by || y0 > by + 7);
        }
        const uint64_t km = __ballot(keep);
        if (keep) L.pend[pn + __popcll(km & lanemask_lt())] = e;
        pn += __popcll(km);
        c0 += 64;
        __syncthreads();
    }
    if (inview) {
        const int gx = bx + pu, gy = by + pv;
        const uint64_t key = L.key[lane];
        const int64_t off = static_cast<int64_t>(gy) * W + gx;
        float* col = vd.color_out ? vd.color_out + 3 * off : a.color + 3 * (vd.pix_base + off);
        if (vd.vis_out) vd.vis_out[off] = key;
        else if (a.vis) a.vis[vd.pix_base + off] = key;
        if (key == kBgKey) {
            col[0] = a.o.bg[0];
            col[1] = a.o.bg[1];
            col[2] = a.o.bg[2];
        } else {
            col[0] = L.rgb[0][lane];
            col[1] = L.rgb[1][lane];
            col[2] = L.rgb[2][lane];
        }
    }
    __syncthreads();
    }   // blocks
    if (a.log_counts && lane == 0) a.log_counts[blockIdx.x] = log_cursor;
}

// Resident waves per CU of the forward (its workgroups are single waves).
template <int TS, class S>
static int fwd_blocks_per_cu() {
    static int n = 0;
    if (n == 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, raster_fwd_kernel<TS, S>, 64, 0) != hipSuccess || b < 1)
            b = 8;
        n = b;
    }
    return n;
}

template <int TS, class S>
static void launch_fwd_t(const RasterArgs& a, hipStream_t s) {
    if (a.n_tiles <= 0 || a.n_blocks <= 0) return;
    hipLaunchKernelGGL((raster_fwd_kernel<TS, S>), dim3(static_cast<unsigned>(a.n_blocks)), dim3(64), 0, s, a);
}


}  // namespace soup
