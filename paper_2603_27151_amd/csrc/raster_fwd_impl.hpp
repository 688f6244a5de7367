#pragma once
// Forward raster: stochastic opacity masking with a 64-bit depth|triangle
// visibility buffer (Eq. (5); Supplement Algorithm A1, part 1).
//
// One wave is one workgroup and owns one region of a screen tile at a time
// (16x16 pixels, four 8x8 blocks, or a single 8x8 block when a call has too
// few 16x16 regions to fill the GPU), taken from a counter (persistent, the
// next region fetched while the current one runs),
// so no barrier ever waits for another wave (the wave's LDS accesses are
// ordered by wavefront-scope fences, which wait on nothing). It walks the tile's triangle
// list (sorted by a lower bound of their depth) in three steps, all in one
// loop with uniform control flow:
//  - scan, lanes over list entries: each entry whose bounding box touches a
//    block of the region, and whose depth bound can still beat a pixel of
//    that block, appends one (triangle, block) pair per such block to a queue
//    of waiting pairs, in list order;
//  - coverage, lanes over 64 waiting pairs: each computes the exact 64-pixel
//    coverage mask of its triangle over its block from float64 edge
//    functions (every value an exact integer); covering pairs leave their
//    edge and vertex data in the wave's LDS;
//  - fragments, lanes over covered (pair, pixel) combinations: the slice's
//    combinations are taken 64 at a time in slice order (a lane finds its pair
//    by a max-scan over the starts of the pairs' runs and its pixel as the
//    k-th set bit of the pair's mask); each computes its fragment's key, and a
//    fragment whose key is below the pixel's current best is a candidate,
//    compacted (ballot + prefix count) into an LDS queue with beta_i / w_i.
// The queue is decoded 64 candidates at a time, one per lane, so the
// expensive texture + MLP decode always runs on full waves. A decoded
// fragment that passes its draw lowers the pixel's key with an LDS 64-bit
// atomicMin; the lane holding the pixel's minimum then writes its colour to
// the output (a later, nearer passing fragment overwrites it).
// Entries whose depth bound is already behind every pixel of a block are
// skipped, and the walk stops once the rest of the list is behind every
// pixel: front-to-back early-out without sorting fragments. The result does
// not depend on the visiting order (the draws are fixed by Philox), only the
// amount of work does.
#include "pform.hpp"

namespace soup {

// A slice pair's geometry, one 16-byte aligned record (five 16-byte reads).
struct alignas(16) PairGeo {
    double e0[3];        // orientation-normalised edge functions at the block's first pixel centre
    int32_t ndx[3];      // ... whose steps per pixel are -256 ndy in x and 256 ndx in y
    int32_t ndy[3];
    float z[3];          // vertex depths
    float iw[3];         // 1 / w at the vertices
    float ra;            // 1 / |2 x area|
    float pad;
};
// A slice pair's run of combinations: coverage mask, list entry, first combination, block.
struct alignas(8) PairMeta {
    uint32_t mlo, mhi;
    uint32_t ent_lo, ent_hi;
    int32_t off, blk;
};

// LDS of one wave owning NB 8x8 blocks.
template <int NB>
struct FwdWaveLds {
    // the current slice: (triangle, block) pairs that cover a pixel of their block
    PairGeo geo[64];
    PairMeta meta[64];
    // (triangle, block) pairs waiting for the coverage step, in list order: a ring of
    // kRing slots (at most 63 wait when a scan of 64 entries appends up to 64 NB more)
    static constexpr int kRing = 64 * (NB + 1);
    uint32_t ptri[kRing];
    uint8_t pblk[kRing];
    // candidate queue: a fragment round starts with fewer than 64 waiting (64
    // are decoded first) and adds at most 64, one per lane
    static constexpr int kQueue = 128;
    uint64_t qkey[kQueue];
    float qt[3][kQueue];    // beta_i / w_i (the decode forms the perspective-correct barycentrics)
    uint16_t qpl[kQueue];   // pixel of the region: block * 64 + pixel of the block
    // the region's pixels: current best key (their colours go straight to the output)
    uint64_t key[64 * NB];
    // per round of the fragment step: the slice pair whose run of combinations starts here
    int32_t head[64];
    // counting only: the region's pixels that some fragment covers, per block (bits 0..31, 32..63)
    uint32_t cov[2 * NB];
};

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), l));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ int wave_incl_scan_i32(int v) {
    return wave_scan_dpp(v, 0, [](int x, int y) { return x + y; });
}

// Position of the k-th set bit (k from 0) of the 64-bit mask hi:lo.
__device__ __forceinline__ int select_bit(uint32_t lo, uint32_t hi, int k) {
    const int cl = __popc(lo);
    uint32_t x = k < cl ? lo : hi;
    int pos = k < cl ? 0 : 32;
    k = k < cl ? k : k - cl;
    int c = __popc(x & 0xFFFFu);
    if (k >= c) { k -= c; x >>= 16; pos += 16; }
    c = __popc(x & 0xFFu);
    if (k >= c) { k -= c; x >>= 8; pos += 8; }
    c = __popc(x & 0xFu);
    if (k >= c) { k -= c; x >>= 4; pos += 4; }
    c = __popc(x & 0x3u);
    if (k >= c) { k -= c; x >>= 2; pos += 2; }
    if (k >= static_cast<int>(x & 1u)) pos += 1;
    return pos;
}

// Element b of a small register array, as masks: a chain of selects of
// array elements would be folded back into an indexed load, which puts the
// array in scratch memory.
template <int N>
__device__ __forceinline__ uint64_t pick(const uint64_t (&arr)[N], int b) {
    uint64_t r = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) r |= arr[i] & (0ull - static_cast<uint64_t>(b == i));
    return r;
}

template <int TS, int RS, class S>
__global__ __launch_bounds__(64, 3) void raster_fwd_kernel(RasterArgs a) {
    static_assert(RS == 8 || (RS == 16 && TS >= 16), "a region is one 8x8 block, or 16x16 pixels of a larger tile");
    constexpr int BR = RS / 8, NB = BR * BR;       // 8x8 blocks per region
    constexpr int RT = TS / RS, RPT = RT * RT;     // regions per tile
    __shared__ FwdWaveLds<NB> L;
    const int lane = threadIdx.x;
    const int pu = lane & 7, pv = lane >> 3;       // the lane's pixel in a block
    const double fx = static_cast<double>(pu), fy = static_cast<double>(pv);
    const int G = a.G;
    const uint64_t n_items = static_cast<uint64_t>(a.n_tiles) * RPT;
    // optional log of every decoded fragment: this wave's region, private cursor
    const uint64_t log_base = static_cast<uint64_t>(blockIdx.x) * a.log_region;
    uint32_t log_cursor = 0;   // wave-uniform
    int vcur = 0;              // view of the previous region, and its tiles [vlo, vhi)
    int64_t vlo = 0, vhi = 0;
    uint32_t next = 0;
    if (lane == 0) next = atomicAdd(a.work, 1u);
    // The walk's scan, coverage and fragment steps wait on memory and LDS; at a
    // raised priority they issue ahead of the other waves' decode batches, long
    // runs of VALU work that then fill the gaps: priority 2 for the scan and the
    // fragment step, 1 for the coverage step, the default for a decode batch
    // (forward 2.26 -> 2.22 ms)
    __builtin_amdgcn_s_setprio(1);

    for (;;) {   // persistent: regions from a counter
    const uint64_t item = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(next)));
    if (item >= n_items) break;
    if (lane == 0) next = atomicAdd(a.work, 1u);   // the following region, fetched while this one runs
    const int64_t tile = static_cast<int64_t>(item / RPT);
    const int rq = static_cast<int>(item % RPT);
    if (tile < vlo || tile >= vhi) {
        vcur = view_of_tile(a.views, a.V, tile);
        vlo = a.views[vcur].tile_base;
        vhi = vcur + 1 < a.V ? a.views[vcur + 1].tile_base : a.n_tiles;
    }
    const int v = vcur;
    const ViewDesc& vd = a.views[v];
    const int W = vd.W, H = vd.H;
    const int64_t tl = tile - vd.tile_base;
    const int rx = static_cast<int>(tl % vd.tiles_x) * TS + (rq % RT) * RS;
    const int ry = static_cast<int>(tl / vd.tiles_x) * TS + (rq / RT) * RS;
    if (rx >= W || ry >= H) continue;   // a region of a ragged tile that lies outside the view
    const SceneDesc sc = a.scenes[vd.scene];
    gfloat* __restrict__ feats = as_global(uniform_ptr(sc.feats));
    const float* mlp_p = uniform_ptr(sc.mlp);
    const TriRec* __restrict__ recs = uniform_ptr(a.recs + vd.rec_base);
    // the view's fields that the batches and the epilogue use, read once: read
    // through vd after a store, they would be loaded again (the store may alias)
    const uint32_t view_id = vd.view_id;
    const int64_t pix_base = vd.pix_base;
    gfloat_w* const color_base = as_global_w(uniform_ptr(vd.color_out ? vd.color_out : a.color + 3 * vd.pix_base));
    guint64_w* const vis_base =
        as_global_w(uniform_ptr(vd.vis_out ? vd.vis_out : (a.vis ? a.vis + vd.pix_base : nullptr)));

    // the pixels' best keys live in L.key; per block, the largest of them (wave-uniform)
    uint64_t wmaxb[NB];
    uint64_t wmax = 0;   // ... over the region
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const bool inview = rx + (b % BR) * 8 + pu < W && ry + (b / BR) * 8 + pv < H;
        const uint64_t k0 = inview ? kBgKey : 0ull;   // pixels outside the view never take fragments
        L.key[b * 64 + lane] = k0;
        wmaxb[b] = wave_max_u64(k0);
        wmax = wmaxb[b] > wmax ? wmaxb[b] : wmax;
    }
    if (a.counter && lane < 2 * NB) L.cov[lane] = 0u;

    // decode a batch of n queued candidates, one per lane
    auto run_batch = [&](int n) __attribute__((always_inline)) {
        // the colour stores below may overwrite a pixel's colour from an earlier
        // batch: those stores complete first (the only wait on global memory
        // that the LDS ordering of this kernel needs)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_setprio(0);
        const bool act = lane < n;
        uint64_t key = 0;
        int pl = 0;
        bool pass = false;
        float o[4] = {0.f, 0.f, 0.f, 0.f};
        constexpr int GW = GateWords<S>::kWords;
        uint32_t gates[GW > 0 ? GW : 1];
#pragma unroll
        for (int w = 0; w < GW; ++w) gates[w] = 0u;
        if (act) {
            key = L.qkey[lane];
            pl = static_cast<int>(L.qpl[lane]);
            float b1, b2;
            persp_from_t(L.qt[0][lane], L.qt[1][lane], L.qt[2][lane], b1, b2);
            const uint32_t tri = static_cast<uint32_t>(key);
            const int blk = pl >> 6, p = pl & 63;
            const int gx = rx + (blk % BR) * 8 + (p & 7), gy = ry + (blk / BR) * 8 + (p >> 3);
            if constexpr (S::kPaper) {
                // the opacity texture alone decides the mask (G holds the texture level R)
                const float alpha = mc_alpha(feats, tri, G, b1, b2);
                if (a.o.mode == 0) {
                    const uint32_t pidx = static_cast<uint32_t>(gy * W + gx);
                    pass = uniform24(a.o.seed, pidx, tri, view_id, a.o.step) < alpha;
                } else {
                    pass = alpha > 0.5f;
                }
            } else {
                const Cell c = cell_of(b1, b2, G);
                float x[S::C];
                fetch_feature<S::C>(feats, tri, G, c, x);
                // an opaque copy of the weight pointer per batch: the compiler may
                // not hoist the weights' scalar loads out of the traversal loops
                // (the ReLU gates are kept for the log; forming them costs two
                // instructions per hidden unit)
                mlp_logits_gates<S>(as_const(opaque_ptr(mlp_p)), x, o, gates);
                if (a.o.mode == 0) {
                    const float alpha = sigmoid_c(o[3]);
                    const uint32_t pidx = static_cast<uint32_t>(gy * W + gx);
                    pass = uniform24(a.o.seed, pidx, tri, view_id, a.o.step) < alpha;
                } else {
                    pass = o[3] > 0.0f;
                }
            }
            if (pass) atomicMin(reinterpret_cast<unsigned long long*>(&L.key[pl]), static_cast<unsigned long long>(key));
            if (a.log_frag) {
                const uint32_t at = log_cursor + static_cast<uint32_t>(lane);
                if (at < a.log_region) {
                    const int64_t pg = pix_base + static_cast<int64_t>(gy) * W + gx;
                    a.log_frag[log_base + at] =
                        make_uint4(static_cast<uint32_t>(pg), tri, __float_as_uint(b1), __float_as_uint(b2));
                    constexpr int AW2 = aux_words(GW) / 2;
                    uint2* ax = a.log_aux + (log_base + at) * AW2;
                    ax[0] = make_uint2(static_cast<uint32_t>(key >> 32), static_cast<uint32_t>(v));
#pragma unroll
                    for (int w = 0; w < GW; w += 2) ax[1 + w / 2] = make_uint2(gates[w], w + 1 < GW ? gates[w + 1] : 0u);
                }
            }
        }
        if (a.log_frag) log_cursor += static_cast<uint32_t>(n);
        wave_fence();
        if (!S::kPaper && pass && L.key[pl] == key) {
            // the pixel's new best: its colour goes to the output now (a later batch that lowers
            // the key again writes after this one, behind the release fence that opens that
            // batch; the paper form shades its winners afterwards)
            const int blk = pl >> 6, p = pl & 63;
            const int64_t off = static_cast<int64_t>(ry + (blk / BR) * 8 + (p >> 3)) * W + rx + (blk % BR) * 8 + (p & 7);
            gfloat_w* col = color_base + 3 * off;
            col[0] = sigmoid_c(o[0]);
            col[1] = sigmoid_c(o[1]);
            col[2] = sigmoid_c(o[2]);
        }
        if (a.counter && lane == 0) atomicAdd(a.counter, static_cast<unsigned long long>(n));
        wave_fence();
        __builtin_amdgcn_s_setprio(1);
        wmax = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            wmaxb[b] = wave_max_u64(L.key[b * 64 + lane]);
            wmax = wmaxb[b] > wmax ? wmaxb[b] : wmax;
        }
    };

    const int64_t beg = a.tile_start[tile], end = a.tile_start[tile + 1];
    int64_t c0 = beg;         // next list entry to scan
    bool listed = false;      // the scan has reached the end of the list or its early-out
    constexpr int kRing = FwdWaveLds<NB>::kRing;
    int ph = 0;               // first waiting pair in the ring (L.ptri, L.pblk)
    int pn = 0;               // pairs waiting for the coverage step
    int qn = 0;               // queued candidates
    uint64_t cent = kBgKey;   // this lane's slice pair: list entry,
    int cblk = 0;             // ... block,
    uint32_t mlo = 0, mhi = 0;   // ... coverage of the block's pixels 0..31, 32..63,
    int cnt = 0, off = 0;     // ... number of covered pixels and the first of its combinations
    int n_comb = 0;           // covered (pair, pixel) combinations of the slice
    int rnd = 0, n_rnd = 0;   // rounds of 64 combinations: next, total
    // Decode when 64 candidates wait (or at the end), else take the next 64
    // covered (pair, pixel) combinations of the slice, else run coverage on the
    // next 64 waiting pairs, else scan the next 64 list entries.
    for (;;) {
        if (qn >= 64 || (rnd >= n_rnd && pn == 0 && listed)) {
            if (qn == 0) break;
            const int n = qn < 64 ? qn : 64;
            run_batch(n);
            // the rest moves to the front, less the candidates that a key this
            // batch set already beats (they were queued against the older keys
            // and would decode to nothing); the reads of each chunk precede its
            // writes, and a chunk writes only where it or the previous chunk has read
            int kept = 0;
            for (int i0 = n; i0 < qn; i0 += 64) {
                const int i = i0 + lane;
                uint64_t k = 0;
                float t0 = 0.f, t1 = 0.f, t2 = 0.f;
                uint16_t qp = 0;
                bool keep = false;
                if (i < qn) {
                    k = L.qkey[i];
                    t0 = L.qt[0][i];
                    t1 = L.qt[1][i];
                    t2 = L.qt[2][i];
                    qp = L.qpl[i];
                    keep = k < L.key[qp];
                }
                const uint64_t m = __ballot(keep);
                if (keep) {
                    const int pos = kept + __popcll(m & lanemask_lt());
                    L.qkey[pos] = k;
                    L.qt[0][pos] = t0;
                    L.qt[1][pos] = t1;
                    L.qt[2][pos] = t2;
                    L.qpl[pos] = qp;
                }
                kept += __popcll(m);
            }
            qn = kept;
            wave_fence();
            continue;
        }
        if (rnd < n_rnd) {
            __builtin_amdgcn_s_setprio(2);
            // ---- fragments of 64 covered (pair, pixel) combinations, in slice order:
            // lane = combination ----
            const int base = 64 * rnd;
            ++rnd;
            // the pair of a combination: the last pair whose run starts at or before it
            L.head[lane] = -1;
            wave_fence();
            if (cnt > 0 && off >= base && off < base + 64) L.head[off - base] = lane;
            wave_fence();
            const uint64_t before = __ballot(cnt > 0 && off < base);
            const int carry = before ? 63 - __builtin_clzll(before) : -1;
            const int h = wave_scan_dpp(L.head[lane], -1, [](int x, int y) { return x > y ? x : y; });
            const int c = base + lane;
            const bool valid = c < n_comb;
            const int j = valid ? (h > carry ? h : carry) : 0;
            // its pixel: the k-th covered pixel of the pair, k its rank in the pair's run
            const PairMeta mj = L.meta[j];
            const PairGeo gj = L.geo[j];
            const int p = select_bit(mj.mlo, mj.mhi, valid ? c - mj.off : 0);
            const int bj = mj.blk;
            const uint64_t zk = (static_cast<uint64_t>(mj.ent_hi) << 32) | mj.ent_lo;
            const uint64_t kp = L.key[bj * 64 + p];   // the pixel's best key as of the last decode batch
            const double px = static_cast<double>(p & 7), py = static_cast<double>(p >> 3);
            Frag f;
            double e[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {   // exact: every term is an integer below 2^51
                const double t = __builtin_fma(py, static_cast<double>(gj.ndx[i]), -(px * static_cast<double>(gj.ndy[i])));
                e[i] = __builtin_fma(static_cast<double>(kSnap), t, gj.e0[i]);
            }
            const float ra = gj.ra;
#pragma unroll
            for (int i = 0; i < 3; ++i) f.beta[i] = static_cast<float>(e[i]) * ra;
            float z = __builtin_fmaf(f.beta[2], gj.z[2], __builtin_fmaf(f.beta[1], gj.z[1], f.beta[0] * gj.z[0]));
            if (!(z > 0.0f)) z = 0.0f;
            if (z > 1.0f) z = 1.0f;
            f.key = (static_cast<uint64_t>(__float_as_uint(z)) << 32) | static_cast<uint32_t>(zk);
            const bool cand = valid & (zk < kp) & (f.key < kp);
            const uint64_t m = __ballot(cand);
            if (cand) {
                const int pos = qn + __popcll(m & lanemask_lt());
                L.qkey[pos] = f.key;
#pragma unroll
                for (int i = 0; i < 3; ++i) L.qt[i][pos] = f.beta[i] * gj.iw[i];
                L.qpl[pos] = static_cast<uint16_t>(bj * 64 + p);
            }
            qn += __popcll(m);
            continue;
        }
        if (pn >= 64 || (listed && pn > 0)) {
            __builtin_amdgcn_s_setprio(1);
            // ---- coverage of up to 64 waiting pairs: lane = (triangle, block) ----
            const int n = pn < 64 ? pn : 64;
            cent = kBgKey;
            int slot = ph + lane;
            if (slot >= kRing) slot -= kRing;
            cblk = lane < n ? static_cast<int>(L.pblk[slot]) : 0;
            mlo = 0;
            mhi = 0;
            uint4 q0, q1, q2, q3;
            if (lane < n) {
                const uint32_t tri = L.ptri[slot];
                guint4* rp = as_global(reinterpret_cast<const uint4*>(recs + tri));
                q0 = rp[0];
                q1 = rp[1];
                q2 = rp[2];
                q3 = rp[3];
                cent = (static_cast<uint64_t>(q3.y) << 32) | tri;   // the list entry: depth bound | triangle
            }
            if (cent < pick<NB>(wmaxb, cblk)) {   // still able to beat a pixel of the block (pads are kBgKey)
                const int32_t X[3] = {static_cast<int32_t>(q0.x), static_cast<int32_t>(q0.y), static_cast<int32_t>(q0.z)};
                const int32_t Y[3] = {static_cast<int32_t>(q0.w), static_cast<int32_t>(q1.x), static_cast<int32_t>(q1.y)};
                const float rA = __uint_as_float(q3.x);
                const int sgn = rA < 0.0f ? -1 : 1;
                // snapped position of the block's first pixel centre
                const int64_t PX0 = static_cast<int64_t>(kSnap) * (rx + (cblk % BR) * 8) + kSnap / 2;
                const int64_t PY0 = static_cast<int64_t>(kSnap) * (ry + (cblk / BR) * 8) + kSnap / 2;
                double e0[3], ea[3], eb[3], thr[3];
                int32_t nx[3], ny[3];
#pragma unroll
                for (int e = 0; e < 3; ++e) {   // edge e joins vertices e+1 and e+2
                    const int va = e == 2 ? 0 : e + 1;
                    const int vb = e == 0 ? 2 : (e == 1 ? 0 : 1);
                    const int32_t dx = X[vb] - X[va], dy = Y[vb] - Y[va];
                    const int64_t E0 =
                        static_cast<int64_t>(dx) * (PY0 - Y[va]) - static_cast<int64_t>(dy) * (PX0 - X[va]);
                    e0[e] = static_cast<double>(sgn * E0);
                    nx[e] = sgn * dx;
                    ny[e] = sgn * dy;
                    ea[e] = -static_cast<double>(kSnap) * static_cast<double>(ny[e]);
                    eb[e] = static_cast<double>(kSnap) * static_cast<double>(nx[e]);
                    // an edge owns the centres exactly on it when it is a top or left edge:
                    // E > 0, or E == 0 on an owning edge, is E > -1/2 for integer E
                    thr[e] = (ny[e] < 0 || (ny[e] == 0 && nx[e] > 0)) ? -0.5 : 0.0;
                }
                // a covered pixel whose best key is already at or below the
                // triangle's depth bound can take no fragment of it (keys only
                // fall), so it is left out of the mask here rather than
                // rejected one combination at a time later
                const uint64_t* __restrict__ kb = &L.key[cblk * 64];
#pragma unroll
                for (int pv2 = 0; pv2 < 8; ++pv2) {
                    double c[3];
#pragma unroll
                    for (int e = 0; e < 3; ++e) c[e] = __builtin_fma(static_cast<double>(pv2), eb[e], e0[e]);
                    uint32_t row = 0;
#pragma unroll
                    for (int pu2 = 0; pu2 < 8; ++pu2) {
                        bool in = cent < kb[pv2 * 8 + pu2];
#pragma unroll
                        for (int e = 0; e < 3; ++e)
                            in = in & (__builtin_fma(static_cast<double>(pu2), ea[e], c[e]) > thr[e]);
                        row |= in ? (1u << pu2) : 0u;
                    }
                    if (pv2 < 4) mlo |= row << (8 * pv2);
                    else mhi |= row << (8 * (pv2 - 4));
                }
                // A pixel left out of the mask already has a passing fragment; every
                // fragment of a pixel without one is in some mask, since the walk
                // then reaches the end of the list.
                if (a.counter && (mlo | mhi) != 0) {
                    atomicOr(&L.cov[2 * cblk], mlo);
                    atomicOr(&L.cov[2 * cblk + 1], mhi);
                }
                if ((mlo | mhi) != 0) {
                    PairGeo g;
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        g.e0[e] = e0[e];
                        g.ndx[e] = nx[e];
                        g.ndy[e] = ny[e];
                    }
                    g.z[0] = __uint_as_float(q1.z);
                    g.z[1] = __uint_as_float(q1.w);
                    g.z[2] = __uint_as_float(q2.x);
                    g.iw[0] = __uint_as_float(q2.y);
                    g.iw[1] = __uint_as_float(q2.z);
                    g.iw[2] = __uint_as_float(q2.w);
                    g.ra = __builtin_fabsf(rA);
                    g.pad = 0.0f;
                    L.geo[lane] = g;
                }
            }
            cnt = __popc(mlo) + __popc(mhi);
            const int incl = wave_incl_scan_i32(cnt);
            off = incl - cnt;
            L.meta[lane] = PairMeta{mlo, mhi, static_cast<uint32_t>(cent), static_cast<uint32_t>(cent >> 32), off, cblk};
            n_comb = __builtin_amdgcn_readlane(incl, 63);
            rnd = 0;
            n_rnd = (n_comb + 63) >> 6;
            ph += n;
            if (ph >= kRing) ph -= kRing;
            pn -= n;
            wave_fence();
            continue;
        }
        __builtin_amdgcn_s_setprio(2);
        // ---- scan the next 64 list entries: lane = entry ----
        if (c0 >= end || remaining_min(a.entries, beg, c0, end) >= wmax) {
            listed = true;
            continue;
        }
        const uint64_t e = c0 + lane < end ? a.entries[c0 + lane] : kBgKey;
        uint32_t touch = 0;   // blocks the entry's bounding box touches and whose pixels it can beat
        if (e < wmax) {
            const uint4 q3 = as_global(reinterpret_cast<const uint4*>(recs + static_cast<uint32_t>(e)))[3];
            const int x0 = static_cast<int16_t>(q3.z & 0xFFFFu), y0 = static_cast<int16_t>(q3.z >> 16);
            const int x1 = static_cast<int16_t>(q3.w & 0xFFFFu), y1 = static_cast<int16_t>(q3.w >> 16);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int bx = rx + (b % BR) * 8, by = ry + (b / BR) * 8;
                if (!(x1 < bx || x0 > bx + 7 || y1 < by || y0 > by + 7) && e < wmaxb[b]) touch |= 1u << b;
            }
        }
        const int cnt = __popc(touch);
        const int incl = wave_incl_scan_i32(cnt);
        int at = ph + pn + incl - cnt;   // below 2 kRing: pn < 64 and pn + 64 NB <= kRing
        if (at >= kRing) at -= kRing;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if ((touch >> b) & 1u) {
                L.ptri[at] = static_cast<uint32_t>(e);
                L.pblk[at] = static_cast<uint8_t>(b);
                if (++at == kRing) at = 0;
            }
        }
        pn += __builtin_amdgcn_readlane(incl, 63);
        c0 += 64;
        wave_fence();
    }
    // every read first, then the stores (a wait for a read issued between
    // stores would also wait for the stores)
    uint64_t okey[NB];
    int64_t ooff[NB];
    bool oin[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int gx = rx + (b % BR) * 8 + pu, gy = ry + (b / BR) * 8 + pv;
        oin[b] = gx < W && gy < H;
        ooff[b] = static_cast<int64_t>(gy) * W + gx;
        okey[b] = L.key[b * 64 + lane];
    }
    if (a.counter) {   // covered = a passing fragment, or a fragment in some coverage mask
        int n_cov = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint64_t won = __ballot(oin[b] && okey[b] != kBgKey);
            n_cov += __popcll(won | (static_cast<uint64_t>(L.cov[2 * b + 1]) << 32) | L.cov[2 * b]);
        }
        if (lane == 0 && n_cov) atomicAdd(a.counter + 8, static_cast<unsigned long long>(n_cov));
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (!oin[b]) continue;
        if (vis_base) vis_base[ooff[b]] = okey[b];
        if (!S::kPaper && okey[b] == kBgKey) {   // covered pixels got their colour when their best key was set
            gfloat_w* col = color_base + 3 * ooff[b];
            col[0] = a.o.bg[0];
            col[1] = a.o.bg[1];
            col[2] = a.o.bg[2];
        }
    }
    wave_fence();
    }   // regions
    if (a.log_counts && lane == 0) a.log_counts[blockIdx.x] = log_cursor;
}

// Resident waves per CU of the forward (its workgroups are single waves).
template <int TS, int RS, class S>
static int fwd_blocks_per_cu_r() {
    static int n = 0;
    if (n == 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, raster_fwd_kernel<TS, RS, S>, 64, 0) != hipSuccess || b < 1)
            b = 8;
        n = b;
    }
    return n;
}

template <int TS, class S>
static int fwd_blocks_per_cu(int region) {
    if constexpr (TS >= 16) {
        if (region == 16) return fwd_blocks_per_cu_r<TS, 16, S>();
    }
    return fwd_blocks_per_cu_r<TS, 8, S>();
}

template <int TS, class S>
static void launch_fwd_t(const RasterArgs& a, hipStream_t s) {
    if (a.n_tiles <= 0 || a.n_blocks <= 0) return;
    if constexpr (TS >= 16) {
        if (a.region == 16) {
            hipLaunchKernelGGL((raster_fwd_kernel<TS, 16, S>), dim3(static_cast<unsigned>(a.n_blocks)), dim3(64), 0,
                               s, a);
            return;
        }
    }
    hipLaunchKernelGGL((raster_fwd_kernel<TS, 8, S>), dim3(static_cast<unsigned>(a.n_blocks)), dim3(64), 0, s, a);
}


}  // namespace soup
