// Tile-raster building blocks shared by the forward and backward kernels:
// the LDS chunk of triangle records of one tile and the exact coverage test.
//
// Edge functions are evaluated in float64. Every operand is an integer below
// 2^51 (snapped coordinates are bounded by 2^24, so products of differences
// are below 2^50), so each value, including the incremental form
// E(x, y) = E(x0, y0) + dx * a + dy * b, is exact and equals the int64 edge
// function of the contract; the tie rule and the conversion to float for the
// barycentrics therefore match it bit for bit.
#pragma once

#include "internal.hpp"

namespace soup {

template <int TS>
struct TileCfg {
    static constexpr int NT = TS * TS >= 256 ? 256 : TS * TS;   // threads per workgroup
    static constexpr int PPT = TS * TS / NT;                    // pixels per thread
    static constexpr int NW = NT / 64;                          // waves
    static_assert(NT % 64 == 0, "tile must hold a multiple of 64 pixels");
};

// Tile-local pixel of index pl: 8x8 blocks in row-major block order, row-major
// inside a block, so each wave (64 consecutive indices) owns one 8x8 block and
// can skip a triangle whose bounding box misses it with one uniform branch.
template <int TS>
__device__ __forceinline__ int px_of(int pl) {
    return ((pl >> 6) % (TS / 8)) * 8 + (pl & 7);
}
template <int TS>
__device__ __forceinline__ int py_of(int pl) {
    return ((pl >> 6) / (TS / 8)) * 8 + ((pl & 63) >> 3);
}

// Does chunk slot j's bounding box touch the 8x8 block b of the tile?
template <int TS>
__device__ __forceinline__ bool box_hits_block(uint32_t box, int b) {
    const int bx0 = (b % (TS / 8)) * 8, by0 = (b / (TS / 8)) * 8;
    return !(static_cast<int>((box >> 16) & 255u) < bx0 || static_cast<int>(box & 255u) > bx0 + 7 ||
             static_cast<int>(box >> 24) < by0 || static_cast<int>((box >> 8) & 255u) > by0 + 7);
}

template <int NT>
struct ChunkLds {
    double e0[3][NT];        // orientation-normalised edge functions at the tile's first pixel centre
    double ea[3][NT];        // ... step per pixel in x
    double eb[3][NT];        // ... step per pixel in y
    float z[3][NT];
    float iw[3][NT];
    float ra[NT];            // 1 / |2 x area|
    uint32_t tri[NT];
    uint32_t zmin[NT];
    uint32_t own[NT];        // bit i: edge i owns centres exactly on it
    uint32_t box[NT];        // tile-local bbox x0 | y0 << 8 | x1 << 16 | y1 << 24
};

// Fill slot i of the chunk from a sorted tile entry.
template <int NT, int TS>
__device__ __forceinline__ void load_slot(ChunkLds<NT>& ch, int i, uint64_t entry, const TriRec& r, int tx0,
                                          int ty0) {
    const uint32_t tri = static_cast<uint32_t>(entry);
    ch.tri[i] = tri;
    ch.zmin[i] = static_cast<uint32_t>(entry >> 32);
    const int bx0 = max(r.x0 - tx0, 0), bx1 = min(r.x1 - tx0, TS - 1);
    const int by0 = max(r.y0 - ty0, 0), by1 = min(r.y1 - ty0, TS - 1);
    ch.box[i] = static_cast<uint32_t>(bx0) | (static_cast<uint32_t>(by0) << 8) | (static_cast<uint32_t>(bx1) << 16) |
                (static_cast<uint32_t>(by1) << 24);
    const int sgn = r.rA < 0.0f ? -1 : 1;
    const int64_t PX0 = static_cast<int64_t>(kSnap) * tx0 + kSnap / 2;
    const int64_t PY0 = static_cast<int64_t>(kSnap) * ty0 + kSnap / 2;
    uint32_t own = 0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int a = e == 2 ? 0 : e + 1;
        const int b = e == 0 ? 2 : (e == 1 ? 0 : 1);
        const int32_t dx = r.X[b] - r.X[a], dy = r.Y[b] - r.Y[a];
        const int64_t E0 = static_cast<int64_t>(dx) * (PY0 - r.Y[a]) - static_cast<int64_t>(dy) * (PX0 - r.X[a]);
        ch.e0[e][i] = static_cast<double>(sgn * E0);
        ch.ea[e][i] = static_cast<double>(-static_cast<int64_t>(sgn) * kSnap * dy);
        ch.eb[e][i] = static_cast<double>(static_cast<int64_t>(sgn) * kSnap * dx);
        const int32_t ndx = sgn * dx, ndy = sgn * dy;
        if (ndy < 0 || (ndy == 0 && ndx > 0)) own |= 1u << e;
        ch.z[e][i] = r.z01[e];
        ch.iw[e][i] = r.iw[e];
    }
    ch.own[i] = own;
    ch.ra[i] = __builtin_fabsf(r.rA);
}

// Exact inside test of tile-local pixel (lx, ly) against chunk slot j: the
// orientation-normalised edge values are left in e, and the pixel is inside
// when every E_i > 0, or E_i == 0 on an edge that owns the centres on it.
// Every operand is read up front and the test has no branches, so a wave
// pays one round of LDS latency per triangle.
template <int NT>
__device__ __forceinline__ bool edge_inside(const ChunkLds<NT>& ch, int j, int lx, int ly, double (&e)[3]) {
    const double dx = static_cast<double>(lx), dy = static_cast<double>(ly);
    const uint32_t own = ch.own[j];
    double e0[3], ea[3], eb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        e0[i] = ch.e0[i][j];
        ea[i] = ch.ea[i][j];
        eb[i] = ch.eb[i][j];
    }
    bool in = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        e[i] = __builtin_fma(dx, ea[i], __builtin_fma(dy, eb[i], e0[i]));
        in = in & ((e[i] > 0.0) | ((e[i] == 0.0) & (((own >> i) & 1u) != 0u)));
    }
    return in;
}

struct Frag {
    uint64_t key;
    float beta[3];
};

// Screen barycentrics and key of a covering fragment from its edge values
// (contract: beta_i = (float)E_i * (1 / (float)A); depth = sum beta_i z_i in
// the stated fma order, clamped to [+0, 1]; key = depth bits << 32 | tri).
template <int NT>
__device__ __forceinline__ void frag_of(const ChunkLds<NT>& ch, int j, const double (&e)[3], Frag& f) {
    const float ra = ch.ra[j];
#pragma unroll
    for (int i = 0; i < 3; ++i) f.beta[i] = static_cast<float>(e[i]) * ra;
    float z = __builtin_fmaf(f.beta[2], ch.z[2][j], __builtin_fmaf(f.beta[1], ch.z[1][j], f.beta[0] * ch.z[0][j]));
    if (!(z > 0.0f)) z = 0.0f;
    if (z > 1.0f) z = 1.0f;
    f.key = (static_cast<uint64_t>(__float_as_uint(z)) << 32) | ch.tri[j];
}

// Perspective-correct barycentrics of vertices 1 and 2 from t_i = beta_i / w_i
// (contract order: r = 1 / ((t0 + t1) + t2), b_i = t_i r).
__device__ __forceinline__ void persp_from_t(float t0, float t1, float t2, float& b1, float& b2) {
    const float r = 1.0f / ((t0 + t1) + t2);
    b1 = t1 * r;
    b2 = t2 * r;
}

// Inclusive scans over the wave on the data-parallel primitives (DPP), with no
// LDS round trip: shifted moves by 1, 2, 4 and 8 lanes within each row of 16
// (a lane with no source in its row keeps its value), then the broadcasts of
// lane 15 into rows 1 and 3 and of lane 31 into rows 2 and 3 (the GFX9
// wave64 controls: row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143).
template <int CTRL, int ROWS, class Op>
__device__ __forceinline__ int dpp_step(int v, int identity, Op op) {
    return op(v, __builtin_amdgcn_update_dpp(identity, v, CTRL, ROWS, 0xF, false));
}
template <class Op>
__device__ __forceinline__ int wave_scan_dpp(int v, int identity, Op op) {
    v = dpp_step<0x111, 0xF>(v, identity, op);
    v = dpp_step<0x112, 0xF>(v, identity, op);
    v = dpp_step<0x114, 0xF>(v, identity, op);
    v = dpp_step<0x118, 0xF>(v, identity, op);
    v = dpp_step<0x142, 0xA>(v, identity, op);
    return dpp_step<0x143, 0xC>(v, identity, op);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_max_step_u64(uint64_t v) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROWS, 0xF, false));
    const uint32_t hi =
        static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v >> 32), CTRL, ROWS, 0xF, false));
    const uint64_t u = (static_cast<uint64_t>(hi) << 32) | lo;
    return u > v ? u : v;
}

// The largest value over the wave (wave-uniform).
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    v = dpp_max_step_u64<0x111, 0xF>(v);
    v = dpp_max_step_u64<0x112, 0xF>(v);
    v = dpp_max_step_u64<0x114, 0xF>(v);
    v = dpp_max_step_u64<0x118, 0xF>(v);
    v = dpp_max_step_u64<0x142, 0xA>(v);
    v = dpp_max_step_u64<0x143, 0xC>(v);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), 63));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Smallest key any not-yet-processed entry of the tile list can produce.
// Lists are sorted in blocks of kSortBlock, so it is the minimum over the
// current position and the first entry of every later block.
__device__ __forceinline__ uint64_t remaining_min(const uint64_t* __restrict__ entries, int64_t beg, int64_t pos,
                                                  int64_t end) {
    uint64_t m = entries[pos];
    for (int64_t b = beg + ((pos - beg) / kSortBlock + 1) * kSortBlock; b < end; b += kSortBlock) {
        const uint64_t e = entries[b];
        m = e < m ? e : m;
    }
    return m;
}

// View that owns global tile `tile` (views sorted by tile_base).
__device__ __forceinline__ int view_of_tile(const ViewDesc* __restrict__ views, int V, int64_t tile) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace soup
