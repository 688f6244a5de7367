// Shared device-side definitions of the gfx950 soup rasterizer: descriptors,
// the float32 arithmetic contract (transform, snap, depth, barycentrics,
// feature fetch, MLP, sigmoid, Philox draw) and small wave helpers.
//
// The contract fixes one float32 operation sequence for everything that
// decides visibility, so that the mask decision u < alpha is reproducible bit
// for bit: explicit fused multiply-adds, no other contraction
// (-ffp-contract=off), correctly rounded division, denormals kept, and an
// exp of our own (Cody-Waite reduction + degree-7 Taylor polynomial).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace soup {

constexpr int kSnap = 256;                          // subpixel steps per pixel
constexpr float kGuard = 16777216.0f;               // |snapped coordinate| < 2^24
constexpr uint64_t kBgKey = 0xFFFFFFFFFFFFFFFFull;  // "no fragment passed"
constexpr uint32_t kZminMargin = 64;                // ulps subtracted from a triangle's min depth
constexpr int kSortBlock = 2048;                    // per-tile lists are sorted in blocks of this size
constexpr int kMaxViews = 1 << 16;

// Address-space qualified pointers: constant (scalar loads of wave-uniform
// data such as the MLP weights) and global (vector loads of per-lane data).
// (The host pass only parses device code; it sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
using cfloat = const float __attribute__((address_space(4)));
using gfloat = const float __attribute__((address_space(1)));
using gfloat4 = const float4 __attribute__((address_space(1)));
using guint4 = const uint4 __attribute__((address_space(1)));
using gfloat_w = float __attribute__((address_space(1)));
using guint64_w = uint64_t __attribute__((address_space(1)));
#else
using cfloat = const float;
using gfloat = const float;
using gfloat4 = const float4;
using guint4 = const uint4;
using gfloat_w = float;
using guint64_w = uint64_t;
#endif

__device__ __forceinline__ cfloat* as_const(const float* p) {
    return reinterpret_cast<cfloat*>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ gfloat* as_global(const float* p) {
    return reinterpret_cast<gfloat*>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ guint4* as_global(const uint4* p) {
    return reinterpret_cast<guint4*>(reinterpret_cast<uintptr_t>(p));
}
// writable global pointers: stores through them are global stores, not flat
// ones (which also count as LDS operations in the wait counters)
__device__ __forceinline__ gfloat_w* as_global_w(float* p) {
    return reinterpret_cast<gfloat_w*>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ guint64_w* as_global_w(uint64_t* p) {
    return reinterpret_cast<guint64_w*>(reinterpret_cast<uintptr_t>(p));
}

// Per-view descriptor (device copy built by the host for every call).
// MI355X has eight XCDs, each with its own L2; consecutive workgroups of a
// launch go to them in turn.
constexpr int kXcds = 8;

struct ViewDesc {
    float M[16];             // view-projection, row-major
    int32_t W, H;
    uint32_t view_id;
    int32_t scene;           // index into the scene descriptors
    int32_t tiles_x, tiles_y;
    int32_t T;               // triangles of this view's scene
    int32_t pad0;
    int64_t tile_base;       // first global tile of this view
    int64_t pix_base;        // first pixel of this view in the output buffers
    int64_t rec_base;        // record index of (this view, triangle 0)
    float* color_out;        // per-request colour buffer (render) or nullptr
    uint64_t* vis_out;       // per-request visibility buffer or nullptr
    float Mi[16];            // inverse view-projection (the paper form's view directions), else zero
};

struct SceneDesc {
    const float* verts;
    const float* feats;
    const float* mlp;
    int32_t T;
    int32_t pad0;
};

// Per (view, triangle) setup record, 64 bytes.
struct __align__(16) TriRec {
    int32_t X[3], Y[3];      // snapped screen positions, 1/256 px, y down
    float z01[3];            // depth in [0,1] at the vertices (unclamped)
    float iw[3];             // 1 / clip w
    float rA;                // +-1 / |2 x area| (1/256^2 px^2); the sign is the orientation
    uint32_t zmin;           // lower bound of the depth bits of any fragment
    int16_t x0, y0, x1, y1;  // inclusive pixel bounding box in the view (x0 > x1: culled)
};
static_assert(sizeof(TriRec) == 64, "TriRec must be 64 bytes");

struct Opts {
    uint64_t seed;
    uint32_t step;
    int32_t mode;            // 0 stochastic, 1 threshold
    float bg[3];
    int32_t edge_pairs;
    float near_w;
    int32_t accumulate;
    int32_t reuse_bins;
};

// --------------------------------------------------------------------------
// float32 contract
// --------------------------------------------------------------------------

// exp(x): x = n ln2 + r with ln2 split into a 17-significant-bit head (so the
// product n * head is exact) and a float tail; e^r by the Taylor polynomial
// of degree 7 in Horner form; times 2^n assembled from exponent bits.
__device__ __forceinline__ float exp_c(float x) {
    const float kLog2e = 0x1.715476p+0f;
    const float kLn2Hi = 0x1.62e4p-1f;
    const float kLn2Lo = 0x1.7f7d1cp-20f;
    if (x != x) return x;
    if (x > 88.0f) return __builtin_huge_valf();
    if (x < -87.0f) return 0.0f;
    const float n = __builtin_rintf(x * kLog2e);
    float r = __builtin_fmaf(-n, kLn2Hi, x);
    r = __builtin_fmaf(-n, kLn2Lo, r);
    float p = 1.0f / 5040.0f;
    p = __builtin_fmaf(p, r, 1.0f / 720.0f);
    p = __builtin_fmaf(p, r, 1.0f / 120.0f);
    p = __builtin_fmaf(p, r, 1.0f / 24.0f);
    p = __builtin_fmaf(p, r, 1.0f / 6.0f);
    p = __builtin_fmaf(p, r, 0.5f);
    p = __builtin_fmaf(p, r, 1.0f);
    p = __builtin_fmaf(p, r, 1.0f);
    const float scale = __uint_as_float(static_cast<uint32_t>(static_cast<int32_t>(n) + 127) << 23);
    return p * scale;
}

__device__ __forceinline__ float sigmoid_c(float x) { return 1.0f / (1.0f + exp_c(-x)); }

// Philox4x32-10 (Salmon et al., SC'11). Counter (pixel, tri, view, step),
// key (seed lo, seed hi); returns the first output word.
__device__ __forceinline__ uint32_t philox_x0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return c0;
}

// 24-bit uniform in [0, 1 - 2^-24] of the fragment (pixel, tri) of a view.
__device__ __forceinline__ float uniform24(uint64_t seed, uint32_t pixel, uint32_t tri,
                                           uint32_t view_id, uint32_t step) {
    const uint32_t r = philox_x0(pixel, tri, view_id, step, static_cast<uint32_t>(seed),
                                 static_cast<uint32_t>(seed >> 32));
    return static_cast<float>(r >> 8) * 0x1p-24f;
}

// Shape of the shared MLP: C inputs, NH hidden layers of width H, 4 outputs.
template <int C_, int H_, int NH_>
struct MlpShape {
    static constexpr bool kPaper = false;   // the paper form's raster policy sets it
    static constexpr int C = C_;
    static constexpr int H = H_;
    static constexpr int NH = NH_;
    static constexpr int kParams = C * H + H + (NH - 1) * (H * H + H) + 4 * H + 4;
    // offsets of layer l's weights and biases in the flat parameter array
    __host__ __device__ static constexpr int w_off(int l) {
        return l == 0 ? 0 : C * H + H + (l - 1) * (H * H + H);
    }
    __host__ __device__ static constexpr int din(int l) { return l == 0 ? C : H; }
    __host__ __device__ static constexpr int dout(int l) { return l == NH ? 4 : H; }
    __host__ __device__ static constexpr int b_off(int l) { return w_off(l) + dout(l) * din(l); }
};

// Orders one wave's LDS accesses for the compiler only: a wave's LDS
// operations execute in issue order, so a lane's read sees another lane's
// earlier write of the same wave without a wait.
__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Texture position of perspective-correct barycentrics (b1, b2) on a G x G
// grid: vertex 0 -> (0,0), vertex 1 -> (G-1,0), vertex 2 -> (0,G-1).

struct Cell {
    int ix, iy;
    float fx, fy;
};

__device__ __forceinline__ Cell cell_of(float b1, float b2, int G) {
    const float gm1 = static_cast<float>(G - 1);
    const float gx = b1 * gm1, gy = b2 * gm1;
    int ix = static_cast<int>(__builtin_floorf(gx));
    int iy = static_cast<int>(__builtin_floorf(gy));
    ix = ix < 0 ? 0 : (ix > G - 2 ? G - 2 : ix);
    iy = iy < 0 ? 0 : (iy > G - 2 ? G - 2 : iy);
    Cell c;
    c.ix = ix;
    c.iy = iy;
    c.fx = gx - static_cast<float>(ix);
    c.fy = gy - static_cast<float>(iy);
    return c;
}

// Bilinear fetch of the C-channel feature at a cell position.
template <int C>
__device__ __forceinline__ void fetch_feature(gfloat* __restrict__ feats, uint32_t tri, int G,
                                              const Cell& c, float (&x)[C]) {
    gfloat* t00 = feats + ((static_cast<size_t>(tri) * G + c.iy) * G + c.ix) * C;
    gfloat* t10 = t00 + C;
    gfloat* t01 = t00 + static_cast<size_t>(G) * C;
    gfloat* t11 = t01 + C;
    const float w00 = (1.0f - c.fx) * (1.0f - c.fy);
    const float w10 = c.fx * (1.0f - c.fy);
    const float w01 = (1.0f - c.fx) * c.fy;
    const float w11 = c.fx * c.fy;
#pragma unroll
    for (int k = 0; k < C; k += 4) {
        const float4 a = *reinterpret_cast<gfloat4*>(t00 + k);
        const float4 b = *reinterpret_cast<gfloat4*>(t10 + k);
        const float4 d = *reinterpret_cast<gfloat4*>(t01 + k);
        const float4 e = *reinterpret_cast<gfloat4*>(t11 + k);
        x[k + 0] = __builtin_fmaf(w11, e.x, __builtin_fmaf(w01, d.x, __builtin_fmaf(w10, b.x, w00 * a.x)));
        x[k + 1] = __builtin_fmaf(w11, e.y, __builtin_fmaf(w01, d.y, __builtin_fmaf(w10, b.y, w00 * a.y)));
        x[k + 2] = __builtin_fmaf(w11, e.z, __builtin_fmaf(w01, d.z, __builtin_fmaf(w10, b.z, w00 * a.z)));
        x[k + 3] = __builtin_fmaf(w11, e.w, __builtin_fmaf(w01, d.w, __builtin_fmaf(w10, b.w, w00 * a.w)));
    }
}

// One dense layer: out_j = b_j + sum_k W[j][k] in_k (k ascending, one FMA each),
// ReLU on hidden layers. W and b are wave-uniform (scalar loads).
template <int DIN, int DOUT, bool RELU>
__device__ __forceinline__ void dense(cfloat* __restrict__ W, cfloat* __restrict__ b,
                                      const float (&in)[DIN], float (&out)[DOUT]) {
#pragma unroll
    for (int j = 0; j < DOUT; ++j) {
        float acc = b[j];
#pragma unroll
        for (int k = 0; k < DIN; ++k) acc = __builtin_fmaf(W[j * DIN + k], in[k], acc);
        out[j] = RELU ? (acc > 0.0f ? acc : 0.0f) : acc;
    }
}

// Forward of the shared MLP; keeps every hidden activation for a backward.
template <class S>
struct MlpAct {
    float h[S::NH][S::H];
    float o[4];
};

template <class S>
__device__ __forceinline__ void mlp_forward(cfloat* __restrict__ p, const float (&x)[S::C],
                                            MlpAct<S>& a) {
    dense<S::C, S::H, true>(p + S::w_off(0), p + S::b_off(0), x, a.h[0]);
#pragma unroll
    for (int l = 1; l < S::NH; ++l)
        dense<S::H, S::H, true>(p + S::w_off(l), p + S::b_off(l), a.h[l - 1], a.h[l]);
    dense<S::H, 4, false>(p + S::w_off(S::NH), p + S::b_off(S::NH), a.h[S::NH - 1], a.o);
}

// Words of ReLU gate bits per decoded fragment: bit l * H + k is set when
// hidden unit k of layer l is positive (the ReLU passes it).
template <class S>
struct GateWords {
    static constexpr int kWords = (S::NH * S::H + 31) / 32;
};

// One dense hidden layer as `dense`, then gate bit (base + j) of `gates` set
// for every positive unit j (read off the layer's output, which is positive
// exactly where the ReLU passes).
template <int DIN, int DOUT, int NW>
__device__ __forceinline__ void dense_relu_gates(cfloat* __restrict__ W, cfloat* __restrict__ b,
                                                 const float (&in)[DIN], float (&out)[DOUT], int base,
                                                 uint32_t (&gates)[NW]) {
    dense<DIN, DOUT, true>(W, b, in, out);
    // out[j] is +0 or positive: its bit pattern is nonzero exactly when the gate is open
#pragma unroll
    for (int j = 0; j < DOUT; ++j)
        gates[(base + j) >> 5] |= min(__float_as_uint(out[j]), 1u) << ((base + j) & 31);
}

// mlp_logits that also returns the hidden units' ReLU gates (same arithmetic).
template <class S>
__device__ __forceinline__ void mlp_logits_gates(cfloat* __restrict__ p, const float (&x)[S::C], float (&o)[4],
                                                 uint32_t (&gates)[GateWords<S>::kWords]) {
#pragma unroll
    for (int w = 0; w < GateWords<S>::kWords; ++w) gates[w] = 0u;
    float h[S::H];
    dense_relu_gates<S::C, S::H>(p + S::w_off(0), p + S::b_off(0), x, h, 0, gates);
#pragma unroll
    for (int l = 1; l < S::NH; ++l) {
        float h2[S::H];
        dense_relu_gates<S::H, S::H>(p + S::w_off(l), p + S::b_off(l), h, h2, l * S::H, gates);
#pragma unroll
        for (int k = 0; k < S::H; ++k) h[k] = h2[k];
    }
    dense<S::H, 4, false>(p + S::w_off(S::NH), p + S::b_off(S::NH), h, o);
}

// Lightweight forward (no stored activations beyond one hidden layer).
template <class S>
__device__ __forceinline__ void mlp_logits(cfloat* __restrict__ p, const float (&x)[S::C],
                                           float (&o)[4]) {
    float h[S::H];
    dense<S::C, S::H, true>(p + S::w_off(0), p + S::b_off(0), x, h);
#pragma unroll
    for (int l = 1; l < S::NH; ++l) {
        float h2[S::H];
        dense<S::H, S::H, true>(p + S::w_off(l), p + S::b_off(l), h, h2);
#pragma unroll
        for (int k = 0; k < S::H; ++k) h[k] = h2[k];
    }
    dense<S::H, 4, false>(p + S::w_off(S::NH), p + S::b_off(S::NH), h, o);
}

// --------------------------------------------------------------------------
// wave helpers (wave64)
// --------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Values the compiler cannot prove wave-uniform (read from LDS, say) are made
// uniform explicitly so that address arithmetic and weight loads stay scalar.
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x)));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x >> 32)));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    return reinterpret_cast<T*>(uniform_i64(reinterpret_cast<int64_t>(p)));
}

// A wave-uniform pointer whose value the compiler cannot see through: loads
// from it can neither be hoisted above this point nor merged with loads
// through another copy.
template <class T>
__device__ __forceinline__ T* opaque_ptr(T* p) {
    uint64_t v = reinterpret_cast<uint64_t>(p);
    asm volatile("" : "+s"(v));
    return reinterpret_cast<T*>(v);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Binary search: index v with base[v] <= x < base[v+1] over V entries.
template <class T>
__device__ __forceinline__ int find_segment(const ViewDesc* __restrict__ views, int V, int64_t x,
                                            T ViewDesc::*field) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].*field <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace soup
