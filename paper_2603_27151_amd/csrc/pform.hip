// Paper form of the step (Section 3.3; Supplement B.3, B.6): kernels besides
// the forward raster (which takes the opacity-only policy PaperTex).
//
//  assemble      sigmoid(sum of the learnable levels sampled at the finest
//                grid's vertices), one workgroup per triangle, and its
//                gradient summed per triangle in LDS;
//  shade         the deferred colour of every pixel's winner: features of its
//                micro-triangle, harmonics of the view direction, the MLP on
//                the vector ALUs in the float32 contract, the RGBA blend;
//  frag          over a fragment list (the forward's log filtered, or a
//                replay): the score term of Eq. (9) on the opacity channel, or
//                log p(f*) of Eq. (6);
//  winner_bwd    per pixel: the colour path of the winner (the MLP's data
//                backward on the vector ALUs; its weight gradient, a
//                contraction over pixels, on the matrix cores), the features'
//                gradient onto the three grid vertices, and the vertex
//                gradient through the barycentrics and the edge term in
//                float64.
#include "decode_mfma.hpp"
#include "pform.hpp"

namespace soup {

// ---------------------------------------------------------------------------
// texture assembly
// ---------------------------------------------------------------------------

// (i, j) of the finest grid's vertex k (row-major storage): row j starts at
// j (n + 1) - j (j - 1) / 2; the float estimate of j is corrected exactly.
__device__ __forceinline__ void mc_ij(int n, int k, int& i, int& j) {
    const float b = static_cast<float>(2 * n + 3);
    int jj = static_cast<int>((b - __builtin_sqrtf(b * b - 8.0f * static_cast<float>(k))) * 0.5f);
    jj = jj < 0 ? 0 : (jj > n ? n : jj);
    while (jj > 0 && mc_index(n, 0, jj) > k) --jj;
    while (jj < n && mc_index(n, 0, jj + 1) <= k) ++jj;
    j = jj;
    i = k - mc_index(n, 0, jj);
}

// Fallback for levels too large to stage in LDS: one thread per (triangle,
// vertex of the finest grid), consecutive threads on consecutive vertices
// (32-byte records, written coalesced), the three grid vertices of every
// level gathered from global memory.
__global__ __launch_bounds__(256) void mc_assemble_kernel(AssembleArgs a) {
    const int nf = 1 << a.Rmax, Vf = mc_count(a.Rmax);
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= static_cast<int64_t>(a.T) * Vf) return;
    const int t = static_cast<int>(g / Vf);
    const int k = static_cast<int>(g - static_cast<int64_t>(t) * Vf);
    float* out = a.tex_out + static_cast<size_t>(t) * Vf * kPCh;
    {
        int i, j;
        mc_ij(nf, k, i, j);
        // i / n and j / n (n a power of two: the product by 1 / n is exact)
        const float b1 = static_cast<float>(i) * (1.0f / static_cast<float>(nf));
        const float b2 = static_cast<float>(j) * (1.0f / static_cast<float>(nf));
        float z[kPCh];
#pragma unroll
        for (int c = 0; c < kPCh; ++c) z[c] = 0.0f;
        for (int R = a.Rmin; R <= a.Rtop; ++R) {
            const Micro m = micro_of(1 << R, b1, b2);
            const float4* g = reinterpret_cast<const float4*>(a.raw[R - a.Rmin] + static_cast<size_t>(t) * mc_count(R) * kPCh);
            float4 v[3][2];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                v[q][0] = g[2 * m.idx[q]];
                v[q][1] = g[2 * m.idx[q] + 1];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                z[4 * h + 0] = z[4 * h + 0] + mc_mix(m, v[0][h].x, v[1][h].x, v[2][h].x);
                z[4 * h + 1] = z[4 * h + 1] + mc_mix(m, v[0][h].y, v[1][h].y, v[2][h].y);
                z[4 * h + 2] = z[4 * h + 2] + mc_mix(m, v[0][h].z, v[1][h].z, v[2][h].z);
                z[4 * h + 3] = z[4 * h + 3] + mc_mix(m, v[0][h].w, v[1][h].w, v[2][h].w);
            }
        }
        float4* o = reinterpret_cast<float4*>(out + static_cast<size_t>(k) * kPCh);
        o[0] = make_float4(sigmoid_c(z[0]), sigmoid_c(z[1]), sigmoid_c(z[2]), sigmoid_c(z[3]));
        o[1] = make_float4(sigmoid_c(z[4]), sigmoid_c(z[5]), sigmoid_c(z[6]), sigmoid_c(z[7]));
    }
}

// TPB consecutive triangles per workgroup: their learnable levels (contiguous
// per level in global memory) are staged in LDS with coalesced 16-byte loads;
// then each thread takes one (finest-grid vertex, half of the channels) for
// all TPB triangles, so the vertex's micro-triangle lookups, which do not
// depend on the triangle, are computed once. Same arithmetic, in the same
// order, as the fallback: the results are identical.
template <int TPB>
__global__ __launch_bounds__(256) void mc_assemble_lds_kernel(AssembleArgs a) {
    extern __shared__ float4 st4[];
    const int t0 = blockIdx.x * TPB;
    const int nt = a.T - t0 < TPB ? a.T - t0 : TPB;
    {
        int off = 0;   // float4 offset of level R's block of TPB triangles
        for (int R = a.Rmin; R <= a.Rtop; ++R) {
            const int v2 = mc_count(R) * 2;
            const float4* src = reinterpret_cast<const float4*>(a.raw[R - a.Rmin]) + static_cast<size_t>(t0) * v2;
            for (int e = threadIdx.x; e < nt * v2; e += blockDim.x) st4[off + e] = src[e];
            off += TPB * v2;
        }
    }
    __syncthreads();
    const int nf = 1 << a.Rmax, Vf = mc_count(a.Rmax);
    for (int e = threadIdx.x; e < 2 * Vf; e += blockDim.x) {
        const int k = e >> 1, h = e & 1;
        int i, j;
        mc_ij(nf, k, i, j);
        const float b1 = static_cast<float>(i) * (1.0f / static_cast<float>(nf));
        const float b2 = static_cast<float>(j) * (1.0f / static_cast<float>(nf));
        float4 z[TPB];
#pragma unroll
        for (int tt = 0; tt < TPB; ++tt) z[tt] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        int off = 0;
        for (int R = a.Rmin; R <= a.Rtop; ++R) {
            const Micro m = micro_of(1 << R, b1, b2);
            const int v2 = mc_count(R) * 2;
#pragma unroll
            for (int tt = 0; tt < TPB; ++tt) {   // rows past nt hold stale LDS; their results are not stored
                const float4* g = st4 + off + tt * v2 + h;
                const float4 v0 = g[2 * m.idx[0]], v1 = g[2 * m.idx[1]], v2v = g[2 * m.idx[2]];
                z[tt].x = z[tt].x + mc_mix(m, v0.x, v1.x, v2v.x);
                z[tt].y = z[tt].y + mc_mix(m, v0.y, v1.y, v2v.y);
                z[tt].z = z[tt].z + mc_mix(m, v0.z, v1.z, v2v.z);
                z[tt].w = z[tt].w + mc_mix(m, v0.w, v1.w, v2v.w);
            }
            off += TPB * v2;
        }
#pragma unroll
        for (int tt = 0; tt < TPB; ++tt) {
            if (tt < nt) {
                float4* o = reinterpret_cast<float4*>(a.tex_out) + static_cast<size_t>(t0 + tt) * Vf * 2 + e;
                *o = make_float4(sigmoid_c(z[tt].x), sigmoid_c(z[tt].y), sigmoid_c(z[tt].z), sigmoid_c(z[tt].w));
            }
        }
    }
}

// Bytes of the learnable levels of one triangle.
static size_t mc_levels_bytes(int Rmin, int Rtop) {
    size_t b = 0;
    for (int R = Rmin; R <= Rtop; ++R) b += static_cast<size_t>(mc_count(R)) * kPCh * sizeof(float);
    return b;
}

// Gradient of the assembly. The lookup of level R at the vertices of level
// Rmax equals prolongation to level R + 1, then R + 2, ..., Rmax (the field of
// a level is linear on each of its micro-triangles, and every micro-triangle
// of the next level lies inside one of them; a vertex of level R + 1 is a
// vertex of level R, weight 1, or the midpoint of an edge, weights 1/2). Its
// transpose is the restriction chain: with dz = tex (1 - tex) d tex on level
// Rmax, g_R(I, J) = g_{R+1}(2I, 2J) + 1/2 sum over the six lattice neighbours
// (2I, 2J) + d, d in +-(1, 0), +-(0, 1), +-(1, -1), that exist. One workgroup
// per triangle keeps the chain in LDS (two buffers of the largest level) and
// writes every learnable level; without room for them the adds go to global
// memory directly, one lookup per level and vertex.
template <bool LDS_SUM>
__global__ __launch_bounds__(256) void mc_assemble_bwd_kernel(AssembleArgs a) {
    extern __shared__ float lds[];
    const int t = blockIdx.x;
    const int nf = 1 << a.Rmax, Vf = mc_count(a.Rmax);
    const float* tx = a.tex + static_cast<size_t>(t) * Vf * kPCh;
    const float* gt = a.grad_tex + static_cast<size_t>(t) * Vf * kPCh;
    if constexpr (LDS_SUM) {
        // level Rmax in the first buffer, the chain's levels then alternate
        // between a second buffer (levels Rmax - 1, Rmax - 3, ...) and the first
        float* cur = lds;
        float* nxt = lds + Vf * kPCh;
        const float4* tx4 = reinterpret_cast<const float4*>(tx);
        const float4* gt4 = reinterpret_cast<const float4*>(gt);
        float4* cur4 = reinterpret_cast<float4*>(cur);
        auto dz4 = [](float4 g, float4 s) {
            return make_float4(g.x * s.x * (1.0f - s.x), g.y * s.y * (1.0f - s.y), g.z * s.z * (1.0f - s.z),
                               g.w * s.w * (1.0f - s.w));
        };
        {   // four loads of each array in flight per thread
            const int n4 = Vf * 2;
            int e = threadIdx.x;
            const int nt = blockDim.x;
            for (; e + 3 * nt < n4; e += 4 * nt) {
                float4 sv[4], gv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    sv[u] = tx4[e + u * nt];
                    gv[u] = gt4[e + u * nt];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) cur4[e + u * nt] = dz4(gv[u], sv[u]);
            }
            for (; e < n4; e += nt) cur4[e] = dz4(gt4[e], tx4[e]);
        }
        __syncthreads();
        for (int R = a.Rmax;; --R) {
            if (R <= a.Rtop) {   // a learnable level: out (32 bytes per vertex, 16-byte aligned)
                const int n4 = mc_count(R) * 2;
                float4* g = reinterpret_cast<float4*>(a.graw[R - a.Rmin]) + static_cast<size_t>(t) * n4;
                const float4* c4 = reinterpret_cast<const float4*>(cur);
                for (int e = threadIdx.x; e < n4; e += blockDim.x) {
                    float4 v = c4[e];
                    if (a.accumulate) {
                        const float4 o = g[e];
                        v = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
                    }
                    g[e] = v;
                }
            }
            if (R == a.Rmin) break;
            // restrict level R (cur) onto level R - 1 (nxt): one thread per
            // (coarse vertex, four channels), the six neighbours in a fixed order
            const int nc = 1 << (R - 1), nfl = 1 << R, Vc = mc_count(R - 1);
            const float4* c4 = reinterpret_cast<const float4*>(cur);
            float4* n4 = reinterpret_cast<float4*>(nxt);
            for (int e = threadIdx.x; e < Vc * 2; e += blockDim.x) {
                const int q = e >> 1, h = e & 1;
                int I, J;
                mc_ij(nc, q, I, J);
                const int i = 2 * I, j = 2 * J;
                float4 side = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                auto add = [&](int ii, int jj) __attribute__((always_inline)) {
                    const float4 v = c4[mc_index(nfl, ii, jj) * 2 + h];
                    side = make_float4(side.x + v.x, side.y + v.y, side.z + v.z, side.w + v.w);
                };
                if (i + 1 + j <= nfl) add(i + 1, j);
                if (i > 0) add(i - 1, j);
                if (i + j + 1 <= nfl) add(i, j + 1);
                if (j > 0) add(i, j - 1);
                if (j > 0) add(i + 1, j - 1);   // i + 1 + j - 1 <= n always
                if (i > 0) add(i - 1, j + 1);
                const float4 c = c4[mc_index(nfl, i, j) * 2 + h];
                n4[e] = make_float4(c.x + 0.5f * side.x, c.y + 0.5f * side.y, c.z + 0.5f * side.z, c.w + 0.5f * side.w);
            }
            __syncthreads();
            float* tmp = cur;
            cur = nxt;
            nxt = tmp;
        }
    } else {
        const int nl = a.Rtop - a.Rmin + 1;
        for (int k = threadIdx.x; k < Vf; k += blockDim.x) {
            int i, j;
            mc_ij(nf, k, i, j);
            const float b1 = static_cast<float>(i) * (1.0f / static_cast<float>(nf));
            const float b2 = static_cast<float>(j) * (1.0f / static_cast<float>(nf));
            float dz[kPCh];
#pragma unroll
            for (int c = 0; c < kPCh; ++c) {
                const float s = tx[k * kPCh + c];
                dz[c] = gt[k * kPCh + c] * s * (1.0f - s);
            }
            for (int l = 0; l < nl; ++l) {
                const int R = a.Rmin + l;
                const Micro m = micro_of(1 << R, b1, b2);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (m.w[q] == 0.0f) continue;
#pragma unroll
                    for (int c = 0; c < kPCh; ++c) {
                        const float v = m.w[q] * dz[c];
                        if (v != 0.0f) atomicAdd(&a.graw[l][(static_cast<size_t>(t) * mc_count(R) + m.idx[q]) * kPCh + c], v);
                    }
                }
            }
        }
    }
}

// LDS one workgroup of the assembly gradient may take: half the CU's, at most 64 KiB.
size_t mc_assemble_bwd_lds_cap(size_t lds_limit) { return lds_limit / 2 < 65536 ? lds_limit / 2 : 65536; }

// The finest level's gradient and the next coarser one's (every later level fits the first).
size_t mc_assemble_bwd_lds(int Rmin, int Rmax) {
    const size_t next = Rmax > Rmin ? static_cast<size_t>(mc_count(Rmax - 1)) : 0;
    return (static_cast<size_t>(mc_count(Rmax)) + next) * kPCh * sizeof(float);
}

void launch_mc_assemble(const AssembleArgs& a, hipStream_t s) {
    if (a.T <= 0) return;
    // four triangles per workgroup while their levels take at most 32 KiB of
    // LDS, fewer up to 64 KiB, else the gathering fallback
    const size_t lb = mc_levels_bytes(a.Rmin, a.Rtop);
    const int tpb = 4 * lb <= 32768 ? 4 : (2 * lb <= 49152 ? 2 : (lb <= 65536 ? 1 : 0));
    const unsigned nb = static_cast<unsigned>((a.T + (tpb > 0 ? tpb : 1) - 1) / (tpb > 0 ? tpb : 1));
    if (tpb == 4) {
        hipLaunchKernelGGL(mc_assemble_lds_kernel<4>, dim3(nb), dim3(256), 4 * lb, s, a);
    } else if (tpb == 2) {
        hipLaunchKernelGGL(mc_assemble_lds_kernel<2>, dim3(nb), dim3(256), 2 * lb, s, a);
    } else if (tpb == 1) {
        hipLaunchKernelGGL(mc_assemble_lds_kernel<1>, dim3(nb), dim3(256), lb, s, a);
    } else {
        const int64_t n = static_cast<int64_t>(a.T) * mc_count(a.Rmax);
        hipLaunchKernelGGL(mc_assemble_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, a);
    }
}

void launch_mc_assemble_bwd(const AssembleArgs& a, size_t lds_limit, hipStream_t s) {
    if (a.T <= 0) return;
    const size_t lds = mc_assemble_bwd_lds(a.Rmin, a.Rmax);
    if (lds <= mc_assemble_bwd_lds_cap(lds_limit)) {
        hipLaunchKernelGGL(mc_assemble_bwd_kernel<true>, dim3(static_cast<unsigned>(a.T)), dim3(256), lds, s, a);
    } else {
        // outputs zeroed by the caller unless accumulating
        hipLaunchKernelGGL(mc_assemble_bwd_kernel<false>, dim3(static_cast<unsigned>(a.T)), dim3(256), 0, s, a);
    }
}

// ---------------------------------------------------------------------------
// per-pixel helpers
// ---------------------------------------------------------------------------

// View of global pixel p (views ordered by pix_base).
__device__ __forceinline__ int view_of_pixel(const ViewDesc* __restrict__ views, int V, int64_t p) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].pix_base <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Workgroups are dealt to the eight XCDs in turn: workgroup b works on block
// (b % 8) * per + b / 8 of the grid's blocks (a bijection when the grid is a
// multiple of eight), so that each XCD takes one contiguous eighth of the
// pixels and a triangle's texture is read into one L2.
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t per = gridDim.x / kXcds;
    return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

// The forward's perspective-correct barycentrics of triangle record tr at the
// centre of pixel (x, y): the exact orientation-normalised edge functions,
// beta_i = (float)E_i |rA|, t_i = beta_i / w_i, then the contract's b1, b2.
__device__ __forceinline__ void frag_bary(const TriRec& tr, int x, int y, float& b1, float& b2, double (&E)[3]) {
    const int64_t PX = static_cast<int64_t>(kSnap) * x + kSnap / 2, PY = static_cast<int64_t>(kSnap) * y + kSnap / 2;
    const double sgn = tr.rA < 0.0f ? -1.0 : 1.0;
    const float ra = __builtin_fabsf(tr.rA);
    float t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int ea = i == 2 ? 0 : i + 1, eb = i == 0 ? 2 : (i == 1 ? 0 : 1);
        const double ex = static_cast<double>(tr.X[eb] - tr.X[ea]), ey = static_cast<double>(tr.Y[eb] - tr.Y[ea]);
        // every factor is an integer below 2^26: the product and the fused sum are exact
        E[i] = sgn * __builtin_fma(ex, static_cast<double>(PY - tr.Y[ea]), -(ey * static_cast<double>(PX - tr.X[ea])));
        t[i] = (static_cast<float>(E[i]) * ra) * tr.iw[i];
    }
    persp_from_t(t[0], t[1], t[2], b1, b2);
}

// The winner's shading inputs: the eight channels of its micro-triangle's
// three grid vertices (v[q][0..1]) and their interpolation (feat).
__device__ __forceinline__ void fetch_texel(gfloat* __restrict__ tex, uint32_t tri, int V, const Micro& m,
                                            float4 (&v)[3][2], float (&feat)[kPCh]) {
    gfloat4* g = reinterpret_cast<gfloat4*>(tex + static_cast<size_t>(tri) * V * kPCh);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        v[q][0] = g[2 * m.idx[q]];
        v[q][1] = g[2 * m.idx[q] + 1];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        feat[4 * h + 0] = mc_mix(m, v[0][h].x, v[1][h].x, v[2][h].x);
        feat[4 * h + 1] = mc_mix(m, v[0][h].y, v[1][h].y, v[2][h].y);
        feat[4 * h + 2] = mc_mix(m, v[0][h].z, v[1][h].z, v[2][h].z);
        feat[4 * h + 3] = mc_mix(m, v[0][h].w, v[1][h].w, v[2][h].w);
    }
}

// ---------------------------------------------------------------------------
// deferred shading (forward)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void pshade_kernel(PShadeArgs a) {
    const int64_t p = static_cast<int64_t>(xcd_block()) * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const uint64_t key = a.vis[p];
    float* out = a.color + 3 * p;
    if (key == kBgKey) {
        out[0] = a.o.bg[0];
        out[1] = a.o.bg[1];
        out[2] = a.o.bg[2];
        return;
    }
    const int v = view_of_pixel(a.views, a.V, p);
    const ViewDesc& vd = a.views[v];
    const uint32_t local = static_cast<uint32_t>(p - vd.pix_base);
    const int y = static_cast<int>(local / static_cast<uint32_t>(vd.W));
    const int x = static_cast<int>(local - static_cast<uint32_t>(y) * static_cast<uint32_t>(vd.W));
    const uint32_t tri = static_cast<uint32_t>(key);
    const TriRec tr = a.recs[vd.rec_base + tri];
    float b1, b2;
    double E[3];
    frag_bary(tr, x, y, b1, b2, E);
    const Micro m = micro_of(1 << a.R, b1, b2);
    float4 tv[3][2];
    float feat[kPCh];
    fetch_texel(as_global(a.tex), tri, mc_count(a.R), m, tv, feat);
    float in[kPIn];
#pragma unroll
    for (int c = 0; c < kPFeat; ++c) in[c] = feat[c];
    float d[3];
    view_dir(vd.Mi, vd.W, vd.H, x, y, d);
    sh2(d, in + kPFeat);
    cfloat* mp = as_const(a.mlp);
    float h1[kPHid], h2[kPHid], o[kPOut];
    dense<kPIn, kPHid, true>(mp + kPW0, mp + kPB0, in, h1);
    dense<kPHid, kPHid, true>(mp + kPW1, mp + kPB1, h1, h2);
    dense<kPHid, kPOut, false>(mp + kPW2, mp + kPB2, h2, o);
    const float A = feat[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float mm = sigmoid_c(o[c]);
        out[c] = __builtin_fmaf(A, feat[c] - mm, mm);   // A RGB + (1 - A) MLP
    }
}

void launch_pshade(const PShadeArgs& a, hipStream_t s) {
    if (a.P <= 0) return;
    const int64_t nb = ((a.P + 255) / 256 + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(pshade_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// fragment list: score term (Eq. (9)) or log p(f*) (Eq. (6))
// ---------------------------------------------------------------------------

template <bool LOGP>
__global__ __launch_bounds__(256) void pfrag_kernel(PFragArgs a) {
    __shared__ uint32_t s_boff[kMaxRegions + 1];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i <= a.n_regions; i += blockDim.x) s_boff[i] = a.boff[i];
    __syncthreads();
    const uint32_t n_batch = s_boff[a.n_regions];
    const uint32_t n_waves = gridDim.x * 4;
    const int n = 1 << a.R, V = mc_count(a.R);
    gfloat* tex = as_global(a.tex);
    for (uint32_t bi = blockIdx.x * 4 + w; bi < n_batch; bi += n_waves) {
        int lo = 0, hi = a.n_regions - 1;   // region: last w with boff[w] <= bi
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_boff[mid] <= bi) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t cr = a.counts[lo];
        const uint32_t in_region = (bi - s_boff[lo]) * 64u + static_cast<uint32_t>(lane);
        if (in_region >= (cr < a.region ? cr : a.region)) continue;
        const FragRec fr = a.frags[static_cast<uint64_t>(lo) * a.region + in_region];
        const uint32_t tri = fr.p0.y & 0x7FFFFFFFu;
        const bool win = (fr.p0.y >> 31) != 0u;
        const float b1 = __uint_as_float(fr.p1.x), b2 = __uint_as_float(fr.p1.y);
        const Micro m = micro_of(n, b1, b2);
        gfloat* t = tex + static_cast<size_t>(tri) * V * kPCh + (kPCh - 1);
        const float alpha = mc_mix(m, t[m.idx[0] * kPCh], t[m.idx[1] * kPCh], t[m.idx[2] * kPCh]);
        if constexpr (LOGP) {
            atomicAdd(&a.logp[fr.p0.x], win ? logf(alpha) : log1pf(-alpha));
        } else {
            const float gl = __uint_as_float(fr.x.x);
            if (gl == 0.0f) continue;
            // d log p / d alpha: 1 / alpha for the winner, -1 / (1 - alpha) in front of it
            const float da = win ? gl / alpha : -gl / (1.0f - alpha);
            float* g = a.grad_tex + static_cast<size_t>(tri) * V * kPCh + (kPCh - 1);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (m.w[q] != 0.0f) atomicAdd(&g[m.idx[q] * kPCh], m.w[q] * da);
        }
    }
}

void launch_pfrag(const PFragArgs& a, bool logp, hipStream_t s) {
    if (a.n_blocks <= 0) return;
    if (logp) hipLaunchKernelGGL(pfrag_kernel<true>, dim3(a.n_blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(pfrag_kernel<false>, dim3(a.n_blocks), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// winners (backward)
// ---------------------------------------------------------------------------

constexpr int kPStage = 64 + 4;   // staged row: 64 pixels, padded

// The world-space gradient of the vertices of the winner's triangle from the
// gradient of its perspective-correct barycentrics (db1, db2) and the edge
// weights (ex, ey), in float64 at the snapped positions (every edge function
// an exact integer), with the clip coordinates recomputed in the setup's
// float32 order.
__device__ __forceinline__ void vertex_grad(const ViewDesc& vd, const TriRec& tr, const float* __restrict__ vp,
                                            int px, int py, const double (&E)[3], double db1, double db2, double ex,
                                            double ey, double (&gw)[9]) {
    const double inv_a = 1.0 / ((E[0] + E[1]) + E[2]);
    double fb[3], iwv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        fb[i] = E[i] * inv_a;
        iwv[i] = tr.iw[i];
    }
    const double tt[3] = {fb[0] * iwv[0], fb[1] * iwv[1], fb[2] * iwv[2]};
    const double inv_s = 1.0 / ((tt[0] + tt[1]) + tt[2]);
    const double bb[3] = {tt[0] * inv_s, tt[1] * inv_s, tt[2] * inv_s};
    const double db[3] = {0.0, db1, db2};
    const double dot = db[1] * bb[1] + db[2] * bb[2];
    double dbeta[3], diw[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double dt = (db[i] - dot) * inv_s;
        dbeta[i] = dt * iwv[i];
        diw[i] = dt * fb[i];
    }
    const int32_t PX = kSnap * px + kSnap / 2, PY = kSnap * py + kSnap / 2;
    const double Ai = __builtin_fma(static_cast<double>(tr.X[1] - tr.X[0]), static_cast<double>(tr.Y[2] - tr.Y[0]),
                                    -(static_cast<double>(tr.Y[1] - tr.Y[0]) * static_cast<double>(tr.X[2] - tr.X[0])));
    const double inv_area = 65536.0 / Ai;   // 1 / (signed 2 x area in px^2)
    const double inv256 = 1.0 / 256.0;
    double gsx[3] = {0., 0., 0.}, gsy[3] = {0., 0., 0.};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        // beta_i = e_i / area with e_i = edge(v_p, v_q, pixel centre)
        const int p = i == 2 ? 0 : i + 1, q = i == 0 ? 2 : (i == 1 ? 0 : 1);
#pragma unroll
        for (int jv = 0; jv < 3; ++jv) {
            const int jp = jv == 2 ? 0 : jv + 1, jq = jv == 0 ? 2 : (jv == 1 ? 0 : 1);
            const double dax = static_cast<double>(tr.Y[jp] - tr.Y[jq]) * inv256;
            const double day = static_cast<double>(tr.X[jq] - tr.X[jp]) * inv256;
            double dex = 0., dey = 0.;
            if (jv == p) {
                dex = static_cast<double>(tr.Y[q] - PY) * inv256;
                dey = static_cast<double>(PX - tr.X[q]) * inv256;
            } else if (jv == q) {
                dex = static_cast<double>(PY - tr.Y[p]) * inv256;
                dey = static_cast<double>(tr.X[p] - PX) * inv256;
            }
            gsx[jv] += dbeta[i] * (dex - fb[i] * dax) * inv_area;
            gsy[jv] += dbeta[i] * (dey - fb[i] * day) * inv_area;
        }
    }
    // edge term (Section 3.2): the boundaries this pixel occludes move with its
    // surface point, w beta_i e on the screen position of vertex i
#pragma unroll
    for (int jv = 0; jv < 3; ++jv) {
        gsx[jv] += ex * fb[jv];
        gsy[jv] += ey * fb[jv];
    }
    // screen position (W/2 (c_x / c_w) + W/2, H/2 - H/2 (c_y / c_w)) and 1/w -> clip -> world
    const double hw = 0.5 * vd.W, hh = 0.5 * vd.H;
#pragma unroll
    for (int jv = 0; jv < 3; ++jv) {
        const float x = vp[3 * jv], y = vp[3 * jv + 1], z = vp[3 * jv + 2];
        float cc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {   // the setup's transform
            float acc = vd.M[j * 4 + 3];
            acc = __builtin_fmaf(vd.M[j * 4 + 0], x, acc);
            acc = __builtin_fmaf(vd.M[j * 4 + 1], y, acc);
            acc = __builtin_fmaf(vd.M[j * 4 + 2], z, acc);
            cc[j] = acc;
        }
        const double cx = cc[0], cy = cc[1], iw = 1.0 / static_cast<double>(cc[3]);
        const double gc0 = gsx[jv] * hw * iw;
        const double gc1 = -gsy[jv] * hh * iw;
        const double gc3 = (-gsx[jv] * hw * cx + gsy[jv] * hh * cy - diw[jv]) * (iw * iw);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            gw[3 * jv + k] = static_cast<double>(vd.M[k]) * gc0 + static_cast<double>(vd.M[4 + k]) * gc1 +
                             static_cast<double>(vd.M[12 + k]) * gc3;
    }
}

// One weight-gradient block of the wave's 64 pixels on the matrix cores:
// D[j][c] += sum over pixels of delta[p][j] act[p][c] (v_mfma_f32_16x16x4f32,
// K = pixels: step s of lane group grp takes pixel 16 grp + s, so that lane
// (grp, col) reads 16 consecutive pixels of unit col from the stage), and
// bsum += the lane's 16 values of delta unit col (the bias gradient).
__device__ __forceinline__ void wgrad_block(float (*st)[kPIn][kPStage], const float (&act)[kPIn], const float* delta,
                                            int nd, int lane, f4v& acc, float& bsum) {
    const int col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int u = 0; u < kPIn; ++u) {
        st[0][u][lane] = act[u];
        st[1][u][lane] = u < nd ? delta[u] : 0.0f;
    }
    wave_fence();
    float4 A4[4], B4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        A4[q] = *reinterpret_cast<const float4*>(&st[1][col][16 * grp + 4 * q]);
        B4[q] = *reinterpret_cast<const float4*>(&st[0][col][16 * grp + 4 * q]);
    }
    wave_fence();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc = mfma4(A4[q].x, B4[q].x, acc);
        acc = mfma4(A4[q].y, B4[q].y, acc);
        acc = mfma4(A4[q].z, B4[q].z, acc);
        acc = mfma4(A4[q].w, B4[q].w, acc);
        bsum += (A4[q].x + A4[q].y) + (A4[q].z + A4[q].w);
    }
}

__global__ __launch_bounds__(256) void pwinner_bwd_kernel(PWinArgs a) {
    __shared__ __align__(16) float stage[4][2][kPIn][kPStage];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, col = lane & 15, grp = lane >> 4;
    float (*st)[kPIn][kPStage] = stage[w];
    // contiguous runs of 64-pixel batches per wave, the waves of one XCD on adjacent runs
    const int64_t nbat = (a.P + 63) / 64;
    const int64_t nw = static_cast<int64_t>(gridDim.x) * 4;
    const int64_t wid = static_cast<int64_t>(xcd_block()) * 4 + w;
    const int64_t bbeg = nbat * wid / nw, bend = nbat * (wid + 1) / nw;
    const int R = a.R, n = 1 << R, V = mc_count(R);
    cfloat* mp = as_const(a.mlp);
    gfloat* tex = as_global(a.tex);
    f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f}, acc2 = {0.f, 0.f, 0.f, 0.f};
    float ab0 = 0.f, ab1 = 0.f, ab2 = 0.f;
    for (int64_t b = bbeg; b < bend; ++b) {
        const int64_t p = b * 64 + lane;
        uint64_t key = kBgKey;
        if (p < a.P) key = a.vis[p];
        const bool on = key != kBgKey;
        float gc[3] = {0.f, 0.f, 0.f};
        float ex = 0.f, ey = 0.f;
        if (on) {
            gc[0] = a.grad_color[3 * p];
            gc[1] = a.grad_color[3 * p + 1];
            gc[2] = a.grad_color[3 * p + 2];
            if (a.edge_w) {
                const float2 e = a.edge_w[p];
                ex = e.x;
                ey = e.y;
            }
        }
        const bool cpath = on && (gc[0] != 0.f || gc[1] != 0.f || gc[2] != 0.f);
        const bool active = cpath || (on && (ex != 0.f || ey != 0.f));
        int x = 0, y = 0, v = 0;
        uint32_t tri = 0;
        TriRec tr{};
        float b1 = 0.f, b2 = 0.f;
        double E[3] = {1.0, 0.0, 0.0};
        Micro m{};
        float4 tv[3][2];
        float feat[kPCh];
        if (active) {
            v = view_of_pixel(a.views, a.V, p);
            const ViewDesc& vd = a.views[v];
            const uint32_t local = static_cast<uint32_t>(p - vd.pix_base);
            y = static_cast<int>(local / static_cast<uint32_t>(vd.W));
            x = static_cast<int>(local - static_cast<uint32_t>(y) * static_cast<uint32_t>(vd.W));
            tri = static_cast<uint32_t>(key);
            tr = a.recs[vd.rec_base + tri];
            frag_bary(tr, x, y, b1, b2, E);
            m = micro_of(n, b1, b2);
        }
        // --- colour path: recompute in the forward's arithmetic, then the data backward ---
        float in[kPIn], h1[kPHid], h2[kPHid], d1[kPHid], d2[kPHid], d3[kPOut];
        float dfeat[kPFeat];
#pragma unroll
        for (int u = 0; u < kPHid; ++u) {
            in[u] = 0.f;
            h1[u] = 0.f;
            h2[u] = 0.f;
            d1[u] = 0.f;
            d2[u] = 0.f;
        }
#pragma unroll
        for (int c = 0; c < kPOut; ++c) d3[c] = 0.f;
#pragma unroll
        for (int c = 0; c < kPFeat; ++c) dfeat[c] = 0.f;
        if (cpath) {
            const ViewDesc& vd = a.views[v];
            fetch_texel(tex, tri, V, m, tv, feat);
#pragma unroll
            for (int c = 0; c < kPFeat; ++c) in[c] = feat[c];
            float d[3];
            view_dir(vd.Mi, vd.W, vd.H, x, y, d);
            sh2(d, in + kPFeat);
            float o[kPOut];
            dense<kPIn, kPHid, true>(mp + kPW0, mp + kPB0, in, h1);
            dense<kPHid, kPHid, true>(mp + kPW1, mp + kPB1, h1, h2);
            dense<kPHid, kPOut, false>(mp + kPW2, mp + kPB2, h2, o);
            const float A = feat[3];
            float dA = 0.f;
#pragma unroll
            for (int c = 0; c < kPOut; ++c) {
                const float mm = sigmoid_c(o[c]);
                dfeat[c] = A * gc[c];
                dA = __builtin_fmaf(gc[c], feat[c] - mm, dA);
                d3[c] = (1.0f - A) * gc[c] * (mm * (1.0f - mm));
            }
            dfeat[3] = dA;
            // through the output layer and the ReLU gates of the recompute (the forward's own)
#pragma unroll
            for (int u = 0; u < kPHid; ++u) {
                float s = 0.f;
#pragma unroll
                for (int c = 0; c < kPOut; ++c) s = __builtin_fmaf(mp[kPW2 + c * kPHid + u], d3[c], s);
                d2[u] = h2[u] > 0.f ? s : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kPHid; ++u) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < kPHid; ++j) s = __builtin_fmaf(mp[kPW1 + j * kPHid + u], d2[j], s);
                d1[u] = h1[u] > 0.f ? s : 0.f;
            }
#pragma unroll
            for (int c = 0; c < kPFeat; ++c) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < kPHid; ++j) s = __builtin_fmaf(mp[kPW0 + j * kPIn + c], d1[j], s);
                dfeat[c] += s;   // the harmonics have no parameters
            }
        }
        // --- MLP weight gradients over the wave's pixels (lanes without a colour path add zeros) ---
        if (__ballot(cpath)) {
            wgrad_block(st, in, d1, kPHid, lane, acc0, ab0);
            wgrad_block(st, h1, d2, kPHid, lane, acc1, ab1);
            wgrad_block(st, h2, d3, kPOut, lane, acc2, ab2);
        }
        // --- features -> the micro-triangle's grid vertices; along (b1, b2) -> the triangle ---
        double gw[9] = {0., 0., 0., 0., 0., 0., 0., 0., 0.};
        if (active) {
            float dfu = 0.f, dfv = 0.f;
            if (cpath) {
                float* gt = a.grad_tex + static_cast<size_t>(tri) * V * kPCh;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (m.w[q] == 0.0f) continue;
#pragma unroll
                    for (int c = 0; c < kPFeat; ++c)
                        if (dfeat[c] != 0.0f) atomicAdd(&gt[m.idx[q] * kPCh + c], m.w[q] * dfeat[c]);
                }
                // upright: w = (1 - fu - fv, fu, fv); inverted: w = (fu + fv - 1, 1 - fv, 1 - fu)
#pragma unroll
                for (int c = 0; c < kPFeat; ++c) {
                    const float t0 = c < 4 ? (&tv[0][0].x)[c] : (&tv[0][1].x)[c - 4];
                    const float t1 = c < 4 ? (&tv[1][0].x)[c] : (&tv[1][1].x)[c - 4];
                    const float t2 = c < 4 ? (&tv[2][0].x)[c] : (&tv[2][1].x)[c - 4];
                    dfu = __builtin_fmaf(dfeat[c], m.inv ? t0 - t2 : t1 - t0, dfu);
                    dfv = __builtin_fmaf(dfeat[c], m.inv ? t0 - t1 : t2 - t0, dfv);
                }
            }
            vertex_grad(a.views[v], tr, a.verts + static_cast<size_t>(tri) * 9, x, y, E,
                        static_cast<double>(dfu) * n, static_cast<double>(dfv) * n, ex, ey, gw);
        }
        // --- the vertex gradient summed over each run of equal triangles among the
        // wave's lanes (neighbouring pixels of a row mostly share their winner), one
        // set of float64 atomics per run ---
        if (__ballot(active)) {
            const uint32_t tk = active ? tri : 0xFFFFFFFFu;
            const uint32_t tp = static_cast<uint32_t>(__shfl_up(static_cast<int>(tk), 1, 64));
            const bool head = lane == 0 || tp != tk;
            const uint64_t heads = __ballot(head);
            double* sd = reinterpret_cast<double*>(&st[0][0][0]);   // [9][64], within the stage
#pragma unroll
            for (int k = 0; k < 9; ++k) sd[k * 64 + lane] = gw[k];
            wave_fence();
            if (head && active) {
                const uint64_t above = lane == 63 ? 0ull : (heads & (~0ull << (lane + 1)));
                const int end = above ? __builtin_ctzll(above) : 64;
                double acc[9] = {0., 0., 0., 0., 0., 0., 0., 0., 0.};
                for (int l = lane; l < end; ++l)
#pragma unroll
                    for (int k = 0; k < 9; ++k) acc[k] += sd[k * 64 + l];
                double* gv = a.gvert + static_cast<size_t>(tri) * 9;
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    if (acc[k] != 0.0) atomicAdd(&gv[k], acc[k]);
            }
            wave_fence();
        }
    }
    // the wave's partial row of the MLP gradient (D[4 grp + i][col] of each block)
    float* row = a.mlp_partial + static_cast<size_t>(blockIdx.x * 4 + w) * kPParams;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        row[kPW0 + (4 * grp + i) * kPIn + col] = acc0[i];
        row[kPW1 + (4 * grp + i) * kPHid + col] = acc1[i];
        if (grp == 0 && i < kPOut) row[kPW2 + i * kPHid + col] = acc2[i];
    }
    ab0 += __shfl_xor(ab0, 16, 64);
    ab0 += __shfl_xor(ab0, 32, 64);
    ab1 += __shfl_xor(ab1, 16, 64);
    ab1 += __shfl_xor(ab1, 32, 64);
    ab2 += __shfl_xor(ab2, 16, 64);
    ab2 += __shfl_xor(ab2, 32, 64);
    if (grp == 0) {
        row[kPB0 + col] = ab0;
        row[kPB1 + col] = ab1;
        if (col < kPOut) row[kPB2 + col] = ab2;
    }
}

int pwinner_blocks(int num_cus) { return ((num_cus * 2 + kXcds - 1) / kXcds) * kXcds; }

void launch_pwinner_bwd(const PWinArgs& a, hipStream_t s) {
    if (a.n_blocks <= 0) return;
    hipLaunchKernelGGL(pwinner_bwd_kernel, dim3(static_cast<unsigned>(a.n_blocks)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// backward over the triangle-sorted fragment list
// ---------------------------------------------------------------------------

// One wave per workgroup walks a contiguous range of the fragment list sorted
// by triangle (every winner, and the fragments in front of it where the pixel
// carries a score weight), 64 fragments per batch, and keeps the gradient of
// the current triangle's texture (V x 8 floats) and its nine float64 vertex
// sums in its LDS. Per fragment: its opacity lookup and the score term;
// per winner also the colour path of pwinner_bwd_kernel (recompute, blend,
// MLP data backward on the VALU, features onto the three grid vertices, the
// float64 vertex chain with the edge term) and the MLP weight gradient on the
// matrix cores. Adds into the row are LDS float atomics (two fragments of a
// run may share a grid vertex). When the triangle changes, the row's nonzero
// entries go to HBM: plain stores when the wave holds all of the triangle's
// fragments, float atomics when the triangle straddles two waves' ranges.
//
// LEVELS: the gradient of the learnable levels instead of the assembled
// texture's (the assembly's backward folded in). Every add into the row is
// multiplied by tex (1 - tex) at its grid vertex (the sigmoid's derivative;
// the texels are the ones the fragment's lookups already read), so the row
// holds the gradient of the level-R sum; when the triangle changes, the
// restriction chain (the transpose of the lookups at the level-R vertices:
// the coincident vertex with weight 1, the six lattice neighbours with 1/2)
// runs in LDS, level R - 1 in the stage buffer (free between batches), level
// R - 2 back in the row, and so on, and each learnable level goes out. The
// restriction is linear, so a triangle split between two waves restricts
// each part and adds them. The seven fine-grid indices of every coarse
// vertex are tabulated once per workgroup (a neighbour outside the grid
// points at a zero vertex one past the level's last), so a restriction step
// is one table read and seven 16-byte reads per (vertex, four channels).
constexpr int kPTabMax = 153 + 45 + 15 + 6 + 1;   // coarse vertices of levels 4..0 (the sorted path has R <= 5)
template <bool LEVELS>
__global__ __launch_bounds__(64) void ptri_bwd_kernel(PTriArgs a) {
    __shared__ __align__(16) float stage[2][kPIn][kPStage];
    __shared__ double vsum[9];
    __shared__ uint4 s_tab[LEVELS ? kPTabMax : 1];   // per coarse vertex: centre, six neighbours (16-bit)
    extern __shared__ __align__(16) float row[];   // [V + 1][8]: the current triangle's texture gradient, a zero vertex
    const int lane = threadIdx.x, col = lane & 15, grp = lane >> 4;
    float (*st)[kPIn][kPStage] = stage;
    const int R = a.R, n = 1 << R, V = mc_count(R), NR = V * kPCh;
    if constexpr (LEVELS) {   // the restriction tables of levels R - 1 down to Rmin, in that order
        int off = 0;
        for (int L = R; L > a.Rmin; --L) {
            const int nc = 1 << (L - 1), nfl = 1 << L, Vc = mc_count(L - 1), Vfl = mc_count(L);
            for (int q = lane; q < Vc; q += 64) {
                int I, J;
                mc_ij(nc, q, I, J);
                const int i = 2 * I, j = 2 * J;
                const uint32_t z = static_cast<uint32_t>(Vfl);   // the zero vertex
                const uint32_t c = mc_index(nfl, i, j);
                const uint32_t n1 = i + 1 + j <= nfl ? mc_index(nfl, i + 1, j) : z;
                const uint32_t n2 = i > 0 ? mc_index(nfl, i - 1, j) : z;
                const uint32_t n3 = i + j + 1 <= nfl ? mc_index(nfl, i, j + 1) : z;
                const uint32_t n4 = j > 0 ? mc_index(nfl, i, j - 1) : z;
                const uint32_t n5 = j > 0 ? mc_index(nfl, i + 1, j - 1) : z;   // i + 1 + j - 1 <= n always
                const uint32_t n6 = i > 0 ? mc_index(nfl, i - 1, j + 1) : z;
                s_tab[off + q] = make_uint4(c | (n1 << 16), n2 | (n3 << 16), n4 | (n5 << 16), n6);
            }
            off += Vc;
        }
    }
    cfloat* mp = as_const(a.mlp);
    gfloat* tex = as_global(a.tex);
    const int64_t E = a.tri_off[a.T];
    const int64_t nb = (E + 63) / 64;
    const int64_t nw = gridDim.x;
    const int64_t wid = xcd_block();
    const int64_t bbeg = nb * wid / nw, bend = nb * (wid + 1) / nw;
    const int64_t f0 = bbeg * 64, f1 = bend * 64 < E ? bend * 64 : E;
    for (int k = lane; k < NR + kPCh; k += 64) row[k] = 0.0f;
    if (lane < 9) vsum[lane] = 0.0;
    f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f}, acc2 = {0.f, 0.f, 0.f, 0.f};
    float ab0 = 0.f, ab1 = 0.f, ab2 = 0.f;
    int cur = -1;   // triangle held in the row (wave-uniform)
    // whether the wave holds all of the current triangle's fragments, loaded
    // when the triangle becomes current (its flush needs it)
    bool cur_owned = false;
    // level L's gradient (n floats at src) out to its grid rows: plain stores
    // when the wave owns the triangle, else atomics of the nonzero entries;
    // two rows per lane and step, their LDS reads issued together
    auto put = [&](float* __restrict__ g, const float* src, int nf4, bool owned) __attribute__((always_inline)) {
        const float4* s4 = reinterpret_cast<const float4*>(src);
        float4* g4 = reinterpret_cast<float4*>(g);
        auto out1 = [&](int k, float4 v) __attribute__((always_inline)) {
            if (owned) {
                if (a.accumulate) {   // the outputs were zero-filled unless accumulating
                    const float4 o = g4[k];
                    v = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
                }
                g4[k] = v;
            } else {
                if (v.x != 0.0f) atomicAdd(&g[4 * k], v.x);
                if (v.y != 0.0f) atomicAdd(&g[4 * k + 1], v.y);
                if (v.z != 0.0f) atomicAdd(&g[4 * k + 2], v.z);
                if (v.w != 0.0f) atomicAdd(&g[4 * k + 3], v.w);
            }
        };
        int k = lane;
        for (; k + 64 < nf4; k += 128) {
            const float4 v0 = s4[k], v1 = s4[k + 64];
            out1(k, v0);
            out1(k + 64, v1);
        }
        if (k < nf4) out1(k, s4[k]);
    };
    // the row's nonzero entries go out and are cleared
    auto flush = [&](int t) __attribute__((always_inline)) {
        wave_fence();
        const bool owned = cur_owned;
        if constexpr (LEVELS) {
            float* cur_l = row;
            float* nxt_l = &st[0][0][0];
            int off = 0;
            for (int L = R;; --L) {
                const int VL = mc_count(L);
                if (L <= a.Rtop) put(a.graw[L - a.Rmin] + static_cast<size_t>(t) * VL * kPCh, cur_l, VL * 2, owned);
                if (L == a.Rmin) break;
                // level L onto level L - 1: lane per (coarse vertex, four channels); the
                // neighbours in a fixed order, an absent one read as the zero vertex
                const int Vc = mc_count(L - 1);
                const float4* c4 = reinterpret_cast<const float4*>(cur_l);
                float4* n4 = reinterpret_cast<float4*>(nxt_l);
                auto one = [&](int e, uint4 ix) __attribute__((always_inline)) {
                    const int h = e & 1;
                    const float4 c = c4[(ix.x & 0xFFFFu) * 2 + h];
                    const float4 v1 = c4[(ix.x >> 16) * 2 + h], v2 = c4[(ix.y & 0xFFFFu) * 2 + h];
                    const float4 v3 = c4[(ix.y >> 16) * 2 + h], v4 = c4[(ix.z & 0xFFFFu) * 2 + h];
                    const float4 v5 = c4[(ix.z >> 16) * 2 + h], v6 = c4[ix.w * 2 + h];
                    const float4 sd = make_float4(((((v1.x + v2.x) + v3.x) + v4.x) + v5.x) + v6.x,
                                                  ((((v1.y + v2.y) + v3.y) + v4.y) + v5.y) + v6.y,
                                                  ((((v1.z + v2.z) + v3.z) + v4.z) + v5.z) + v6.z,
                                                  ((((v1.w + v2.w) + v3.w) + v4.w) + v5.w) + v6.w);
                    n4[e] = make_float4(c.x + 0.5f * sd.x, c.y + 0.5f * sd.y, c.z + 0.5f * sd.z, c.w + 0.5f * sd.w);
                };
                int e = lane;
                for (; e + 64 < Vc * 2; e += 128) {   // two items per step: both table reads first
                    const uint4 i0 = s_tab[off + (e >> 1)], i1 = s_tab[off + ((e + 64) >> 1)];
                    one(e, i0);
                    one(e + 64, i1);
                }
                if (e < Vc * 2) one(e, s_tab[off + (e >> 1)]);
                if (lane < 2) n4[Vc * 2 + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);   // level L - 1's zero vertex
                off += Vc;
                wave_fence();
                float* tmp = cur_l;
                cur_l = nxt_l;
                nxt_l = tmp;
            }
            float4* r4 = reinterpret_cast<float4*>(row);   // the row and its zero vertex
            for (int k = lane; k < (NR + kPCh) / 4; k += 64) r4[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        } else {
            float4* r4 = reinterpret_cast<float4*>(row);
            float4* g4 = reinterpret_cast<float4*>(a.grad_tex + static_cast<size_t>(t) * NR);
            float* g = a.grad_tex + static_cast<size_t>(t) * NR;
            for (int k = lane; k < NR / 4; k += 64) {
                float4 v = r4[k];
                if (v.x != 0.0f || v.y != 0.0f || v.z != 0.0f || v.w != 0.0f) {
                    r4[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (owned) {   // the texture gradient was zero-filled unless accumulating
                        if (a.accumulate) {
                            const float4 o = g4[k];
                            v = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
                        }
                        g4[k] = v;
                    } else {
                        if (v.x != 0.0f) atomicAdd(&g[4 * k], v.x);
                        if (v.y != 0.0f) atomicAdd(&g[4 * k + 1], v.y);
                        if (v.z != 0.0f) atomicAdd(&g[4 * k + 2], v.z);
                        if (v.w != 0.0f) atomicAdd(&g[4 * k + 3], v.w);
                    }
                }
            }
        }
        if (lane < 9) {
            const double v = vsum[lane];
            vsum[lane] = 0.0;
            if (v != 0.0) atomicAdd(&a.gvert[static_cast<size_t>(t) * 9 + lane], v);
        }
        wave_fence();
    };
    // Memory is pipelined across batches: a batch's records are loaded two
    // batches ahead, and its per-fragment loads (the opacity texels; for a
    // winner its eight-channel texels, colour gradient and edge weights) are
    // issued before the previous batch's adds into the row and its flush, so
    // that their latency falls behind that work.
    struct Pre {
        FragRec fr;
        bool on;
        Micro m;
        float s7[3];        // the opacity texels of the micro-triangle's vertices
        float gc[3];        // the winner's colour gradient
        float ex, ey;       // ... and its pixel's edge weights
        float4 tv[3][2];    // ... and its eight-channel texels
    };
    auto load_rec = [&](int64_t b, FragRec& fr) __attribute__((always_inline)) {
        const int64_t fi = b * 64 + lane;
        fr = {make_uint2(0u, 0u), make_uint2(0u, 0u), make_uint2(0u, 0u)};
        if (b < bend && fi < E) fr = a.sorted[fi];
    };
    auto issue = [&](const FragRec& fr, int64_t b, Pre& P) __attribute__((always_inline)) {
        P.fr = fr;
        P.on = b < bend && b * 64 + lane < E;
        P.m = Micro{};
        P.ex = P.ey = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            P.s7[q] = 0.f;
            P.gc[q] = 0.f;
        }
        if (P.on) {
            const uint32_t tri = fr.p0.y & 0x7FFFFFFFu;
            P.m = micro_of(n, __uint_as_float(fr.p1.x), __uint_as_float(fr.p1.y));
            gfloat* t7 = tex + static_cast<size_t>(tri) * NR + (kPCh - 1);
#pragma unroll
            for (int q = 0; q < 3; ++q) P.s7[q] = t7[P.m.idx[q] * kPCh];
            if (fr.p0.y >> 31) {   // a winner
                const uint32_t p = fr.p0.x;
#pragma unroll
                for (int c = 0; c < 3; ++c) P.gc[c] = a.grad_color[3 * static_cast<size_t>(p) + c];
                if (a.edge_w) {
                    const float2 e = a.edge_w[p];
                    P.ex = e.x;
                    P.ey = e.y;
                }
                gfloat4* g = reinterpret_cast<gfloat4*>(tex + static_cast<size_t>(tri) * NR);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    P.tv[q][0] = g[2 * P.m.idx[q]];
                    P.tv[q][1] = g[2 * P.m.idx[q] + 1];
                }
            }
        }
    };
    Pre nx;
    FragRec rec1;
    {
        FragRec rec0;
        load_rec(bbeg, rec0);
        issue(rec0, bbeg, nx);
        load_rec(bbeg + 1, rec1);
    }
    for (int64_t b = bbeg; b < bend; ++b) {
        const Pre P = nx;       // this batch's records and loads
        FragRec rec2;           // the records two batches ahead
        load_rec(b + 2, rec2);
        const FragRec& fr = P.fr;
        const bool on = P.on;
        const uint32_t tri = on ? (fr.p0.y & 0x7FFFFFFFu) : 0xFFFFFFFFu;
        const bool win = on && (fr.p0.y >> 31) != 0u;
        const float gl = a.score ? __uint_as_float(fr.x.x) : 0.0f;
        const Micro& m = P.m;
        const float(&s7)[3] = P.s7;
        const float alpha = on ? mc_mix(m, s7[0], s7[1], s7[2]) : 1.0f;
        // d log p / d alpha: 1 / alpha for the winner, -1 / (1 - alpha) in front of it
        const float da = gl == 0.0f ? 0.0f : (win ? gl / alpha : -gl / (1.0f - alpha));
        // --- the winner's colour path ---
        const float(&gc)[3] = P.gc;
        const float ex = P.ex, ey = P.ey;
        int x = 0, y = 0, v = 0;
        if (win) {
            const uint32_t p = fr.p0.x;
            v = static_cast<int>(fr.x.y);
            const ViewDesc& vd = a.views[v];
            const uint32_t local = p - static_cast<uint32_t>(vd.pix_base);
            y = static_cast<int>(local / static_cast<uint32_t>(vd.W));
            x = static_cast<int>(local - static_cast<uint32_t>(y) * static_cast<uint32_t>(vd.W));
        }
        const bool cpath = win && (gc[0] != 0.f || gc[1] != 0.f || gc[2] != 0.f);
        const bool vpath = cpath || (win && (ex != 0.f || ey != 0.f));
        // the winner's setup record and vertices, for its vertex chain after the MLP
        TriRec tr{};
        float vx[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) vx[k] = 0.f;
        if (vpath) {
            tr = a.recs[a.views[v].rec_base + tri];
#pragma unroll
            for (int k = 0; k < 9; ++k) vx[k] = a.verts[static_cast<size_t>(tri) * 9 + k];
        }
        const float4(&tv)[3][2] = P.tv;
        float in[kPIn], h1[kPHid], h2[kPHid], d1[kPHid], d2[kPHid], d3[kPOut];
        float dfeat[kPFeat];
#pragma unroll
        for (int u = 0; u < kPHid; ++u) {
            in[u] = 0.f;
            h1[u] = 0.f;
            h2[u] = 0.f;
            d1[u] = 0.f;
            d2[u] = 0.f;
        }
#pragma unroll
        for (int c = 0; c < kPOut; ++c) d3[c] = 0.f;
#pragma unroll
        for (int c = 0; c < kPFeat; ++c) dfeat[c] = 0.f;
        if (cpath) {
            const ViewDesc& vd = a.views[v];
            float feat[kPCh];
#pragma unroll
            for (int h = 0; h < 2; ++h) {   // the texels' interpolation, as fetch_texel
                feat[4 * h + 0] = mc_mix(m, tv[0][h].x, tv[1][h].x, tv[2][h].x);
                feat[4 * h + 1] = mc_mix(m, tv[0][h].y, tv[1][h].y, tv[2][h].y);
                feat[4 * h + 2] = mc_mix(m, tv[0][h].z, tv[1][h].z, tv[2][h].z);
                feat[4 * h + 3] = mc_mix(m, tv[0][h].w, tv[1][h].w, tv[2][h].w);
            }
#pragma unroll
            for (int c = 0; c < kPFeat; ++c) in[c] = feat[c];
            float d[3];
            view_dir(vd.Mi, vd.W, vd.H, x, y, d);
            sh2(d, in + kPFeat);
            float o[kPOut];
            dense<kPIn, kPHid, true>(mp + kPW0, mp + kPB0, in, h1);
            dense<kPHid, kPHid, true>(mp + kPW1, mp + kPB1, h1, h2);
            dense<kPHid, kPOut, false>(mp + kPW2, mp + kPB2, h2, o);
            const float A = feat[3];
            float dA = 0.f;
#pragma unroll
            for (int c = 0; c < kPOut; ++c) {
                const float mm = sigmoid_c(o[c]);
                dfeat[c] = A * gc[c];
                dA = __builtin_fmaf(gc[c], feat[c] - mm, dA);
                d3[c] = (1.0f - A) * gc[c] * (mm * (1.0f - mm));
            }
            dfeat[3] = dA;
#pragma unroll
            for (int u = 0; u < kPHid; ++u) {
                float sacc = 0.f;
#pragma unroll
                for (int c = 0; c < kPOut; ++c) sacc = __builtin_fmaf(mp[kPW2 + c * kPHid + u], d3[c], sacc);
                d2[u] = h2[u] > 0.f ? sacc : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kPHid; ++u) {
                float sacc = 0.f;
#pragma unroll
                for (int j = 0; j < kPHid; ++j) sacc = __builtin_fmaf(mp[kPW1 + j * kPHid + u], d2[j], sacc);
                d1[u] = h1[u] > 0.f ? sacc : 0.f;
            }
#pragma unroll
            for (int c = 0; c < kPFeat; ++c) {
                float sacc = 0.f;
#pragma unroll
                for (int j = 0; j < kPHid; ++j) sacc = __builtin_fmaf(mp[kPW0 + j * kPIn + c], d1[j], sacc);
                dfeat[c] += sacc;
            }
        }
        if (__ballot(cpath)) {
            wgrad_block(st, in, d1, kPHid, lane, acc0, ab0);
            wgrad_block(st, h1, d2, kPHid, lane, acc1, ab1);
            wgrad_block(st, h2, d3, kPOut, lane, acc2, ab2);
        }
        // --- the winner's vertex gradient (colour path and edge term), float64 ---
        double gw[9] = {0., 0., 0., 0., 0., 0., 0., 0., 0.};
        if (vpath) {
            float dfu = 0.f, dfv = 0.f;
            if (cpath) {
#pragma unroll
                for (int c = 0; c < kPFeat; ++c) {
                    const float t0 = c < 4 ? (&tv[0][0].x)[c] : (&tv[0][1].x)[c - 4];
                    const float t1 = c < 4 ? (&tv[1][0].x)[c] : (&tv[1][1].x)[c - 4];
                    const float t2 = c < 4 ? (&tv[2][0].x)[c] : (&tv[2][1].x)[c - 4];
                    dfu = __builtin_fmaf(dfeat[c], m.inv ? t0 - t2 : t1 - t0, dfu);
                    dfv = __builtin_fmaf(dfeat[c], m.inv ? t0 - t1 : t2 - t0, dfv);
                }
            }
            const ViewDesc& vd = a.views[v];
            float pb1, pb2;
            double E3[3];
            frag_bary(tr, x, y, pb1, pb2, E3);
            vertex_grad(vd, tr, vx, x, y, E3, static_cast<double>(dfu) * n, static_cast<double>(dfv) * n, ex, ey, gw);
        }
        // the next batch's loads go out before this batch's adds and flush
        issue(rec1, b + 1, nx);
        rec1 = rec2;
        // --- into the wave's row, one run of equal triangles at a time ---
        const uint32_t tp = static_cast<uint32_t>(__shfl_up(static_cast<int>(tri), 1, 64));
        uint64_t heads = __ballot(lane == 0 || tp != tri);
        while (heads) {
            const int h = __builtin_ctzll(heads);
            heads &= heads - 1;
            const int t = __builtin_amdgcn_readlane(static_cast<int>(tri), h);
            if (t < 0) break;   // the sentinel run: empty lanes at the list's end
            if (t != cur) {
                if (cur >= 0) flush(cur);
                cur = t;
                cur_owned = a.tri_off[t] >= f0 && a.tri_off[t + 1] <= f1;
            }
            const int end = heads ? __builtin_ctzll(heads) : 64;
            const bool in_run = lane >= h && lane < end;
            if (in_run) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (m.w[q] == 0.0f) continue;
                    float* rv = row + m.idx[q] * kPCh;
                    // LEVELS: times the sigmoid's derivative at the grid vertex
                    const float w7 = LEVELS ? m.w[q] * (s7[q] * (1.0f - s7[q])) : m.w[q];
                    if (da != 0.0f) atomicAdd(rv + (kPCh - 1), w7 * da);
                    if (cpath) {
#pragma unroll
                        for (int c = 0; c < kPFeat; ++c) {
                            const float tq = c < 4 ? (&tv[q][0].x)[c] : (&tv[q][1].x)[c - 4];
                            const float wc = LEVELS ? m.w[q] * (tq * (1.0f - tq)) : m.w[q];
                            if (dfeat[c] != 0.0f) atomicAdd(rv + c, wc * dfeat[c]);
                        }
                    }
                }
            }
            if (__ballot(in_run && vpath)) {   // the run's winners: vertex sums over the wave
                double vv[9], q[3];
#pragma unroll
                for (int k = 0; k < 9; ++k) vv[k] = in_run ? gw[k] : 0.0;
                wave_sum9(vv, q);
                if ((lane & 15) == 0) {   // row g's first lane: components c, c + 2 (and 4 in row 0)
                    const int g = lane >> 4, c0 = (g & 1) + 5 * (g >> 1);
                    vsum[c0] += q[0];
                    vsum[c0 + 2] += q[1];
                    if (g == 0) vsum[4] += q[2];
                }
            }
            wave_fence();
        }
    }
    if (cur >= 0) flush(cur);
    // the wave's partial row of the MLP gradient
    float* prow = a.mlp_partial + static_cast<size_t>(blockIdx.x) * kPParams;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        prow[kPW0 + (4 * grp + i) * kPIn + col] = acc0[i];
        prow[kPW1 + (4 * grp + i) * kPHid + col] = acc1[i];
        if (grp == 0 && i < kPOut) prow[kPW2 + i * kPHid + col] = acc2[i];
    }
    ab0 += __shfl_xor(ab0, 16, 64);
    ab0 += __shfl_xor(ab0, 32, 64);
    ab1 += __shfl_xor(ab1, 16, 64);
    ab1 += __shfl_xor(ab1, 32, 64);
    ab2 += __shfl_xor(ab2, 16, 64);
    ab2 += __shfl_xor(ab2, 32, 64);
    if (grp == 0) {
        prow[kPB0 + col] = ab0;
        prow[kPB1 + col] = ab1;
        if (col < kPOut) prow[kPB2 + col] = ab2;
    }
}

size_t ptri_bwd_lds(int R) { return static_cast<size_t>(mc_count(R) + 1) * kPCh * sizeof(float); }

// As many single-wave workgroups as are resident at once (the LDS row bounds them), a
// multiple of eight: the wave ranges are static, so a second round of workgroups
// would double the time.
int ptri_blocks(int num_cus, int R) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ptri_bwd_kernel<true>, 64, ptri_bwd_lds(R)) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return (num_cus * per_cu / kXcds) * kXcds > 0 ? (num_cus * per_cu / kXcds) * kXcds : kXcds;
}

bool ptri_levels_fit(int R) {
    // level R - 1 and its zero vertex in the stage buffer; the tables of levels R - 1.. (R <= 5)
    return R < 1 || (R <= 5 && static_cast<size_t>(mc_count(R - 1) + 1) * kPCh <= 2 * kPIn * kPStage);
}

void launch_ptri_bwd(const PTriArgs& a, hipStream_t s) {
    if (a.n_blocks <= 0) return;
    if (a.levels)
        hipLaunchKernelGGL(ptri_bwd_kernel<true>, dim3(static_cast<unsigned>(a.n_blocks)), dim3(64), ptri_bwd_lds(a.R),
                           s, a);
    else
        hipLaunchKernelGGL(ptri_bwd_kernel<false>, dim3(static_cast<unsigned>(a.n_blocks)), dim3(64), ptri_bwd_lds(a.R),
                           s, a);
}

__global__ __launch_bounds__(256) void pvert_finish_kernel(const double* __restrict__ g, float* __restrict__ out,
                                                           int64_t n, int accumulate) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = static_cast<float>((accumulate ? static_cast<double>(out[i]) : 0.0) + g[i]);
}

void launch_pvert_finish(const double* g, float* out, int64_t n, bool accumulate, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(pvert_finish_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, g, out, n,
                       accumulate ? 1 : 0);
}

}  // namespace soup
