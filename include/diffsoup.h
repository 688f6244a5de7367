/*
 * diffsoup.h -- C ABI of the MI355X (gfx950) differentiable triangle-soup
 * rasterizer: one rasterization step of an opaque triangle soup under
 * stochastic opacity masking (DiffSoup, arXiv 2603.27151).
 *
 * The problem statement follows Section 3.1 and Supplement B.6 of the paper:
 * a soup of |T| independent triangles (nine floats each), per-triangle
 * textures, a shared MLP decoder (Section 3.3) and pinhole cameras in; an
 * image of colours out; gradients for vertices, textures and the MLP back,
 * as a custom differentiable operator (Supplement A.1).
 *
 * Conventions
 *  - Every pointer marked "device" is a device pointer owned by the caller;
 *    every pointer marked "host" is read during the call only.
 *  - All compute calls are ordered on the given stream (a hipStream_t, passed
 *    as void*; NULL = the default stream). A call returns once its work is
 *    enqueued, except where noted; it synchronises the stream once to size
 *    its tile lists (see soup_rasterize_fwd).
 *  - Argument errors are detected before any work is enqueued: the call
 *    returns SOUP_ERR_INVALID (or SOUP_ERR_UNSUPPORTED) and soup_last_error()
 *    describes the problem. No C++ exception crosses this interface.
 *  - Views of one call are concatenated in the output buffers: view v owns
 *    pixels [sum_{u<v} W_u H_u, sum_{u<=v} W_u H_u), row-major (y * W + x),
 *    row 0 at the top of the image.
 *  - A context is not thread safe; use one context per host thread/stream.
 */
#ifndef DIFFSOUP_H
#define DIFFSOUP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct soup_ctx soup_ctx;

typedef enum {
    SOUP_OK = 0,
    SOUP_ERR_INVALID = 1,      /* bad argument (message via soup_last_error) */
    SOUP_ERR_OOM = 2,          /* device allocation failed */
    SOUP_ERR_CAPACITY = 3,     /* a fixed workspace capacity was exceeded */
    SOUP_ERR_HIP = 4,          /* a HIP runtime call failed */
    SOUP_ERR_UNSUPPORTED = 5   /* valid but not compiled in (e.g. an MLP shape) */
} soup_status;

/* A triangle soup with its neural texture (Section 3.1; Section 3.3 in the
 * form of a G x G feature grid per triangle, sampled bilinearly at the
 * perspective-correct barycentrics (b1, b2) -> grid (b1 (G-1), b2 (G-1)),
 * and a shared MLP C -> h ... -> 4 with ReLU hidden layers whose outputs are
 * the RGB logits and the opacity logit; colour = sigmoid(o0..o2),
 * alpha = sigmoid(o3)). */
typedef struct {
    int32_t T;                 /* triangles, >= 0 */
    int32_t G;                 /* feature grid side, >= 2; G * G * C <= 4096 (else SOUP_ERR_UNSUPPORTED) */
    int32_t C;                 /* feature channels = dims[0] */
    int32_t n_layers;          /* MLP layers (linear maps), >= 1 */
    const int32_t* dims;       /* host [n_layers+1]; dims[0] == C, dims[n_layers] == 4 */
    const float* verts;        /* device [T,3,3] world positions, float32 */
    const float* feats;        /* device [T,G,G,C], texel [t][iy][ix][c] */
    const float* mlp;          /* device, per layer: W[d_out][d_in] row-major, then b[d_out] */
} soup_scene;

/* Pinhole views. clip = M [x, y, z, 1]; screen x = W/2 (c_x/c_w + 1),
 * screen y = H/2 (1 - c_y/c_w), depth = (c_z/c_w + 1)/2 clamped to [0, 1]. */
typedef struct {
    int32_t V;                 /* number of views, >= 1 */
    const int32_t* width;      /* host [V], 1..16384 */
    const int32_t* height;     /* host [V], 1..16384 */
    const uint32_t* view_id;   /* host [V]: enters the random draws (not the batch position) */
    const float* view_proj;    /* host [V,4,4] row-major float32 */
} soup_views;

typedef struct {
    uint64_t seed;             /* Philox4x32-10 key (low word, high word) */
    uint32_t step;             /* fourth counter word (e.g. the iteration) */
    int32_t mode;              /* 0: stochastic masking, Eq. (5); 1: threshold alpha > 1/2, Eq. (3) */
    float background[3];       /* colour where no fragment passes */
    int32_t edge_pairs;        /* 0: every adjacent pixel pair (Section 3.2); 1: only pairs whose
                                  triangle id differs; 2: no edge term */
    float near_w;              /* triangles with any vertex at clip w < near_w are culled (0.1) */
    int32_t accumulate;        /* backward: 0 overwrite the gradient outputs, 1 add into them */
    int32_t reuse_bins;        /* backward: 1 = reuse the triangle setup and tile lists of the last
                                  forward on this context when its views, scenes, tile size and near_w
                                  are the same (else they are rebuilt); the caller guarantees that the
                                  vertex data did not change in between. 0 = always rebuild. */
} soup_opts;

/* Work counts of the last compute call on a context (filled on request). */
typedef struct {
    int64_t pixels;            /* pixels of all views */
    int64_t tiles;             /* screen tiles of all views */
    int64_t bin_entries;       /* (tile, triangle) pairs after binning */
    int64_t visible_tris;      /* (view, triangle) records that survived culling */
    int64_t decodes;           /* texture + MLP decodes performed by the raster kernel (forward,
                                  render) or by the backward's decode (the fragments it needs) */
    int64_t covered_pixels;    /* forward and render: pixels that at least one fragment covers
                                  (Eq. (1)); -1 for the backward */
} soup_stats;

/* Create a context on HIP device `device`. Owns the workspaces (triangle
 * records, tile lists, partial sums), grown on demand and freed by
 * soup_ctx_destroy. Returns SOUP_ERR_HIP if the device cannot be used. */
soup_status soup_ctx_create(soup_ctx** out, int device);
void soup_ctx_destroy(soup_ctx* ctx);

/* Message of the last error on this context ("" if none). Valid until the
 * next call on the context. */
const char* soup_last_error(const soup_ctx* ctx);

/* Screen tile side in pixels: 8, 16 (default) or 32. */
soup_status soup_ctx_set_tile(soup_ctx* ctx, int32_t tile);
int32_t soup_ctx_get_tile(const soup_ctx* ctx);

/* Per-kernel timing. When enabled, every launch group of a compute call is
 * bracketed by a pair of HIP events recorded on the call's stream (no
 * synchronisation is added). soup_read_timings synchronises those events,
 * adds their elapsed times into ms[k] and the number of launches into
 * count[k] for k < SOUP_TIMING_KINDS (arrays of that length, host), and
 * forgets them. Kinds: */
enum {
    SOUP_T_SETUP = 0,    /* triangle setup + per-tile counts */
    SOUP_T_SCAN = 1,     /* tile offsets */
    SOUP_T_SCATTER = 2,  /* tile lists */
    SOUP_T_SORT = 3,     /* per-tile depth sort */
    SOUP_T_FWD = 4,      /* forward raster */
    SOUP_T_BWD = 5,      /* backward fragment decode (MLP backward, gradient records) */
    SOUP_T_EDGE = 6,     /* per-pixel edge weights (the edge term joins the decode's vertex chain) */
    SOUP_T_CHAIN = 7,    /* reserved (the vertex chain runs inside the backward decode) */
    SOUP_T_REDUCE = 8,   /* MLP-gradient reduction */
    SOUP_T_LOGP = 9,     /* log p(f*) pass (includes its replay and decode) */
    SOUP_T_LOSS = 10,    /* L2 loss */
    SOUP_T_FILL = 11,    /* zero fills */
    SOUP_T_REPLAY = 12,  /* backward front-set replay (coverage, fragment list) */
    SOUP_T_GRAD = 13,    /* per-triangle feature and vertex gradient reduction */
    SOUP_T_COVER = 14,   /* adaptive control: coverage counts */
    SOUP_T_EDGELEN = 15, /* adaptive control: screen-space edge lengths */
    SOUP_T_APPLY = 16,   /* adaptive control: applying a plan */
    SOUP_T_TLOSS = 17,   /* L1 + SSIM loss */
    SOUP_T_ADAM = 18,    /* optimiser steps */
    SOUP_T_SHADE = 19,   /* paper form: deferred shading of the winners */
    SOUP_T_ASSEMBLE = 20, /* paper form: texture assembly */
    SOUP_T_ASSEMBLE_BWD = 21, /* paper form: texture assembly gradient */
    SOUP_TIMING_KINDS = 22
};
soup_status soup_ctx_set_timing(soup_ctx* ctx, int32_t on);
soup_status soup_read_timings(soup_ctx* ctx, double* ms, int64_t* count);

/* Static-capacity mode, for callers that capture a sequence of calls into a
 * HIP graph (hipStreamBeginCapture / torch.cuda.graph) and replay it.
 * When on, soup_rasterize_fwd / soup_rasterize_bwd / soup_render neither
 * synchronise nor allocate: every workspace keeps the size an earlier call
 * outside static mode gave it (run the captured sequence once eagerly first,
 * with the same scene, views and tile), the views and scenes must equal
 * those of the previous call (their device copies are reused), and the
 * lists whose length is only known on the device (tile lists, backward
 * fragments) are bounded by the capacity in place. A call that would exceed
 * it produces no fragments for the overflowing part and sets a sticky flag
 * instead of failing. Counting and timing must be off.
 * soup_ctx_check synchronises the device, returns SOUP_ERR_CAPACITY (and
 * clears the flag) if any static-mode call since the last check overflowed,
 * else SOUP_OK; the caller then reruns outside static mode, which grows the
 * workspaces, and captures again. */
soup_status soup_ctx_set_static(soup_ctx* ctx, int32_t on);
soup_status soup_ctx_check(soup_ctx* ctx);

/* Device bytes the context's workspaces hold now (they grow on demand and
 * are released by soup_ctx_destroy): what a caller that admits work by
 * memory has to count besides its own buffers. */
soup_status soup_ctx_workspace_bytes(const soup_ctx* ctx, int64_t* bytes);

/* Enable (1) or disable (0, default) counting of decodes in soup_stats. */
soup_status soup_ctx_set_counting(soup_ctx* ctx, int32_t on);
soup_status soup_last_stats(const soup_ctx* ctx, soup_stats* out);

/*
 * Forward pass (Eq. (1), (2), (5); Supplement Algorithm A1, part 1).
 * For every pixel centre: the fragments are the triangles covering it; each
 * fragment f draws u_f = Philox(seed; pixel index, triangle, view_id, step)
 * (24-bit uniform) and passes when u_f < alpha_f (mode 0) or when its opacity
 * logit is > 0 (mode 1); the winner is the passing fragment with the smallest
 * key (depth bits << 32 | triangle), found without sorting fragments.
 * Outputs (device, caller-allocated, overwritten):
 *   vis   [P] uint64   winner key, 0xFFFFFFFFFFFFFFFF where no fragment passes
 *   color [P,3] float  sigmoid of the winner's RGB logits, or background
 *   logp  [P] float    log p(f*) of Eq. (6) (mode 0), or NULL
 * The call synchronises `stream` once (after binning) to size the tile list
 * workspace; everything else is asynchronous.
 */
soup_status soup_rasterize_fwd(soup_ctx* ctx, const soup_scene* scene, const soup_views* views,
                               const soup_opts* opts, uint64_t* vis, float* color, float* logp,
                               void* stream);

/*
 * Backward pass (Eq. (8), (9); Supplement Algorithm A1, part 2; Section 3.2
 * edge term), recomputing fragments from the saved visibility buffer.
 * Inputs: vis and color from soup_rasterize_fwd with the same arguments;
 * grad_color [P,3] = dL/dcolor; grad_logp [P] = per-pixel weight of the score
 * term (the sampled pixel loss for Algorithm A1's L * s), or NULL.
 * Outputs (device): grad_verts [T,3,3], grad_feats [T,G,G,C], grad_mlp
 * [n_params]; overwritten, or added into when opts->accumulate is 1 (a loop
 * over views can then sum its gradients in place).
 *   winner f*:        colour path (exact derivative with draws fixed),
 *                     through the texture position to the vertices, plus
 *                     score g_L (1 - alpha*) on its opacity logit (features
 *                     and MLP only: the score term moves no vertex, Section
 *                     3.2);
 *   f in front of f*: score -g_L alpha_f on its opacity logit (features and
 *                     MLP only, no vertex motion);
 *   adjacent pixel pairs (a, b = a + e): w = 1/2 (g_a + g_b).(C_a - C_b)
 *                     moves the nearer pixel's triangle vertices by
 *                     w beta_i e in screen space.
 * Floating-point sums are order-dependent (atomics); results agree with an
 * exact evaluation to about 1e-6 relative.
 */
soup_status soup_rasterize_bwd(soup_ctx* ctx, const soup_scene* scene, const soup_views* views,
                               const soup_opts* opts, const uint64_t* vis, const float* color,
                               const float* grad_color, const float* grad_logp,
                               float* grad_verts, float* grad_feats, float* grad_mlp,
                               void* stream);

/*
 * Batched forward-only render of R requests (serving): request r renders
 * scenes[r] from view r of `views` (views->V == R) into color[r] (device
 * [H_r, W_r, 3], overwritten). All scenes must share G, C and the MLP shape;
 * their triangle counts may differ. The mode in opts applies to all
 * requests (1 = the deterministic threshold render of Eq. (3)).
 */
soup_status soup_render(soup_ctx* ctx, const soup_scene* scenes, int32_t R, const soup_views* views,
                        const soup_opts* opts, float* const* color, void* stream);

/*
 * Per-pixel L2 photometric loss against `target` (device [P,3]) over P pixels
 * (the benchmark's loss; any per-pixel loss can feed soup_rasterize_bwd):
 *   L = mean over P*3 of (color - target)^2,
 *   grad_color = 2 (color - target) / (3P),
 *   grad_logp  = sum_c (color - target)^2 / (3P)   (so sum_p grad_logp = L).
 * loss (device scalar, may be NULL) receives L.
 */
soup_status soup_loss_l2(soup_ctx* ctx, const float* color, const float* target, int64_t P,
                         float* grad_color, float* grad_logp, float* loss, void* stream);

/*
 * Adaptive control of primitives (Section 3.4, "Adaptive control of
 * primitives"; Supplement B, resampling of a random initialisation): split
 * edges that look long on a sample of views, prune the triangles that cover
 * the fewest pixels, keep the triangle budget. Measure (soup_coverage_count,
 * soup_edge_lengths, device), decide (soup_adaptive_plan, host), rebuild
 * (soup_adaptive_apply, device).
 */

/* Pixel coverage: counts[t] += the number of keys of vis [n] (device uint64,
 * from soup_rasterize_fwd over any views of one scene) whose low 32 bits,
 * the winner's triangle index, equal t. Background keys and indices >= T
 * are skipped. counts: device [T] uint32, added into (zero it for a fresh
 * count); the order of the additions does not matter (integers). */
soup_status soup_coverage_count(soup_ctx* ctx, const uint64_t* vis, int64_t n, int32_t T, uint32_t* counts,
                                void* stream);

/* Screen-space edge lengths: rel_len (device [T,3] float, overwritten)
 * receives for edge k of triangle t (vertex k to vertex (k+1) mod 3) its
 * largest length in pixels divided by the view's height, over the views in
 * which every vertex is at clip w >= near_w and the screen bounding box meets
 * [0,W] x [0,H]; 0 where no view qualifies. The projection is the one of
 * soup_views, evaluated in float64 (products, then sums left to right), the
 * result rounded to float32 once. verts: device [T,3,3]; views->view_id is
 * not read. Any number of views (launched 32 at a time). */
soup_status soup_edge_lengths(soup_ctx* ctx, const float* verts, int32_t T, const soup_views* views, float near_w,
                              float* rel_len, void* stream);

enum { SOUP_ACT_REMOVE = 0, SOUP_ACT_KEEP = 1, SOUP_ACT_SPLIT0 = 2 }; /* SPLIT0 + k: split edge k */
enum { SOUP_PLAN_PRUNE_ZERO = 1, SOUP_PLAN_FILL = 2 };

/* Plan (host code on host arrays; synchronous; ctx may be NULL).
 *  1. a triangle whose longest edge (lowest k among equals) has
 *     rel_len > split_frac (float32 comparison) splits on that edge;
 *  2. SOUP_PLAN_PRUNE_ZERO: triangles with counts == 0 are removed;
 *  3. while the triangle count after the splits exceeds target, triangles
 *     are removed in order of (counts, index) ascending, each with its split;
 *  4. SOUP_PLAN_FILL: while the count is below target, kept unsplit
 *     triangles split on their longest edge, longest first (index order
 *     among equals).
 * Outputs: actions [T] (SOUP_ACT_*), offsets [T] (each triangle's first
 * output slot: the exclusive prefix sum of 0 / 1 / 2 outputs), *n_new.
 * 0 <= T <= 2^30, target >= 0. */
soup_status soup_adaptive_plan(soup_ctx* ctx, const uint32_t* counts, const float* rel_len, int32_t T,
                               float split_frac, int32_t target, int32_t flags, int32_t* actions, int32_t* offsets,
                               int32_t* n_new);

/* Apply a plan (device): verts_out [n_new,3,3] and feats_out [n_new,G,G,C]
 * (device, overwritten) receive the kept triangles in order and, for a
 * split of edge k, two halves at offsets[t] and offsets[t]+1: half 0 takes
 * the midpoint in place of vertex k+1, half 1 in place of vertex k (the
 * vertex order, hence the orientation, is kept). A half's texel (ix, iy),
 * at (ix, iy)/(G-1) in its barycentrics, samples the parent's grid
 * bilinearly at the same surface point (grid coordinates clamped to
 * [0, G-1]). Uses scene->T, G, C, verts, feats; the MLP is unchanged.
 * actions, offsets: device [T], a plan from soup_adaptive_plan; entries whose
 * outputs would fall outside [0, n_new) are not written. feats and
 * feats_out must be 16-byte aligned (as any device allocation is). */
soup_status soup_adaptive_apply(soup_ctx* ctx, const soup_scene* scene, const int32_t* actions,
                                const int32_t* offsets, int32_t n_new, float* verts_out, float* feats_out,
                                void* stream);

/*
 * Paper form of the step (Section 3.3, "Learnable multi-resolution triangle
 * texture" and "Neural deferred shading"; Supplement B.3 and B.6).
 *
 * Texture: per triangle the level-R mesh-colour grid: n = 2^R segments per
 * edge, grid vertex (i, j), i + j <= n, at perspective-correct barycentrics
 * (b1, b2) = (i/n, j/n), V(R) = (n + 1)(n + 2)/2 vertices (561 at R = 5)
 * stored row-major: vertex (i, j) at index j (n + 1) - j (j - 1)/2 + i. Each
 * vertex holds 8 floats (32 bytes): 7 colour features, then the opacity, all
 * in [0, 1] (after the sigmoid). A fragment's values are interpolated
 * linearly in the micro-triangle that contains it: u = b1 n, v = b2 n,
 * i = floor(u) in [0, n-1], j = floor(v) in [0, n-1-i], fu = u - i,
 * fv = v - j; if fu + fv > 1 and i + j <= n - 2, the vertices (i+1, j+1),
 * (i+1, j), (i, j+1) with weights (fu + fv - 1, 1 - fv, 1 - fu), else
 * (i, j), (i+1, j), (i, j+1) with ((1 - fu) - fv, fu, fv).
 * Mask: the opacity alpha of a fragment is channel 7 (no MLP); the draws and
 * the winner are those of soup_rasterize_fwd (mode 1: alpha > 1/2).
 * Colour (deferred, winners only): input = the 7 features and the 9 real
 * spherical harmonics of degree <= 2 of the pixel's view direction (order
 * Y00; Y1: y, z, x; Y2: xy, yz, 2z^2 - x^2 - y^2, xz, x^2 - y^2, orthonormal,
 * no Condon-Shortley sign); MLP 16 -> 16 -> 16 -> 3, ReLU hidden layers,
 * sigmoid outputs m; features 0..3 read as RGBA: colour = A RGB + (1 - A) m.
 * The view direction of pixel (x, y) is normalize(P(+1) - P(-1)) with P(z)
 * the point of normalised device coordinates ((2x + 1)/W - 1, 1 - (2y + 1)/H,
 * z) through the view's inverse view-projection (divided by w).
 */
typedef struct {
    int32_t T;                 /* triangles, >= 0 */
    int32_t R;                 /* texture level, 0..7 */
    const float* verts;        /* device [T,3,3] world positions */
    const float* tex;          /* device [T,V(R),8], 16-byte aligned */
    const float* mlp;          /* device [595]: W0[16][16], b0[16], W1[16][16], b1[16], W2[3][16], b2[3]
                                  (W[out][in] row-major) */
} soup_pscene;

/*
 * Paper-form forward (Eq. (1), (2), (5) with the texture's opacity; the
 * deferred colour). inv_view_proj: host [V,4,4] row-major, the inverse of
 * each view's view_proj (the caller's, used as given). Outputs as in
 * soup_rasterize_fwd: vis [P] (bit-identical to an evaluation of the same
 * float32 operations), color [P,3], logp [P] or NULL. With opts->reuse_bins
 * (or logp in mode 0) the call keeps a log of its opacity decodes for
 * soup_pbackward / the logp pass. Synchronises the stream as
 * soup_rasterize_fwd does.
 */
soup_status soup_pforward(soup_ctx* ctx, const soup_pscene* scene, const soup_views* views,
                          const float* inv_view_proj, const soup_opts* opts, uint64_t* vis, float* color,
                          float* logp, void* stream);

/*
 * Paper-form backward (Algorithm A1, part 2; Eq. (8), (9); the edge term of
 * Section 3.2). Inputs as in soup_rasterize_bwd. Outputs (device):
 * grad_verts [T,3,3], grad_tex [T,V(R),8], grad_mlp [595]; overwritten, or
 * added into when opts->accumulate is 1.
 *   winner f*:   colour path (d colour / d RGB = A, d / d A = RGB - m, the
 *                MLP backward to the 7 features), onto the micro-triangle's
 *                3 grid vertices with its weights, and through (b1, b2) to
 *                the vertices; score g_L / alpha* on its opacity channel;
 *   f in front:  score -g_L / (1 - alpha_f) on its opacity channel;
 *   the score term moves no vertex; the edge term as in soup_rasterize_bwd.
 * Floating-point sums use atomics (order-dependent, about 1e-6 relative).
 * For an empty soup (T = 0) grad_verts and grad_tex may be NULL.
 */
soup_status soup_pbackward(soup_ctx* ctx, const soup_pscene* scene, const soup_views* views,
                           const float* inv_view_proj, const soup_opts* opts, const uint64_t* vis,
                           const float* color, const float* grad_color, const float* grad_logp,
                           float* grad_verts, float* grad_tex, float* grad_mlp, void* stream);

/*
 * soup_pbackward followed by the assembly's backward (Section 3.3; the
 * gradient of soup_mc_assemble), in one call: scene->tex must be the
 * assembly of the learnable levels Rmin..Rtop onto level scene->R, and
 * grad_raw (host array of Rtop - Rmin + 1 device pointers, [T,V(Rmin + l),8],
 * 16-byte aligned) receives the gradient of those levels instead of a
 * gradient of the texture; overwritten, or added into when opts->accumulate
 * is 1. grad_verts and grad_mlp as in soup_pbackward. Where one triangle's
 * grids fit the backward's LDS (R <= 5) the restriction to the levels runs
 * inside it and no texture-sized gradient is written; otherwise the call
 * uses a context workspace of T * V(R) * 32 bytes. Errors as soup_pbackward,
 * and SOUP_ERR_INVALID for levels outside 0 <= Rmin <= Rtop <= R or a NULL
 * level pointer.
 */
soup_status soup_pbackward_levels(soup_ctx* ctx, const soup_pscene* scene, const soup_views* views,
                                  const float* inv_view_proj, const soup_opts* opts, const uint64_t* vis,
                                  const float* color, const float* grad_color, const float* grad_logp,
                                  int32_t Rmin, int32_t Rtop, float* grad_verts, float* const* grad_raw,
                                  float* grad_mlp, void* stream);

/*
 * Multi-resolution texture assembly (Section 3.3): the learnable grids of
 * levels Rmin..Rtop (raw: host array of Rtop - Rmin + 1 device pointers,
 * level Rmin + l at raw[l], [T,V(Rmin + l),8], before the sigmoid) are each
 * sampled at the vertices of the level-Rmax grid by the micro-triangle
 * lookup, summed (Rmin first) and passed through the sigmoid:
 * tex [T,V(Rmax),8] (device, overwritten). 0 <= Rmin <= Rtop <= Rmax <= 7.
 * The paper keeps grids up to Rmax - 1 (Rtop = Rmax - 1); Rtop = Rmax makes
 * the finest grid learnable as well. Buffers 16-byte aligned.
 */
soup_status soup_mc_assemble(soup_ctx* ctx, int32_t T, int32_t Rmin, int32_t Rtop, int32_t Rmax,
                             const float* const* raw, float* tex, void* stream);

/* Gradient of soup_mc_assemble: grad_raw[l] (device, [T,V(Rmin + l),8])
 * receives the sum over the level-Rmax vertices of the lookup weight times
 * tex (1 - tex) grad_tex; overwritten, or added into when accumulate is 1. */
soup_status soup_mc_assemble_bwd(soup_ctx* ctx, int32_t T, int32_t Rmin, int32_t Rtop, int32_t Rmax,
                                 const float* tex, const float* grad_tex, float* const* grad_raw,
                                 int32_t accumulate, void* stream);

/*
 * Photometric loss of training (Section 3.4, "Loss function"):
 *   L = lambda L1 + (1 - lambda) (1 - SSIM), lambda = 0.8 in the paper,
 * L1 = mean over the P pixels of all views and 3 channels of |color - target|;
 * SSIM = mean over pixels and channels of the SSIM map (Wang et al. 2004):
 * 11 x 11 Gaussian window (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, local
 * statistics per view and channel with zero padding outside the image.
 * color, target: device [P,3] (views concatenated, as in soup_rasterize_fwd);
 * views: only width and height are read. Outputs (device, overwritten):
 *   grad_color [P,3] = dL/dcolor (the L1 part uses sign, 0 at equality);
 *   grad_logp  [P]   = pixel p's share of L, [lambda sum_c |d| +
 *                      (1 - lambda) sum_c (1 - S_c(p))] / (3P), so the shares
 *                      sum to L (the score term's per-pixel loss);
 *   loss (device scalar, may be NULL) = L (summed with atomics).
 * Uses a context workspace of 48 bytes per pixel of the largest view. */
soup_status soup_loss_l1_ssim(soup_ctx* ctx, const float* color, const float* target, const soup_views* views,
                              float lambda, float* grad_color, float* grad_logp, float* loss, void* stream);

/*
 * soup_loss_l1_ssim for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc): the same arguments, kernels and results, with the
 * statistics record in a static device array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends, instead of a
 * context workspace. The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine; no timing events). A view of more than
 * 1,398,101 pixels (64 MiB / 48 B) is rejected with SOUP_ERR_CAPACITY.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other contexts, other threads) race and must be
 * ordered by the caller. Nothing in the array needs to start at zero: each
 * pixel's record is written before it is read within the same call.
 */
soup_status soup_loss_l1_ssim_noalloc(soup_ctx* ctx, const float* color, const float* target,
                                      const soup_views* views, float lambda, float* grad_color, float* grad_logp,
                                      float* loss, void* stream);

/*
 * One optimiser step (Section 3.4; Supplement, hyperparameters): Adam for
 * vec = 1, VectorAdam for vec = 3 (vertex positions: one second moment per
 * 3-vector, from its squared norm). For each vector i of n / vec:
 *   m = b1 m + (1 - b1) g;   v_i = b2 v_i + (1 - b2) |g_i|^2;
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v_i / (1 - b2^t)) + eps).
 * p, m: device [n] float, updated; g: device [n]; v: device [n / vec],
 * updated; t >= 1 is the step count; n must be a multiple of vec. The
 * betas are double so that 1 - beta and the bias corrections are formed from
 * the exact hyperparameters (in float, 1 - 0.999 is off by 1.3e-5).
 */
soup_status soup_adam_step(soup_ctx* ctx, float* p, const float* g, float* m, float* v, int64_t n, int32_t vec,
                           float lr, double beta1, double beta2, float eps, int32_t t, void* stream);

/* Contract self-test: y[i] = the device sigmoid of x[i] (the opacity
 * sigmoid whose value decides the mask), for checking it bit for bit
 * against an independent implementation. x, y device [n]. */
soup_status soup_selftest_sigmoid(soup_ctx* ctx, const float* x, float* y, int64_t n, void* stream);

/* Contract self-test: u[i] = the device 24-bit uniform draw for counter
 * (pixel[i], tri[i], view_id, step) under `seed`. pixel, tri, u device [n]. */
soup_status soup_selftest_uniform(soup_ctx* ctx, uint64_t seed, const uint32_t* pixel,
                                  const uint32_t* tri, uint32_t view_id, uint32_t step,
                                  float* u, int64_t n, void* stream);

/*
 * Measured ceilings: kernels of known work that a caller times on `stream`
 * to put the method's kernels on a measured roofline beside the published
 * peaks (they compute nothing of the method). Each leaves a result that can
 * be checked exactly. Device buffers, 16-byte aligned where noted; errors
 * SOUP_ERR_INVALID for bad arguments.
 *   soup_probe_copy:   dst = src, `bytes` (a multiple of 16) read and written.
 *   soup_probe_read:   reads `bytes` of src (a multiple of 16); partial
 *                      [n_partial] receives per-workgroup sums of its floats
 *                      (min(bytes / 4096, n_partial) of them, rounded up,
 *                      are written).
 *   soup_probe_atomic: n_ops float atomic adds of 1 into slots [n_slots],
 *                      op k to slot (k * 2654435761) mod n_slots (scattered).
 *   soup_probe_fma:    n_threads (a multiple of 256) threads each run eight
 *                      independent chains of iters float32 FMAs (2^20 at most):
 *                      16 iters n_threads FLOP; out [n_threads] = 8 iters + 28.
 *   soup_probe_mfma:   n_threads / 64 waves each run four independent chains
 *                      of iters v_mfma_f32_16x16x4f32 (2^18 at most): 8192
 *                      iters n_threads / 64 FLOP; out [n_threads] = 64 iters.
 */
soup_status soup_probe_copy(soup_ctx* ctx, const void* src, void* dst, int64_t bytes, void* stream);
soup_status soup_probe_read(soup_ctx* ctx, const void* src, int64_t bytes, float* partial, int64_t n_partial,
                            void* stream);
soup_status soup_probe_atomic(soup_ctx* ctx, float* slots, int64_t n_slots, int64_t n_ops, void* stream);
soup_status soup_probe_fma(soup_ctx* ctx, float* out, int64_t n_threads, int32_t iters, void* stream);
soup_status soup_probe_mfma(soup_ctx* ctx, float* out, int64_t n_threads, int32_t iters, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DIFFSOUP_H */
