/*
 * CPU oracle for one differentiable rasterization step of a triangle soup
 * under stochastic opacity masking (DiffSoup, Sections 3.1-3.2,
 * Supplement B.1 and C).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, plain statement of what
 * the step computes. Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it. It shares no source with the GPU library.
 *
 * Forward (per view, per pixel), following Eq. (1), (2), (3) and (5):
 *   1. enumerate every triangle whose interior covers the pixel centre
 *      (the fragments f = (b_f, D_f, t_f) of Eq. (1));
 *   2. sort the fragments by the packed key K = (depth bits << 32) | tri;
 *   3. walk them front to back; the first fragment whose draw passes its
 *      opacity test is the winner f* (stochastic mode: u_f < alpha_f, the
 *      threshold test of Eq. (5); threshold mode: opacity logit > 0, Eq. (3));
 *   4. colour = the winner's decoded RGB (Eq. (2)), or the background.
 * Backward: the likelihood-ratio estimator of Eq. (8) with the score values
 * of Eq. (9) (Supplement Algorithm A1, part 2), plus the all-adjacent-pixel-
 * pairs edge term of Section 3.2, chained to world-space vertices. All
 * gradient accumulation is in double precision.
 *
 * Everything up to and including the mask decision follows one float32
 * operation sequence (explicit fmaf, no contraction, correctly rounded
 * division, an own exp), so that the decision is reproducible bit for bit.
 */
#ifndef SOUP_ORACLE_H
#define SOUP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t T, G, C, n_layers;
    const int32_t* dims;      /* [n_layers+1], dims[0]==C, dims[n_layers]==4 */
    const float* verts;       /* [T,3,3] world positions */
    const float* feats;       /* [T,G,G,C] feature grid, texel [t][iy][ix][c] */
    const float* mlp;         /* W0[d1][d0], b0[d1], W1[d2][d1], b1, ... */
} orc_scene;

typedef struct {
    int32_t W, H;
    uint32_t view_id;
    const float* M;           /* [4,4] row-major, clip = M @ [x,y,z,1] */
} orc_view;

typedef struct {
    uint64_t seed;            /* Philox key (lo, hi) */
    uint32_t step;            /* fourth counter word */
    int32_t mode;             /* 0 stochastic masking, 1 threshold (Eq. 3) */
    float background[3];
    int32_t edge_pairs;       /* 0 all pairs, 1 pairs whose triangle id changes, 2 none */
    float near_w;             /* cull triangles with any clip w below this */
    int32_t analysis;         /* backward only: 1 = float64, unsnapped evaluation */
} orc_opts;

typedef struct {
    int64_t covered_pixels;      /* pixels with at least one fragment */
    int64_t covering_fragments;  /* all fragments */
    int64_t decodes;             /* fragments whose opacity the walk evaluates */
    int64_t winners;             /* pixels where some fragment passes */
    int64_t front_fragments;     /* fragments in front of the winner (or all, for background) */
} orc_stats;

/* Forward over the whole view. vis [H*W], color [H*W*3], logp [H*W] (may be
 * NULL), stats (may be NULL). Returns 0, or -1 on invalid arguments. */
int orc_forward(const orc_scene* s, const orc_view* v, const orc_opts* o,
                uint64_t* vis, float* color, double* logp, orc_stats* st);

/* Backward over the whole view. vis/color must be this oracle's own forward
 * output for the same inputs. grad_logp may be NULL (no score term).
 * Gradients are ADDED to g_verts [T*9], g_feats [T*G*G*C], g_mlp [n_params]. */
int orc_backward(const orc_scene* s, const orc_view* v, const orc_opts* o,
                 const uint64_t* vis, const float* color,
                 const float* grad_color, const float* grad_logp,
                 double* g_verts, double* g_feats, double* g_mlp);

/* Forward at n listed pixels xy [n,2] = (x, y), by brute force over every
 * triangle. Outputs are per listed pixel. */
int orc_forward_pixels(const orc_scene* s, const orc_view* v, const orc_opts* o,
                       int64_t n, const int32_t* xy,
                       uint64_t* vis, float* color, double* logp);

/* Backward when the upstream gradients are zero everywhere except at the n
 * listed (distinct) pixels: grad_color [n,3], grad_logp [n] (may be NULL).
 * Adds the colour, score and edge contributions of exactly those gradients. */
int orc_backward_pixels(const orc_scene* s, const orc_view* v, const orc_opts* o,
                        int64_t n, const int32_t* xy,
                        const float* grad_color, const float* grad_logp,
                        double* g_verts, double* g_feats, double* g_mlp);

/* One pixel in detail: its sorted fragments (up to cap), their opacity,
 * opacity logit, draw u and score-path logit gradient per unit grad_logp
 * (0 for fragments behind the winner). Returns the fragment count; *winner
 * is the winner's position in the list or -1. */
int orc_pixel_fragments(const orc_scene* s, const orc_view* v, const orc_opts* o,
                        int32_t x, int32_t y, int32_t cap,
                        uint32_t* tri, uint64_t* key, float* alpha, float* o3,
                        float* u, double* dlogit, int32_t* winner);

/* float64, unsnapped colour of triangle tri at pixel centre (x, y), ignoring
 * visibility: rgb[3] and alpha. Returns 0 if the triangle setup culls it. */
int orc_color_f64(const orc_scene* s, const orc_view* v, const orc_opts* o,
                  int32_t tri, int32_t x, int32_t y, double* rgb, double* alpha);

/* ------------------------------------------------------------------------- */
/* Paper form (Section 3.3; Supplement B.3, B.6): multi-resolution mesh-colour */
/* texture, opacity outside the MLP, deferred MLP with spherical harmonics.   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t T;
    int32_t R;                /* finest texture level: n = 2^R segments per edge */
    const float* verts;       /* [T,3,3] */
    const float* tex;         /* [T, V(R), 8]: 7 colour features, then the opacity, in [0,1] */
    const float* mlp;         /* W0[16][16], b0[16], W1[16][16], b1[16], W2[3][16], b2[3] */
} orc_pscene;

/* Grid vertices of level R: (2^(R-1) + 1)(2^R + 1) = (n + 1)(n + 2) / 2. */
int orc_mc_count(int R);
/* The contract lookup: grid vertices (row-major indices) and weights of the
 * micro-triangle of level R containing perspective-correct barycentrics (b1, b2). */
int orc_mc_lookup(int R, float b1, float b2, int32_t idx[3], float w[3]);
/* tex [T, V(Rmax), 8] = sigmoid(sum of the learnable levels Rmin..Rtop
 * (Rtop <= Rmax) sampled at the level-Rmax grid's vertices);
 * raw[l] = [T, V(Rmin + l), 8]. */
int orc_mc_assemble(int T, int Rmin, int Rtop, int Rmax, const float* const* raw, float* tex);
/* Adds d loss / d raw[l] (float64) given tex and d loss / d tex. */
int orc_mc_assemble_bwd(int T, int Rmin, int Rtop, int Rmax, const float* tex, const float* grad_tex,
                        double* const* grad_raw);
/* The 9 real spherical harmonics of degree <= 2 of a unit vector (float32). */
void orc_sh2(const float d[3], float out[9]);
int orc_pmlp_params(void);
/* Unit view direction through the centre of pixel (x, y) (float32). */
int orc_view_dir(const orc_view* v, const float* Minv, int32_t x, int32_t y, float d[3]);
/* Forward / backward of the paper form; Minv = this view's inverse
 * view-projection [4,4] (row-major). Gradients are ADDED (g_tex [T,V,8]). */
int orc_pforward(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o,
                 uint64_t* vis, float* color, double* logp, orc_stats* st);
int orc_pbackward(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o,
                  const uint64_t* vis, const float* color, const float* grad_color, const float* grad_logp,
                  double* g_verts, double* g_tex, double* g_mlp);
/* The same at a list of pixels xy [n,2] of one view (distinct for the
 * backward, whose grad_color [n,3] and grad_logp [n] belong to them). */
int orc_pforward_pixels(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o, int64_t n,
                        const int32_t* xy, uint64_t* vis, float* color, double* logp);
int orc_pbackward_pixels(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o, int64_t n,
                         const int32_t* xy, const float* grad_color, const float* grad_logp, double* g_verts,
                         double* g_tex, double* g_mlp);
int orc_pcolor_f64(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o,
                   int32_t tri, int32_t x, int32_t y, double* rgb, double* alpha);

/* Contract pieces, exposed for their own tests. */
float orc_exp(float x);
float orc_sigmoid(float x);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float orc_uniform(uint64_t seed, uint32_t pixel, uint32_t tri, uint32_t view_id, uint32_t step);
/* Number of triangles a setup would keep (not culled) in this view. */
int64_t orc_count_valid(const orc_scene* s, const orc_view* v, const orc_opts* o);
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
