/*
 * CPU oracle for the triangle-soup rasterization step (DiffSoup,
 * arXiv 2603.27151). TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the product never does.
 *
 * Plain C, no SIMD intrinsics, built with -ffp-contract=off. Each function
 * names the passage of the paper it follows. Where the paper is silent, the
 * reading taken is stated at the place it is used.
 *
 * Float32 contract (identical operation sequence in both implementations,
 * written independently): vertex transform, perspective divide, snap to
 * 1/256 px, integer edge functions, screen barycentrics, depth, perspective-
 * correct barycentrics, bilinear feature fetch, MLP, sigmoid, Philox draw,
 * mask decision. Everything after the decision (colour output aside) is
 * evaluated in double precision.
 */
#include "soup_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXW 128            /* widest MLP layer supported by the oracle */
#define MAXL 8              /* deepest MLP supported by the oracle */
#define SNAP 256            /* subpixel steps per pixel */
#define GUARD 16777216.0f   /* |snapped coordinate| limit, 2^24 */
#define BG_KEY 0xFFFFFFFFFFFFFFFFull

/* ------------------------------------------------------------------------- */
/* Contract scalar functions                                                   */
/* ------------------------------------------------------------------------- */

/* exp by Cody-Waite reduction x = n ln2 + r (ln2 split into a 17-bit head and
 * a float tail so n*head is exact) and the degree-7 Taylor polynomial of e^r
 * in Horner form, scaled by 2^n built from its exponent bits. Used instead of
 * the C library's exp so that the sigmoid, and therefore the mask decision,
 * is reproducible bit for bit. */
float orc_exp(float x)
{
    const float log2e = 0x1.715476p+0f;   /* log2(e) rounded to float */
    const float ln2_hi = 0x1.62e4p-1f;    /* ln 2 truncated to 17 significant bits */
    const float ln2_lo = 0x1.7f7d1cp-20f; /* ln 2 - ln2_hi rounded to float */
    if (x != x) return x;
    if (x > 88.0f) return INFINITY;
    if (x < -87.0f) return 0.0f;
    float n = rintf(x * log2e);
    float r = fmaf(-n, ln2_hi, x);
    r = fmaf(-n, ln2_lo, r);
    float p = 1.0f / 5040.0f;             /* 1/7! */
    p = fmaf(p, r, 1.0f / 720.0f);        /* 1/6! */
    p = fmaf(p, r, 1.0f / 120.0f);        /* 1/5! */
    p = fmaf(p, r, 1.0f / 24.0f);         /* 1/4! */
    p = fmaf(p, r, 1.0f / 6.0f);          /* 1/3! */
    p = fmaf(p, r, 0.5f);                 /* 1/2! */
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    int32_t e = (int32_t)n + 127;         /* n in [-126, 127] here */
    uint32_t bits = (uint32_t)e << 23;
    float scale;
    memcpy(&scale, &bits, 4);
    return p * scale;
}

float orc_sigmoid(float x)
{
    return 1.0f / (1.0f + orc_exp(-x));
}

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplies with the published multipliers, a Weyl key schedule
 * with the published increments. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The per-fragment threshold tau_f of Eq. (5): one independent uniform per
 * fragment. A fragment is one (pixel, triangle) pair, so the counter is
 * (pixel index y*W+x in its view, triangle, view id, step). u = top 24 bits
 * of the first output word times 2^-24, in [0, 1 - 2^-24]. */
float orc_uniform(uint64_t seed, uint32_t pixel, uint32_t tri, uint32_t view_id, uint32_t step)
{
    uint32_t ctr[4] = {pixel, tri, view_id, step};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    return (float)(r[0] >> 8) * 0x1p-24f;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Triangle setup (Section 3.1: triangles transformed to camera space and      */
/* rasterized; Supplement B.6: 9 floats per triangle)                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    int valid;
    int32_t X[3], Y[3];      /* snapped screen position, 1/256 px, y down */
    float z01[3], iw[3];     /* depth in [0,1] (unclamped) and 1/w per vertex */
    float cx[3], cy[3], cw[3];
    double sx[3], sy[3];     /* unsnapped screen position (float value) */
    int64_t A;               /* |2 x signed area|, 1/256^2 px^2 */
    int sgn;                 /* orientation: edge functions multiplied by sgn */
    int x0, x1, y0, y1;      /* inclusive pixel bounding box, clipped to the view */
} tri_setup;

static int64_t edge_i64(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py)
{
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

static int64_t floor_div(int64_t a, int64_t b)   /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static int64_t ceil_div(int64_t a, int64_t b)    /* b > 0 */
{
    return -floor_div(-a, b);
}

/* Readings where the paper is silent: pixel centres at +0.5 (the pixel-centre
 * sample of Eq. (1)); 8 subpixel bits; no clipping, a triangle with any vertex
 * at w < near is culled; degenerate (zero snapped area) and non-finite
 * triangles are culled; both orientations are kept (no backface culling). */
static void setup_triangle(const orc_scene* s, const orc_view* v, const orc_opts* o,
                           int t, tri_setup* out)
{
    memset(out, 0, sizeof(*out));
    const float* M = v->M;
    const float hw = 0.5f * (float)v->W, hh = 0.5f * (float)v->H;
    for (int i = 0; i < 3; ++i) {
        const float* p = s->verts + ((size_t)t * 3 + i) * 3;
        float c[4];
        for (int j = 0; j < 4; ++j) {
            float a = M[j * 4 + 3];
            a = fmaf(M[j * 4 + 0], p[0], a);
            a = fmaf(M[j * 4 + 1], p[1], a);
            a = fmaf(M[j * 4 + 2], p[2], a);
            c[j] = a;
        }
        if (!(c[3] >= o->near_w)) return;            /* also rejects NaN */
        if (!isfinite(c[0]) || !isfinite(c[1]) || !isfinite(c[2]) || !isfinite(c[3])) return;
        float iw = 1.0f / c[3];
        float sx = fmaf(c[0] * iw, hw, hw);
        float sy = fmaf(-(c[1] * iw), hh, hh);
        float z01 = fmaf(c[2] * iw, 0.5f, 0.5f);
        float fx = sx * 256.0f, fy = sy * 256.0f;
        if (!(fabsf(fx) <= GUARD) || !(fabsf(fy) <= GUARD)) return;
        if (!isfinite(z01)) return;
        out->X[i] = (int32_t)rintf(fx);
        out->Y[i] = (int32_t)rintf(fy);
        out->z01[i] = z01;
        out->iw[i] = iw;
        out->cx[i] = c[0]; out->cy[i] = c[1]; out->cw[i] = c[3];
        out->sx[i] = sx; out->sy[i] = sy;
    }
    int64_t A = edge_i64(out->X[0], out->Y[0], out->X[1], out->Y[1], out->X[2], out->Y[2]);
    if (A == 0) return;
    out->sgn = A > 0 ? 1 : -1;
    out->A = A > 0 ? A : -A;
    int32_t mnx = out->X[0], mxx = out->X[0], mny = out->Y[0], mxy = out->Y[0];
    for (int i = 1; i < 3; ++i) {
        if (out->X[i] < mnx) mnx = out->X[i];
        if (out->X[i] > mxx) mxx = out->X[i];
        if (out->Y[i] < mny) mny = out->Y[i];
        if (out->Y[i] > mxy) mxy = out->Y[i];
    }
    /* pixel x is a candidate when mnx <= 256x+128 <= mxx */
    int64_t x0 = ceil_div((int64_t)mnx - SNAP / 2, SNAP), x1 = floor_div((int64_t)mxx - SNAP / 2, SNAP);
    int64_t y0 = ceil_div((int64_t)mny - SNAP / 2, SNAP), y1 = floor_div((int64_t)mxy - SNAP / 2, SNAP);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > v->W - 1) x1 = v->W - 1;
    if (y1 > v->H - 1) y1 = v->H - 1;
    if (x0 > x1 || y0 > y1) return;
    out->x0 = (int)x0; out->x1 = (int)x1; out->y0 = (int)y0; out->y1 = (int)y1;
    out->valid = 1;
}

/* ------------------------------------------------------------------------- */
/* Fragments (Eq. (1)): barycentrics b_f, depth D_f, triangle t_f               */
/* ------------------------------------------------------------------------- */

typedef struct {
    uint32_t tri;
    uint64_t key;            /* (depth bits << 32) | tri */
    int64_t E[3];            /* orientation-normalised edge functions, >= 0 */
    float beta[3];           /* screen-space barycentrics */
    float b1, b2;            /* perspective-correct barycentrics of v1, v2 */
    int ix, iy;              /* texture cell */
    float fx, fy;            /* position inside the cell */
} frag_t;

/* Edge i runs from vertex i+1 to vertex i+2. A pixel centre exactly on an
 * edge belongs to the triangle when the edge's direction (after orientation
 * normalisation) has dy < 0, or dy == 0 and dx > 0: the tie is broken as if
 * the sample sat an infinitesimal step along (1, +eps), so a centre on an edge
 * shared by two triangles, or on a vertex of a closed fan, is covered once. */
static int owns_edge(const tri_setup* t, int i)
{
    int a = (i + 1) % 3, b = (i + 2) % 3;
    int64_t dx = (int64_t)t->sgn * ((int64_t)t->X[b] - t->X[a]);
    int64_t dy = (int64_t)t->sgn * ((int64_t)t->Y[b] - t->Y[a]);
    return dy < 0 || (dy == 0 && dx > 0);
}

static int make_fragment(const tri_setup* t, uint32_t tri, int x, int y, int G, frag_t* f)
{
    if (!t->valid || x < t->x0 || x > t->x1 || y < t->y0 || y > t->y1) return 0;
    int64_t px = (int64_t)SNAP * x + SNAP / 2, py = (int64_t)SNAP * y + SNAP / 2;
    for (int i = 0; i < 3; ++i) {
        int a = (i + 1) % 3, b = (i + 2) % 3;
        int64_t e = t->sgn * edge_i64(t->X[a], t->Y[a], t->X[b], t->Y[b], px, py);
        if (e < 0 || (e == 0 && !owns_edge(t, i))) return 0;
        f->E[i] = e;
    }
    f->tri = tri;
    float rA = 1.0f / (float)t->A;
    for (int i = 0; i < 3; ++i) f->beta[i] = (float)f->E[i] * rA;
    /* D_f: screen-linear depth, clamped to [+0, 1] (reading: NDC z mapped to
     * [0,1]); its IEEE bits order like the values for non-negative floats. */
    float z = fmaf(f->beta[2], t->z01[2], fmaf(f->beta[1], t->z01[1], f->beta[0] * t->z01[0]));
    if (!(z > 0.0f)) z = 0.0f;
    if (z > 1.0f) z = 1.0f;
    uint32_t zb;
    memcpy(&zb, &z, 4);
    f->key = ((uint64_t)zb << 32) | tri;
    /* perspective-correct barycentrics (reading: attributes are interpolated
     * perspective-correctly, depth screen-linearly) */
    float t0 = f->beta[0] * t->iw[0], t1 = f->beta[1] * t->iw[1], t2 = f->beta[2] * t->iw[2];
    float r = 1.0f / ((t0 + t1) + t2);
    f->b1 = t1 * r;
    f->b2 = t2 * r;
    /* feature grid coordinates: vertex 0 -> texel (0,0), vertex 1 -> (G-1,0),
     * vertex 2 -> (0,G-1) */
    float gm1 = (float)(G - 1);
    float gx = f->b1 * gm1, gy = f->b2 * gm1;
    int ix = (int)floorf(gx), iy = (int)floorf(gy);
    if (ix < 0) ix = 0;
    if (ix > G - 2) ix = G - 2;
    if (iy < 0) iy = 0;
    if (iy > G - 2) iy = G - 2;
    f->ix = ix; f->iy = iy;
    f->fx = gx - (float)ix;
    f->fy = gy - (float)iy;
    return 1;
}

static int cmp_frag(const void* a, const void* b)
{
    uint64_t ka = ((const frag_t*)a)->key, kb = ((const frag_t*)b)->key;
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

/* ------------------------------------------------------------------------- */
/* Neural texture decode (Section 3.3 in the workloads' form: a G x G feature  */
/* grid sampled bilinearly and a shared MLP producing RGB + opacity logit)     */
/* ------------------------------------------------------------------------- */

/* float32 contract decode. act[l] holds the input of layer l (act[0] = the
 * bilinear feature); out[4] = logits (RGB, opacity). */
static void decode_f32(const orc_scene* s, const frag_t* f, float act[MAXL + 1][MAXW])
{
    const int G = s->G, C = s->C;
    const float* T00 = s->feats + (((size_t)f->tri * G + f->iy) * G + f->ix) * C;
    const float* T10 = T00 + C;
    const float* T01 = T00 + (size_t)G * C;
    const float* T11 = T01 + C;
    float fx = f->fx, fy = f->fy;
    float w00 = (1.0f - fx) * (1.0f - fy), w10 = fx * (1.0f - fy);
    float w01 = (1.0f - fx) * fy, w11 = fx * fy;
    for (int c = 0; c < C; ++c)
        act[0][c] = fmaf(w11, T11[c], fmaf(w01, T01[c], fmaf(w10, T10[c], w00 * T00[c])));
    const float* p = s->mlp;
    for (int l = 0; l < s->n_layers; ++l) {
        int din = s->dims[l], dout = s->dims[l + 1];
        const float* W = p;
        const float* b = p + (size_t)dout * din;
        for (int j = 0; j < dout; ++j) {
            float h = b[j];
            for (int k = 0; k < din; ++k) h = fmaf(W[j * din + k], act[l][k], h);
            if (l < s->n_layers - 1) h = h > 0.0f ? h : 0.0f;   /* hidden ReLU */
            act[l + 1][j] = h;
        }
        p += (size_t)dout * din + dout;
    }
}

/* Mask test of one fragment: Eq. (5) (u < alpha) or Eq. (3) (logit > 0, read
 * as alpha > 0.5 without rounding the sigmoid). */
static int passes(const orc_view* v, const orc_opts* o, int x, int y, uint32_t tri, float o3,
                  float* alpha_out, float* u_out)
{
    float a = orc_sigmoid(o3);
    if (alpha_out) *alpha_out = a;
    if (o->mode == 1) {
        if (u_out) *u_out = 0.5f;
        return o3 > 0.0f;
    }
    float u = orc_uniform(o->seed, (uint32_t)(y * v->W + x), tri, v->view_id, o->step);
    if (u_out) *u_out = u;
    return u < a;
}

/* ------------------------------------------------------------------------- */
/* Per-view context: setups and per-pixel candidate lists                       */
/* ------------------------------------------------------------------------- */

typedef struct {
    const orc_scene* s;
    const orc_view* v;
    const orc_opts* o;
    tri_setup* ts;           /* [T] */
    int64_t* start;          /* [H*W+1] CSR over candidates, or NULL for brute force */
    uint32_t* cand;
    uint32_t* valid_list;    /* triangles kept by setup (brute force) */
    int64_t n_valid;
} view_ctx;

static int scene_ok(const orc_scene* s)
{
    if (!s || s->T < 0 || s->G < 2 || s->C < 1 || s->C > MAXW || s->n_layers < 1 ||
        s->n_layers > MAXL || !s->dims)
        return 0;
    if (s->dims[0] != s->C || s->dims[s->n_layers] != 4) return 0;
    for (int l = 0; l <= s->n_layers; ++l)
        if (s->dims[l] < 1 || s->dims[l] > MAXW) return 0;
    return 1;
}

static int ctx_init(view_ctx* c, const orc_scene* s, const orc_view* v, const orc_opts* o, int csr)
{
    memset(c, 0, sizeof(*c));
    if (!scene_ok(s) || !v || !o || v->W <= 0 || v->H <= 0) return -1;
    c->s = s; c->v = v; c->o = o;
    c->ts = (tri_setup*)calloc((size_t)(s->T > 0 ? s->T : 1), sizeof(tri_setup));
    c->valid_list = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(s->T > 0 ? s->T : 1));
    #pragma omp parallel for schedule(static)
    for (int t = 0; t < s->T; ++t) setup_triangle(s, v, o, t, &c->ts[t]);
    for (int t = 0; t < s->T; ++t)
        if (c->ts[t].valid) c->valid_list[c->n_valid++] = (uint32_t)t;
    if (csr) {
        size_t npix = (size_t)v->W * v->H;
        c->start = (int64_t*)calloc(npix + 1, sizeof(int64_t));
        for (int t = 0; t < s->T; ++t) {
            const tri_setup* q = &c->ts[t];
            if (!q->valid) continue;
            for (int y = q->y0; y <= q->y1; ++y)
                for (int x = q->x0; x <= q->x1; ++x) c->start[(size_t)y * v->W + x + 1] += 1;
        }
        for (size_t i = 0; i < npix; ++i) c->start[i + 1] += c->start[i];
        c->cand = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(c->start[npix] > 0 ? c->start[npix] : 1));
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * npix);
        memcpy(fill, c->start, sizeof(int64_t) * npix);
        for (int t = 0; t < s->T; ++t) {
            const tri_setup* q = &c->ts[t];
            if (!q->valid) continue;
            for (int y = q->y0; y <= q->y1; ++y)
                for (int x = q->x0; x <= q->x1; ++x) c->cand[fill[(size_t)y * v->W + x]++] = (uint32_t)t;
        }
        free(fill);
    }
    return 0;
}

static void ctx_free(view_ctx* c)
{
    free(c->ts); free(c->start); free(c->cand); free(c->valid_list);
}

typedef struct { frag_t* f; int n, cap; } frag_buf;

static void buf_push(frag_buf* b, const frag_t* f)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 64;
        b->f = (frag_t*)realloc(b->f, sizeof(frag_t) * (size_t)b->cap);
    }
    b->f[b->n++] = *f;
}

/* All fragments of pixel (x, y), sorted front to back by key. */
static void pixel_fragments(const view_ctx* c, int x, int y, frag_buf* b)
{
    b->n = 0;
    frag_t f;
    if (c->start) {
        size_t p = (size_t)y * c->v->W + x;
        for (int64_t i = c->start[p]; i < c->start[p + 1]; ++i) {
            uint32_t t = c->cand[i];
            if (make_fragment(&c->ts[t], t, x, y, c->s->G, &f)) buf_push(b, &f);
        }
    } else {
        for (int64_t i = 0; i < c->n_valid; ++i) {
            uint32_t t = c->valid_list[i];
            if (make_fragment(&c->ts[t], t, x, y, c->s->G, &f)) buf_push(b, &f);
        }
    }
    qsort(b->f, (size_t)b->n, sizeof(frag_t), cmp_frag);
}

/* ------------------------------------------------------------------------- */
/* Forward                                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int winner;              /* index in the sorted list, -1 = background */
    uint64_t key;
    float rgb[3];
    double logp;
    int decodes;
} pixel_result;

/* Front-to-back walk: the first fragment passing its test is the argmin of
 * Eq. (5) over passing fragments. log p(f*) of Eq. (6)/(A2) is accumulated
 * along the way; for the background (no fragment passes) it is the log of the
 * probability that every fragment fails. */
static void pixel_forward(const view_ctx* c, int x, int y, const frag_buf* b, pixel_result* r)
{
    float act[MAXL + 1][MAXW];
    r->winner = -1;
    r->key = BG_KEY;
    r->rgb[0] = c->o->background[0];
    r->rgb[1] = c->o->background[1];
    r->rgb[2] = c->o->background[2];
    r->logp = 0.0;
    r->decodes = 0;
    const int L = c->s->n_layers;
    for (int i = 0; i < b->n; ++i) {
        decode_f32(c->s, &b->f[i], act);
        r->decodes++;
        float alpha;
        int pass = passes(c->v, c->o, x, y, b->f[i].tri, act[L][3], &alpha, NULL);
        if (pass) {
            r->winner = i;
            r->key = b->f[i].key;
            for (int k = 0; k < 3; ++k) r->rgb[k] = orc_sigmoid(act[L][k]);
            if (c->o->mode == 0) r->logp += log((double)alpha);
            return;
        }
        if (c->o->mode == 0) r->logp += log1p(-(double)alpha);
    }
}

int orc_forward(const orc_scene* s, const orc_view* v, const orc_opts* o,
                uint64_t* vis, float* color, double* logp, orc_stats* st)
{
    view_ctx c;
    if (ctx_init(&c, s, v, o, 1) != 0) return -1;
    int64_t cov = 0, frags = 0, dec = 0, win = 0, front = 0;
    #pragma omp parallel reduction(+ : cov, frags, dec, win, front)
    {
        frag_buf b = {0};
        #pragma omp for schedule(dynamic, 4)
        for (int y = 0; y < v->H; ++y) {
            for (int x = 0; x < v->W; ++x) {
                size_t p = (size_t)y * v->W + x;
                pixel_fragments(&c, x, y, &b);
                pixel_result r;
                pixel_forward(&c, x, y, &b, &r);
                vis[p] = r.key;
                color[3 * p + 0] = r.rgb[0];
                color[3 * p + 1] = r.rgb[1];
                color[3 * p + 2] = r.rgb[2];
                if (logp) logp[p] = r.logp;
                cov += b.n > 0;
                frags += b.n;
                dec += r.decodes;
                win += r.winner >= 0;
                front += r.winner >= 0 ? r.winner : b.n;
            }
        }
        free(b.f);
    }
    if (st) {
        st->covered_pixels = cov;
        st->covering_fragments = frags;
        st->decodes = dec;
        st->winners = win;
        st->front_fragments = front;
    }
    ctx_free(&c);
    return 0;
}

int orc_forward_pixels(const orc_scene* s, const orc_view* v, const orc_opts* o,
                       int64_t n, const int32_t* xy, uint64_t* vis, float* color, double* logp)
{
    view_ctx c;
    if (ctx_init(&c, s, v, o, 0) != 0) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (xy[2 * i] < 0 || xy[2 * i] >= v->W || xy[2 * i + 1] < 0 || xy[2 * i + 1] >= v->H) {
            ctx_free(&c);
            return -1;
        }
    #pragma omp parallel
    {
        frag_buf b = {0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            int x = xy[2 * i], y = xy[2 * i + 1];
            pixel_fragments(&c, x, y, &b);
            pixel_result r;
            pixel_forward(&c, x, y, &b, &r);
            vis[i] = r.key;
            for (int k = 0; k < 3; ++k) color[3 * i + k] = r.rgb[k];
            if (logp) logp[i] = r.logp;
        }
        free(b.f);
    }
    ctx_free(&c);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Backward                                                                     */
/* ------------------------------------------------------------------------- */

static void atomic_add(double* p, double v)
{
    #pragma omp atomic
    *p += v;
}

/* Geometry of a fragment for the backward: barycentrics and their
 * derivatives with respect to the screen positions of the three vertices.
 * The forward snaps positions to 1/256 px; its derivative is taken as the
 * identity (straight-through), evaluated at the snapped positions. In the
 * analysis mode everything is unsnapped float64. */
typedef struct {
    double vx[3], vy[3];     /* vertex screen positions, px */
    double px, py;           /* pixel centre, px */
    double beta[3];
    double iw[3];
} frag_geom;

static double edge_d(double ax, double ay, double bx, double by, double px, double py)
{
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

static void geom_of(const view_ctx* c, const tri_setup* t, int x, int y, frag_geom* g)
{
    for (int i = 0; i < 3; ++i) {
        if (c->o->analysis) {
            g->vx[i] = t->sx[i];
            g->vy[i] = t->sy[i];
        } else {
            g->vx[i] = (double)t->X[i] / SNAP;
            g->vy[i] = (double)t->Y[i] / SNAP;
        }
        g->iw[i] = t->iw[i];
    }
    g->px = x + 0.5;
    g->py = y + 0.5;
    double a = edge_d(g->vx[0], g->vy[0], g->vx[1], g->vy[1], g->vx[2], g->vy[2]);
    for (int i = 0; i < 3; ++i) {
        int p = (i + 1) % 3, q = (i + 2) % 3;
        g->beta[i] = edge_d(g->vx[p], g->vy[p], g->vx[q], g->vy[q], g->px, g->py) / a;
    }
}

/* d beta_i / d (vx_j, vy_j): beta_i = e_i / a with e_i the edge function of
 * the edge opposite vertex i and a = e_0 + e_1 + e_2 (twice the signed area). */
static void dbeta(const frag_geom* g, double d[3][3][2])
{
    double a = edge_d(g->vx[0], g->vy[0], g->vx[1], g->vy[1], g->vx[2], g->vy[2]);
    /* da/dv_j: the edge function of (v_{j+1}, v_{j+2}) differentiated in its
     * third argument is (-(b.y-a.y), b.x-a.x); by the cyclic symmetry of a,
     * da/dv_j = (v_{j+1}.y - v_{j+2}.y, v_{j+2}.x - v_{j+1}.x). */
    double da[3][2];
    for (int j = 0; j < 3; ++j) {
        int p = (j + 1) % 3, q = (j + 2) % 3;
        da[j][0] = g->vy[p] - g->vy[q];
        da[j][1] = g->vx[q] - g->vx[p];
    }
    for (int i = 0; i < 3; ++i) {
        int p = (i + 1) % 3, q = (i + 2) % 3;   /* e_i = edge(v_p, v_q, pixel) */
        double de[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        /* d edge(a,b,P)/da = (b.y - P.y, P.x - b.x); d/db = (P.y - a.y, a.x - P.x) */
        de[p][0] = g->vy[q] - g->py;
        de[p][1] = g->px - g->vx[q];
        de[q][0] = g->py - g->vy[p];
        de[q][1] = g->vx[p] - g->px;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 2; ++k) d[i][j][k] = (de[j][k] - g->beta[i] * da[j][k]) / a;
    }
}

/* float64 decode used by the analysis mode: the same function as decode_f32
 * evaluated in double with the cell (ix, iy) given. */
static void decode_f64_at(const orc_scene* s, uint32_t tri, int ix, int iy, double fx, double fy,
                          double act[MAXL + 1][MAXW])
{
    const int G = s->G, C = s->C;
    const float* T00 = s->feats + (((size_t)tri * G + iy) * G + ix) * C;
    const float* T10 = T00 + C;
    const float* T01 = T00 + (size_t)G * C;
    const float* T11 = T01 + C;
    for (int c = 0; c < C; ++c)
        act[0][c] = (1 - fx) * (1 - fy) * T00[c] + fx * (1 - fy) * T10[c] + (1 - fx) * fy * T01[c] +
                    fx * fy * T11[c];
    const float* p = s->mlp;
    for (int l = 0; l < s->n_layers; ++l) {
        int din = s->dims[l], dout = s->dims[l + 1];
        const float* W = p;
        const float* b = p + (size_t)dout * din;
        for (int j = 0; j < dout; ++j) {
            double h = b[j];
            for (int k = 0; k < din; ++k) h += (double)W[j * din + k] * act[l][k];
            if (l < s->n_layers - 1) h = h > 0 ? h : 0;
            act[l + 1][j] = h;
        }
        p += (size_t)dout * din + dout;
    }
}

static double sigmoid_d(double x) { return 1.0 / (1.0 + exp(-x)); }

typedef struct {
    double* g_verts_screen;  /* [T][3][3]: d/d(sx, sy, iw) of each vertex */
    double* g_feats;
    double* g_mlp;
} grad_out;

/* Back-propagate logit gradients dout[4] of one fragment through the MLP and
 * the bilinear fetch. With want_pos, also through the barycentrics to the
 * screen positions and 1/w of the triangle's vertices (colour path of
 * Algorithm A1, 2(a)); the opacity score path stops at the texture (the
 * score term carries opacity gradients only, Section 3.2). */
static void backprop_at(const view_ctx* c, const frag_t* f, int x, int y, const double dout_in[4],
                        int want_pos, grad_out* go)
{
    const orc_scene* s = c->s;
    const int L = s->n_layers, G = s->G, C = s->C;
    const tri_setup* t = &c->ts[f->tri];
    frag_geom g;
    geom_of(c, t, x, y, &g);

    /* perspective-correct barycentrics and texture position, float64 */
    double tt[3], S = 0;
    for (int i = 0; i < 3; ++i) { tt[i] = g.beta[i] * g.iw[i]; S += tt[i]; }
    double b[3] = {tt[0] / S, tt[1] / S, tt[2] / S};
    double gx = b[1] * (G - 1), gy = b[2] * (G - 1);
    int ix = f->ix, iy = f->iy;      /* the forward's cell */
    double fx = gx - ix, fy = gy - iy;

    /* forward activations at which the derivative is taken */
    double act[MAXL + 1][MAXW];
    if (c->o->analysis) {
        decode_f64_at(s, f->tri, ix, iy, fx, fy, act);
    } else {
        float a32[MAXL + 1][MAXW];
        decode_f32(s, f, a32);
        for (int l = 0; l <= L; ++l)
            for (int k = 0; k < s->dims[l]; ++k) act[l][k] = a32[l][k];
    }

    /* MLP backward */
    double delta[MAXW], prev[MAXW];
    for (int j = 0; j < 4; ++j) delta[j] = dout_in[j];
    /* parameter offsets per layer */
    size_t off[MAXL];
    {
        size_t o = 0;
        for (int l = 0; l < L; ++l) { off[l] = o; o += (size_t)s->dims[l + 1] * s->dims[l] + s->dims[l + 1]; }
    }
    for (int l = L - 1; l >= 0; --l) {
        int din = s->dims[l], dout = s->dims[l + 1];
        const float* W = s->mlp + off[l];
        double* gW = go->g_mlp + off[l];
        double* gb = gW + (size_t)dout * din;
        for (int j = 0; j < dout; ++j) {
            if (delta[j] == 0.0) continue;
            atomic_add(&gb[j], delta[j]);
            for (int k = 0; k < din; ++k)
                if (act[l][k] != 0.0) atomic_add(&gW[(size_t)j * din + k], delta[j] * act[l][k]);
        }
        for (int k = 0; k < din; ++k) {
            double acc = 0;
            for (int j = 0; j < dout; ++j) acc += (double)W[j * din + k] * delta[j];
            /* ReLU gate of the hidden layer feeding this one */
            if (l > 0 && !(act[l][k] > 0)) acc = 0;
            prev[k] = acc;
        }
        memcpy(delta, prev, sizeof(double) * (size_t)din);
    }
    /* delta = d loss / d feature (bilinear output) */
    const float* T00 = s->feats + (((size_t)f->tri * G + iy) * G + ix) * C;
    const float* T10 = T00 + C;
    const float* T01 = T00 + (size_t)G * C;
    const float* T11 = T01 + C;
    double* g00 = go->g_feats + (((size_t)f->tri * G + iy) * G + ix) * C;
    double* g10 = g00 + C;
    double* g01 = g00 + (size_t)G * C;
    double* g11 = g01 + C;
    double dfx = 0, dfy = 0;
    for (int k = 0; k < C; ++k) {
        double d = delta[k];
        if (d == 0.0) continue;
        atomic_add(&g00[k], d * (1 - fx) * (1 - fy));
        atomic_add(&g10[k], d * fx * (1 - fy));
        atomic_add(&g01[k], d * (1 - fx) * fy);
        atomic_add(&g11[k], d * fx * fy);
        dfx += d * ((1 - fy) * ((double)T10[k] - T00[k]) + fy * ((double)T11[k] - T01[k]));
        dfy += d * ((1 - fx) * ((double)T01[k] - T00[k]) + fx * ((double)T11[k] - T10[k]));
    }
    if (!want_pos) return;

    /* texture position -> perspective-correct barycentrics -> screen
     * barycentrics and 1/w -> vertex screen positions */
    double db[3] = {0.0, dfx * (G - 1), dfy * (G - 1)};
    double dot = db[0] * b[0] + db[1] * b[1] + db[2] * b[2];
    double dtt[3];
    for (int i = 0; i < 3; ++i) dtt[i] = (db[i] - dot) / S;      /* b_i = tt_i / S */
    double dbeta_v[3], diw[3];
    for (int i = 0; i < 3; ++i) {
        dbeta_v[i] = dtt[i] * g.iw[i];
        diw[i] = dtt[i] * g.beta[i];
    }
    double D[3][3][2];
    dbeta(&g, D);
    double* gv = go->g_verts_screen + (size_t)f->tri * 9;
    for (int j = 0; j < 3; ++j) {
        double sx = 0, sy = 0;
        for (int i = 0; i < 3; ++i) { sx += dbeta_v[i] * D[i][j][0]; sy += dbeta_v[i] * D[i][j][1]; }
        atomic_add(&gv[3 * j + 0], sx);
        atomic_add(&gv[3 * j + 1], sy);
        atomic_add(&gv[3 * j + 2], diw[j]);
    }
}

/* Algorithm A1, part 2, for one pixel: (a) colour gradient of the winner;
 * (b) score term g_L * dlog p(f*)/dalpha_f' (Eq. (9)) for the winner and every
 * fragment in front of it, pushed through the sigmoid:
 *   winner:  g_L * (1/alpha) * alpha(1-alpha) = g_L (1 - alpha)
 *   in front: g_L * (-1/(1-alpha)) * alpha(1-alpha) = -g_L alpha
 * The score term is an opacity gradient only (Eq. (8), second term; Section
 * 3.2 opens its discussion of visibility discontinuities by noting that the
 * masking gives no motion gradient): for every fragment, the winner
 * included, it reaches the texture and the MLP but not the vertices. Only
 * the winner's colour logits are chained to its vertex positions.
 * Reading for the background (no fragment passes): it is an always-opaque
 * layer behind everything with no parameters, so every fragment is in front. */
static void pixel_backward(const view_ctx* c, int x, int y, const frag_buf* b, uint64_t key_star,
                           const double gC[3], double gL, grad_out* go)
{
    const int L = c->s->n_layers;
    float act[MAXL + 1][MAXW];
    for (int i = 0; i < b->n; ++i) {
        const frag_t* f = &b->f[i];
        if (f->key > key_star) break;                 /* behind the winner: s = 0 */
        decode_f32(c->s, f, act);
        double alpha = orc_sigmoid(act[L][3]);
        double d[4] = {0, 0, 0, 0};
        if (f->key == key_star) {
            for (int k = 0; k < 3; ++k) {
                double rgb = orc_sigmoid(act[L][k]);
                d[k] = gC[k] * rgb * (1.0 - rgb);
            }
            if (c->o->mode == 0) d[3] = gL * (1.0 - alpha);
            if (c->o->analysis) {
                /* analysis mode: sigmoid derivatives from the float64 decode */
                double a64[MAXL + 1][MAXW];
                frag_geom g;
                geom_of(c, &c->ts[f->tri], x, y, &g);
                double tt[3], S = 0;
                for (int k = 0; k < 3; ++k) { tt[k] = g.beta[k] * g.iw[k]; S += tt[k]; }
                double gx = tt[1] / S * (c->s->G - 1), gy = tt[2] / S * (c->s->G - 1);
                decode_f64_at(c->s, f->tri, f->ix, f->iy, gx - f->ix, gy - f->iy, a64);
                for (int k = 0; k < 3; ++k) {
                    double rgb = sigmoid_d(a64[L][k]);
                    d[k] = gC[k] * rgb * (1.0 - rgb);
                }
                if (c->o->mode == 0) d[3] = gL * (1.0 - sigmoid_d(a64[L][3]));
            }
            /* colour logits: through the texture position to the vertices;
             * the score logit: texture and MLP only */
            const double d_col[4] = {d[0], d[1], d[2], 0.0};
            const double d_score[4] = {0.0, 0.0, 0.0, d[3]};
            backprop_at(c, f, x, y, d_col, 1, go);
            if (d[3] != 0.0) backprop_at(c, f, x, y, d_score, 0, go);
            break;
        }
        if (c->o->mode != 0 || gL == 0.0) continue;
        d[3] = -gL * alpha;
        backprop_at(c, f, x, y, d, 0, go);
    }
}

/* Edge term (Section 3.2, extending rasterized edge gradients to every
 * horizontally and vertically adjacent pixel pair of the sampled image).
 * The paper prints no formula; reading: for the pair (a, b = a + e), a box
 * filter across the boundary between the two centres gives
 *   dL/d(boundary displacement along e) = 1/2 (g_a + g_b) . (C_a - C_b),
 * the same sign whichever side the occluder is on. The occluder o is the
 * pixel with the smaller key; the boundary moves with o's surface point, so
 * vertex i of tri(o) receives w * beta_i(o) * e in screen space. */
static void pair_edge(const view_ctx* c, int xa, int ya, int xb, int yb, uint64_t ka, uint64_t kb,
                      const float* Ca, const float* Cb, const double ga[3], const double gb[3], grad_out* go)
{
    if (ka == BG_KEY && kb == BG_KEY) return;
    if (c->o->edge_pairs == 2) return;
    if (c->o->edge_pairs == 1 && ka != BG_KEY && kb != BG_KEY && (uint32_t)ka == (uint32_t)kb) return;
    double w = 0;
    for (int k = 0; k < 3; ++k) w += 0.5 * (ga[k] + gb[k]) * ((double)Ca[k] - (double)Cb[k]);
    if (w == 0.0) return;
    int xo = ka < kb ? xa : xb, yo = ka < kb ? ya : yb;
    uint32_t to = (uint32_t)(ka < kb ? ka : kb);
    frag_geom g;
    geom_of(c, &c->ts[to], xo, yo, &g);
    double ex = xb - xa, ey = yb - ya;
    double* gv = go->g_verts_screen + (size_t)to * 9;
    for (int i = 0; i < 3; ++i) {
        atomic_add(&gv[3 * i + 0], w * g.beta[i] * ex);
        atomic_add(&gv[3 * i + 1], w * g.beta[i] * ey);
    }
}

/* Screen position and 1/w back to world space through the projection
 * (clip = M [x,y,z,1]; s = W/2 (c_x/c_w) + W/2, H/2 - H/2 (c_y/c_w); 1/w). */
static void vertex_chain(const view_ctx* c, const double* gs, double* g_verts)
{
    const orc_scene* s = c->s;
    const float* M = c->v->M;
    const double hw = 0.5 * c->v->W, hh = 0.5 * c->v->H;
    for (int t = 0; t < s->T; ++t) {
        const tri_setup* q = &c->ts[t];
        if (!q->valid) continue;
        for (int i = 0; i < 3; ++i) {
            const double* g = gs + (size_t)t * 9 + 3 * i;
            if (g[0] == 0 && g[1] == 0 && g[2] == 0) continue;
            double cx = q->cx[i], cy = q->cy[i], cw = q->cw[i];
            if (c->o->analysis) {
                /* exact float64 clip coordinates */
                const float* p = s->verts + ((size_t)t * 3 + i) * 3;
                double cc[4];
                for (int j = 0; j < 4; ++j)
                    cc[j] = (double)M[j * 4 + 3] + (double)M[j * 4] * p[0] + (double)M[j * 4 + 1] * p[1] +
                            (double)M[j * 4 + 2] * p[2];
                cx = cc[0]; cy = cc[1]; cw = cc[3];
            }
            double gc[4];
            gc[0] = g[0] * hw / cw;
            gc[1] = -g[1] * hh / cw;
            gc[2] = 0;
            gc[3] = -g[0] * hw * cx / (cw * cw) + g[1] * hh * cy / (cw * cw) - g[2] / (cw * cw);
            for (int k = 0; k < 3; ++k) {
                double acc = 0;
                for (int j = 0; j < 4; ++j) acc += (double)M[j * 4 + k] * gc[j];
                g_verts[(size_t)t * 9 + 3 * i + k] += acc;
            }
        }
    }
}

int orc_backward(const orc_scene* s, const orc_view* v, const orc_opts* o,
                 const uint64_t* vis, const float* color,
                 const float* grad_color, const float* grad_logp,
                 double* g_verts, double* g_feats, double* g_mlp)
{
    view_ctx c;
    if (ctx_init(&c, s, v, o, 1) != 0) return -1;
    grad_out go;
    go.g_verts_screen = (double*)calloc((size_t)(s->T > 0 ? s->T : 1) * 9, sizeof(double));
    go.g_feats = g_feats;
    go.g_mlp = g_mlp;
    const int W = v->W, H = v->H;
    #pragma omp parallel
    {
        frag_buf b = {0};
        #pragma omp for schedule(dynamic, 4)
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                size_t p = (size_t)y * W + x;
                double gC[3] = {grad_color[3 * p], grad_color[3 * p + 1], grad_color[3 * p + 2]};
                double gL = grad_logp ? grad_logp[p] : 0.0;
                if (gC[0] == 0 && gC[1] == 0 && gC[2] == 0 && gL == 0) continue;
                pixel_fragments(&c, x, y, &b);
                pixel_backward(&c, x, y, &b, vis[p], gC, gL, &go);
            }
        }
        free(b.f);
        #pragma omp for schedule(dynamic, 4)
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                size_t a = (size_t)y * W + x;
                double ga[3] = {grad_color[3 * a], grad_color[3 * a + 1], grad_color[3 * a + 2]};
                if (x + 1 < W) {
                    size_t q = a + 1;
                    double gb[3] = {grad_color[3 * q], grad_color[3 * q + 1], grad_color[3 * q + 2]};
                    pair_edge(&c, x, y, x + 1, y, vis[a], vis[q], color + 3 * a, color + 3 * q, ga, gb, &go);
                }
                if (y + 1 < H) {
                    size_t q = a + (size_t)W;
                    double gb[3] = {grad_color[3 * q], grad_color[3 * q + 1], grad_color[3 * q + 2]};
                    pair_edge(&c, x, y, x, y + 1, vis[a], vis[q], color + 3 * a, color + 3 * q, ga, gb, &go);
                }
            }
        }
    }
    vertex_chain(&c, go.g_verts_screen, g_verts);
    free(go.g_verts_screen);
    ctx_free(&c);
    return 0;
}

static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int orc_backward_pixels(const orc_scene* s, const orc_view* v, const orc_opts* o,
                        int64_t n, const int32_t* xy,
                        const float* grad_color, const float* grad_logp,
                        double* g_verts, double* g_feats, double* g_mlp)
{
    view_ctx c;
    if (ctx_init(&c, s, v, o, 0) != 0) return -1;
    const int W = v->W, H = v->H;
    /* sorted (linear index, position in the list) for gradient lookup */
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * (n > 0 ? n : 1)));
    for (int64_t i = 0; i < n; ++i) {
        int x = xy[2 * i], y = xy[2 * i + 1];
        if (x < 0 || x >= W || y < 0 || y >= H) { free(idx); ctx_free(&c); return -1; }
        idx[2 * i] = (int64_t)y * W + x;
        idx[2 * i + 1] = i;
    }
    qsort(idx, (size_t)n, 2 * sizeof(int64_t), cmp_i64);
    for (int64_t i = 1; i < n; ++i)
        if (idx[2 * i] == idx[2 * i - 2]) { free(idx); ctx_free(&c); return -1; }
    /* every pixel that takes part: the listed ones and their 4 neighbours */
    int64_t m = 0;
    int64_t* all = (int64_t*)malloc(sizeof(int64_t) * (size_t)(5 * (n > 0 ? n : 1)));
    static const int nb[5][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 5; ++k) {
            int x = xy[2 * i] + nb[k][0], y = xy[2 * i + 1] + nb[k][1];
            if (x >= 0 && x < W && y >= 0 && y < H) all[m++] = (int64_t)y * W + x;
        }
    qsort(all, (size_t)m, sizeof(int64_t), cmp_i64);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i)
        if (u == 0 || all[i] != all[u - 1]) all[u++] = all[i];
    m = u;
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
    float* col = (float*)malloc(sizeof(float) * 3 * (size_t)(m > 0 ? m : 1));
    grad_out go;
    go.g_verts_screen = (double*)calloc((size_t)(s->T > 0 ? s->T : 1) * 9, sizeof(double));
    go.g_feats = g_feats;
    go.g_mlp = g_mlp;
    #pragma omp parallel
    {
        frag_buf b = {0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < m; ++i) {
            int x = (int)(all[i] % W), y = (int)(all[i] / W);
            pixel_fragments(&c, x, y, &b);
            pixel_result r;
            pixel_forward(&c, x, y, &b, &r);
            key[i] = r.key;
            for (int k = 0; k < 3; ++k) col[3 * i + k] = r.rgb[k];
            /* colour and score paths of listed pixels */
            int64_t lin = all[i];
            int64_t lo = 0, hi = n - 1, pos = -1;
            while (lo <= hi) {
                int64_t mid = (lo + hi) / 2;
                if (idx[2 * mid] == lin) { pos = idx[2 * mid + 1]; break; }
                if (idx[2 * mid] < lin) lo = mid + 1; else hi = mid - 1;
            }
            if (pos >= 0) {
                double gC[3] = {grad_color[3 * pos], grad_color[3 * pos + 1], grad_color[3 * pos + 2]};
                double gL = grad_logp ? grad_logp[pos] : 0.0;
                pixel_backward(&c, x, y, &b, r.key, gC, gL, &go);
            }
        }
        free(b.f);
    }
    /* edge pairs touching a listed pixel, each pair once */
    for (int64_t i = 0; i < m; ++i) {
        int x = (int)(all[i] % W), y = (int)(all[i] / W);
        for (int dir = 0; dir < 2; ++dir) {
            int xb = x + (dir == 0), yb = y + (dir == 1);
            if (xb >= W || yb >= H) continue;
            int64_t lb = (int64_t)yb * W + xb;
            /* position of b among the participating pixels */
            int64_t lo = 0, hi = m - 1, jb = -1;
            while (lo <= hi) {
                int64_t mid = (lo + hi) / 2;
                if (all[mid] == lb) { jb = mid; break; }
                if (all[mid] < lb) lo = mid + 1; else hi = mid - 1;
            }
            if (jb < 0) continue;
            double ga[3] = {0, 0, 0}, gb[3] = {0, 0, 0};
            int in_a = 0, in_b = 0;
            int64_t lo2 = 0, hi2 = n - 1;
            while (lo2 <= hi2) {
                int64_t mid = (lo2 + hi2) / 2;
                if (idx[2 * mid] == all[i]) { int64_t p = idx[2 * mid + 1]; for (int k = 0; k < 3; ++k) ga[k] = grad_color[3 * p + k]; in_a = 1; break; }
                if (idx[2 * mid] < all[i]) lo2 = mid + 1; else hi2 = mid - 1;
            }
            lo2 = 0; hi2 = n - 1;
            while (lo2 <= hi2) {
                int64_t mid = (lo2 + hi2) / 2;
                if (idx[2 * mid] == lb) { int64_t p = idx[2 * mid + 1]; for (int k = 0; k < 3; ++k) gb[k] = grad_color[3 * p + k]; in_b = 1; break; }
                if (idx[2 * mid] < lb) lo2 = mid + 1; else hi2 = mid - 1;
            }
            if (!in_a && !in_b) continue;
            pair_edge(&c, x, y, xb, yb, key[i], key[jb], col + 3 * i, col + 3 * jb, ga, gb, &go);
        }
    }
    vertex_chain(&c, go.g_verts_screen, g_verts);
    free(go.g_verts_screen);
    free(key); free(col); free(all); free(idx);
    ctx_free(&c);
    return 0;
}

int orc_pixel_fragments(const orc_scene* s, const orc_view* v, const orc_opts* o,
                        int32_t x, int32_t y, int32_t cap,
                        uint32_t* tri, uint64_t* key, float* alpha, float* o3,
                        float* u, double* dlogit, int32_t* winner)
{
    view_ctx c;
    if (ctx_init(&c, s, v, o, 0) != 0) return -1;
    if (x < 0 || x >= v->W || y < 0 || y >= v->H) { ctx_free(&c); return -1; }
    frag_buf b = {0};
    pixel_fragments(&c, x, y, &b);
    pixel_result r;
    pixel_forward(&c, x, y, &b, &r);
    float act[MAXL + 1][MAXW];
    const int L = s->n_layers;
    for (int i = 0; i < b.n && i < cap; ++i) {
        decode_f32(s, &b.f[i], act);
        float a, uu;
        passes(v, o, x, y, b.f[i].tri, act[L][3], &a, &uu);
        tri[i] = b.f[i].tri;
        key[i] = b.f[i].key;
        alpha[i] = a;
        o3[i] = act[L][3];
        u[i] = uu;
        if (r.winner >= 0 && i == r.winner) dlogit[i] = 1.0 - (double)a;
        else if (r.winner < 0 || i < r.winner) dlogit[i] = -(double)a;
        else dlogit[i] = 0.0;
    }
    *winner = r.winner;
    int n = b.n;
    free(b.f);
    ctx_free(&c);
    return n;
}

int orc_color_f64(const orc_scene* s, const orc_view* v, const orc_opts* o,
                  int32_t tri, int32_t x, int32_t y, double* rgb, double* alpha)
{
    if (!scene_ok(s) || tri < 0 || tri >= s->T) return -1;
    tri_setup t;
    setup_triangle(s, v, o, tri, &t);
    if (!t.sgn) return 0;
    const float* M = v->M;
    double vx[3], vy[3], iw[3];
    for (int i = 0; i < 3; ++i) {
        const float* p = s->verts + ((size_t)tri * 3 + i) * 3;
        double cc[4];
        for (int j = 0; j < 4; ++j)
            cc[j] = (double)M[j * 4 + 3] + (double)M[j * 4] * p[0] + (double)M[j * 4 + 1] * p[1] +
                    (double)M[j * 4 + 2] * p[2];
        iw[i] = 1.0 / cc[3];
        vx[i] = 0.5 * v->W * (cc[0] * iw[i]) + 0.5 * v->W;
        vy[i] = 0.5 * v->H - 0.5 * v->H * (cc[1] * iw[i]);
    }
    double px = x + 0.5, py = y + 0.5;
    double a = edge_d(vx[0], vy[0], vx[1], vy[1], vx[2], vy[2]);
    double tt[3], S = 0;
    for (int i = 0; i < 3; ++i) {
        int p = (i + 1) % 3, q = (i + 2) % 3;
        double beta = edge_d(vx[p], vy[p], vx[q], vy[q], px, py) / a;
        tt[i] = beta * iw[i];
        S += tt[i];
    }
    const int G = s->G;
    double gx = tt[1] / S * (G - 1), gy = tt[2] / S * (G - 1);
    int ix = (int)floor(gx), iy = (int)floor(gy);
    if (ix < 0) ix = 0;
    if (ix > G - 2) ix = G - 2;
    if (iy < 0) iy = 0;
    if (iy > G - 2) iy = G - 2;
    double act[MAXL + 1][MAXW];
    decode_f64_at(s, (uint32_t)tri, ix, iy, gx - ix, gy - iy, act);
    for (int k = 0; k < 3; ++k) rgb[k] = sigmoid_d(act[s->n_layers][k]);
    *alpha = sigmoid_d(act[s->n_layers][3]);
    return 1;
}

int64_t orc_count_valid(const orc_scene* s, const orc_view* v, const orc_opts* o)
{
    view_ctx c;
    if (ctx_init(&c, s, v, o, 0) != 0) return -1;
    int64_t n = c.n_valid;
    ctx_free(&c);
    return n;
}

/* ========================================================================= */
/* Paper form of the step (Section 3.3, "Learnable multi-resolution triangle   */
/* texture" and "Neural deferred shading"; Supplement B.3, MLP architecture;   */
/* Supplement B.6, 561 grid points at R = 5).                                  */
/*                                                                             */
/* Texture: per triangle, the finest mesh-colour grid of level R: the          */
/* triangle subdivided into n = 2^R segments per edge, grid vertex (i, j)      */
/* (i, j >= 0, i + j <= n) at barycentrics (b1, b2) = (i/n, j/n); 8 channels    */
/* per vertex, activated (in [0,1]): 7 colour features, then the opacity.      */
/* Opacity stays outside the MLP: a fragment's alpha is the opacity channel     */
/* interpolated in the micro-triangle that contains it. The MLP runs once per   */
/* pixel, on the winner (deferred): input = the 7 interpolated features and     */
/* the 9 real spherical harmonics of degree <= 2 of the view direction; two     */
/* hidden layers of 16 (ReLU); 3 outputs through the sigmoid. Reading of the    */
/* skip blend: features 0..3 are RGBA, and the colour is                        */
/* A * RGB + (1 - A) * MLP.                                                     */
/* Everything up to the mask decision and the deferred colour follows one      */
/* float32 operation sequence, so both are reproducible bit for bit.           */
/* ========================================================================= */

#define PCH 8            /* channels per grid vertex */
#define PFEAT 7          /* colour features */
#define PIN 16           /* MLP input: 7 features + 9 harmonics */
#define PHID 16

int orc_mc_count(int R)
{
    const int n = 1 << R;
    return (n + 1) * (n + 2) / 2;
}

/* Row-major layout: row j holds n + 1 - j vertices, i ascending. */
static int mc_index(int n, int i, int j)
{
    return j * (n + 1) - j * (j - 1) / 2 + i;
}

/* The micro-triangle of the level with n segments per edge that contains the
 * point (b1, b2), and the point's barycentric weights in it (float32): u = b1 n
 * and v = b2 n (exact: n is a power of two), i = floor(u) clamped to
 * [0, n - 1], j = floor(v) clamped to [0, n - 1 - i], fu = u - i, fv = v - j.
 * If fu + fv > 1 and the inverted micro-triangle exists (i + j <= n - 2) the
 * point lies in it: vertices (i+1, j+1), (i+1, j), (i, j+1), weights
 * (fu + fv - 1, 1 - fv, 1 - fu); otherwise in the upright one: (i, j),
 * (i+1, j), (i, j+1), weights ((1 - fu) - fv, fu, fv). */
static void mc_lookup(int n, float b1, float b2, int idx[3], float w[3], float* fu_out, float* fv_out, int* inv_out)
{
    const float u = b1 * (float)n, v = b2 * (float)n;
    int i = (int)floorf(u);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    int j = (int)floorf(v);
    if (j < 0) j = 0;
    if (j > n - 1 - i) j = n - 1 - i;
    const float fu = u - (float)i, fv = v - (float)j;
    const float s = fu + fv;
    int inv = s > 1.0f && i + j <= n - 2;
    if (inv) {
        idx[0] = mc_index(n, i + 1, j + 1); idx[1] = mc_index(n, i + 1, j); idx[2] = mc_index(n, i, j + 1);
        w[0] = s - 1.0f; w[1] = 1.0f - fv; w[2] = 1.0f - fu;
    } else {
        idx[0] = mc_index(n, i, j); idx[1] = mc_index(n, i + 1, j); idx[2] = mc_index(n, i, j + 1);
        w[0] = (1.0f - fu) - fv; w[1] = fu; w[2] = fv;
    }
    if (fu_out) *fu_out = fu;
    if (fv_out) *fv_out = fv;
    if (inv_out) *inv_out = inv;
}

static float mc_interp(const float* tex, int ch, const int idx[3], const float w[3])
{
    return fmaf(w[2], tex[(size_t)idx[2] * PCH + ch], fmaf(w[1], tex[(size_t)idx[1] * PCH + ch],
                                                          w[0] * tex[(size_t)idx[0] * PCH + ch]));
}

int orc_mc_lookup(int R, float b1, float b2, int32_t idx[3], float w[3])
{
    int ii[3];
    mc_lookup(1 << R, b1, b2, ii, w, NULL, NULL, NULL);
    for (int k = 0; k < 3; ++k) idx[k] = ii[k];
    return 0;
}

/* Multi-resolution texture (Section 3.3): learnable grids of levels Rmin ..
 * Rtop (Rtop <= Rmax), raw[l] of level Rmin + l, [T][V(level)][8], each
 * sampled at the vertices of the level-Rmax grid by the micro-triangle lookup
 * and summed (Rmin first) before the sigmoid: tex [T][V(Rmax)][8] =
 * sigmoid(sum). The paper keeps grids up to Rmax - 1 and accumulates them on
 * the finest grid (Rtop = Rmax - 1); Rtop = Rmax makes the finest grid
 * learnable as well. */
static int levels_ok(int T, int Rmin, int Rtop, int Rmax)
{
    return T >= 0 && Rmin >= 0 && Rtop >= Rmin && Rmax >= Rtop && Rmax <= 10;
}

int orc_mc_assemble(int T, int Rmin, int Rtop, int Rmax, const float* const* raw, float* tex)
{
    if (!levels_ok(T, Rmin, Rtop, Rmax)) return -1;
    const int n = 1 << Rmax, V = orc_mc_count(Rmax);
    #pragma omp parallel for schedule(static)
    for (int t = 0; t < T; ++t) {
        for (int j = 0; j <= n; ++j)
            for (int i = 0; i + j <= n; ++i) {
                const float b1 = (float)i / (float)n, b2 = (float)j / (float)n;
                float z[PCH] = {0, 0, 0, 0, 0, 0, 0, 0};
                for (int R = Rmin; R <= Rtop; ++R) {
                    const float* g = raw[R - Rmin] + (size_t)t * orc_mc_count(R) * PCH;
                    int idx[3];
                    float w[3];
                    mc_lookup(1 << R, b1, b2, idx, w, NULL, NULL, NULL);
                    for (int c = 0; c < PCH; ++c) z[c] = z[c] + mc_interp(g, c, idx, w);
                }
                float* out = tex + ((size_t)t * V + mc_index(n, i, j)) * PCH;
                for (int c = 0; c < PCH; ++c) out[c] = orc_sigmoid(z[c]);
            }
    }
    return 0;
}

/* Gradient of orc_mc_assemble: d raw[l] += sum over finest vertices of
 * sigmoid' * d tex * (the vertex's weight in the level's lookup). The
 * sigmoid derivative is taken from the assembled value: tex (1 - tex). */
int orc_mc_assemble_bwd(int T, int Rmin, int Rtop, int Rmax, const float* tex, const float* grad_tex,
                        double* const* grad_raw)
{
    if (!levels_ok(T, Rmin, Rtop, Rmax)) return -1;
    const int n = 1 << Rmax, V = orc_mc_count(Rmax);
    #pragma omp parallel for schedule(static)
    for (int t = 0; t < T; ++t) {
        for (int j = 0; j <= n; ++j)
            for (int i = 0; i + j <= n; ++i) {
                const size_t at = ((size_t)t * V + mc_index(n, i, j)) * PCH;
                const float b1 = (float)i / (float)n, b2 = (float)j / (float)n;
                for (int R = Rmin; R <= Rtop; ++R) {
                    double* g = grad_raw[R - Rmin] + (size_t)t * orc_mc_count(R) * PCH;
                    int idx[3];
                    float w[3];
                    mc_lookup(1 << R, b1, b2, idx, w, NULL, NULL, NULL);
                    for (int c = 0; c < PCH; ++c) {
                        const double s = tex[at + c];
                        const double dz = (double)grad_tex[at + c] * s * (1.0 - s);
                        for (int k = 0; k < 3; ++k) g[(size_t)idx[k] * PCH + c] += (double)w[k] * dz;
                    }
                }
            }
    }
    return 0;
}

/* The view direction through the centre of pixel (x, y), float32: the pixel's
 * normalised device coordinates at the near (-1) and far (+1) depth mapped
 * back through Minv (the inverse view-projection, given with the view), each
 * row as the vertex transform (bias first, then x, y, z by FMA), divided by
 * w; the difference normalised. */
static void view_dir(const orc_view* v, const float* Minv, int x, int y, float d[3])
{
    const float nx = (2.0f * (float)x + 1.0f) / (float)v->W - 1.0f;
    const float ny = 1.0f - (2.0f * (float)y + 1.0f) / (float)v->H;
    float p[2][4];
    for (int e = 0; e < 2; ++e) {
        const float nz = e == 0 ? -1.0f : 1.0f;
        for (int r = 0; r < 4; ++r) {
            float a = Minv[r * 4 + 3];
            a = fmaf(Minv[r * 4 + 0], nx, a);
            a = fmaf(Minv[r * 4 + 1], ny, a);
            a = fmaf(Minv[r * 4 + 2], nz, a);
            p[e][r] = a;
        }
    }
    for (int k = 0; k < 3; ++k) d[k] = p[1][k] / p[1][3] - p[0][k] / p[0][3];
    const float len = sqrtf(fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0])));
    for (int k = 0; k < 3; ++k) d[k] = d[k] / len;
}

int orc_view_dir(const orc_view* v, const float* Minv, int32_t x, int32_t y, float d[3])
{
    if (!v || !Minv || x < 0 || y < 0 || x >= v->W || y >= v->H) return -1;
    view_dir(v, Minv, x, y, d);
    return 0;
}

/* The 9 real spherical harmonics of degree <= 2 (orthonormal on the sphere,
 * no Condon-Shortley sign) of a unit vector, float32:
 *   1/(2 sqrt(pi));  sqrt(3/(4 pi)) (y, z, x);
 *   sqrt(15/(4 pi)) (xy, yz), sqrt(5/(16 pi)) (2z^2 - x^2 - y^2),
 *   sqrt(15/(4 pi)) xz, sqrt(15/(16 pi)) (x^2 - y^2). */
void orc_sh2(const float d[3], float out[9])
{
    const float x = d[0], y = d[1], z = d[2];
    const float c0 = 0.28209479177387814f, c1 = 0.48860251190291992f;
    const float c2 = 1.0925484305920792f, c3 = 0.31539156525252005f, c4 = 0.54627421529603959f;
    out[0] = c0;
    out[1] = c1 * y;
    out[2] = c1 * z;
    out[3] = c1 * x;
    out[4] = c2 * (x * y);
    out[5] = c2 * (y * z);
    out[6] = c3 * fmaf(2.0f * z, z, -fmaf(x, x, y * y));
    out[7] = c2 * (x * z);
    out[8] = c4 * fmaf(x, x, -(y * y));
}

/* orc_sh2 in double, constants from their closed forms. */
static void sh2_d(const double d[3], double out[9])
{
    const double PI = 3.14159265358979323846;
    const double x = d[0], y = d[1], z = d[2];
    const double c0 = 0.5 / sqrt(PI), c1 = sqrt(3.0 / (4 * PI)), c2 = sqrt(15.0 / (4 * PI)),
                 c3 = sqrt(5.0 / (16 * PI)), c4 = sqrt(15.0 / (16 * PI));
    out[0] = c0;
    out[1] = c1 * y; out[2] = c1 * z; out[3] = c1 * x;
    out[4] = c2 * x * y; out[5] = c2 * y * z; out[6] = c3 * (2 * z * z - x * x - y * y);
    out[7] = c2 * x * z; out[8] = c4 * (x * x - y * y);
}

/* Deferred MLP, float32 contract (as decode_f32): act[0] = input, act[1],
 * act[2] = hidden layers, act[3][0..2] = output logits. Parameters: W0[16][16],
 * b0[16], W1[16][16], b1[16], W2[3][16], b2[3]. */
static void pmlp_f32(const float* p, const float in[PIN], float act[4][PHID])
{
    for (int k = 0; k < PIN; ++k) act[0][k] = in[k];
    const int din[3] = {PIN, PHID, PHID}, dout[3] = {PHID, PHID, 3};
    for (int l = 0; l < 3; ++l) {
        const float* W = p;
        const float* b = p + dout[l] * din[l];
        for (int j = 0; j < dout[l]; ++j) {
            float h = b[j];
            for (int k = 0; k < din[l]; ++k) h = fmaf(W[j * din[l] + k], act[l][k], h);
            if (l < 2) h = h > 0.0f ? h : 0.0f;
            act[l + 1][j] = h;
        }
        p += dout[l] * din[l] + dout[l];
    }
}

int orc_pmlp_params(void) { return PIN * PHID + PHID + PHID * PHID + PHID + 3 * PHID + 3; }

typedef struct {
    const float* tex;        /* [T][V][8] */
    const float* mlp;
    const float* Minv;       /* this view's inverse view-projection */
    int R, n, V;
} pctx;

/* Colour of the winner fragment f at pixel (x, y) (float32 contract): the
 * features and A at its barycentrics, the MLP on features + harmonics, the
 * blend. act/feat/mlp_rgb are returned for the backward. */
static void pshade(const pctx* P, const orc_view* v, const frag_t* f, int x, int y, float rgb[3],
                   float feat[PFEAT], float act[4][PHID], int idx[3], float w[3])
{
    const float* tt = P->tex + (size_t)f->tri * P->V * PCH;
    mc_lookup(P->n, f->b1, f->b2, idx, w, NULL, NULL, NULL);
    for (int c = 0; c < PFEAT; ++c) feat[c] = mc_interp(tt, c, idx, w);
    float d[3], in[PIN];
    view_dir(v, P->Minv, x, y, d);
    for (int c = 0; c < PFEAT; ++c) in[c] = feat[c];
    orc_sh2(d, in + PFEAT);
    pmlp_f32(P->mlp, in, act);
    const float A = feat[3];
    for (int c = 0; c < 3; ++c) {
        const float m = orc_sigmoid(act[3][c]);
        rgb[c] = fmaf(A, feat[c] - m, m);     /* A RGB + (1 - A) MLP */
    }
}

static float palpha(const pctx* P, const frag_t* f)
{
    int idx[3];
    float w[3];
    mc_lookup(P->n, f->b1, f->b2, idx, w, NULL, NULL, NULL);
    return mc_interp(P->tex + (size_t)f->tri * P->V * PCH, PFEAT, idx, w);
}

/* Mask test with the opacity texture: Eq. (5) (u < alpha) or Eq. (3) read as
 * alpha > 0.5. */
static int ppasses(const orc_view* v, const orc_opts* o, int x, int y, uint32_t tri, float a)
{
    if (o->mode == 1) return a > 0.5f;
    return orc_uniform(o->seed, (uint32_t)(y * v->W + x), tri, v->view_id, o->step) < a;
}

static void ppixel_forward(const view_ctx* c, const pctx* P, int x, int y, const frag_buf* b, pixel_result* r)
{
    r->winner = -1;
    r->key = BG_KEY;
    for (int k = 0; k < 3; ++k) r->rgb[k] = c->o->background[k];
    r->logp = 0.0;
    r->decodes = 0;
    for (int i = 0; i < b->n; ++i) {
        const float a = palpha(P, &b->f[i]);
        r->decodes++;
        if (ppasses(c->v, c->o, x, y, b->f[i].tri, a)) {
            r->winner = i;
            r->key = b->f[i].key;
            float feat[PFEAT], act[4][PHID], w[3];
            int idx[3];
            pshade(P, c->v, &b->f[i], x, y, r->rgb, feat, act, idx, w);
            if (c->o->mode == 0) r->logp += log((double)a);
            return;
        }
        if (c->o->mode == 0) r->logp += log1p(-(double)a);
    }
}

/* geometry-only scene for the shared setup and coverage code */
static orc_scene pgeom(const orc_pscene* s, int32_t* dims)
{
    orc_scene g;
    dims[0] = 1; dims[1] = 4;
    g.T = s->T; g.G = 2; g.C = 1; g.n_layers = 1; g.dims = dims;
    g.verts = s->verts; g.feats = NULL; g.mlp = NULL;
    return g;
}

static int pscene_ok(const orc_pscene* s)
{
    return s && s->T >= 0 && s->R >= 0 && s->R <= 10 && (s->T == 0 || (s->verts && s->tex && s->mlp));
}

int orc_pforward(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o,
                 uint64_t* vis, float* color, double* logp, orc_stats* st)
{
    if (!pscene_ok(s) || !Minv) return -1;
    int32_t dims[2];
    orc_scene g = pgeom(s, dims);
    view_ctx c;
    if (ctx_init(&c, &g, v, o, 1) != 0) return -1;
    pctx P = {s->tex, s->mlp, Minv, s->R, 1 << s->R, orc_mc_count(s->R)};
    int64_t cov = 0, frags = 0, dec = 0, win = 0, front = 0;
    #pragma omp parallel reduction(+ : cov, frags, dec, win, front)
    {
        frag_buf b = {0};
        #pragma omp for schedule(dynamic, 4)
        for (int y = 0; y < v->H; ++y)
            for (int x = 0; x < v->W; ++x) {
                size_t p = (size_t)y * v->W + x;
                pixel_fragments(&c, x, y, &b);
                pixel_result r;
                ppixel_forward(&c, &P, x, y, &b, &r);
                vis[p] = r.key;
                for (int k = 0; k < 3; ++k) color[3 * p + k] = r.rgb[k];
                if (logp) logp[p] = r.logp;
                cov += b.n > 0;
                frags += b.n;
                dec += r.decodes;
                win += r.winner >= 0;
                front += r.winner >= 0 ? r.winner : b.n;
            }
        free(b.f);
    }
    if (st) {
        st->covered_pixels = cov;
        st->covering_fragments = frags;
        st->decodes = dec;
        st->winners = win;
        st->front_fragments = front;
    }
    ctx_free(&c);
    return 0;
}

/* d loss / d (perspective-correct b1, b2) of fragment f -> the screen
 * positions and 1/w of its triangle's vertices (as the colour path of the
 * workloads' form: perspective division, screen barycentrics). */
static void push_bary(const view_ctx* c, const frag_t* f, int x, int y, double db1, double db2, grad_out* go)
{
    const tri_setup* t = &c->ts[f->tri];
    frag_geom g;
    geom_of(c, t, x, y, &g);
    double tt[3], S = 0;
    for (int i = 0; i < 3; ++i) { tt[i] = g.beta[i] * g.iw[i]; S += tt[i]; }
    const double b[3] = {tt[0] / S, tt[1] / S, tt[2] / S};
    const double db[3] = {0.0, db1, db2};
    const double dot = db[0] * b[0] + db[1] * b[1] + db[2] * b[2];
    double dbeta_v[3], diw[3];
    for (int i = 0; i < 3; ++i) {
        const double dtt = (db[i] - dot) / S;
        dbeta_v[i] = dtt * g.iw[i];
        diw[i] = dtt * g.beta[i];
    }
    double D[3][3][2];
    dbeta(&g, D);
    double* gv = go->g_verts_screen + (size_t)f->tri * 9;
    for (int j = 0; j < 3; ++j) {
        double sx = 0, sy = 0;
        for (int i = 0; i < 3; ++i) { sx += dbeta_v[i] * D[i][j][0]; sy += dbeta_v[i] * D[i][j][1]; }
        atomic_add(&gv[3 * j + 0], sx);
        atomic_add(&gv[3 * j + 1], sy);
        atomic_add(&gv[3 * j + 2], diw[j]);
    }
}

/* The winner's shading inputs at which the backward differentiates: the
 * float32 contract values, or in analysis mode float64 values at the exact
 * perspective-correct barycentrics (the micro-triangle kept from the float32
 * lookup) with the view direction, harmonics and MLP in double. feat[0..7],
 * act[0] = MLP input, act[1..2] hidden, act[3][0..2] logits. */
static void pshade_d(const view_ctx* c, const pctx* P, const frag_t* f, int x, int y, const int idx[3], int inv,
                     float fu32, float fv32, double feat[PCH], double act[4][PHID], double w[3])
{
    const float* tt = P->tex + (size_t)f->tri * P->V * PCH;
    if (!c->o->analysis) {
        float rgb[3], ft[PFEAT], a32[4][PHID], w32[3];
        int id[3];
        pshade(P, c->v, f, x, y, rgb, ft, a32, id, w32);
        for (int k = 0; k < 3; ++k) w[k] = w32[k];
        for (int k = 0; k < PFEAT; ++k) feat[k] = ft[k];
        feat[PFEAT] = palpha(P, f);
        for (int l = 0; l < 4; ++l)
            for (int k = 0; k < PHID; ++k) act[l][k] = a32[l][k];
        return;
    }
    const tri_setup* t = &c->ts[f->tri];
    frag_geom g;
    geom_of(c, t, x, y, &g);
    double q[3], S = 0;
    for (int i = 0; i < 3; ++i) { q[i] = g.beta[i] * g.iw[i]; S += q[i]; }
    const int n = P->n;
    /* cell origin from the float32 lookup: u = i + fu */
    const double i0 = (double)(f->b1 * (float)n) - fu32, j0 = (double)(f->b2 * (float)n) - fv32;
    const double fu = q[1] / S * n - i0, fv = q[2] / S * n - j0;
    w[0] = inv ? fu + fv - 1.0 : 1.0 - fu - fv;
    w[1] = inv ? 1.0 - fv : fu;
    w[2] = inv ? 1.0 - fu : fv;
    for (int ch = 0; ch < PCH; ++ch)
        feat[ch] = w[0] * tt[(size_t)idx[0] * PCH + ch] + w[1] * tt[(size_t)idx[1] * PCH + ch] +
                   w[2] * tt[(size_t)idx[2] * PCH + ch];
    const float* Mi = P->Minv;
    const double nx = (2.0 * x + 1.0) / c->v->W - 1.0, ny = 1.0 - (2.0 * y + 1.0) / c->v->H;
    double pr[2][4], d[3], len = 0;
    for (int e = 0; e < 2; ++e)
        for (int r = 0; r < 4; ++r)
            pr[e][r] = Mi[r * 4 + 3] + Mi[r * 4] * nx + Mi[r * 4 + 1] * ny + Mi[r * 4 + 2] * (e ? 1.0 : -1.0);
    for (int k = 0; k < 3; ++k) { d[k] = pr[1][k] / pr[1][3] - pr[0][k] / pr[0][3]; len += d[k] * d[k]; }
    len = sqrt(len);
    for (int k = 0; k < 3; ++k) d[k] /= len;
    double* in = act[0];
    for (int k = 0; k < PFEAT; ++k) in[k] = feat[k];
    sh2_d(d, in + PFEAT);
    const int din[3] = {PIN, PHID, PHID}, dout[3] = {PHID, PHID, 3};
    const float* p = P->mlp;
    for (int l = 0; l < 3; ++l) {
        for (int j = 0; j < dout[l]; ++j) {
            double h = p[dout[l] * din[l] + j];
            for (int k = 0; k < din[l]; ++k) h += (double)p[j * din[l] + k] * act[l][k];
            act[l + 1][j] = l < 2 ? (h > 0 ? h : 0) : h;
        }
        p += dout[l] * din[l] + dout[l];
    }
}

/* Algorithm A1, part 2, for one pixel of the paper form.
 * (a) colour of the winner: out = A RGB + (1 - A) m, m = sigmoid(MLP logits):
 *     d RGB = A gC, d A = gC . (RGB - m), d m = (1 - A) gC, back through the
 *     sigmoid and the MLP (its ReLU gates those of the float32 forward) to the
 *     7 features; the features' gradient goes to the 3 grid vertices of the
 *     micro-triangle (weights w) and, through the interpolation's derivative
 *     along (b1, b2), to the vertices of the triangle.
 * (b) score term (Eq. (9)): the winner's opacity d alpha = g_L / alpha, each
 *     fragment in front d alpha = -g_L / (1 - alpha) (alpha is the texture
 *     value itself, no sigmoid here); to the opacity channel of the 3 grid
 *     vertices, no vertex motion (Section 3.2). */
static void ppixel_backward(const view_ctx* c, const pctx* P, int x, int y, const frag_buf* b, uint64_t key_star,
                            const double gC[3], double gL, double* g_tex, double* g_mlp, grad_out* go)
{
    for (int i = 0; i < b->n; ++i) {
        const frag_t* f = &b->f[i];
        if (f->key > key_star) break;
        const float a = palpha(P, f);
        int idx[3], inv;
        float w[3], fu, fv;
        mc_lookup(P->n, f->b1, f->b2, idx, w, &fu, &fv, &inv);
        double* gt = g_tex + (size_t)f->tri * P->V * PCH;
        if (f->key == key_star) {
            if (c->o->mode == 0 && gL != 0.0)
                for (int k = 0; k < 3; ++k) atomic_add(&gt[(size_t)idx[k] * PCH + PFEAT], (double)w[k] * gL / (double)a);
            if (gC[0] == 0.0 && gC[1] == 0.0 && gC[2] == 0.0) break;
            double feat[PCH], act[4][PHID], wd[3];
            pshade_d(c, P, f, x, y, idx, inv, fu, fv, feat, act, wd);
            const double A = feat[3];
            double dfeat[PFEAT] = {0, 0, 0, 0, 0, 0, 0};
            double delta[PHID], prev[PHID];
            double dA = 0;
            for (int k = 0; k < 3; ++k) {
                const double m = 1.0 / (1.0 + exp(-act[3][k]));
                dfeat[k] += A * gC[k];
                dA += gC[k] * (feat[k] - m);
                delta[k] = (1.0 - A) * gC[k] * m * (1.0 - m);
            }
            dfeat[3] += dA;
            /* MLP backward (parameter offsets per layer) */
            const int din[3] = {PIN, PHID, PHID}, dout[3] = {PHID, PHID, 3};
            int off[3] = {0, 0, 0};
            for (int l = 1; l < 3; ++l) off[l] = off[l - 1] + dout[l - 1] * din[l - 1] + dout[l - 1];
            for (int l = 2; l >= 0; --l) {
                const float* Wl = P->mlp + off[l];
                double* gW = g_mlp + off[l];
                double* gb = gW + dout[l] * din[l];
                for (int j = 0; j < dout[l]; ++j) {
                    if (delta[j] == 0.0) continue;
                    atomic_add(&gb[j], delta[j]);
                    for (int k = 0; k < din[l]; ++k)
                        if (act[l][k] != 0.0) atomic_add(&gW[j * din[l] + k], delta[j] * act[l][k]);
                }
                for (int k = 0; k < din[l]; ++k) {
                    double acc = 0;
                    for (int j = 0; j < dout[l]; ++j) acc += (double)Wl[j * din[l] + k] * delta[j];
                    if (l > 0 && !(act[l][k] > 0.0)) acc = 0;
                    prev[k] = acc;
                }
                memcpy(delta, prev, sizeof(double) * (size_t)din[l]);
            }
            for (int k = 0; k < PFEAT; ++k) dfeat[k] += delta[k];   /* the harmonics have no parameters */
            /* features -> grid vertices, and along (b1, b2) -> triangle vertices */
            const float* tt = P->tex + (size_t)f->tri * P->V * PCH;
            double dfu = 0, dfv = 0;
            for (int k = 0; k < PFEAT; ++k) {
                for (int q = 0; q < 3; ++q) atomic_add(&gt[(size_t)idx[q] * PCH + k], wd[q] * dfeat[k]);
                const double t0 = tt[(size_t)idx[0] * PCH + k], t1 = tt[(size_t)idx[1] * PCH + k],
                             t2 = tt[(size_t)idx[2] * PCH + k];
                /* upright: w = (1 - fu - fv, fu, fv); inverted: w = (fu + fv - 1, 1 - fv, 1 - fu) */
                dfu += dfeat[k] * (inv ? t0 - t2 : t1 - t0);
                dfv += dfeat[k] * (inv ? t0 - t1 : t2 - t0);
            }
            push_bary(c, f, x, y, dfu * P->n, dfv * P->n, go);
            break;
        }
        if (c->o->mode != 0 || gL == 0.0) continue;
        for (int k = 0; k < 3; ++k)
            atomic_add(&gt[(size_t)idx[k] * PCH + PFEAT], -(double)w[k] * gL / (1.0 - (double)a));
    }
}

int orc_pbackward(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o,
                  const uint64_t* vis, const float* color, const float* grad_color, const float* grad_logp,
                  double* g_verts, double* g_tex, double* g_mlp)
{
    if (!pscene_ok(s) || !Minv) return -1;
    int32_t dims[2];
    orc_scene g = pgeom(s, dims);
    view_ctx c;
    if (ctx_init(&c, &g, v, o, 1) != 0) return -1;
    pctx P = {s->tex, s->mlp, Minv, s->R, 1 << s->R, orc_mc_count(s->R)};
    grad_out go;
    go.g_verts_screen = (double*)calloc((size_t)(s->T > 0 ? s->T : 1) * 9, sizeof(double));
    go.g_feats = NULL;
    go.g_mlp = NULL;
    const int W = v->W, H = v->H;
    #pragma omp parallel
    {
        frag_buf b = {0};
        #pragma omp for schedule(dynamic, 4)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t p = (size_t)y * W + x;
                double gC[3] = {grad_color[3 * p], grad_color[3 * p + 1], grad_color[3 * p + 2]};
                double gL = grad_logp ? grad_logp[p] : 0.0;
                if (gC[0] == 0 && gC[1] == 0 && gC[2] == 0 && gL == 0) continue;
                pixel_fragments(&c, x, y, &b);
                ppixel_backward(&c, &P, x, y, &b, vis[p], gC, gL, g_tex, g_mlp, &go);
            }
        free(b.f);
        #pragma omp for schedule(dynamic, 4)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t a = (size_t)y * W + x;
                double ga[3] = {grad_color[3 * a], grad_color[3 * a + 1], grad_color[3 * a + 2]};
                if (x + 1 < W) {
                    size_t q = a + 1;
                    double gb[3] = {grad_color[3 * q], grad_color[3 * q + 1], grad_color[3 * q + 2]};
                    pair_edge(&c, x, y, x + 1, y, vis[a], vis[q], color + 3 * a, color + 3 * q, ga, gb, &go);
                }
                if (y + 1 < H) {
                    size_t q = a + (size_t)W;
                    double gb[3] = {grad_color[3 * q], grad_color[3 * q + 1], grad_color[3 * q + 2]};
                    pair_edge(&c, x, y, x, y + 1, vis[a], vis[q], color + 3 * a, color + 3 * q, ga, gb, &go);
                }
            }
    }
    vertex_chain(&c, go.g_verts_screen, g_verts);
    free(go.g_verts_screen);
    ctx_free(&c);
    return 0;
}

/* float64, unsnapped colour and opacity of triangle tri at the centre of
 * pixel (x, y), ignoring visibility (the paper form's counterpart of
 * orc_color_f64, for finite differences): geometry from the exact clip
 * coordinates, the micro-triangle chosen at that point, harmonics and MLP in
 * double. Returns 0 if the triangle's setup culls it. */
int orc_pcolor_f64(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o,
                   int32_t tri, int32_t x, int32_t y, double* rgb, double* alpha)
{
    if (!pscene_ok(s) || !Minv || tri < 0 || tri >= s->T) return -1;
    int32_t dims[2];
    orc_scene g = pgeom(s, dims);
    tri_setup t;
    setup_triangle(&g, v, o, tri, &t);
    if (!t.sgn) return 0;
    const float* M = v->M;
    double vx[3], vy[3], iw[3];
    for (int i = 0; i < 3; ++i) {
        const float* p = s->verts + ((size_t)tri * 3 + i) * 3;
        double cc[4];
        for (int j = 0; j < 4; ++j)
            cc[j] = (double)M[j * 4 + 3] + (double)M[j * 4] * p[0] + (double)M[j * 4 + 1] * p[1] +
                    (double)M[j * 4 + 2] * p[2];
        iw[i] = 1.0 / cc[3];
        vx[i] = 0.5 * v->W * (cc[0] * iw[i]) + 0.5 * v->W;
        vy[i] = 0.5 * v->H - 0.5 * v->H * (cc[1] * iw[i]);
    }
    const double px = x + 0.5, py = y + 0.5;
    const double a = edge_d(vx[0], vy[0], vx[1], vy[1], vx[2], vy[2]);
    double tt[3], S = 0;
    for (int i = 0; i < 3; ++i) {
        const int p = (i + 1) % 3, q = (i + 2) % 3;
        tt[i] = edge_d(vx[p], vy[p], vx[q], vy[q], px, py) / a * iw[i];
        S += tt[i];
    }
    const int n = 1 << s->R, V = orc_mc_count(s->R);
    const double u = tt[1] / S * n, vv = tt[2] / S * n;
    int i = (int)floor(u);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    int j = (int)floor(vv);
    if (j < 0) j = 0;
    if (j > n - 1 - i) j = n - 1 - i;
    const double fu = u - i, fv = vv - j;
    int idx[3];
    double w[3];
    if (fu + fv > 1.0 && i + j <= n - 2) {
        idx[0] = mc_index(n, i + 1, j + 1); idx[1] = mc_index(n, i + 1, j); idx[2] = mc_index(n, i, j + 1);
        w[0] = fu + fv - 1.0; w[1] = 1.0 - fv; w[2] = 1.0 - fu;
    } else {
        idx[0] = mc_index(n, i, j); idx[1] = mc_index(n, i + 1, j); idx[2] = mc_index(n, i, j + 1);
        w[0] = 1.0 - fu - fv; w[1] = fu; w[2] = fv;
    }
    const float* tx = s->tex + (size_t)tri * V * PCH;
    double feat[PCH];
    for (int ch = 0; ch < PCH; ++ch)
        feat[ch] = w[0] * tx[(size_t)idx[0] * PCH + ch] + w[1] * tx[(size_t)idx[1] * PCH + ch] +
                   w[2] * tx[(size_t)idx[2] * PCH + ch];
    /* view direction and harmonics in double */
    double pr[2][4];
    const double nx = (2.0 * x + 1.0) / v->W - 1.0, ny = 1.0 - (2.0 * y + 1.0) / v->H;
    for (int e = 0; e < 2; ++e)
        for (int r = 0; r < 4; ++r)
            pr[e][r] = Minv[r * 4 + 3] + Minv[r * 4] * nx + Minv[r * 4 + 1] * ny + Minv[r * 4 + 2] * (e ? 1.0 : -1.0);
    double d[3], len = 0;
    for (int k = 0; k < 3; ++k) { d[k] = pr[1][k] / pr[1][3] - pr[0][k] / pr[0][3]; len += d[k] * d[k]; }
    len = sqrt(len);
    for (int k = 0; k < 3; ++k) d[k] /= len;
    double in[PIN];
    for (int k = 0; k < PFEAT; ++k) in[k] = feat[k];
    sh2_d(d, in + PFEAT);
    double h[3][PHID];
    const float* p = s->mlp;
    const int din[3] = {PIN, PHID, PHID}, dout[3] = {PHID, PHID, 3};
    const double* src = in;
    for (int l = 0; l < 3; ++l) {
        for (int jj = 0; jj < dout[l]; ++jj) {
            double acc = p[dout[l] * din[l] + jj];
            for (int k = 0; k < din[l]; ++k) acc += (double)p[jj * din[l] + k] * src[k];
            h[l][jj] = l < 2 ? (acc > 0 ? acc : 0) : acc;
        }
        src = h[l];
        p += dout[l] * din[l] + dout[l];
    }
    const double A = feat[3];
    for (int k = 0; k < 3; ++k) {
        const double m = 1.0 / (1.0 + exp(-h[2][k]));
        rgb[k] = A * feat[k] + (1.0 - A) * m;
    }
    *alpha = feat[PFEAT];
    return 1;
}

/* The paper form's forward at a list of pixels (x, y) of one view: vis,
 * colour and log p of each (as orc_pforward computes them). */
int orc_pforward_pixels(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o, int64_t n,
                        const int32_t* xy, uint64_t* vis, float* color, double* logp)
{
    if (!pscene_ok(s) || !Minv) return -1;
    int32_t dims[2];
    orc_scene g = pgeom(s, dims);
    view_ctx c;
    if (ctx_init(&c, &g, v, o, 0) != 0) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (xy[2 * i] < 0 || xy[2 * i] >= v->W || xy[2 * i + 1] < 0 || xy[2 * i + 1] >= v->H) {
            ctx_free(&c);
            return -1;
        }
    pctx P = {s->tex, s->mlp, Minv, s->R, 1 << s->R, orc_mc_count(s->R)};
    #pragma omp parallel
    {
        frag_buf b = {0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            const int x = xy[2 * i], y = xy[2 * i + 1];
            pixel_fragments(&c, x, y, &b);
            pixel_result r;
            ppixel_forward(&c, &P, x, y, &b, &r);
            vis[i] = r.key;
            for (int k = 0; k < 3; ++k) color[3 * i + k] = r.rgb[k];
            if (logp) logp[i] = r.logp;
        }
        free(b.f);
    }
    ctx_free(&c);
    return 0;
}

/* The paper form's backward of the loss terms of a list of distinct pixels
 * (grad_color [n,3], grad_logp [n] or NULL, in list order; every other
 * pixel's gradients are zero): their colour and score paths, and the edge
 * pairs that touch a listed pixel. Gradients are ADDED. */
int orc_pbackward_pixels(const orc_pscene* s, const orc_view* v, const float* Minv, const orc_opts* o, int64_t n,
                         const int32_t* xy, const float* grad_color, const float* grad_logp, double* g_verts,
                         double* g_tex, double* g_mlp)
{
    if (!pscene_ok(s) || !Minv) return -1;
    int32_t dims[2];
    orc_scene g = pgeom(s, dims);
    view_ctx c;
    if (ctx_init(&c, &g, v, o, 0) != 0) return -1;
    const int W = v->W, H = v->H;
    pctx P = {s->tex, s->mlp, Minv, s->R, 1 << s->R, orc_mc_count(s->R)};
    /* the listed pixels' linear indices, sorted, with their list positions */
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * (n > 0 ? n : 1)));
    for (int64_t i = 0; i < n; ++i) {
        const int x = xy[2 * i], y = xy[2 * i + 1];
        if (x < 0 || x >= W || y < 0 || y >= H) { free(idx); ctx_free(&c); return -1; }
        idx[2 * i] = (int64_t)y * W + x;
        idx[2 * i + 1] = i;
    }
    qsort(idx, (size_t)n, 2 * sizeof(int64_t), cmp_i64);
    for (int64_t i = 1; i < n; ++i)
        if (idx[2 * i] == idx[2 * i - 2]) { free(idx); ctx_free(&c); return -1; }
    /* every pixel that takes part: the listed ones and their 4 neighbours */
    int64_t m = 0;
    int64_t* all = (int64_t*)malloc(sizeof(int64_t) * (size_t)(5 * (n > 0 ? n : 1)));
    static const int nb[5][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 5; ++k) {
            const int x = xy[2 * i] + nb[k][0], y = xy[2 * i + 1] + nb[k][1];
            if (x >= 0 && x < W && y >= 0 && y < H) all[m++] = (int64_t)y * W + x;
        }
    qsort(all, (size_t)m, sizeof(int64_t), cmp_i64);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i)
        if (u == 0 || all[i] != all[u - 1]) all[u++] = all[i];
    m = u;
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
    float* col = (float*)malloc(sizeof(float) * 3 * (size_t)(m > 0 ? m : 1));
    int64_t* pos_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i) {
        int64_t lo = 0, hi = n - 1;
        pos_of[i] = -1;
        while (lo <= hi) {
            const int64_t mid = (lo + hi) / 2;
            if (idx[2 * mid] == all[i]) { pos_of[i] = idx[2 * mid + 1]; break; }
            if (idx[2 * mid] < all[i]) lo = mid + 1; else hi = mid - 1;
        }
    }
    grad_out go;
    go.g_verts_screen = (double*)calloc((size_t)(s->T > 0 ? s->T : 1) * 9, sizeof(double));
    go.g_feats = NULL;
    go.g_mlp = NULL;
    #pragma omp parallel
    {
        frag_buf b = {0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < m; ++i) {
            const int x = (int)(all[i] % W), y = (int)(all[i] / W);
            pixel_fragments(&c, x, y, &b);
            pixel_result r;
            ppixel_forward(&c, &P, x, y, &b, &r);
            key[i] = r.key;
            for (int k = 0; k < 3; ++k) col[3 * i + k] = r.rgb[k];
            const int64_t pos = pos_of[i];
            if (pos >= 0) {
                const double gC[3] = {grad_color[3 * pos], grad_color[3 * pos + 1], grad_color[3 * pos + 2]};
                const double gL = grad_logp ? grad_logp[pos] : 0.0;
                if (gC[0] != 0 || gC[1] != 0 || gC[2] != 0 || gL != 0)
                    ppixel_backward(&c, &P, x, y, &b, r.key, gC, gL, g_tex, g_mlp, &go);
            }
        }
        free(b.f);
    }
    /* edge pairs (a, b = a + e) with a listed pixel among them, each once */
    for (int64_t i = 0; i < m; ++i) {
        const int x = (int)(all[i] % W), y = (int)(all[i] / W);
        for (int dir = 0; dir < 2; ++dir) {
            const int xb = x + (dir == 0), yb = y + (dir == 1);
            if (xb >= W || yb >= H) continue;
            const int64_t lb = (int64_t)yb * W + xb;
            int64_t lo = 0, hi = m - 1, jb = -1;
            while (lo <= hi) {
                const int64_t mid = (lo + hi) / 2;
                if (all[mid] == lb) { jb = mid; break; }
                if (all[mid] < lb) lo = mid + 1; else hi = mid - 1;
            }
            if (jb < 0 || (pos_of[i] < 0 && pos_of[jb] < 0)) continue;
            double ga[3] = {0, 0, 0}, gb[3] = {0, 0, 0};
            for (int k = 0; k < 3; ++k) {
                if (pos_of[i] >= 0) ga[k] = grad_color[3 * pos_of[i] + k];
                if (pos_of[jb] >= 0) gb[k] = grad_color[3 * pos_of[jb] + k];
            }
            pair_edge(&c, x, y, xb, yb, key[i], key[jb], col + 3 * i, col + 3 * jb, ga, gb, &go);
        }
    }
    vertex_chain(&c, go.g_verts_screen, g_verts);
    free(go.g_verts_screen);
    free(idx); free(all); free(key); free(col); free(pos_of);
    ctx_free(&c);
    return 0;
}
