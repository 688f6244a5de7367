// C ABI of the gfx950 soup rasterizer: context, argument validation,
// workspace management and the launch sequence of each entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/diffsoup.h"
#include "internal.hpp"
#include "pform.hpp"

namespace {

using namespace soup;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct soup_ctx {
    int device = 0;
    int num_cus = 256;
    size_t lds_limit = 163840;   // LDS bytes one workgroup may use (the CU's whole LDS on this GPU)
    int tile = 16;
    bool counting = false;
    bool fixed = false;              // static-capacity mode: no synchronisation, no allocation
    bool flags_ready = false;        // sticky overflow flags cleared after allocation
    // the forward's fragment log: region size and count, hint for the next,
    // and the draws it was made with (valid only with bins_valid)
    bool log_valid = false;
    uint64_t log_region = 0, log_hint = 0;
    int log_regions = 0;
    uint64_t log_seed = 0;
    uint32_t log_step = 0;
    int log_mode = 0;
    // the setup records and tile lists in place: built for desc_cache, this tile size and near_w
    bool bins_valid = false;
    int bins_tile = 0;
    float bins_near_w = 0.0f;
    std::vector<char> desc_cache;    // descriptors of the last upload (static mode reuses them)
    std::string err;
    soup_stats stats{};
    DevBuf views, scenes, recs, tile_count, tile_fill, tile_start, bsum, entries, edge_w, partial, counters;
    DevBuf chunk_base;   // [binning chunks][tiles] first slot of a chunk in each tile list
    DevBuf tri_count, tri_fill, tri_off, tri_bsum, mlp_mid, frags, sorted;
    DevBuf region_counts, region_boff, flags;
    DevBuf log_frag, log_aux, log_counts, log_boff;   // the forward's fragment log
    DevBuf frag_gates, sorted_gates;                  // ReLU gates of the kept and sorted fragments
    bool frags_gated = false;        // the current fragment list carries the forward's gates
    DevBuf ssim;                                      // SSIM statistics of the training loss
    DevBuf gvert;                                     // the paper form's float64 vertex gradient sums
    DevBuf gtex;                                      // its texture gradient when levels are asked for and the sorted path cannot fold them in
    uint64_t region_hint = 0;        // largest replay-region count of the last call, to size the next
    uint64_t frag_region = 0;        // region size and count of the current fragment list
    int frag_regions = 0;
    void* host_stage = nullptr;      // pinned: descriptors up, totals down
    float* scratch = nullptr;        // this device's address of the allocation-free loss's static scratch
    size_t host_stage_bytes = 0;
    // optional per-kernel timing: recorded event pairs and a pool of free events
    bool timing = false;
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
};

namespace {

soup_status fail(soup_ctx* c, soup_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(ctx, SOUP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

soup_status ensure(soup_ctx* c, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return SOUP_OK;
    if (c->fixed)
        return fail(c, SOUP_ERR_CAPACITY, "static mode: a workspace of %zu bytes is needed (have %zu); run the "
                    "call once outside static mode to size it", bytes, b.bytes);
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return fail(c, SOUP_ERR_HIP, "hipFree failed: %s", hipGetErrorString(e));
    }
    size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(c, SOUP_ERR_OOM, "device allocation of %zu bytes failed", want);
    }
    b.bytes = want;
    return SOUP_OK;
}

soup_status ensure_host(soup_ctx* c, size_t bytes) {
    if (c->host_stage_bytes >= bytes) return SOUP_OK;
    if (c->host_stage) (void)hipHostFree(c->host_stage);
    c->host_stage = nullptr;
    c->host_stage_bytes = 0;
    size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
    if (hipHostMalloc(&c->host_stage, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, SOUP_ERR_OOM, "pinned host allocation of %zu bytes failed", want);
    }
    c->host_stage_bytes = want;
    return SOUP_OK;
}

}  // namespace

namespace {

hipEvent_t take_event(soup_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Brackets the launches made during its lifetime with two events (timing on).
struct Timed {
    soup_ctx* c;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Timed(soup_ctx* c_, int k, hipStream_t s_) : c(c_), kind(k), s(s_) {
        if (c->timing && !c->fixed && (a = take_event(c))) (void)hipEventRecord(a, s);
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) {
            c->pool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, s);
        c->marks.push_back({kind, a, b});
    }
};

}  // namespace

namespace soup {

int gate_words(MlpKind k) {
    switch (k) {
        case MlpKind::k8_16_1: return 1;
        case MlpKind::k16_32_2: return 2;
        case MlpKind::k32_64_2: return 4;
        default: return 0;
    }
}

MlpKind mlp_kind(int n_layers, const int32_t* dims) {
    if (n_layers == 2 && dims[0] == 8 && dims[1] == 16 && dims[2] == 4) return MlpKind::k8_16_1;
    if (n_layers == 3 && dims[0] == 16 && dims[1] == 32 && dims[2] == 32 && dims[3] == 4) return MlpKind::k16_32_2;
    if (n_layers == 3 && dims[0] == 32 && dims[1] == 64 && dims[2] == 64 && dims[3] == 4) return MlpKind::k32_64_2;
    return MlpKind::kNone;
}

int mlp_params(int n_layers, const int32_t* dims) {
    int n = 0;
    for (int l = 0; l < n_layers; ++l) n += dims[l + 1] * dims[l] + dims[l + 1];
    return n;
}

}  // namespace soup

namespace {

soup_status check_scene(soup_ctx* c, const soup_scene* s, MlpKind* kind) {
    if (!s) return fail(c, SOUP_ERR_INVALID, "scene is NULL");
    if (s->T < 0) return fail(c, SOUP_ERR_INVALID, "scene.T = %d < 0", s->T);
    if (s->G < 2 || s->G > 256) return fail(c, SOUP_ERR_INVALID, "scene.G = %d outside [2, 256]", s->G);
    if (s->n_layers < 1 || s->n_layers > 16 || !s->dims)
        return fail(c, SOUP_ERR_INVALID, "scene.n_layers = %d or dims missing", s->n_layers);
    if (s->dims[0] != s->C) return fail(c, SOUP_ERR_INVALID, "dims[0] = %d != C = %d", s->dims[0], s->C);
    if (s->dims[s->n_layers] != 4) return fail(c, SOUP_ERR_INVALID, "dims[last] = %d != 4", s->dims[s->n_layers]);
    if (static_cast<int64_t>(s->G) * s->G * s->C > 4096)
        return fail(c, SOUP_ERR_UNSUPPORTED, "G*G*C = %d exceeds the per-wave LDS gradient grid (4096 floats)",
                    s->G * s->G * s->C);
    if (s->T > 0 && (!s->verts || !s->feats || !s->mlp))
        return fail(c, SOUP_ERR_INVALID, "scene device pointers are NULL");
    *kind = soup::mlp_kind(s->n_layers, s->dims);
    if (*kind == MlpKind::kNone) {
        std::string d;
        for (int i = 0; i <= s->n_layers; ++i) d += (i ? "->" : "") + std::to_string(s->dims[i]);
        return fail(c, SOUP_ERR_UNSUPPORTED, "MLP shape %s is not compiled in (8->16->4, 16->32->32->4, 32->64->64->4)",
                    d.c_str());
    }
    return SOUP_OK;
}

// The backward decode keeps one triangle's gradient grid per wave in LDS: refuse a
// grid that would not fit one workgroup's LDS rather than launch it.
soup_status check_decode_lds(soup_ctx* c, MlpKind kind, int G, bool logp) {
    const size_t need = decode_bwd_lds(kind, G, logp);
    if (need > c->lds_limit)
        return fail(c, SOUP_ERR_UNSUPPORTED, "the backward decode needs %zu bytes of LDS per workgroup for G = %d "
                    "(the device has %zu): use a smaller texture grid", need, G, c->lds_limit);
    return SOUP_OK;
}

soup_status check_views(soup_ctx* c, const soup_views* v) {
    if (!v) return fail(c, SOUP_ERR_INVALID, "views is NULL");
    if (v->V < 1 || v->V > soup::kMaxViews) return fail(c, SOUP_ERR_INVALID, "views.V = %d outside [1, 65536]", v->V);
    if (!v->width || !v->height || !v->view_id || !v->view_proj)
        return fail(c, SOUP_ERR_INVALID, "views host arrays are NULL");
    for (int i = 0; i < v->V; ++i)
        if (v->width[i] < 1 || v->width[i] > 16384 || v->height[i] < 1 || v->height[i] > 16384)
            return fail(c, SOUP_ERR_INVALID, "view %d size %dx%d outside [1, 16384]", i, v->width[i], v->height[i]);
    return SOUP_OK;
}

soup_status check_opts(soup_ctx* c, const soup_opts* o) {
    if (!o) return fail(c, SOUP_ERR_INVALID, "opts is NULL");
    if (o->mode != 0 && o->mode != 1) return fail(c, SOUP_ERR_INVALID, "opts.mode = %d (0 or 1)", o->mode);
    if (o->accumulate != 0 && o->accumulate != 1)
        return fail(c, SOUP_ERR_INVALID, "opts.accumulate = %d (0 or 1)", o->accumulate);
    if (o->edge_pairs < 0 || o->edge_pairs > 2)
        return fail(c, SOUP_ERR_INVALID, "opts.edge_pairs = %d (0, 1 or 2)", o->edge_pairs);
    if (o->reuse_bins != 0 && o->reuse_bins != 1)
        return fail(c, SOUP_ERR_INVALID, "opts.reuse_bins = %d (0 or 1)", o->reuse_bins);
    if (!(o->near_w > 0.0f)) return fail(c, SOUP_ERR_INVALID, "opts.near_w must be > 0");
    return SOUP_OK;
}

Opts to_opts(const soup_opts* o) {
    Opts r{};
    r.seed = o->seed;
    r.step = o->step;
    r.mode = o->mode;
    r.bg[0] = o->background[0];
    r.bg[1] = o->background[1];
    r.bg[2] = o->background[2];
    r.edge_pairs = o->edge_pairs;
    r.near_w = o->near_w;
    r.accumulate = o->accumulate;
    r.reuse_bins = o->reuse_bins;
    return r;
}

// Per-call plan: descriptors and sizes.
struct Plan {
    std::vector<ViewDesc> views;
    std::vector<SceneDesc> scenes;
    int64_t n_tiles = 0, n_pix = 0, n_recs = 0;
    int maxT = 0;
    int G = 0;
    MlpKind kind = MlpKind::kNone;
    int n_params = 0;
};

void plan_views(Plan& p, const soup_views* v, int tile, const std::vector<int>& scene_of_view,
                const std::vector<int64_t>& rec_base) {
    p.views.resize(v->V);
    int64_t tb = 0, pb = 0;
    for (int i = 0; i < v->V; ++i) {
        ViewDesc& d = p.views[i];
        memset(&d, 0, sizeof(d));
        memcpy(d.M, v->view_proj + 16 * i, sizeof(d.M));
        d.W = v->width[i];
        d.H = v->height[i];
        d.view_id = v->view_id[i];
        d.scene = scene_of_view[i];
        d.tiles_x = (d.W + tile - 1) / tile;
        d.tiles_y = (d.H + tile - 1) / tile;
        d.T = p.scenes[d.scene].T;
        d.tile_base = tb;
        d.pix_base = pb;
        d.rec_base = rec_base[i];
        tb += static_cast<int64_t>(d.tiles_x) * d.tiles_y;
        pb += static_cast<int64_t>(d.W) * d.H;
        p.maxT = std::max(p.maxT, d.T);
    }
    p.n_tiles = tb;
    p.n_pix = pb;
}

bool same_descriptors(const soup_ctx* c, const Plan& p) {
    const size_t vbytes = p.views.size() * sizeof(ViewDesc), sbytes = p.scenes.size() * sizeof(SceneDesc);
    return c->desc_cache.size() == vbytes + sbytes && memcmp(c->desc_cache.data(), p.views.data(), vbytes) == 0 &&
           memcmp(c->desc_cache.data() + vbytes, p.scenes.data(), sbytes) == 0;
}

// Upload descriptors, run setup + scan, read the list size, scatter + sort.
soup_status bin(soup_ctx* c, Plan& p, const Opts& o, hipStream_t s) {
    const size_t vbytes = p.views.size() * sizeof(ViewDesc), sbytes = p.scenes.size() * sizeof(SceneDesc);
    const int chunk = bin_chunk_size(static_cast<int>(p.views.size()), p.maxT, c->num_cus);
    soup_status st;
    // the forward counts its regions in 32 bits
    if (p.n_tiles * fwd_regions_per_tile(c->tile, 8) >= (int64_t(1) << 32))
        return fail(c, SOUP_ERR_CAPACITY, "too many pixels in one call (2^32 forward regions)");
    if ((st = ensure(c, c->views, vbytes)) || (st = ensure(c, c->scenes, sbytes)) ||
        (st = ensure(c, c->recs, static_cast<size_t>(p.n_recs) * sizeof(TriRec))) ||
        (st = ensure(c, c->tile_count, static_cast<size_t>(p.n_tiles) * 4)) ||
        (st = ensure(c, c->tile_fill, static_cast<size_t>(p.n_tiles) * 4)) ||
        // per-chunk tile slots exist only for the LDS-histogram chunks (a small render's
        // one-triangle-per-thread chunks count with global atomics and need none)
        (st = ensure(c, c->chunk_base,
                     chunk >= kBinChunk ? static_cast<size_t>(bin_chunks(p.maxT, chunk)) * p.n_tiles * 4 : 0)) ||
        (st = ensure(c, c->tile_start, static_cast<size_t>(p.n_tiles + 1) * 8)) ||
        (st = ensure(c, c->bsum, static_cast<size_t>((p.n_tiles + 1023) / 1024 + 1) * 8)) ||
        (st = ensure(c, c->counters, 128)) || (st = ensure(c, c->flags, 256)) ||
        (st = ensure_host(c, vbytes + sbytes + 64)))
        return st;
    if (!c->flags_ready) {   // first allocation (never in static mode): clear the sticky flags
        launch_fill_i32(static_cast<int32_t*>(c->flags.p), 64, 0, s);
        c->flags_ready = true;
    }
    const bool same = same_descriptors(c, p);
    c->bins_valid = false;
    c->log_valid = false;
    if (c->fixed) {
        // a captured call must not depend on host memory at replay time
        if (!same) return fail(c, SOUP_ERR_INVALID, "static mode needs the views and scenes of the previous call");
    } else {
        // the previous call has drained this stream's use of the staging buffer
        HIP_TRY(c, hipStreamSynchronize(s));
        char* hs = static_cast<char*>(c->host_stage);
        memcpy(hs, p.views.data(), vbytes);
        memcpy(hs + vbytes, p.scenes.data(), sbytes);
        HIP_TRY(c, hipMemcpyAsync(c->views.p, hs, vbytes, hipMemcpyHostToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(c->scenes.p, hs + vbytes, sbytes, hipMemcpyHostToDevice, s));
        c->desc_cache.assign(hs, hs + vbytes + sbytes);
    }
    char* hs = static_cast<char*>(c->host_stage);
    unsigned long long* cnt = static_cast<unsigned long long*>(c->counters.p);
    {
        Timed t(c, SOUP_T_FILL, s);
        launch_fill_i32(reinterpret_cast<int32_t*>(cnt), 32, 0, s);
        launch_fill_i32(static_cast<int32_t*>(c->tile_count.p), p.n_tiles, 0, s);
    }
    {
    Timed t_setup(c, SOUP_T_SETUP, s);
    launch_setup(static_cast<ViewDesc*>(c->views.p), static_cast<int>(p.views.size()), p.maxT, chunk,
                 static_cast<SceneDesc*>(c->scenes.p), o, c->tile, static_cast<TriRec*>(c->recs.p),
                 static_cast<int32_t*>(c->tile_count.p), static_cast<int32_t*>(c->chunk_base.p), p.n_tiles,
                 c->counting ? cnt + 1 : nullptr, s);
    }
    {
        Timed t(c, SOUP_T_SCAN, s);
        launch_scan(static_cast<int32_t*>(c->tile_count.p), p.n_tiles, static_cast<int64_t*>(c->bsum.p),
                    static_cast<int64_t*>(c->tile_start.p), s);
    }
    int64_t total = -1;
    if (c->fixed) {
        // the capacity in place bounds the lists; an overflow empties them and is flagged
        launch_clip(static_cast<int64_t*>(c->tile_start.p), p.n_tiles, static_cast<int64_t>(c->entries.bytes / 8),
                    reinterpret_cast<unsigned int*>(cnt + 7), static_cast<unsigned int*>(c->flags.p), s);
    } else {
        int64_t* htotal = reinterpret_cast<int64_t*>(hs + vbytes + sbytes);
        HIP_TRY(c, hipMemcpyAsync(htotal, static_cast<int64_t*>(c->tile_start.p) + p.n_tiles, 8,
                                  hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipStreamSynchronize(s));
        total = *htotal;
        if ((st = ensure(c, c->entries, static_cast<size_t>(total) * 8))) return st;
    }
    {
        Timed t(c, SOUP_T_SCATTER, s);
        launch_fill_i32(static_cast<int32_t*>(c->tile_fill.p), p.n_tiles, 0, s);
        launch_scatter(static_cast<ViewDesc*>(c->views.p), static_cast<int>(p.views.size()), p.maxT, chunk, c->tile,
                       static_cast<TriRec*>(c->recs.p), static_cast<int64_t*>(c->tile_start.p), p.n_tiles,
                       static_cast<int32_t*>(c->chunk_base.p), static_cast<int32_t*>(c->tile_fill.p),
                       static_cast<uint64_t*>(c->entries.p), s);
    }
    {
        Timed t(c, SOUP_T_SORT, s);
        launch_sort(static_cast<int64_t*>(c->tile_start.p), p.n_tiles, static_cast<uint64_t*>(c->entries.p), s);
    }
    HIP_TRY(c, hipGetLastError());
    c->stats.pixels = p.n_pix;
    c->stats.tiles = p.n_tiles;
    c->stats.bin_entries = total;
    c->bins_valid = true;
    c->bins_tile = c->tile;
    c->bins_near_w = o.near_w;
    return SOUP_OK;
}

RasterArgs raster_args(soup_ctx* c, const Plan& p, const Opts& o) {
    RasterArgs a{};
    a.views = static_cast<ViewDesc*>(c->views.p);
    a.V = static_cast<int>(p.views.size());
    a.scenes = static_cast<SceneDesc*>(c->scenes.p);
    a.o = o;
    a.G = p.G;
    a.recs = static_cast<TriRec*>(c->recs.p);
    a.tile_start = static_cast<int64_t*>(c->tile_start.p);
    a.entries = static_cast<uint64_t*>(c->entries.p);
    a.n_tiles = p.n_tiles;
    unsigned long long* cnt = static_cast<unsigned long long*>(c->counters.p);
    a.counter = c->counting ? cnt : nullptr;
    a.work = reinterpret_cast<unsigned int*>(cnt + 2);
    // the forward's workgroups are single waves, one region of a tile at a time: 16x16 pixels, or a
    // single 8x8 block for 8-pixel tiles and for calls with fewer 16x16 regions than two per resident
    // wave (a small render); as many waves as are resident
    int region = 8;
    if (c->tile >= 16) {
        const int64_t r16 = p.n_tiles * fwd_regions_per_tile(c->tile, 16);
        const int64_t res16 = static_cast<int64_t>(c->num_cus) * raster_fwd_blocks_per_cu(c->tile, p.kind, 16);
        region = r16 >= 2 * res16 ? 16 : 8;
    }
    a.region = region;
    const int64_t items = p.n_tiles * fwd_regions_per_tile(c->tile, region);
    const int64_t resident = static_cast<int64_t>(c->num_cus) * raster_fwd_blocks_per_cu(c->tile, p.kind, region);
    a.n_blocks = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(resident, kMaxRegions), items)));
    return a;
}

soup_status finish_stats(soup_ctx* c, hipStream_t s, bool raster = true) {
    if (!c->counting || c->fixed) {
        c->stats.visible_tris = -1;
        c->stats.decodes = -1;
        c->stats.covered_pixels = -1;
        return SOUP_OK;
    }
    unsigned long long h[9];
    HIP_TRY(c, hipMemcpyAsync(h, c->counters.p, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    c->stats.decodes = static_cast<int64_t>(h[0]);
    c->stats.visible_tris = static_cast<int64_t>(h[1]);
    c->stats.covered_pixels = raster ? static_cast<int64_t>(h[8]) : -1;
    return SOUP_OK;
}

int persistent_blocks(soup_ctx* c, const Plan& p) {
    const int64_t want = static_cast<int64_t>(c->num_cus) * 4;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, p.n_tiles)));
}


soup_status plan_single(soup_ctx* c, Plan& p, const soup_scene* scene, const soup_views* views) {
    soup_status st = check_scene(c, scene, &p.kind);
    if (st) return st;
    if ((st = check_views(c, views))) return st;
    SceneDesc sd{};
    sd.verts = scene->verts;
    sd.feats = scene->feats;
    sd.mlp = scene->mlp;
    sd.T = scene->T;
    p.scenes = {sd};
    p.G = scene->G;
    p.n_params = mlp_params(scene->n_layers, scene->dims);
    std::vector<int> sov(views->V, 0);
    std::vector<int64_t> rb(views->V);
    for (int i = 0; i < views->V; ++i) rb[i] = static_cast<int64_t>(i) * scene->T;
    p.n_recs = static_cast<int64_t>(views->V) * scene->T;
    plan_views(p, views, c->tile, sov, rb);
    return SOUP_OK;
}

soup_status check_pscene(soup_ctx* c, const soup_pscene* s) {
    if (!s) return fail(c, SOUP_ERR_INVALID, "scene is NULL");
    if (s->T < 0) return fail(c, SOUP_ERR_INVALID, "scene.T = %d < 0", s->T);
    if (s->R < 0 || s->R > kPMaxR) return fail(c, SOUP_ERR_INVALID, "scene.R = %d outside [0, %d]", s->R, kPMaxR);
    if (s->T > 0 && (!s->verts || !s->tex || !s->mlp)) return fail(c, SOUP_ERR_INVALID, "scene device pointers are NULL");
    return SOUP_OK;
}

soup_status plan_paper(soup_ctx* c, Plan& p, const soup_pscene* scene, const soup_views* views,
                       const float* inv_view_proj) {
    soup_status st;
    if ((st = check_pscene(c, scene)) || (st = check_views(c, views))) return st;
    if (!inv_view_proj) return fail(c, SOUP_ERR_INVALID, "inv_view_proj is NULL");
    SceneDesc sd{};
    sd.verts = scene->verts;
    sd.feats = scene->tex;   // the raster reads the opacity channel through the feature pointer
    sd.mlp = scene->mlp;
    sd.T = scene->T;
    p.scenes = {sd};
    p.G = scene->R;          // ... and the texture level through the grid side
    p.kind = MlpKind::kPaper;
    p.n_params = kPParams;
    std::vector<int> sov(views->V, 0);
    std::vector<int64_t> rb(views->V);
    for (int i = 0; i < views->V; ++i) rb[i] = static_cast<int64_t>(i) * scene->T;
    p.n_recs = static_cast<int64_t>(views->V) * scene->T;
    plan_views(p, views, c->tile, sov, rb);
    for (int i = 0; i < views->V; ++i) memcpy(p.views[i].Mi, inv_view_proj + 16 * i, sizeof(p.views[i].Mi));
    return SOUP_OK;
}

}  // namespace

namespace {

// Scratch of soup_loss_l1_ssim_noalloc: the SSIM statistics record (12
// floats per pixel) of one view at a time. Every GPU the library runs on
// holds its own copy of this array until the process ends. Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): it uses the address hipGetSymbolAddress gives on each
// device, kept in noalloc_scratch_ptr.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];

std::mutex noalloc_scratch_mu;
float* noalloc_scratch_ptr[kNoAllocMaxDevices] = {};

// Once per device, with that device current: the device address of scratch.
soup_status noalloc_scratch_setup(soup_ctx* c) {
    std::lock_guard<std::mutex> lock(noalloc_scratch_mu);
    if (c->device >= kNoAllocMaxDevices)
        return fail(c, SOUP_ERR_UNSUPPORTED, "device %d: the allocation-free entry point supports devices 0..%d",
                    c->device, kNoAllocMaxDevices - 1);
    if (!noalloc_scratch_ptr[c->device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(c, SOUP_ERR_HIP, "hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
        }
        noalloc_scratch_ptr[c->device] = static_cast<float*>(p);
    }
    c->scratch = noalloc_scratch_ptr[c->device];
    return SOUP_OK;
}

}  // namespace

extern "C" {

soup_status soup_ctx_create(soup_ctx** out, int device) {
    if (!out) return SOUP_ERR_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return SOUP_ERR_HIP;
    }
    if (hipSetDevice(device) != hipSuccess) return SOUP_ERR_HIP;
    soup_ctx* c = new soup_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) == hipSuccess && lds > 0)
        c->lds_limit = static_cast<size_t>(lds);
    else
        (void)hipGetLastError();
    // error messages are formatted into a 512-byte buffer: with this capacity in
    // place, reporting one allocates no memory
    c->err.reserve(512);
    if (noalloc_scratch_setup(c) != SOUP_OK) {
        delete c;
        return SOUP_ERR_HIP;
    }
    *out = c;
    return SOUP_OK;
}

void soup_ctx_destroy(soup_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    DevBuf* bufs[] = {&c->views,     &c->scenes,    &c->recs,          &c->tile_count,  &c->tile_fill,
                      &c->tile_start, &c->bsum,      &c->entries,       &c->edge_w,      &c->partial,
                      &c->counters,   &c->tri_count, &c->tri_fill,      &c->tri_off,     &c->tri_bsum,
                      &c->mlp_mid,    &c->frags,     &c->sorted,        &c->region_counts, &c->region_boff,
                      &c->flags,      &c->log_frag,  &c->log_aux,       &c->log_counts,  &c->log_boff, &c->ssim,
                      &c->chunk_base, &c->frag_gates, &c->sorted_gates, &c->gvert, &c->gtex};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (c->host_stage) (void)hipHostFree(c->host_stage);
    for (auto& m : c->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

const char* soup_last_error(const soup_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

soup_status soup_ctx_set_tile(soup_ctx* c, int32_t tile) {
    if (!c) return SOUP_ERR_INVALID;
    if (tile != 8 && tile != 16 && tile != 32) return fail(c, SOUP_ERR_INVALID, "tile = %d (8, 16 or 32)", tile);
    c->tile = tile;
    return SOUP_OK;
}

int32_t soup_ctx_get_tile(const soup_ctx* c) { return c ? c->tile : 0; }

soup_status soup_ctx_set_timing(soup_ctx* c, int32_t on) {
    if (!c) return SOUP_ERR_INVALID;
    c->timing = on != 0;
    return SOUP_OK;
}

soup_status soup_read_timings(soup_ctx* c, double* ms, int64_t* count) {
    if (!c || !ms || !count) return SOUP_ERR_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    for (auto& m : c->marks) {
        HIP_TRY(c, hipEventSynchronize(m.b));
        float t = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&t, m.a, m.b));
        if (m.kind >= 0 && m.kind < SOUP_TIMING_KINDS) {
            ms[m.kind] += t;
            count[m.kind] += 1;
        }
        c->pool.push_back(m.a);
        c->pool.push_back(m.b);
    }
    c->marks.clear();
    return SOUP_OK;
}

soup_status soup_ctx_set_static(soup_ctx* c, int32_t on) {
    if (!c) return SOUP_ERR_INVALID;
    if (on && (c->counting || c->timing))
        return fail(c, SOUP_ERR_INVALID, "static mode excludes counting and timing (both synchronise)");
    c->fixed = on != 0;
    return SOUP_OK;
}

soup_status soup_ctx_check(soup_ctx* c) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (!c->flags.p) return SOUP_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    unsigned int h[2] = {0, 0};
    HIP_TRY(c, hipMemcpy(h, c->flags.p, sizeof(h), hipMemcpyDeviceToHost));
    h[0] &= kOverflowBins | kOverflowFragments;
    if (!h[0]) return SOUP_OK;
    const unsigned int zero[2] = {0, 0};
    HIP_TRY(c, hipMemcpy(c->flags.p, zero, sizeof(zero), hipMemcpyHostToDevice));
    return fail(c, SOUP_ERR_CAPACITY, "a static-mode call overflowed its %s%s%s; rerun outside static mode to grow "
                "the workspaces", (h[0] & kOverflowBins) ? "tile lists" : "",
                (h[0] & kOverflowBins) && (h[0] & kOverflowFragments) ? " and " : "",
                (h[0] & kOverflowFragments) ? "fragment list" : "");
}

soup_status soup_ctx_set_counting(soup_ctx* c, int32_t on) {
    if (!c) return SOUP_ERR_INVALID;
    c->counting = on != 0;
    return SOUP_OK;
}

soup_status soup_ctx_workspace_bytes(const soup_ctx* c, int64_t* bytes) {
    if (!c || !bytes) return SOUP_ERR_INVALID;
    const DevBuf* bufs[] = {&c->views,     &c->scenes,    &c->recs,          &c->tile_count,  &c->tile_fill,
                            &c->tile_start, &c->bsum,      &c->entries,       &c->edge_w,      &c->partial,
                            &c->counters,   &c->tri_count, &c->tri_fill,      &c->tri_off,     &c->tri_bsum,
                            &c->mlp_mid,    &c->frags,     &c->sorted,        &c->region_counts, &c->region_boff,
                            &c->flags,      &c->log_frag,  &c->log_aux,       &c->log_counts,  &c->log_boff, &c->ssim,
                            &c->chunk_base, &c->frag_gates, &c->sorted_gates, &c->gvert, &c->gtex};
    int64_t n = 0;
    for (const DevBuf* b : bufs) n += static_cast<int64_t>(b->bytes);
    *bytes = n;
    return SOUP_OK;
}

soup_status soup_last_stats(const soup_ctx* c, soup_stats* out) {
    if (!c || !out) return SOUP_ERR_INVALID;
    *out = c->stats;
    return SOUP_OK;
}

// Persistent grid of the replay: 4 workgroups per CU, at most kMaxRegions waves.
int replay_blocks(soup_ctx* c, const Plan& p) {
    const int wpb = replay_waves_per_block(c->tile);
    const int64_t want = std::min<int64_t>(static_cast<int64_t>(c->num_cus) * 4, kMaxRegions / wpb);
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, p.n_tiles)));
}

// Persistent grid of the decode kernel: 4 waves per workgroup, 4 workgroups per CU.
int decode_blocks(soup_ctx* c) { return std::max(1, std::min(c->num_cus * 4, kMaxRegions / 4)); }

// Backward, part 1: gather the fragments the backward needs into c->frags,
// one region per wave, then scan the region counts into batch offsets. The
// fragments come from the replay (coverage re-run from the tile lists) or,
// when from_log, from the filter of the forward's log. Regions are sized
// from the last call's largest count, doubled (else from 1.5
// fragments per pixel); an overflow is detected from the counts and the
// gather runs again, sized exactly. Returns the number of fragments in
// *n_frag and of decode batches in *n_batch.
soup_status replay(soup_ctx* c, const Plan& p, const RasterArgs& a, const uint64_t* vis, const float* grad_color,
                   const float* grad_logp, const float2* edge_w, bool all_front, int32_t* tri_count, int T,
                   hipStream_t s, int64_t* n_frag, int64_t* n_batch, bool from_log = false, bool want_gates = false) {
    // the forward's ReLU gates travel with the fragments when they come from its log
    want_gates = want_gates && from_log;
    c->frags_gated = want_gates;
    if (p.n_pix >= (int64_t(1) << 32)) return fail(c, SOUP_ERR_CAPACITY, "backward needs fewer than 2^32 pixels per call");
    unsigned long long* cnt = static_cast<unsigned long long*>(c->counters.p);
    const int nb = from_log ? decode_blocks(c) : replay_blocks(c, p);
    const int nr = nb * (from_log ? 4 : replay_waves_per_block(c->tile));
    // per-wave counts vary between calls (tiles are handed out dynamically):
    // twice the last call's largest, so that a static-mode call fits
    uint64_t hint = c->region_hint;
    if (hint && c->frag_regions && c->frag_regions != nr) hint = hint * c->frag_regions / nr + 64;
    uint64_t region = hint ? 2 * hint + 1024 : (static_cast<uint64_t>(p.n_pix) * 3 / 2) / nr + 1024;
    soup_status st;
    if ((st = ensure(c, c->region_counts, static_cast<size_t>(kMaxRegions) * 4)) ||
        (st = ensure(c, c->region_boff, static_cast<size_t>(kMaxRegions + 1) * 4)))
        return st;
    const int gw = gate_words(p.kind);
    auto launch = [&](uint64_t reg) {
        if (from_log) {
            CollectArgs ca{};
            ca.log_frag = static_cast<uint4*>(c->log_frag.p);
            ca.log_aux = static_cast<uint2*>(c->log_aux.p);
            ca.gate_words = gw;   // the log's record layout
            if (want_gates) ca.frag_gates = static_cast<uint32_t*>(c->frag_gates.p);
            ca.log_region = static_cast<uint32_t>(c->log_region);
            ca.log_counts = static_cast<uint32_t*>(c->log_counts.p);
            ca.log_boff = static_cast<uint32_t*>(c->log_boff.p);
            ca.log_regions = c->log_regions;
            ca.vis = vis;
            ca.grad_logp = grad_logp;
            ca.all_front = all_front ? 1 : 0;
            ca.frags = static_cast<FragRec*>(c->frags.p);
            ca.region = static_cast<uint32_t>(reg);
            ca.counts = static_cast<uint32_t*>(c->region_counts.p);
            ca.tri_count = tri_count;
            ca.n_blocks = nb;
            launch_collect(ca, s);
        } else {
            ReplayArgs ra{};
            ra.r = a;
            ra.vis = vis;
            ra.grad_color = grad_color;
            ra.grad_logp = grad_logp;
            ra.edge_w = edge_w;
            ra.all_front = all_front ? 1 : 0;
            ra.frags = static_cast<FragRec*>(c->frags.p);
            ra.region = static_cast<uint32_t>(reg);
            ra.counts = static_cast<uint32_t*>(c->region_counts.p);
            ra.tri_count = tri_count;
            ra.n_blocks = nb;
            launch_replay(ra, c->tile, s);
        }
        launch_region_scan(static_cast<uint32_t*>(c->region_counts.p), nr, static_cast<uint32_t>(reg),
                           static_cast<uint32_t*>(c->region_boff.p), cnt + 4, static_cast<unsigned int*>(c->flags.p),
                           s);
    };
    if (c->fixed) {
        // the fragment list in place bounds the regions; an overflow is flagged
        if (c->frag_regions != nr || c->frag_region == 0)
            return fail(c, SOUP_ERR_CAPACITY, "static mode: no fragment list sized for this call; run it once "
                        "outside static mode");
        if (want_gates && c->frag_gates.bytes < static_cast<size_t>(c->frag_region) * nr * gate_stride(gw) * 4)
            return fail(c, SOUP_ERR_CAPACITY, "static mode: no gate list sized for this call; run it once "
                        "outside static mode");
        launch_fill_i32(reinterpret_cast<int32_t*>(a.work), 1, 0, s);
        if (tri_count) launch_fill_i32(tri_count, T, 0, s);
        launch(c->frag_region);
        HIP_TRY(c, hipGetLastError());
        *n_frag = -1;
        *n_batch = static_cast<int64_t>(nr) * static_cast<int64_t>((c->frag_region + 63) / 64);   // upper bound
        return SOUP_OK;
    }
    uint64_t summary[3] = {0, 0, 0};
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (region >= (uint64_t(1) << 31)) return fail(c, SOUP_ERR_CAPACITY, "fragment region too large");
        if ((st = ensure(c, c->frags, static_cast<size_t>(region) * nr * sizeof(FragRec)))) return st;
        if (want_gates && (st = ensure(c, c->frag_gates, static_cast<size_t>(region) * nr * gate_stride(gw) * 4)))
            return st;
        {
            Timed t(c, SOUP_T_FILL, s);
            launch_fill_i32(reinterpret_cast<int32_t*>(a.work), 1, 0, s);
            if (tri_count) launch_fill_i32(tri_count, T, 0, s);
        }
        {
            Timed t(c, SOUP_T_REPLAY, s);
            launch(region);
        }
        HIP_TRY(c, hipGetLastError());
        uint64_t* h = reinterpret_cast<uint64_t*>(c->host_stage);
        HIP_TRY(c, hipMemcpyAsync(h, cnt + 4, 24, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        memcpy(summary, h, sizeof(summary));
        if (summary[2] <= region) break;
        region = summary[2] + summary[2] / 8 + 64;
    }
    if (summary[2] > region) return fail(c, SOUP_ERR_CAPACITY, "fragment list overflowed twice");
    c->region_hint = summary[2];
    c->frag_region = region;
    c->frag_regions = nr;
    *n_frag = static_cast<int64_t>(summary[0]);
    *n_batch = static_cast<int64_t>(summary[1]);
    return SOUP_OK;
}

// The forward raster, with the log of its decoded fragments when `keep`: the
// log is sized from the last call's largest region count (twice, so that a
// static-mode call fits), its counts are scanned, and an eager call reads
// whether it overflowed (an overflowing log is simply not used: the backward
// replays).
static soup_status raster_forward(soup_ctx* c, const Plan& p, const Opts& o, RasterArgs& a, bool keep,
                                  hipStream_t s) {
    soup_status st;
    const int log_nr = a.n_blocks;   // one log region per forward wave
    uint64_t log_region = 0;
    if (keep) {
        if (c->fixed) {
            if (c->log_regions != log_nr || c->log_region == 0)
                return fail(c, SOUP_ERR_CAPACITY, "static mode: no fragment log sized for this call; run it once "
                            "outside static mode");
            log_region = c->log_region;
        } else {
            // twice the last call's largest count: per-wave counts vary from call to
            // call (regions are handed out dynamically), and a static-mode call
            // (which cannot grow the log) must fit
            log_region = c->log_hint ? 2 * c->log_hint + 1024
                                     : (static_cast<uint64_t>(p.n_pix) * 2) / log_nr + 1024;
            if (log_region >= (uint64_t(1) << 31)) return fail(c, SOUP_ERR_CAPACITY, "fragment log region too large");
            if ((st = ensure(c, c->log_frag, static_cast<size_t>(log_region) * log_nr * sizeof(uint4))) ||
                (st = ensure(c, c->log_aux, static_cast<size_t>(log_region) * log_nr * aux_words(gate_words(p.kind)) * 4)) ||
                (st = ensure(c, c->log_counts, static_cast<size_t>(kMaxRegions) * 4)) ||
                (st = ensure(c, c->log_boff, static_cast<size_t>(kMaxRegions + 1) * 4)))
                return st;
        }
        a.log_frag = static_cast<uint4*>(c->log_frag.p);
        a.log_aux = static_cast<uint2*>(c->log_aux.p);
        a.log_region = static_cast<uint32_t>(log_region);
        a.log_counts = static_cast<uint32_t*>(c->log_counts.p);
    }
    launch_fill_i32(reinterpret_cast<int32_t*>(a.work), 1, 0, s);
    {
        Timed t(c, SOUP_T_FWD, s);
        launch_raster_fwd(a, c->tile, p.kind, s);
    }
    HIP_TRY(c, hipGetLastError());
    if (keep) {
        unsigned long long* cnt = static_cast<unsigned long long*>(c->counters.p);
        // an eager call reads the largest count: an overflowing log is simply not
        // used (the backward replays); in static mode the overflow is flagged
        launch_region_scan(a.log_counts, log_nr, a.log_region, static_cast<uint32_t*>(c->log_boff.p), cnt + 4,
                           c->fixed ? static_cast<unsigned int*>(c->flags.p) : nullptr, s);
        HIP_TRY(c, hipGetLastError());
        bool ok = true;
        if (!c->fixed) {
            uint64_t* h = reinterpret_cast<uint64_t*>(c->host_stage);
            HIP_TRY(c, hipMemcpyAsync(h, cnt + 4, 24, hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipStreamSynchronize(s));
            ok = h[2] <= log_region;
            c->log_hint = h[2];
        }
        c->log_valid = ok;
        c->log_region = log_region;
        c->log_regions = log_nr;
        c->log_seed = o.seed;
        c->log_step = o.step;
        c->log_mode = o.mode;
    }
    return SOUP_OK;
}

DecodeArgs decode_args(soup_ctx* c, const Plan& p, const RasterArgs& a) {
    DecodeArgs d{};
    d.views = a.views;
    d.V = a.V;
    d.recs = a.recs;
    d.feats = p.scenes[0].feats;
    d.mlp = p.scenes[0].mlp;
    d.G = p.G;
    d.T = p.scenes[0].T;
    d.verts = p.scenes[0].verts;
    d.frags = static_cast<FragRec*>(c->frags.p);
    d.region = static_cast<uint32_t>(c->frag_region);
    d.counts = static_cast<uint32_t*>(c->region_counts.p);
    d.boff = static_cast<uint32_t*>(c->region_boff.p);
    d.n_regions = c->frag_regions;
    d.counter = a.counter;
    d.n_blocks = decode_blocks(c);
    return d;
}

soup_status soup_rasterize_fwd(soup_ctx* c, const soup_scene* scene, const soup_views* views, const soup_opts* opts,
                               uint64_t* vis, float* color, float* logp, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    hipStream_t s = static_cast<hipStream_t>(stream);
    soup_status st;
    Plan p;
    if ((st = plan_single(c, p, scene, views))) return st;
    if ((st = check_opts(c, opts))) return st;
    if (!vis || !color) return fail(c, SOUP_ERR_INVALID, "vis and color outputs are required");
    if (logp && (st = check_decode_lds(c, p.kind, p.G, true))) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    const Opts o = to_opts(opts);
    if ((st = bin(c, p, o, s))) return st;
    RasterArgs a = raster_args(c, p, o);
    a.vis = vis;
    a.color = color;
    // reuse_bins: keep a log of the decoded fragments for the backward
    const bool keep = o.reuse_bins != 0;
    if ((st = raster_forward(c, p, o, a, keep, s))) return st;
    if (logp) {
        Timed t(c, SOUP_T_LOGP, s);
        launch_fill_f32(logp, p.n_pix, 0.0f, s);
        if (o.mode == 0) {
            RasterArgs ra = a;
            ra.counter = nullptr;
            int64_t n_frag = 0, n_batch = 0;
            if ((st = replay(c, p, ra, vis, nullptr, nullptr, nullptr, true, nullptr, 0, s, &n_frag, &n_batch,
                             keep && c->log_valid)))
                return st;
            DecodeArgs d = decode_args(c, p, ra);
            d.logp = logp;
            launch_decode_bwd(d, p.kind, true, s);
        }
        HIP_TRY(c, hipGetLastError());
    }
    return finish_stats(c, s);
}

soup_status soup_rasterize_bwd(soup_ctx* c, const soup_scene* scene, const soup_views* views, const soup_opts* opts,
                               const uint64_t* vis, const float* color, const float* grad_color,
                               const float* grad_logp, float* grad_verts, float* grad_feats, float* grad_mlp,
                               void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    hipStream_t s = static_cast<hipStream_t>(stream);
    soup_status st;
    Plan p;
    if ((st = plan_single(c, p, scene, views))) return st;
    if ((st = check_opts(c, opts))) return st;
    if (!vis || !color || !grad_color) return fail(c, SOUP_ERR_INVALID, "vis, color and grad_color are required");
    if (!grad_verts || !grad_feats || !grad_mlp) return fail(c, SOUP_ERR_INVALID, "gradient outputs are required");
    if ((st = check_decode_lds(c, p.kind, p.G, false))) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    const Opts o = to_opts(opts);
    bool reused = false;
    if (o.reuse_bins && c->bins_valid && c->bins_tile == c->tile && c->bins_near_w == o.near_w &&
        same_descriptors(c, p)) {
        // the last forward's setup records and tile lists are those of these inputs
        launch_fill_i32(static_cast<int32_t*>(c->counters.p), 32, 0, s);
        reused = true;
    } else if ((st = bin(c, p, o, s))) {
        return st;
    }
    // ... and its fragment log, if it was made with these draws
    const bool from_log = reused && c->log_valid && c->log_seed == o.seed && c->log_step == o.step &&
                          c->log_mode == o.mode;
    const int nb = decode_blocks(c);
    const int rows = nb * 4;
    const int T = scene->T;
    const int64_t n_grid = static_cast<int64_t>(scene->G) * scene->G * scene->C;
    if ((st = ensure(c, c->edge_w, static_cast<size_t>(p.n_pix) * sizeof(float2))) ||
        (st = ensure(c, c->partial, static_cast<size_t>(rows) * p.n_params * 4)) ||
        (st = ensure(c, c->mlp_mid, static_cast<size_t>(mlp_reduce_mid_rows(rows)) * p.n_params * 8)) ||
        (st = ensure(c, c->tri_count, static_cast<size_t>(T) * 4)) ||
        (st = ensure(c, c->tri_fill, static_cast<size_t>(T) * 8)) ||
        (st = ensure(c, c->tri_off, static_cast<size_t>(T + 1) * 8)) ||
        (st = ensure(c, c->tri_bsum, static_cast<size_t>((T + 1023) / 1024 + 1) * 8)))
        return st;
    RasterArgs a = raster_args(c, p, o);
    const float* gl = o.mode == 0 ? grad_logp : nullptr;
    const float2* ew = nullptr;
    if (o.edge_pairs != 2) {
        Timed t(c, SOUP_T_EDGE, s);
        launch_edge_weights(a.views, a.V, p.n_pix, o, vis, color, grad_color, static_cast<float2*>(c->edge_w.p), s);
        ew = static_cast<float2*>(c->edge_w.p);
    }
    int64_t n_frag = 0, n_batch = 0;
    if ((st = replay(c, p, a, vis, grad_color, gl, ew, false, static_cast<int32_t*>(c->tri_count.p), T, s, &n_frag,
                     &n_batch, from_log, true)))
        return st;
    // the list sorted by triangle has at most as many entries as the regions hold
    const int64_t frag_cap = static_cast<int64_t>(c->frag_regions) * static_cast<int64_t>(c->frag_region);
    const int gw = gate_words(p.kind);
    if (!c->frags_gated) {
        // replayed fragments: their ReLU gates from a decode in the forward's arithmetic
        if ((st = ensure(c, c->frag_gates, static_cast<size_t>(frag_cap) * gate_stride(gw) * 4))) return st;
        Timed t(c, SOUP_T_REPLAY, s);
        launch_fragment_gates(decode_args(c, p, a), p.kind, static_cast<uint32_t*>(c->frag_gates.p), s);
        c->frags_gated = true;
    }
    if ((st = ensure(c, c->sorted, static_cast<size_t>(frag_cap) * sizeof(FragRec)))) return st;
    if (c->frags_gated && (st = ensure(c, c->sorted_gates, static_cast<size_t>(frag_cap) * gate_stride(gw) * 4)))
        return st;
    {
        Timed t(c, SOUP_T_GRAD, s);
        launch_scan(static_cast<int32_t*>(c->tri_count.p), T, static_cast<int64_t*>(c->tri_bsum.p),
                    static_cast<int64_t*>(c->tri_off.p), s);
        launch_fill_i32(static_cast<int32_t*>(c->tri_fill.p), 2 * T, 0, s);
        PlaceArgs pa{};
        pa.frags = static_cast<FragRec*>(c->frags.p);
        pa.region = static_cast<uint32_t>(c->frag_region);
        pa.counts = static_cast<uint32_t*>(c->region_counts.p);
        pa.boff = static_cast<uint32_t*>(c->region_boff.p);
        pa.n_regions = c->frag_regions;
        pa.tri_off = static_cast<int64_t*>(c->tri_off.p);
        pa.tri_fill = static_cast<unsigned long long*>(c->tri_fill.p);
        pa.sorted = static_cast<FragRec*>(c->sorted.p);
        if (c->frags_gated) {
            pa.frag_gates = static_cast<uint32_t*>(c->frag_gates.p);
            pa.sorted_gates = static_cast<uint32_t*>(c->sorted_gates.p);
            pa.gate_words = gw;
        }
        pa.n_blocks = decode_blocks(c);
        launch_place(pa, s);
    }
    {
        Timed t(c, SOUP_T_FILL, s);
        if (!o.accumulate) {
            launch_fill_f32(grad_feats, static_cast<int64_t>(T) * n_grid, 0.0f, s);
            launch_fill_f32(grad_verts, static_cast<int64_t>(T) * 9, 0.0f, s);
        }
    }
    {
        DecodeArgs d = decode_args(c, p, a);
        d.sorted = static_cast<FragRec*>(c->sorted.p);
        d.sorted_gates = c->frags_gated ? static_cast<uint32_t*>(c->sorted_gates.p) : nullptr;
        d.tri_off = static_cast<int64_t*>(c->tri_off.p);
        d.grad_color = grad_color;
        d.edge_w = ew;
        d.grad_feats = grad_feats;
        d.grad_verts = grad_verts;
        d.accumulate = o.accumulate;
        d.mlp_partial = static_cast<float*>(c->partial.p);
        Timed t(c, SOUP_T_BWD, s);
        launch_decode_bwd(d, p.kind, false, s);
    }
    HIP_TRY(c, hipGetLastError());
    {
        Timed t(c, SOUP_T_REDUCE, s);
        launch_mlp_reduce(static_cast<float*>(c->partial.p), rows, p.n_params, static_cast<double*>(c->mlp_mid.p),
                          grad_mlp, o.accumulate != 0, s);
    }
    HIP_TRY(c, hipGetLastError());
    return finish_stats(c, s, false);
}

soup_status soup_render(soup_ctx* c, const soup_scene* scenes, int32_t R, const soup_views* views,
                        const soup_opts* opts, float* const* color, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    hipStream_t s = static_cast<hipStream_t>(stream);
    soup_status st;
    if (R < 1 || !scenes || !color) return fail(c, SOUP_ERR_INVALID, "render needs R >= 1 scenes and outputs");
    if ((st = check_views(c, views))) return st;
    if (views->V != R) return fail(c, SOUP_ERR_INVALID, "views.V = %d != R = %d", views->V, R);
    if ((st = check_opts(c, opts))) return st;
    Plan p;
    std::vector<int> sov(R);
    std::vector<int64_t> rb(R);
    int64_t recs = 0;
    for (int r = 0; r < R; ++r) {
        MlpKind k;
        if ((st = check_scene(c, &scenes[r], &k))) return st;
        if (r == 0) {
            p.kind = k;
            p.G = scenes[0].G;
        } else if (k != p.kind || scenes[r].G != p.G || scenes[r].C != scenes[0].C) {
            return fail(c, SOUP_ERR_INVALID, "request %d: all scenes of a batch must share G, C and the MLP shape", r);
        }
        if (!color[r]) return fail(c, SOUP_ERR_INVALID, "request %d: color output is NULL", r);
        SceneDesc sd{};
        sd.verts = scenes[r].verts;
        sd.feats = scenes[r].feats;
        sd.mlp = scenes[r].mlp;
        sd.T = scenes[r].T;
        p.scenes.push_back(sd);
        sov[r] = r;
        rb[r] = recs;
        recs += scenes[r].T;
    }
    p.n_recs = recs;
    plan_views(p, views, c->tile, sov, rb);
    for (int r = 0; r < R; ++r) p.views[r].color_out = color[r];
    HIP_TRY(c, hipSetDevice(c->device));
    const Opts o = to_opts(opts);
    if ((st = bin(c, p, o, s))) return st;
    RasterArgs a = raster_args(c, p, o);
    a.vis = nullptr;
    a.color = nullptr;
    launch_fill_i32(reinterpret_cast<int32_t*>(a.work), 1, 0, s);
    {
        Timed t(c, SOUP_T_FWD, s);
        launch_raster_fwd(a, c->tile, p.kind, s);
    }
    HIP_TRY(c, hipGetLastError());
    return finish_stats(c, s);
}

soup_status soup_pforward(soup_ctx* c, const soup_pscene* scene, const soup_views* views, const float* inv_view_proj,
                          const soup_opts* opts, uint64_t* vis, float* color, float* logp, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    hipStream_t s = static_cast<hipStream_t>(stream);
    soup_status st;
    Plan p;
    if ((st = plan_paper(c, p, scene, views, inv_view_proj))) return st;
    if ((st = check_opts(c, opts))) return st;
    if (!vis || !color) return fail(c, SOUP_ERR_INVALID, "vis and color outputs are required");
    HIP_TRY(c, hipSetDevice(c->device));
    const Opts o = to_opts(opts);
    if ((st = bin(c, p, o, s))) return st;
    RasterArgs a = raster_args(c, p, o);
    a.vis = vis;
    a.color = color;
    const bool keep = o.reuse_bins != 0 || (logp && o.mode == 0);
    if ((st = raster_forward(c, p, o, a, keep, s))) return st;
    {
        Timed t(c, SOUP_T_SHADE, s);
        PShadeArgs sa{};
        sa.views = a.views;
        sa.V = a.V;
        sa.P = p.n_pix;
        sa.recs = a.recs;
        sa.tex = scene->tex;
        sa.mlp = scene->mlp;
        sa.R = scene->R;
        sa.vis = vis;
        sa.color = color;
        sa.o = o;
        launch_pshade(sa, s);
    }
    HIP_TRY(c, hipGetLastError());
    if (logp) {
        Timed t(c, SOUP_T_LOGP, s);
        launch_fill_f32(logp, p.n_pix, 0.0f, s);
        if (o.mode == 0) {
            RasterArgs ra = a;
            ra.counter = nullptr;
            int64_t n_frag = 0, n_batch = 0;
            if ((st = replay(c, p, ra, vis, nullptr, nullptr, nullptr, true, nullptr, 0, s, &n_frag, &n_batch,
                             c->log_valid)))
                return st;
            PFragArgs fa{};
            fa.frags = static_cast<FragRec*>(c->frags.p);
            fa.region = static_cast<uint32_t>(c->frag_region);
            fa.counts = static_cast<uint32_t*>(c->region_counts.p);
            fa.boff = static_cast<uint32_t*>(c->region_boff.p);
            fa.n_regions = c->frag_regions;
            fa.tex = scene->tex;
            fa.R = scene->R;
            fa.logp = logp;
            fa.n_blocks = decode_blocks(c);
            launch_pfrag(fa, true, s);
        }
        HIP_TRY(c, hipGetLastError());
    }
    return finish_stats(c, s);
}

static soup_status check_levels(soup_ctx* c, int32_t T, int32_t Rmin, int32_t Rtop, int32_t Rmax) {
    if (T < 0) return fail(c, SOUP_ERR_INVALID, "T = %d < 0", T);
    if (Rmin < 0 || Rtop < Rmin || Rmax < Rtop || Rmax > kPMaxR || Rtop - Rmin + 1 > kPMaxLevels)
        return fail(c, SOUP_ERR_INVALID, "levels Rmin = %d, Rtop = %d, Rmax = %d: need 0 <= Rmin <= Rtop <= Rmax <= %d",
                    Rmin, Rtop, Rmax, kPMaxR);
    return SOUP_OK;
}

// The learnable levels a backward writes instead of the assembled texture's gradient.
struct LevelsOut {
    int Rmin, Rtop;
    float* const* graw;
};

static soup_status pbackward_impl(soup_ctx* c, const soup_pscene* scene, const soup_views* views,
                                  const float* inv_view_proj, const soup_opts* opts, const uint64_t* vis,
                                  const float* color, const float* grad_color, const float* grad_logp,
                                  float* grad_verts, float* grad_tex, const LevelsOut* lv, float* grad_mlp,
                                  void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    hipStream_t s = static_cast<hipStream_t>(stream);
    soup_status st;
    Plan p;
    if ((st = plan_paper(c, p, scene, views, inv_view_proj))) return st;
    if ((st = check_opts(c, opts))) return st;
    if (!vis || !color || !grad_color) return fail(c, SOUP_ERR_INVALID, "vis, color and grad_color are required");
    // an empty soup has empty vertex and texture gradients (their pointers may be NULL)
    if (!grad_mlp || (scene->T > 0 && (!grad_verts || (!lv && !grad_tex))))
        return fail(c, SOUP_ERR_INVALID, "gradient outputs are required");
    if (lv) {
        if ((st = check_levels(c, scene->T, lv->Rmin, lv->Rtop, scene->R))) return st;
        if (scene->T > 0) {
            if (!lv->graw) return fail(c, SOUP_ERR_INVALID, "grad_raw is NULL");
            for (int l = 0; l <= lv->Rtop - lv->Rmin; ++l)
                if (!lv->graw[l]) return fail(c, SOUP_ERR_INVALID, "grad_raw[%d] (level %d) is NULL", l, lv->Rmin + l);
        }
    }
    HIP_TRY(c, hipSetDevice(c->device));
    const Opts o = to_opts(opts);
    bool reused = false;
    if (o.reuse_bins && c->bins_valid && c->bins_tile == c->tile && c->bins_near_w == o.near_w &&
        same_descriptors(c, p)) {
        launch_fill_i32(static_cast<int32_t*>(c->counters.p), 32, 0, s);
        reused = true;
    } else if ((st = bin(c, p, o, s))) {
        return st;
    }
    const bool from_log = reused && c->log_valid && c->log_seed == o.seed && c->log_step == o.step &&
                          c->log_mode == o.mode;
    const int T = scene->T;
    const int64_t n_tex = static_cast<int64_t>(T) * mc_count(scene->R) * kPCh;
    // the triangle-sorted path keeps one triangle's texture gradient per wave in LDS
    // (18 KB at R = 5); a texture too large for that takes the per-pixel path with
    // global atomics
    const bool sorted_path = ptri_bwd_lds(scene->R) <= 65536;
    // levels: folded into the sorted path's flush where level R - 1 fits its stage;
    // otherwise the texture gradient goes to a workspace and through the assembly's
    // backward
    const bool fused = lv && sorted_path && ptri_levels_fit(scene->R);
    if (lv && !fused) {
        if ((st = ensure(c, c->gtex, static_cast<size_t>(n_tex) * sizeof(float)))) return st;
        grad_tex = static_cast<float*>(c->gtex.p);
    }
    const int nb = sorted_path ? ptri_blocks(c->num_cus, scene->R) : pwinner_blocks(c->num_cus);
    const int rows = sorted_path ? nb : nb * 4;
    if ((st = ensure(c, c->edge_w, static_cast<size_t>(p.n_pix) * sizeof(float2))) ||
        (st = ensure(c, c->partial, static_cast<size_t>(rows) * kPParams * 4)) ||
        (st = ensure(c, c->mlp_mid, static_cast<size_t>(mlp_reduce_mid_rows(rows)) * kPParams * 8)) ||
        (st = ensure(c, c->gvert, static_cast<size_t>(T) * 9 * sizeof(double))) ||
        (st = ensure(c, c->tri_count, static_cast<size_t>(T) * 4)) ||
        (st = ensure(c, c->tri_fill, static_cast<size_t>(T) * 8)) ||
        (st = ensure(c, c->tri_off, static_cast<size_t>(T + 1) * 8)) ||
        (st = ensure(c, c->tri_bsum, static_cast<size_t>((T + 1023) / 1024 + 1) * 8)))
        return st;
    RasterArgs a = raster_args(c, p, o);
    const float2* ew = nullptr;
    if (o.edge_pairs != 2) {
        Timed t(c, SOUP_T_EDGE, s);
        launch_edge_weights(a.views, a.V, p.n_pix, o, vis, color, grad_color, static_cast<float2*>(c->edge_w.p), s);
        ew = static_cast<float2*>(c->edge_w.p);
    }
    {
        Timed t(c, SOUP_T_FILL, s);
        if (fused) {
            if (!o.accumulate)
                for (int l = 0; l <= lv->Rtop - lv->Rmin; ++l)
                    launch_fill_f32(lv->graw[l], static_cast<int64_t>(T) * mc_count(lv->Rmin + l) * kPCh, 0.0f, s);
        } else if (!o.accumulate || lv) {   // the workspace starts from zero
            launch_fill_f32(grad_tex, n_tex, 0.0f, s);
        }
        launch_fill_i32(static_cast<int32_t*>(c->gvert.p), static_cast<int64_t>(T) * 18, 0, s);
    }
    const float* gl = o.mode == 0 ? grad_logp : nullptr;
    if (sorted_path) {
        // every winner and, where the pixel carries a score weight, every fragment in
        // front of it (Eq. (9)), sorted by triangle
        int64_t n_frag = 0, n_batch = 0;
        if ((st = replay(c, p, a, vis, grad_color, gl, ew, false, static_cast<int32_t*>(c->tri_count.p), T, s,
                         &n_frag, &n_batch, from_log)))
            return st;
        const int64_t frag_cap = static_cast<int64_t>(c->frag_regions) * static_cast<int64_t>(c->frag_region);
        if ((st = ensure(c, c->sorted, static_cast<size_t>(frag_cap) * sizeof(FragRec)))) return st;
        {
            Timed t(c, SOUP_T_GRAD, s);
            launch_scan(static_cast<int32_t*>(c->tri_count.p), T, static_cast<int64_t*>(c->tri_bsum.p),
                        static_cast<int64_t*>(c->tri_off.p), s);
            launch_fill_i32(static_cast<int32_t*>(c->tri_fill.p), 2 * T, 0, s);
            PlaceArgs pa{};
            pa.frags = static_cast<FragRec*>(c->frags.p);
            pa.region = static_cast<uint32_t>(c->frag_region);
            pa.counts = static_cast<uint32_t*>(c->region_counts.p);
            pa.boff = static_cast<uint32_t*>(c->region_boff.p);
            pa.n_regions = c->frag_regions;
            pa.tri_off = static_cast<int64_t*>(c->tri_off.p);
            pa.tri_fill = static_cast<unsigned long long*>(c->tri_fill.p);
            pa.sorted = static_cast<FragRec*>(c->sorted.p);
            pa.n_blocks = decode_blocks(c);
            launch_place(pa, s);
        }
        Timed t(c, SOUP_T_BWD, s);
        PTriArgs ta{};
        ta.views = a.views;
        ta.recs = a.recs;
        ta.verts = scene->verts;
        ta.tex = scene->tex;
        ta.mlp = scene->mlp;
        ta.R = scene->R;
        ta.T = T;
        ta.sorted = static_cast<FragRec*>(c->sorted.p);
        ta.tri_off = static_cast<int64_t*>(c->tri_off.p);
        ta.grad_color = grad_color;
        ta.edge_w = ew;
        ta.score = gl ? 1 : 0;
        ta.accumulate = lv && !fused ? 0 : o.accumulate;
        ta.grad_tex = fused ? nullptr : grad_tex;
        if (fused) {
            ta.levels = 1;
            ta.Rmin = lv->Rmin;
            ta.Rtop = lv->Rtop;
            for (int l = 0; l <= lv->Rtop - lv->Rmin; ++l) ta.graw[l] = lv->graw[l];
        }
        ta.gvert = static_cast<double*>(c->gvert.p);
        ta.mlp_partial = static_cast<float*>(c->partial.p);
        ta.n_blocks = nb;
        launch_ptri_bwd(ta, s);
    } else {
        if (gl) {
            // the score term (Eq. (9)): every fragment in front of a winner, and the winner
            int64_t n_frag = 0, n_batch = 0;
            if ((st = replay(c, p, a, vis, grad_color, gl, nullptr, false, nullptr, 0, s, &n_frag, &n_batch,
                             from_log)))
                return st;
            Timed t(c, SOUP_T_GRAD, s);
            PFragArgs fa{};
            fa.frags = static_cast<FragRec*>(c->frags.p);
            fa.region = static_cast<uint32_t>(c->frag_region);
            fa.counts = static_cast<uint32_t*>(c->region_counts.p);
            fa.boff = static_cast<uint32_t*>(c->region_boff.p);
            fa.n_regions = c->frag_regions;
            fa.tex = scene->tex;
            fa.R = scene->R;
            fa.grad_tex = grad_tex;
            fa.n_blocks = decode_blocks(c);
            launch_pfrag(fa, false, s);
        }
        Timed t(c, SOUP_T_BWD, s);
        PWinArgs wa{};
        wa.views = a.views;
        wa.V = a.V;
        wa.P = p.n_pix;
        wa.recs = a.recs;
        wa.verts = scene->verts;
        wa.tex = scene->tex;
        wa.mlp = scene->mlp;
        wa.R = scene->R;
        wa.vis = vis;
        wa.grad_color = grad_color;
        wa.edge_w = ew;
        wa.grad_tex = grad_tex;
        wa.gvert = static_cast<double*>(c->gvert.p);
        wa.mlp_partial = static_cast<float*>(c->partial.p);
        wa.n_blocks = nb;
        launch_pwinner_bwd(wa, s);
    }
    HIP_TRY(c, hipGetLastError());
    if (lv && !fused) {   // the workspace's texture gradient through the assembly's backward
        Timed t(c, SOUP_T_ASSEMBLE_BWD, s);
        AssembleArgs aa{};
        for (int l = 0; l <= lv->Rtop - lv->Rmin; ++l) aa.graw[l] = lv->graw[l];
        aa.Rmin = lv->Rmin;
        aa.Rtop = lv->Rtop;
        aa.Rmax = scene->R;
        aa.T = T;
        aa.tex = scene->tex;
        aa.grad_tex = grad_tex;
        aa.accumulate = o.accumulate;
        if (mc_assemble_bwd_lds(aa.Rmin, aa.Rmax) > mc_assemble_bwd_lds_cap(c->lds_limit) && !o.accumulate && T > 0)
            for (int l = 0; l <= aa.Rtop - aa.Rmin; ++l)
                launch_fill_f32(aa.graw[l], static_cast<int64_t>(T) * mc_count(aa.Rmin + l) * kPCh, 0.0f, s);
        launch_mc_assemble_bwd(aa, c->lds_limit, s);
    }
    {
        Timed t(c, SOUP_T_REDUCE, s);
        launch_pvert_finish(static_cast<double*>(c->gvert.p), grad_verts, static_cast<int64_t>(T) * 9,
                            o.accumulate != 0, s);
        launch_mlp_reduce(static_cast<float*>(c->partial.p), rows, kPParams, static_cast<double*>(c->mlp_mid.p),
                          grad_mlp, o.accumulate != 0, s);
    }
    HIP_TRY(c, hipGetLastError());
    return finish_stats(c, s, false);
}

soup_status soup_pbackward(soup_ctx* c, const soup_pscene* scene, const soup_views* views, const float* inv_view_proj,
                           const soup_opts* opts, const uint64_t* vis, const float* color, const float* grad_color,
                           const float* grad_logp, float* grad_verts, float* grad_tex, float* grad_mlp,
                           void* stream) {
    return pbackward_impl(c, scene, views, inv_view_proj, opts, vis, color, grad_color, grad_logp, grad_verts, grad_tex,
                          nullptr, grad_mlp, stream);
}

soup_status soup_pbackward_levels(soup_ctx* c, const soup_pscene* scene, const soup_views* views,
                                  const float* inv_view_proj, const soup_opts* opts, const uint64_t* vis,
                                  const float* color, const float* grad_color, const float* grad_logp,
                                  int32_t Rmin, int32_t Rtop, float* grad_verts, float* const* grad_raw,
                                  float* grad_mlp, void* stream) {
    const LevelsOut lv{Rmin, Rtop, grad_raw};
    return pbackward_impl(c, scene, views, inv_view_proj, opts, vis, color, grad_color, grad_logp, grad_verts, nullptr,
                          &lv, grad_mlp, stream);
}

soup_status soup_mc_assemble(soup_ctx* c, int32_t T, int32_t Rmin, int32_t Rtop, int32_t Rmax, const float* const* raw,
                             float* tex, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    soup_status st;
    if ((st = check_levels(c, T, Rmin, Rtop, Rmax))) return st;
    if (T > 0 && (!raw || !tex)) return fail(c, SOUP_ERR_INVALID, "mc_assemble: NULL buffers");
    AssembleArgs aa{};
    for (int l = 0; l <= Rtop - Rmin; ++l) {
        if (T > 0 && !raw[l]) return fail(c, SOUP_ERR_INVALID, "mc_assemble: level %d is NULL", Rmin + l);
        aa.raw[l] = raw[l];
    }
    aa.Rmin = Rmin;
    aa.Rtop = Rtop;
    aa.Rmax = Rmax;
    aa.T = T;
    aa.tex_out = tex;
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        Timed t(c, SOUP_T_ASSEMBLE, s);
        launch_mc_assemble(aa, s);
    }
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_mc_assemble_bwd(soup_ctx* c, int32_t T, int32_t Rmin, int32_t Rtop, int32_t Rmax, const float* tex,
                                 const float* grad_tex, float* const* grad_raw, int32_t accumulate, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    soup_status st;
    if ((st = check_levels(c, T, Rmin, Rtop, Rmax))) return st;
    if (accumulate != 0 && accumulate != 1) return fail(c, SOUP_ERR_INVALID, "accumulate = %d (0 or 1)", accumulate);
    if (T > 0 && (!tex || !grad_tex || !grad_raw)) return fail(c, SOUP_ERR_INVALID, "mc_assemble_bwd: NULL buffers");
    AssembleArgs aa{};
    for (int l = 0; l <= Rtop - Rmin; ++l) {
        if (T > 0 && !grad_raw[l]) return fail(c, SOUP_ERR_INVALID, "mc_assemble_bwd: level %d is NULL", Rmin + l);
        aa.graw[l] = grad_raw[l];
    }
    aa.Rmin = Rmin;
    aa.Rtop = Rtop;
    aa.Rmax = Rmax;
    aa.T = T;
    aa.tex = tex;
    aa.grad_tex = grad_tex;
    aa.accumulate = accumulate;
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        Timed t(c, SOUP_T_ASSEMBLE_BWD, s);
        if (mc_assemble_bwd_lds(Rmin, Rmax) > mc_assemble_bwd_lds_cap(c->lds_limit) && !accumulate && T > 0)
            for (int l = 0; l <= Rtop - Rmin; ++l)
                launch_fill_f32(grad_raw[l], static_cast<int64_t>(T) * mc_count(Rmin + l) * kPCh, 0.0f, s);
        launch_mc_assemble_bwd(aa, c->lds_limit, s);
    }
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_loss_l2(soup_ctx* c, const float* color, const float* target, int64_t P, float* grad_color,
                         float* grad_logp, float* loss, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (P < 0 || (P > 0 && (!color || !target || !grad_color || !grad_logp)))
        return fail(c, SOUP_ERR_INVALID, "loss_l2: bad arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    {
        Timed t(c, SOUP_T_LOSS, static_cast<hipStream_t>(stream));
        launch_loss_l2(color, target, P, grad_color, grad_logp, loss, static_cast<hipStream_t>(stream));
    }
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_coverage_count(soup_ctx* c, const uint64_t* vis, int64_t n, int32_t T, uint32_t* counts,
                                void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (n < 0 || T < 0 || (n > 0 && !vis) || (T > 0 && !counts))
        return fail(c, SOUP_ERR_INVALID, "coverage_count: bad arguments (n = %lld, T = %d)", (long long)n, T);
    HIP_TRY(c, hipSetDevice(c->device));
    {
        Timed t(c, SOUP_T_COVER, static_cast<hipStream_t>(stream));
        launch_coverage(vis, n, T, counts, c->num_cus, static_cast<hipStream_t>(stream));
    }
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_edge_lengths(soup_ctx* c, const float* verts, int32_t T, const soup_views* v, float near_w,
                              float* rel_len, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (T < 0 || (T > 0 && (!verts || !rel_len))) return fail(c, SOUP_ERR_INVALID, "edge_lengths: bad arguments");
    if (!v || v->V < 1 || !v->width || !v->height || !v->view_proj)
        return fail(c, SOUP_ERR_INVALID, "edge_lengths: views missing");
    for (int i = 0; i < v->V; ++i)
        if (v->width[i] < 1 || v->width[i] > 16384 || v->height[i] < 1 || v->height[i] > 16384)
            return fail(c, SOUP_ERR_INVALID, "view %d size %dx%d outside [1, 16384]", i, v->width[i], v->height[i]);
    if (!(near_w > 0.0f)) return fail(c, SOUP_ERR_INVALID, "edge_lengths: near_w must be > 0");
    HIP_TRY(c, hipSetDevice(c->device));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    {
        Timed t(c, SOUP_T_EDGELEN, s);
        for (int v0 = 0; v0 < v->V; v0 += soup::kEdgeViews) {
            soup::EdgeViews ev{};
            ev.n = std::min(soup::kEdgeViews, v->V - v0);
            for (int i = 0; i < ev.n; ++i) {
                std::memcpy(ev.m[i], v->view_proj + static_cast<size_t>(v0 + i) * 16, 16 * sizeof(float));
                ev.w[i] = static_cast<float>(v->width[v0 + i]);
                ev.h[i] = static_cast<float>(v->height[v0 + i]);
            }
            launch_edge_lengths(verts, T, ev, near_w, v0 == 0, rel_len, s);
        }
    }
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_adaptive_plan(soup_ctx* c, const uint32_t* counts, const float* rel_len, int32_t T, float split_frac,
                               int32_t target, int32_t flags, int32_t* actions, int32_t* offsets, int32_t* n_new) {
    if (c) c->err.clear();
    if (!n_new || T < 0 || T > (1 << 30) || target < 0 || (flags & ~3) != 0 ||
        (T > 0 && (!counts || !rel_len || !actions || !offsets)))
        return fail(c, SOUP_ERR_INVALID, "adaptive_plan: bad arguments (T = %d, target = %d, flags = %d)", T, target,
                    flags);
    if (!(split_frac == split_frac)) return fail(c, SOUP_ERR_INVALID, "adaptive_plan: split_frac is NaN");
    *n_new = soup::plan_host(counts, rel_len, T, split_frac, target, (flags & SOUP_PLAN_PRUNE_ZERO) != 0,
                             (flags & SOUP_PLAN_FILL) != 0, actions, offsets);
    return SOUP_OK;
}

soup_status soup_adaptive_apply(soup_ctx* c, const soup_scene* sc, const int32_t* actions, const int32_t* offsets,
                                int32_t n_new, float* verts_out, float* feats_out, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (!sc || sc->T < 0 || sc->G < 2 || sc->G > 256 || sc->C < 1 || n_new < 0)
        return fail(c, SOUP_ERR_INVALID, "adaptive_apply: bad scene or n_new");
    if (sc->T > 0 && (!sc->verts || !sc->feats || !actions || !offsets))
        return fail(c, SOUP_ERR_INVALID, "adaptive_apply: device pointers are NULL");
    if (n_new > 0 && (!verts_out || !feats_out))
        return fail(c, SOUP_ERR_INVALID, "adaptive_apply: output pointers are NULL");
    if ((reinterpret_cast<uintptr_t>(sc->feats) | reinterpret_cast<uintptr_t>(feats_out)) & 15)
        return fail(c, SOUP_ERR_INVALID, "adaptive_apply: feats and feats_out must be 16-byte aligned");
    HIP_TRY(c, hipSetDevice(c->device));
    {
        Timed t(c, SOUP_T_APPLY, static_cast<hipStream_t>(stream));
        launch_apply(sc->verts, sc->feats, actions, offsets, sc->T, sc->G, sc->C, n_new, verts_out, feats_out,
                     static_cast<hipStream_t>(stream));
    }
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

namespace {

// Arguments of the L1 + D-SSIM loss: the total and the largest view's pixels.
soup_status check_loss_l1_ssim(soup_ctx* c, const float* color, const float* target, const soup_views* v,
                               float lambda, const float* grad_color, const float* grad_logp, int64_t* P_out,
                               int64_t* maxp_out) {
    if (!v || v->V < 1 || !v->width || !v->height) return fail(c, SOUP_ERR_INVALID, "loss_l1_ssim: views missing");
    if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(c, SOUP_ERR_INVALID, "loss_l1_ssim: lambda outside [0, 1]");
    int64_t P = 0, maxp = 0;
    for (int i = 0; i < v->V; ++i) {
        if (v->width[i] < 1 || v->width[i] > 16384 || v->height[i] < 1 || v->height[i] > 16384)
            return fail(c, SOUP_ERR_INVALID, "view %d size %dx%d outside [1, 16384]", i, v->width[i], v->height[i]);
        const int64_t np = static_cast<int64_t>(v->width[i]) * v->height[i];
        P += np;
        maxp = std::max(maxp, np);
    }
    if (!color || !target || !grad_color || !grad_logp)
        return fail(c, SOUP_ERR_INVALID, "loss_l1_ssim: device pointers are NULL");
    *P_out = P;
    *maxp_out = maxp;
    return SOUP_OK;
}

// The loss's launches, view by view, with the statistics record in `stats`
// (12 floats per pixel of the largest view). Allocates nothing when `timed`
// is false (the timing events come from a pool that may grow).
void loss_l1_ssim_launch(soup_ctx* c, const float* color, const float* target, const soup_views* v, float lambda,
                         float* grad_color, float* grad_logp, float* loss, int64_t P, float* stats, bool timed,
                         hipStream_t s) {
    // the window: normalised 1-D Gaussian, sigma 1.5, summed in double
    soup::SsimWindow win{};
    double g[2 * soup::kSsimR + 1], sum = 0.0;
    for (int i = 0; i <= 2 * soup::kSsimR; ++i) {
        const double x = i - soup::kSsimR;
        g[i] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
        sum += g[i];
    }
    for (int i = 0; i <= 2 * soup::kSsimR; ++i) win.g[i] = static_cast<float>(g[i] / sum);
    const float inv_n = static_cast<float>(1.0 / (3.0 * static_cast<double>(P)));
    auto run = [&]() {
        if (loss) launch_fill_f32(loss, 1, 0.0f, s);
        int64_t off = 0;
        for (int i = 0; i < v->V; ++i) {
            const int64_t np = static_cast<int64_t>(v->width[i]) * v->height[i];
            launch_loss_l1_ssim(color + off * 3, target + off * 3, v->width[i], v->height[i], lambda, inv_n, win,
                                stats, grad_color + off * 3, grad_logp + off, loss, s);
            off += np;
        }
    };
    if (timed) {
        Timed t(c, SOUP_T_TLOSS, s);
        run();
    } else {
        run();
    }
}

}  // namespace

soup_status soup_loss_l1_ssim(soup_ctx* c, const float* color, const float* target, const soup_views* v,
                              float lambda, float* grad_color, float* grad_logp, float* loss, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    int64_t P = 0, maxp = 0;
    soup_status st = check_loss_l1_ssim(c, color, target, v, lambda, grad_color, grad_logp, &P, &maxp);
    if (st != SOUP_OK) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    if ((st = ensure(c, c->ssim, static_cast<size_t>(maxp) * 12 * sizeof(float)))) return st;
    loss_l1_ssim_launch(c, color, target, v, lambda, grad_color, grad_logp, loss, P, static_cast<float*>(c->ssim.p),
                        true, static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_loss_l1_ssim_noalloc(soup_ctx* c, const float* color, const float* target, const soup_views* v,
                                      float lambda, float* grad_color, float* grad_logp, float* loss, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    int64_t P = 0, maxp = 0;
    soup_status st = check_loss_l1_ssim(c, color, target, v, lambda, grad_color, grad_logp, &P, &maxp);
    if (st != SOUP_OK) return st;
    const int64_t max_pixels = static_cast<int64_t>(kNoAllocScratchBytes / (12 * sizeof(float)));
    if (maxp > max_pixels)
        return fail(c, SOUP_ERR_CAPACITY, "loss_l1_ssim_noalloc: a view of %lld pixels exceeds the static scratch "
                    "(%zu MiB: views of at most %lld pixels); use soup_loss_l1_ssim", static_cast<long long>(maxp),
                    kNoAllocScratchBytes >> 20, static_cast<long long>(max_pixels));
    if (!c->scratch) return fail(c, SOUP_ERR_HIP, "loss_l1_ssim_noalloc: the static scratch has no device address");
    HIP_TRY(c, hipSetDevice(c->device));
    loss_l1_ssim_launch(c, color, target, v, lambda, grad_color, grad_logp, loss, P, c->scratch, false,
                        static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_adam_step(soup_ctx* c, float* p, const float* g, float* m, float* v, int64_t n, int32_t vec, float lr,
                           double beta1, double beta2, float eps, int32_t t, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (n < 0 || vec < 1 || vec > 4 || n % vec != 0 || t < 1 || (n > 0 && (!p || !g || !m || !v)))
        return fail(c, SOUP_ERR_INVALID, "adam_step: bad arguments (n = %lld, vec = %d, t = %d)", (long long)n, vec, t);
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps >= 0.0f))
        return fail(c, SOUP_ERR_INVALID, "adam_step: betas must lie in [0, 1) and eps >= 0");
    HIP_TRY(c, hipSetDevice(c->device));
    const float bc1 = static_cast<float>(1.0 - std::pow(beta1, t));
    const float bc2 = static_cast<float>(1.0 - std::pow(beta2, t));
    {
        Timed tm(c, SOUP_T_ADAM, static_cast<hipStream_t>(stream));
        launch_adam(p, g, m, v, n / vec, vec, lr, static_cast<float>(beta1), static_cast<float>(1.0 - beta1),
                    static_cast<float>(beta2), static_cast<float>(1.0 - beta2), eps, bc1, bc2,
                    static_cast<hipStream_t>(stream));
    }
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_selftest_sigmoid(soup_ctx* c, const float* x, float* y, int64_t n, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    if (n < 0 || (n > 0 && (!x || !y))) return fail(c, SOUP_ERR_INVALID, "selftest_sigmoid: bad arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    launch_selftest_sigmoid(x, y, n, static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_selftest_uniform(soup_ctx* c, uint64_t seed, const uint32_t* pixel, const uint32_t* tri,
                                  uint32_t view_id, uint32_t step, float* u, int64_t n, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    if (n < 0 || (n > 0 && (!pixel || !tri || !u))) return fail(c, SOUP_ERR_INVALID, "selftest_uniform: bad arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    launch_selftest_uniform(seed, pixel, tri, view_id, step, u, n, static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// measured ceilings
// ---------------------------------------------------------------------------

soup_status soup_probe_copy(soup_ctx* c, const void* src, void* dst, int64_t bytes, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (bytes < 0 || bytes % 16 != 0 || (bytes > 0 && (!src || !dst)) ||
        ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) != 0)
        return fail(c, SOUP_ERR_INVALID, "probe_copy: need 16-byte aligned buffers and a multiple of 16 bytes");
    HIP_TRY(c, hipSetDevice(c->device));
    soup::launch_probe_copy(static_cast<const float4*>(src), static_cast<float4*>(dst), bytes / 16, c->num_cus,
                            static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_probe_read(soup_ctx* c, const void* src, int64_t bytes, float* partial, int64_t n_partial,
                            void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (bytes < 0 || bytes % 16 != 0 || (bytes > 0 && (!src || !partial)) || n_partial < 1 ||
        (reinterpret_cast<uintptr_t>(src) & 15) != 0)
        return fail(c, SOUP_ERR_INVALID, "probe_read: need a 16-byte aligned buffer, a multiple of 16 bytes and "
                    "n_partial >= 1");
    HIP_TRY(c, hipSetDevice(c->device));
    soup::launch_probe_read(static_cast<const float4*>(src), bytes / 16, partial, n_partial,
                            static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_probe_atomic(soup_ctx* c, float* slots, int64_t n_slots, int64_t n_ops, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (n_slots < 1 || n_ops < 0 || !slots) return fail(c, SOUP_ERR_INVALID, "probe_atomic: bad arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    soup::launch_probe_atomic(slots, n_slots, n_ops, c->num_cus, static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_probe_fma(soup_ctx* c, float* out, int64_t n_threads, int32_t iters, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (!out || n_threads < 256 || n_threads % 256 != 0 || n_threads / 256 > INT32_MAX || iters < 0 ||
        iters > (1 << 20))
        return fail(c, SOUP_ERR_INVALID, "probe_fma: n_threads a positive multiple of 256, 0 <= iters <= 2^20");
    HIP_TRY(c, hipSetDevice(c->device));
    soup::launch_probe_fma(out, n_threads, iters, static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}

soup_status soup_probe_mfma(soup_ctx* c, float* out, int64_t n_threads, int32_t iters, void* stream) {
    if (!c) return SOUP_ERR_INVALID;
    c->err.clear();
    if (!out || n_threads < 256 || n_threads % 256 != 0 || n_threads / 256 > INT32_MAX || iters < 0 ||
        iters > (1 << 18))
        return fail(c, SOUP_ERR_INVALID, "probe_mfma: n_threads a positive multiple of 256, 0 <= iters <= 2^18");
    HIP_TRY(c, hipSetDevice(c->device));
    soup::launch_probe_mfma(out, n_threads, iters, static_cast<hipStream_t>(stream));
    HIP_TRY(c, hipGetLastError());
    return SOUP_OK;
}
