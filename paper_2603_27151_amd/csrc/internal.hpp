// Host-side declarations of the kernel launchers (internal to the library).
#pragma once

#include "common.hpp"

namespace soup {

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
// Binning works on chunks of triangles per view. Large chunks (kBinChunk) of
// a view with at most kHistBins tiles are counted in an LDS histogram, and
// chunk_base ([chunks][tiles] int32) receives each chunk's first slot in every
// tile list it touches; when large chunks would leave the GPU idle (few views,
// few triangles) the chunks are one triangle per thread, counted with global
// atomics.
constexpr int kBinChunk = 2048;
constexpr int kHistBins = 8192;
int bin_chunk_size(int V, int maxT, int num_cus);
inline int bin_chunks(int maxT, int chunk) { return maxT <= 0 ? 0 : (maxT + chunk - 1) / chunk; }
void launch_setup(const ViewDesc* views, int V, int maxT, int chunk, const SceneDesc* scenes, const Opts& o,
                  int tile, TriRec* recs, int32_t* tile_count, int32_t* chunk_base, int64_t n_tiles,
                  unsigned long long* visible, hipStream_t s);
void launch_scan(const int32_t* in, int64_t n, int64_t* bsum, int64_t* out, hipStream_t s);
void launch_scatter(const ViewDesc* views, int V, int maxT, int chunk, int tile, const TriRec* recs,
                    const int64_t* tile_start, int64_t n_tiles, const int32_t* chunk_base, int32_t* tile_fill,
                    uint64_t* entries, hipStream_t s);
void launch_sort(const int64_t* tile_start, int64_t n_tiles, uint64_t* entries, hipStream_t s);
void launch_clip(int64_t* tile_start, int64_t n_tiles, int64_t cap, unsigned int* local, unsigned int* sticky,
                 hipStream_t s);

// Sticky overflow bits of the static-capacity mode.
constexpr unsigned kOverflowBins = 1u;
constexpr unsigned kOverflowFragments = 2u;

// MLP shapes compiled in: (C, H, NH); kPaper is the paper form's raster (opacity
// texture only, the shading MLP deferred)
enum class MlpKind { k8_16_1, k16_32_2, k32_64_2, kPaper, kNone };
MlpKind mlp_kind(int n_layers, const int32_t* dims);
int mlp_params(int n_layers, const int32_t* dims);

struct RasterArgs {
    const ViewDesc* views;
    int V;
    const SceneDesc* scenes;
    Opts o;
    int G;
    const TriRec* recs;
    const int64_t* tile_start;
    const uint64_t* entries;
    int64_t n_tiles;
    uint64_t* vis;                 // concatenated outputs (may be null when views carry their own)
    float* color;
    unsigned long long* counter;   // counters or null: [0] decodes, [8] pixels that some fragment covers
    unsigned int* work;            // persistent-kernel tile counter (zeroed by the launcher's caller)
    int n_blocks;                  // persistent grid of the forward (single-wave workgroups)
    int region;                    // side of a forward wave's region: 16 (tiles of 16, 32) or 8
    // optional log of the forward's decoded fragments, one region per wave (= workgroup):
    // log_frag = (pixel, triangle, b1, b2); log_aux = aux_words(gate_words) words per
    // fragment: depth bits, view, then the decode's ReLU gates (zero-padded to an even count)
    uint4* log_frag;
    uint2* log_aux;
    uint32_t log_region;
    uint32_t* log_counts;
};

// Words of ReLU gate bits a decode of this MLP shape logs (one bit per hidden unit).
int gate_words(MlpKind k);
// Words of one log_aux record: depth bits, view and the gates, rounded up to an even count.
__host__ __device__ constexpr int aux_words(int gate_words) { return (2 + gate_words + 1) & ~1; }
// Words per fragment in the gate arrays beside the fragment lists: the gates padded to an
// even count, so that every copy moves 8-byte units.
__host__ __device__ constexpr int gate_stride(int gate_words) { return (gate_words + 1) & ~1; }

void launch_raster_fwd(const RasterArgs& a, int tile, MlpKind k, hipStream_t s);
// Resident single-wave workgroups per CU of the forward kernel for a tile side, MLP shape and
// region side (16: 16x16 pixels of a tile of 16 or 32; 8: one 8x8 block).
int raster_fwd_blocks_per_cu(int tile, MlpKind k, int region);
// The forward's unit of work: a region of `region` x `region` pixels of a tile.
inline int fwd_regions_per_tile(int tile, int region) { return (tile / region) * (tile / region); }

// One fragment the backward needs (24 bytes): p0 = (pixel, triangle | winner
// << 31), p1 = the perspective-correct barycentrics (b1, b2) as bits, x =
// (the pixel's score weight as bits, view). A winner's colour gradient and
// edge weights are read from the per-pixel arrays by the decode (half of the
// fragments are winners; the list is written, placed and read again, so the
// smaller record moves 1.2 GB less per step on the batched workload).
struct FragRec {
    uint2 p0;
    uint2 p1;
    uint2 x;
};

// The fragment list is split into one region of `region` entries per replay
// wave (wave w owns [w * region, (w + 1) * region)), so that no two waves
// share a counter. counts[w] is the number of fragments wave w found (it may
// exceed `region`: the call then runs again with larger regions).
constexpr int kMaxRegions = 4096;

struct ReplayArgs {
    RasterArgs r;
    const uint64_t* vis;
    const float* grad_color;       // [P,3] (null in the logp pass)
    const float* grad_logp;        // [P] or null
    const float2* edge_w;          // [P] edge weights or null
    int all_front;                 // logp pass: every pixel needs its whole front set
    FragRec* frags;                // [n_regions * region]
    uint32_t region;
    uint32_t* counts;              // [n_regions]
    int32_t* tri_count;            // [T] fragments per triangle (added to; null: not counted)
    int n_blocks;                  // persistent grid size (n_regions = n_blocks * waves per block)
};

void launch_replay(const ReplayArgs& a, int tile, hipStream_t s);

// The same fragment list as the replay, filtered from the forward's log:
// every fragment with key <= the pixel's winner key was decoded (and logged)
// by the forward, since the forward's best key never drops below the winner's.
struct CollectArgs {
    const uint4* log_frag;
    const uint2* log_aux;          // aux_words(gate_words) words per logged fragment
    uint32_t* frag_gates;          // the log's ReLU gates of every kept fragment (same slots as frags, gate_stride
                                   // words each), or null
    int gate_words;
    uint32_t log_region;
    const uint32_t* log_counts;    // [log_regions]
    const uint32_t* log_boff;      // [log_regions + 1] batch offsets of the log
    int log_regions;
    const uint64_t* vis;
    const float* grad_logp;        // [P] or null
    int all_front;                 // logp pass
    FragRec* frags;
    uint32_t region;
    uint32_t* counts;              // [n_blocks * 4]
    int32_t* tri_count;            // [T] or null
    int n_blocks;
};

void launch_collect(const CollectArgs& a, hipStream_t s);
int replay_waves_per_block(int tile);

// Batch offsets of the regions: boff[w] = sum over v < w of ceil(min(counts[v],
// region) / 64), boff[n] = total batches; summary = (fragments, batches,
// largest region count); an overflow sets kOverflowFragments in *sticky
// (when not null).
void launch_region_scan(const uint32_t* counts, int n, uint32_t region, uint32_t* boff,
                        unsigned long long* summary, unsigned int* sticky, hipStream_t s);

// Counting-sort placement of the fragment list by triangle. Within triangle
// t's range [tri_off[t], tri_off[t + 1]) its winners come first (filled
// upwards from the start) and the fragments in front of winners last (filled
// downwards from the end), so that most 64-fragment batches of the decode
// hold winners only or none.
struct PlaceArgs {
    const FragRec* frags;
    uint32_t region;
    const uint32_t* counts;        // [n_regions]
    const uint32_t* boff;          // [n_regions + 1]
    int n_regions;
    const int64_t* tri_off;        // [T + 1] exclusive scan of the per-triangle counts
    unsigned long long* tri_fill;  // [T] zeroed: winners placed (low 32 bits), others (high 32 bits)
    FragRec* sorted;               // [tri_off[T]]
    const uint32_t* frag_gates;    // ReLU gates of frags (gate_words each), or null
    uint32_t* sorted_gates;        // ... placed as sorted
    int gate_words;
    int n_blocks;
};

void launch_place(const PlaceArgs& a, hipStream_t s);

struct DecodeArgs {
    const ViewDesc* views;
    int V;
    const TriRec* recs;
    const float* feats;
    const float* mlp;
    int G;
    int T;
    // logp pass: the region list
    const FragRec* frags;
    uint32_t region;
    const uint32_t* counts;        // [n_regions]
    const uint32_t* boff;          // [n_regions + 1]
    int n_regions;
    // backward: the list sorted by triangle
    const FragRec* sorted;         // [tri_off[T]]
    const uint32_t* sorted_gates;  // the forward's ReLU gates of each sorted fragment, or null (recomputed)
    const int64_t* tri_off;        // [T + 1]
    const float* verts;            // [T, 3, 3]: the winners' clip coordinates are recomputed
    const float* grad_color;       // [P, 3]: the winners' colour gradients
    const float2* edge_w;          // [P] the winners' edge weights, or null (none)
    float* grad_feats;             // [T, G, G, C]: zeroed by the caller unless accumulate
    float* grad_verts;             // [T, 9]: zeroed by the caller unless accumulate
    int accumulate;
    float* mlp_partial;            // [n_blocks * 4, n_params]
    float* logp;                   // logp output (logp pass only; zeroed by the caller)
    unsigned long long* counter;   // decode counter or null
    int n_blocks;
};

void launch_decode_bwd(const DecodeArgs& a, MlpKind k, bool logp_pass, hipStream_t s);
// The forward's ReLU gates of a replayed fragment list (a.frags, a.region, a.counts,
// a.boff, a.n_regions), gate_words(k) words per slot into gates_out.
void launch_fragment_gates(const DecodeArgs& a, MlpKind k, uint32_t* gates_out, hipStream_t s);
// LDS bytes one workgroup of the decode needs for a grid side G (0: unknown).
size_t decode_bwd_lds(MlpKind k, int G, bool logp_pass);
// ew[p] = (x, y) edge weights of the pairs pixel p occludes (Section 3.2),
// written for covered pixels only (a background pixel occludes nothing)
void launch_edge_weights(const ViewDesc* views, int V, int64_t P, const Opts& o, const uint64_t* vis,
                         const float* color, const float* grad_color, float2* ew, hipStream_t s);
void launch_mlp_reduce(const float* partial, int n_rows, int n_params, double* mid, float* out, bool accumulate,
                       hipStream_t s);
int mlp_reduce_mid_rows(int n_rows);
void launch_loss_l2(const float* color, const float* target, int64_t P, float* gc, float* gl, float* loss,
                    hipStream_t s);
void launch_selftest_sigmoid(const float* x, float* y, int64_t n, hipStream_t s);
void launch_selftest_uniform(uint64_t seed, const uint32_t* pixel, const uint32_t* tri, uint32_t view_id,
                             uint32_t step, float* u, int64_t n, hipStream_t s);


// Paper form (Section 3.3; Supplement B.3, B.6): mesh-colour texture assembly,
// deferred shading, the score term and log p over a fragment list, the
// winners' backward.
constexpr int kPMaxLevels = 8;
struct AssembleArgs {
    const float* raw[kPMaxLevels];   // learnable level Rmin + l: [T][V(level)][8]
    float* graw[kPMaxLevels];        // backward: their gradients
    int Rmin, Rtop, Rmax, T;
    float* tex_out;                  // forward: [T][V(Rmax)][8]
    const float* tex;                // backward: the assembled texture and its gradient
    const float* grad_tex;
    int accumulate;
};
void launch_mc_assemble(const AssembleArgs& a, hipStream_t s);
size_t mc_assemble_bwd_lds(int Rmin, int Rmax);
size_t mc_assemble_bwd_lds_cap(size_t lds_limit);
void launch_mc_assemble_bwd(const AssembleArgs& a, size_t lds_limit, hipStream_t s);

struct PShadeArgs {
    const ViewDesc* views;
    int V;
    int64_t P;
    const TriRec* recs;
    const float* tex;
    const float* mlp;
    int R;
    const uint64_t* vis;
    float* color;
    Opts o;
};
void launch_pshade(const PShadeArgs& a, hipStream_t s);

struct PFragArgs {
    const FragRec* frags;
    uint32_t region;
    const uint32_t* counts;
    const uint32_t* boff;
    int n_regions;
    const float* tex;
    int R;
    float* grad_tex;                 // score pass: d / d opacity channel (added to)
    float* logp;                     // logp pass (zeroed by the caller)
    int n_blocks;
};
void launch_pfrag(const PFragArgs& a, bool logp, hipStream_t s);

struct PWinArgs {
    const ViewDesc* views;
    int V;
    int64_t P;
    const TriRec* recs;
    const float* verts;
    const float* tex;
    const float* mlp;
    int R;
    const uint64_t* vis;
    const float* grad_color;
    const float2* edge_w;            // or null
    float* grad_tex;                 // added to
    double* gvert;                   // [T, 9] float64 sums (zeroed by the caller)
    float* mlp_partial;              // [n_blocks * 4, 595]
    int n_blocks;
};
struct PTriArgs {
    const ViewDesc* views;
    const TriRec* recs;
    const float* verts;
    const float* tex;
    const float* mlp;
    int R;
    int T;
    const FragRec* sorted;           // [tri_off[T]] the fragment list sorted by triangle
    const int64_t* tri_off;          // [T + 1]
    const float* grad_color;
    const float2* edge_w;            // or null
    int score;                       // 1: the score term (mode 0 with score weights)
    int accumulate;                  // 1: add into grad_tex rows (else they were zero-filled)
    float* grad_tex;
    double* gvert;                   // [T, 9] float64 sums (zeroed by the caller)
    float* mlp_partial;              // [n_blocks, 595]
    int n_blocks;                    // single-wave workgroups, a multiple of 8
    // levels = 1: the learnable levels' gradients instead of grad_tex (tex is
    // their assembly onto level R); graw[l] = level Rmin + l, zero-filled by
    // the caller unless accumulating
    int levels;
    int Rmin, Rtop;
    float* graw[kPMaxLevels];
};
size_t ptri_bwd_lds(int R);
bool ptri_levels_fit(int R);   // level R - 1 fits the kernel's stage buffer

// measured ceilings (probe.hip)
void launch_probe_copy(const float4* src, float4* dst, int64_t n, int num_cus, hipStream_t s);
void launch_probe_read(const float4* src, int64_t n, float* partial, int64_t n_partial, hipStream_t s);
void launch_probe_atomic(float* slots, int64_t n_slots, int64_t n_ops, int num_cus, hipStream_t s);
void launch_probe_fma(float* out, int64_t n_threads, int iters, hipStream_t s);
void launch_probe_mfma(float* out, int64_t n_threads, int iters, hipStream_t s);
int ptri_blocks(int num_cus, int R);
void launch_ptri_bwd(const PTriArgs& a, hipStream_t s);
int pwinner_blocks(int num_cus);
void launch_pwinner_bwd(const PWinArgs& a, hipStream_t s);
void launch_pvert_finish(const double* g, float* out, int64_t n, bool accumulate, hipStream_t s);

// Adaptive control of primitives.
constexpr int kEdgeViews = 32;  // views per edge-length launch (kernel argument)
struct EdgeViews {
    float m[kEdgeViews][16];    // row-major view-projection matrices
    float w[kEdgeViews], h[kEdgeViews];
    int n;
};
constexpr int kActRemove = 0, kActKeep = 1, kActSplit0 = 2;
void launch_coverage(const uint64_t* vis, int64_t n, int32_t T, uint32_t* counts, int num_cus, hipStream_t s);
void launch_edge_lengths(const float* verts, int32_t T, const EdgeViews& ev, float near_w, bool first, float* rel,
                         hipStream_t s);
void launch_apply(const float* verts, const float* feats, const int32_t* actions, const int32_t* offsets, int32_t T,
                  int32_t G, int32_t C, int32_t n_new, float* vout, float* fout, hipStream_t s);
int32_t plan_host(const uint32_t* counts, const float* rel, int32_t T, float split_frac, int32_t target,
                  bool prune_zero, bool fill, int32_t* actions, int32_t* offsets);

// Training step: L1 + SSIM loss, Adam / VectorAdam.
constexpr int kSsimR = 5;  // 11 x 11 window
struct SsimWindow {
    float g[2 * kSsimR + 1];   // normalised 1-D Gaussian, sigma 1.5; the window is its outer product
};
void launch_loss_l1_ssim(const float* color, const float* target, int W, int H, float lam, float inv_n,
                         const SsimWindow& win, float* stats, float* grad_color, float* grad_logp, float* loss,
                         hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int64_t nvec, int vec, float lr, float b1, float omb1,
                 float b2, float omb2, float eps, float bc1, float bc2, hipStream_t s);

}  // namespace soup
