// kernels.h -- argument blocks and host launchers of the libgsr kernels.
#pragma once
#include "gsr_device.h"

namespace gsr {

struct ProjectArgs {
    int64_t n;
    const float *mean, *quat, *log_scale, *opacity_logit, *colour;
    const float* poses;        // [V][12]
    const ViewTable* views;    // device copy
    DevCfg cfg;
    float4 *geom, *conic_o, *rgb_d;
    float* qthr;
    void* stage;               // StageRec or (mixed) StageRecM per slot
    double* grad2d;            // [slots][9], zeroed for live slots
    unsigned long long* acc;   // [slots][GSR_FIX_LIMBS][9] (deterministic mode) or null, zeroed for live slots
    Counters* counters;
    unsigned long long* stamps;  // [V + 1]: [V] = device wall clock when the projection starts
    uint64_t* live_mask;       // [mask_words][views]: bit k of word [w][v] set when slot (v, 64 w + k) is live
    int64_t mask_words;        // ceil(n / 64)
};

struct BinArgs {
    int64_t n;                 // Gaussians per view
    int32_t n_views;
    const ViewTable* views;
    DevCfg cfg;
    const float4* geom;
    const float4* conic_o;
    const float* qthr;
    const float4* rgb_d;
    int32_t chunks;            // most chunks of GSR_BIN_CHUNK * chunk_mult live slots a view can have
    int32_t chunk_mult;
    const uint64_t* live_mask; // [mask_words][views]: the projection's liveness ballots
    int64_t mask_words;
    uint32_t* live;            // [views][n]: per view, the live Gaussians (built by the binning)
    uint32_t* live_count;      // their number, view v's at [GSR_LIVE_STRIDE v]
    int32_t total_tiles;
    uint32_t* cnt;             // per view: [chunks][tiles of the view] pair counts, then offsets
    Counters* counters;
    uint2* ranges;             // [total_tiles]: [first, last + 1) of each tile's pairs
    unsigned long long* seg;   // [capacity]: (depth bits << 32 | Gaussian index), grouped by tile
    unsigned long long* tile_blocks;  // [ceil(total_tiles / 64)]: pairs of each run of 64 tiles
};

struct SegArgs {
    const Counters* counters;
    const ViewTable* views;
    const uint2* ranges;
    const uint32_t* order;     // tiles by pair count, descending
    unsigned long long* seg;   // [capacity]: emitted keys, sorted in place per tile (scratch)
    unsigned long long* keys;  // [capacity]: sorted (tile << 32 | depth bits)
    uint32_t* vals;            // [capacity]: sorted slots
    uint32_t* queue;           // [1]: next list of the short class (zeroed by the ordering)
    int64_t n;
};

struct RangeArgs {
    const Counters* counters;
    const uint2* ranges;
    int32_t total_tiles;
    uint32_t* order;           // [tiles]: tiles by pair count, descending
    uint32_t* buckets;         // [66]: per log2-bucket counts, cursors, then the sort queue head
};

struct RasterArgs {
    const ViewTable* views;
    DevCfg cfg;
    Counters* counters;         // overflow flag (read), accumulator flag (written)
    const uint2* ranges;
    const uint32_t* order;     // processing order of the tiles
    const uint32_t* vals;
    const float4* geom;        // liveness of a slot (rx >= 0)
    const void* stage;         // per-slot staging records (StageRec, or StageRecM when cfg.mixed)
    void* rgb;                 // [sum 3 H W], float (or binary16 when cfg.mixed)
    float* T_final;            // [sum H W]
    int32_t* n_contrib;        // [sum H W]
    int32_t* n_blend;          // nullable
    uint32_t* fwd_queue;       // [1]: next (long tile, part) item of the split forward
    // backward only
    const float* T_final_in;   // forward outputs, read by the backward
    const int32_t* n_contrib_in;
    const float* dL_drgb;
    const float* dL_dT;        // nullable
    double* grad2d;            // [slots][9]
    unsigned long long* acc;   // [slots][GSR_FIX_LIMBS][9] in deterministic mode, else null
    int64_t slots;
    unsigned long long* tiles_done;  // [V]: backward tiles of each view completed, over all calls
    unsigned long long* stamps;  // [V + 1]: wall clock when a view's last backward tile ends
};

struct ProjectBwdArgs {
    int64_t n;
    const float *mean, *quat, *log_scale, *opacity_logit, *colour;
    const float* poses;
    const ViewTable* views;
    DevCfg cfg;
    const uint64_t* live_mask;      // [mask_words][views]: the projection's liveness ballots
    const double* grad2d;
    unsigned long long pose_only;   // bit v set: view v updates the pose only
    float *d_mean, *d_quat, *d_log_scale, *d_opacity_logit, *d_colour;
    double* xi_partial;             // [V][blocks][6]
    double* xi_partial_sh;          // [V][blocks][6], the SH chain's (degree >= 1)
    int32_t blocks;
};

struct LossArgs {
    const void* rgb;           // float, or binary16 (half_image)
    int32_t half_image;
    const float* target;
    float* dL_drgb;
    int64_t count;      // 3 * total pixels
    float scale;        // 1 / count
};

struct TrackArgs {
    const ViewTable* views;
    const float* rgb;          // render [3][H][W] per view, concatenated
    const float* T_final;      // [H][W] per view
    const float* target;       // observation, like rgb
    double tau_alpha, tau_grad;
    double* part;              // [views][GSR_TRACK_BLOCKS][GSR_TRACK_SLOTS] partial sums
    double* loss;              // [views]
    double* exposure;          // [views][2]: g, b
    float* dL_drgb;            // like rgb
    float* dL_dT;              // like T_final, nullable
};

struct MapLossArgs {
    const ViewTable* views;
    const float* rgb;          // render [3][H][W] per view, concatenated
    const float* target;       // like rgb
    float w[11];               // window weights of offsets -5..5
    float c1, c2;              // SSIM stabilisers
    float scale_ssim;          // -lambda / (3 P), P = pixels of all views
    float scale_l1;            // (1 - lambda) / (3 P)
    double lambda, inv_n;      // lambda, 1 / (3 P)
    int32_t max_tiles;         // most 32 x 32 tiles of one view
    double* part;              // [views][max_tiles][2]: sum SSIM, sum |x - y| per block
    double* loss;              // [1]
    float* dL_drgb;            // like rgb
};

#define GSR_ADAM_BLOCKS 1024         // blocks of the gradient-norm pass
#define GSR_PRUNE_CHUNK 2048         // Gaussians per block of the pruning scan

struct AdamArgs {
    float* p[5];               // planes: mean, quat, log_scale, opacity_logit, colour
    const float* g[5];
    float* m[5];
    float* v[5];
    int64_t len[5];            // floats per plane
    float step_size[5];        // lr / (1 - beta1^t) per plane
    float inv_sqrt_bc2;        // 1 / sqrt(1 - beta2^t)
    float beta1, beta2, omb1, omb2;  // beta and 1 - beta, each rounded once from double
    float eps, max_norm, ema;
    float* anchor;             // [3][n] or null
    double* part;              // [GSR_ADAM_BLOCKS + 1]: norm partials, then the clip factor
    double* norm;              // [1] or null
};

struct CovisArgs {
    int64_t pixels;
    int32_t frames;
    float tau;
    const float* T_key;        // [pixels]
    const float* T_frames;     // [frames][pixels]
    unsigned long long* counts;  // [frames][2]: intersection, union
    double* iou;               // [frames]
};

struct PruneArgs {
    int64_t n;
    int32_t blocks;            // ceil(n / GSR_PRUNE_CHUNK)
    const int32_t* m_obs;
    const float* v_vis;
    const float* log_scale;    // [3][n]
    const float* opacity_logit;
    const int32_t* mask;       // null: the pruning rule; else keep where mask != 0
    int32_t m_min;
    double v_min, sigma_max2, alpha_min;
    uint32_t* block_count;     // [blocks]: kept per block, then offsets
    int32_t* keep_index;       // [n]: kept indices in order
    long long* kept;           // [1]
};

struct MergeArgs {
    int64_t n;
    int32_t colour_rows;
    const float* in[5];        // planes: mean, quat, log_scale, opacity_logit, colour
    float* out[5];             // the same layout
    const float* v_vis;        // [n] merge weights
    const int32_t* nn;         // [n] nearest other Gaussian (-1: none)
    double radius, colour_tol;
    int32_t* keep;             // [n] 1 kept, 0 merged into its partner
};

struct CompactArgs {
    int64_t n;
    int32_t rows;
    const float* src;          // [rows][n]
    const int32_t* keep_index;
    const long long* kept;
    float* dst;                // [rows][n], columns < kept written
};

#define GSR_SEED_MAX_NEIGHBOURS 8
#define GSR_KNN_BLOCKS 256          // blocks of the seeds' bounding-box pass
#define GSR_KNN_LEVELS 8            // fine hashed grid levels (cell sizes h1 * 2^l)

struct SeedView {
    double P[12];              // 3x4 projection matrix K [R | t], row-major
    double centre[3];          // camera centre, world
    int32_t width, height;
    const float* image;        // [3][H][W]
    double gain, bias;         // exposure: observed = gain * radiance + bias
};

struct SeedArgs {
    SeedView views[GSR_SEED_MAX_NEIGHBOURS + 1];  // reference, then neighbours
    int64_t n;
    int32_t K;
    double max_reproj, min_parallax, alpha_lo, alpha_hi;
    const float* x_ref;        // [2][n]
    const float* x_nb;         // [K][2][n]
    const float* kappa;        // [K][n]
    float* mean;               // [3][n]
    float* colour;             // [3][n]
    float* opacity_logit;      // [n]
    int32_t* valid;            // [n]
    int32_t* best;             // [n]
    float* err;                // [n]
    float* angle;              // [n]
    float* kappa_bar;          // [n]
};

struct KnnGrid {
    double origin[3];
    double h;                  // coarse cell size
    int32_t dims[3];           // coarse grid
    int64_t cells;
    int64_t count;             // valid seeds
    double h1, inv_h1;         // fine cell size (when fine)
    int32_t fine;
};

struct KnnArgs {
    int64_t n;
    const float* mean;         // [3][n]
    const int32_t* valid;      // [n]
    float floor_scale;
    int64_t max_cells;
    float* bpart;              // [GSR_KNN_BLOCKS][8]
    KnnGrid* grid;
    uint32_t* cell_count;      // [max_cells + 1]
    uint32_t* cell_start;      // [max_cells + 1]
    uint32_t* cell_of;         // [n]
    uint32_t* rank;            // [n]
    uint32_t* sorted;          // [n]
    int32_t table_bits;        // fine grid: hash table of 2^table_bits buckets
    double* opart;             // [GSR_KNN_BLOCKS]
    uint32_t* fine_count;      // [GSR_KNN_LEVELS][2^table_bits + 1]
    uint32_t* fine_start;      // [GSR_KNN_LEVELS][2^table_bits + 1]
    uint32_t* fine_of;         // [GSR_KNN_LEVELS][n]
    uint32_t* fine_rank;       // [GSR_KNN_LEVELS][n]
    float4* fine_pts;          // [GSR_KNN_LEVELS][n]: (x, y, z, index bits) in fine-bucket order
    float4* cell_pts;          // [n]: the same in coarse-cell order
    int32_t* nn_index;         // [n] or null: each seed's nearest other seed (-1: none)
    uint32_t* scan_tot;        // block totals of the scans
    uint32_t* bf_list;         // [n] queries left to the exhaustive search
    uint32_t* bf_count;        // their number
    float* log_scale;          // [3][n]
    int32_t fine_levels;       // fine levels built (0: all GSR_KNN_LEVELS)
};

// anisotropic initialisation of the seeds (after the coarse grid of KnnArgs)
struct FrameArgs {
    double P[12];              // reference projection, row-major 3 x 4
    double centre[3];          // reference camera centre
    double radius;             // plane-fit neighbourhood
    double c_par;              // calibration of the axial scale
    double floor_scale;
    const float* err;          // [n] reprojection error of the kept hypothesis (px)
    const float* angle;        // [n] its baseline angle (rad)
    float* quat;               // [4][n] out
    float* log_scale;          // [3][n] out
};

#define GSR_TRACK_BLOCKS 256        // blocks per view of the tracking-loss kernels
#define GSR_TRACK_SLOTS 8           // partial sums per block (4 exposure sums, 3 loss/sign sums)
#define GSR_BIN_CHUNK 256           // Gaussians staged in LDS at a time by the binning blocks (x256)
#define GSR_BIN_LDS_TILES 16384     // views with more tiles count and place with global atomics
#ifndef GSR_BIN_CHUNK_MULT
#define GSR_BIN_CHUNK_MULT 1        // live slots per binning chunk, in units of GSR_BIN_CHUNK
#endif
#define GSR_LIVE_STRIDE 64          // uint32 between two views' live counters (one 256-byte line each)
#define GSR_XCDS 8                  // accelerator dies; workgroups are dealt to them in turn
#define GSR_SEG_SMALL_THREADS 256   // segments below GSR_SEG_SMALL_ITEMS keys: 256-thread blocks
#define GSR_SEG_SMALL_ITEMS 2048
#define GSR_SEG_THREADS 512
#define GSR_SEG_ITEMS 8192          // segments below this size are sorted in LDS by 512-thread blocks
#define GSR_SEG_LONG_THREADS 1024   // longer segments: one 1024-thread block each
#define GSR_SEG_LONG_ITEMS 16384    // ... holding this many keys in LDS
#define GSR_FWD_LONG 4096           // least list length of a tile composited in parts (power of 2)
#define GSR_FWD_WAVES 5120          // resident compositing waves (256 CUs x 4 SIMDs x 5)
#ifndef GSR_FWD_SPLIT
#define GSR_FWD_SPLIT 2             // parts of a long tile (at most the pixels per lane)
#endif
#define GSR_FWD_LONG_WAVES 2048     // persistent waves of the long tiles' parts (two per SIMD)

hipError_t launch_project(const ProjectArgs& a, int sh_degree, hipStream_t s);
// pair counting, offsets, emission into per-tile segments; max_tiles_view is
// the largest tile count of one view
hipError_t launch_bin(const BinArgs& a, int max_tiles_view, hipStream_t s);
hipError_t launch_order(const RangeArgs& a, hipStream_t s);
hipError_t launch_seg_sort(const SegArgs& a, int total_tiles, int64_t capacity, hipStream_t s, hipStream_t side,
                           hipEvent_t fork, hipEvent_t join);
hipError_t launch_raster_fwd(const RasterArgs& a, int total_tiles, int tile_px, int batch, hipStream_t s,
                             hipStream_t side, hipEvent_t fork, hipEvent_t join);
hipError_t launch_clear_grad2d(const RasterArgs& a, hipStream_t s);
hipError_t launch_raster_bwd(const RasterArgs& a, int total_tiles, int tile_px, int batch, hipStream_t s);
hipError_t launch_project_bwd(const ProjectBwdArgs& a, int sh_degree, float* d_xi, int n_views,
                              hipStream_t s);
hipError_t launch_loss_l1(const LossArgs& a, hipStream_t s);
hipError_t launch_loss_track(const TrackArgs& a, int n_views, hipStream_t s);
hipError_t launch_loss_mapping(const MapLossArgs& a, int n_views, hipStream_t s);
hipError_t launch_adam(const AdamArgs& a, bool vec, hipStream_t s);
hipError_t launch_covis(const CovisArgs& a, hipStream_t s);
hipError_t launch_prune(const PruneArgs& a, hipStream_t s);
hipError_t launch_compact(const CompactArgs& a, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_seed_triangulate(const SeedArgs& a, hipStream_t s);
hipError_t launch_seed_scale(const KnnArgs& a, hipStream_t s);
hipError_t launch_seed_frame(const KnnArgs& a, const FrameArgs& f, hipStream_t s);

}  // namespace gsr
