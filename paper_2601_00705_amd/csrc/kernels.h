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
    StageRec* stage;
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
    uint32_t* block_sums;      // [n_views * chunks]
    unsigned long long* block_offs;
    int32_t chunks;            // chunks of BIN_CHUNK Gaussians per view
    Counters* counters;
    unsigned long long* keys;  // [capacity]
    uint32_t* vals;
};

struct SortArgs {
    const Counters* counters;
    const unsigned long long* keys_in;
    const uint32_t* vals_in;
    unsigned long long* keys_out;
    uint32_t* vals_out;
    uint32_t* hist;            // [256][max_blocks]
    uint32_t* digit_total;     // [256]
    int32_t max_blocks;
    int32_t shift;
};

struct RangeArgs {
    const Counters* counters;
    const unsigned long long* keys;
    uint2* ranges;
    int32_t total_tiles;
    uint32_t* order;           // [tiles]: tiles by pair count, descending
    uint32_t* buckets;         // [64]: per log2-bucket counts, then cursors
};

struct RasterArgs {
    const ViewTable* views;
    DevCfg cfg;
    const Counters* counters;
    const uint2* ranges;
    const uint32_t* order;     // processing order of the tiles
    const uint32_t* vals;
    const float4* geom;        // liveness of a slot (rx >= 0)
    const StageRec* stage;     // per-slot staging records
    float* rgb;                // [sum 3 H W]
    float* T_final;            // [sum H W]
    int32_t* n_contrib;        // [sum H W]
    int32_t* n_blend;          // nullable
    // backward only
    const float* T_final_in;   // forward outputs, read by the backward
    const int32_t* n_contrib_in;
    const float* dL_drgb;
    const float* dL_dT;        // nullable
    double* grad2d;            // [9][slots]
    int64_t slots;
};

struct ProjectBwdArgs {
    int64_t n;
    const float *mean, *quat, *log_scale, *opacity_logit, *colour;
    const float* poses;
    const ViewTable* views;
    DevCfg cfg;
    const float4* geom;
    const double* grad2d;
    unsigned long long pose_only;   // bit v set: view v updates the pose only
    float *d_mean, *d_quat, *d_log_scale, *d_opacity_logit, *d_colour;
    double* xi_partial;             // [V][blocks][6]
    int32_t blocks;
};

struct LossArgs {
    const float* rgb;
    const float* target;
    float* dL_drgb;
    int64_t count;      // 3 * total pixels
    float scale;        // 1 / count
};

#define GSR_BIN_CHUNK 1024
#define GSR_SORT_ITEMS 4096
#define GSR_SORT_THREADS 256

hipError_t launch_project(const ProjectArgs& a, int sh_degree, hipStream_t s);
hipError_t launch_bin(const BinArgs& a, hipStream_t s);
hipError_t launch_sort_pass(const SortArgs& a, int grid_blocks, hipStream_t s);
hipError_t launch_ranges(const RangeArgs& a, int grid_blocks, hipStream_t s);
hipError_t launch_raster_fwd(const RasterArgs& a, int total_tiles, int tile_px, int batch, hipStream_t s);
hipError_t launch_clear_grad2d(const RasterArgs& a, hipStream_t s);
hipError_t launch_raster_bwd(const RasterArgs& a, int total_tiles, int tile_px, int batch, hipStream_t s);
hipError_t launch_project_bwd(const ProjectBwdArgs& a, int sh_degree, float* d_xi, int n_views,
                              hipStream_t s);
hipError_t launch_loss_l1(const LossArgs& a, hipStream_t s);

}  // namespace gsr
