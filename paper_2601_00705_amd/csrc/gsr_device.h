// gsr_device.h -- device-side definitions shared by the HIP kernels of libgsr.
//
// Layouts (all in the caller-owned workspace, one record per slot, where a
// slot is (view v, Gaussian i) at index v * n + i):
//   geom    float4 (u, v, rx, ry)     projected mean and extent half-widths;
//                                      rx < 0 marks a culled slot
//   conic_o float4 (A, B, C, o)       inverse screen covariance, opacity
//   rgb_d   float4 (r, g, b, depth)   colour in this view, camera depth z
//   grad2d  double [9][slots]         screen-space gradient accumulators
//                                      (du, dv, dA, dB, dC, do, dr, dg, db)
// The rectangle function below is the binning contract: a pure function of
// the float32 (u, v, rx, ry) of a slot, single IEEE operations only, so the
// host reference reproduces it bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GSR_MAX_VIEWS 64
#define GSR_G2 9  // screen-space gradient fields per slot

namespace gsr {

struct ViewInfo {
    int32_t width, height, tiles_x, tiles_y;
    int32_t tile_base;   // first global tile of the view
    int32_t pix_base;    // first pixel of the view in the concatenated images
    float fx, fy, cx, cy;
};

struct ViewTable {
    int32_t n;
    int32_t total_tiles;
    ViewInfo v[GSR_MAX_VIEWS];
};

struct DevCfg {
    int32_t tile_w, tile_h, log2_tw, log2_th;
    int32_t sh_degree;
    float z_near, dilation, alpha_min, alpha_max, T_min;
    float bg0, bg1, bg2;
};

// Device-side counters at the head of the workspace.
struct Counters {
    unsigned long long pairs;   // required pair count of the last binning
    uint32_t overflow;          // 1 when pairs > capacity
    uint32_t pad0;
    unsigned long long capacity;
    uint32_t pad[10];
};

// ---------------------------------------------------------------------------
// binning contract: tile rectangle of a projected record.
// Returns false when the slot touches no tile.  Tile sizes are powers of two,
// so multiplying by the exact reciprocal equals IEEE division.
__device__ __forceinline__ bool tile_rect(float u, float v, float rx, float ry, float inv_tw,
                                          float inv_th, int tiles_x, int tiles_y, int& x0,
                                          int& y0, int& x1, int& y1)
{
    if (!(rx >= 0.0f) || !(ry >= 0.0f) || u != u || v != v) return false;
    float fx0 = floorf(__fsub_rn(u, rx) * inv_tw);
    float fx1 = floorf(__fadd_rn(u, rx) * inv_tw);
    float fy0 = floorf(__fsub_rn(v, ry) * inv_th);
    float fy1 = floorf(__fadd_rn(v, ry) * inv_th);
    float mx = (float)(tiles_x - 1), my = (float)(tiles_y - 1);
    if (fx1 < 0.0f || fy1 < 0.0f || fx0 > mx || fy0 > my) return false;
    x0 = fx0 < 0.0f ? 0 : (int)fx0;
    y0 = fy0 < 0.0f ? 0 : (int)fy0;
    x1 = fx1 > mx ? tiles_x - 1 : (int)fx1;
    y1 = fy1 > my ? tiles_y - 1 : (int)fy1;
    return true;
}

// view owning a global tile (views are few; a uniform linear scan)
__device__ __forceinline__ int view_of_tile(const ViewTable* vt, int tile)
{
    int v = 0;
    for (int k = 1; k < vt->n; ++k)
        if (tile >= vt->v[k].tile_base) v = k;
    return v;
}

// ---------------------------------------------------------------------------
// wave64 helpers
__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ void atomic_add_f64(double* p, double v)
{
    unsafeAtomicAdd(p, v);
}

}  // namespace gsr
