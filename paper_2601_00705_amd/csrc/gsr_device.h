// gsr_device.h -- device-side definitions shared by the HIP kernels of libgsr.
//
// Layouts (all in the caller-owned workspace, one record per slot, where a
// slot is (view v, Gaussian i) at index v * n + i):
//   geom    float4 (u, v, rx, ry)     projected mean and extent half-widths;
//                                      rx < 0 marks a culled slot
//   conic_o float4 (A, B, C, o)       inverse screen covariance, opacity
//   rgb_d   float4 (r, g, b, depth)   colour in this view, camera depth z
//   qthr    float                     level of the quadratic form d^T conic d
//                                      below which a tile is binned
//   grad2d  double [9][slots]         screen-space gradient accumulators
//                                      (du, dv, dA, dB, dC, do, dr, dg, db)
// The rectangle function below is the binning contract: a pure function of
// the float32 (u, v, rx, ry) of a slot, single IEEE operations only, so the
// host reference reproduces it bit for bit.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GSR_MAX_VIEWS 64
#define GSR_G2 9  // screen-space gradient fields per slot
// deterministic backward: each field is a fixed-point number in 4 signed
// 64-bit limbs of 32 significant bits each; the lowest bit weighs 2^-96
#define GSR_FIX_LIMBS 4
#define GSR_FIX_UNIT 96

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
    int32_t mixed;        // 1: 32-byte staging records (StageRecM)
    float z_near, dilation, alpha_min, alpha_max, T_min;
    float bg0, bg1, bg2;
};

// Device-side counters at the head of the workspace.
struct Counters {
    unsigned long long pairs;   // required pair count of the last binning
    uint32_t overflow;          // 1 when pairs > capacity
    uint32_t grad_dirty;        // 1 once a backward has added to the accumulators
                                // since the last projection zeroed them
    unsigned long long capacity;
    uint32_t pad[10];
};
static_assert(sizeof(Counters) == 64, "Counters is 64 bytes");

// Per live slot, the record the compositing kernels stage from: the projected
// centre and conic in double (each tile expands the quadratic form around its
// own centre, so that a Gaussian far from the pixels it reaches keeps its
// accuracy) and the opacity and colour.
struct __align__(16) StageRec {
    double u, v, A, B, C;
    float o, r, g, b;
    float pad[2];
};
static_assert(sizeof(StageRec) == 64, "StageRec is 64 bytes");

// The mixed-precision staging record: centre, conic and opacity in float32,
// colour in binary16 (32 bytes, half the gather of StageRec).
struct __align__(16) StageRecM {
    float u, v, A, B, C, o;
    __half r, g, b;
    uint16_t pad;
};
static_assert(sizeof(StageRecM) == 32, "StageRecM is 32 bytes");

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

// Second half of the binning contract: candidate tile (tx, ty) of a slot is
// kept iff q(d) = A dx^2 + 2 B dx dy + C dy^2 (d = pixel centre - (u, v))
// reaches qthr on the box spanned by the tile's pixel centres.  Inside the
// box the minimum is 0; otherwise it lies on an edge, at the edge's
// unconstrained minimiser clamped to the edge.  Float32, this exact order.
// iA = 1 / A and iC = 1 / C (float32 divisions) are passed in, so that a
// caller testing many tiles of one ellipse divides once.
__device__ __forceinline__ bool tile_hit(float u, float v, float A, float B, float C, float iA, float iC, float qthr,
                                         int tx, int ty, int tw, int th)
{
    const float x0 = ((float)(tx * tw) + 0.5f) - u;
    const float x1 = ((float)(tx * tw + tw - 1) + 0.5f) - u;
    const float y0 = ((float)(ty * th) + 0.5f) - v;
    const float y1 = ((float)(ty * th + th - 1) + 0.5f) - v;
    if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return true;
    const float B2 = 2.0f * B;
    float m = INFINITY;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float X = e ? x1 : x0;
        float ys = -(B * X) * iC;
        ys = ys < y0 ? y0 : (ys > y1 ? y1 : ys);
        const float q = (A * X) * X + (B2 * X) * ys + (C * ys) * ys;
        m = q < m ? q : m;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float Y = e ? y1 : y0;
        float xs = -(B * Y) * iA;
        xs = xs < x0 ? x0 : (xs > x1 ? x1 : xs);
        const float q = (A * xs) * xs + (B2 * xs) * Y + (C * Y) * Y;
        m = q < m ? q : m;
    }
    return m <= qthr;
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
// wave64 cross-lane helpers on VALU instructions (no LDS round trip):
// v_permlane32_swap / v_permlane16_swap exchange lane i with lane i ^ 32 /
// i ^ 16 between their two operands; DPP row_mirror pairs lane i with
// 15 - i of its row, row_half_mirror with 7 - i of its half-row, quad_perm
// permutes within quads.

// (every lane's source lies inside the wave for these patterns; bound_ctrl
// lets the compiler fold the move into the consuming add as a DPP operand)
template <int CTRL>
__device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
#define GSR_DPP_QUAD_XOR1 0xB1
#define GSR_DPP_QUAD_XOR2 0x4E
#define GSR_DPP_ROW_MIRROR 0x140
#define GSR_DPP_ROW_HALF_MIRROR 0x141

// Sum of a and b after exchanging the upper 32 lanes of a with the lower 32
// lanes of b: lanes 0-31 get a + a(lane + 32), lanes 32-63 get
// b(lane - 32) + b.  permlane16 does the same between rows 0/1 and 2/3.
__device__ __forceinline__ float swap_sum32(float a, float b)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap_sum16(float a, float b)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Transposed reduction of 8 values over the wave.  Afterwards lane 8k holds
// the 64-lane total of v[k].  Each exchange keeps half of the values and adds
// the partner lane's copy of that half.
__device__ __forceinline__ float wave_sum8_transposed(const float (&v)[9], int lane)
{
    float a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = swap_sum32(v[j], v[4 + j]);  // lane ^ 32
    const float b0 = swap_sum16(a[0], a[2]), b1 = swap_sum16(a[1], a[3]);  // lane ^ 16
    // mirror partner in the row (bit 3 complemented)
    const bool hi = lane & 8;
    float s = (hi ? b1 : b0) + dpp<GSR_DPP_ROW_MIRROR>(hi ? b0 : b1);
    s += dpp<GSR_DPP_ROW_HALF_MIRROR>(s);
    s += dpp<GSR_DPP_QUAD_XOR2>(s);
    s += dpp<GSR_DPP_QUAD_XOR1>(s);
    return s;
}

// Totals of two values over the wave in one chain: afterwards every lane of
// rows 0 and 1 holds the total of x, every lane of rows 2 and 3 that of y
// (lanes 1 and 33, say).  The exchange at distance 32 folds x into the lower
// half and y into the upper; the one at distance 16, of that result with
// itself, leaves each half's two rows with their sum; four DPP adds finish
// inside each row.
__device__ __forceinline__ float wave_sum_pair(float x, float y)
{
    float w = swap_sum32(x, y);
    w = swap_sum16(w, w);
    w += dpp<GSR_DPP_QUAD_XOR1>(w);
    w += dpp<GSR_DPP_QUAD_XOR2>(w);
    w += dpp<GSR_DPP_ROW_HALF_MIRROR>(w);
    w += dpp<GSR_DPP_ROW_MIRROR>(w);
    return w;
}

__device__ __forceinline__ void atomic_add_f64(double* p, double v)
{
    unsafeAtomicAdd(p, v);
}

}  // namespace gsr
