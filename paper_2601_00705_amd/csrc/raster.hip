// raster.hip -- per-tile alpha compositing, Eq. (alpha), forward and backward.
//
// One workgroup per (view, tile), one thread per pixel.  The tile's
// depth-sorted pair range is walked in batches: each thread stages one
// record into LDS (precomputed in exp2 form: power2 = a dx^2 + b dx dy +
// c dy^2 with the conic scaled by -log2(e)/2, -log2(e), -log2(e)/2, and the
// alpha_min test as power2 < log2(alpha_min / o)), then every pixel walks the
// batch.  Forward: alpha = min(alpha_max, o 2^power2); entries below
// alpha_min are skipped; compositing stops before an entry that would take T
// below T_min; out = C + T bg, plus T_final and n_contrib (list position + 1
// of the last blended entry), optionally the number of blended entries.
//
// Backward: the same range is replayed from the block's largest n_contrib
// down.  Each pixel recovers T before an entry as T / (1 - alpha) and keeps
// g . (colour behind) as a running scalar, giving
//   dL/dalpha_i = T_i g.c_i - (g.S_i + dL/dT_final T_final) / (1 - alpha_i).
// Per entry the 9 screen-space partials are reduced over the wavefront
// (transposed exchange: 8 values in 10 shuffles, plus one), accumulated per
// batch in LDS across the workgroup's waves, then added to the per-slot
// accumulators with one global float atomic per field and batch entry.
#include "kernels.h"

namespace gsr {

#define GSR_LOG2E 1.4426950408889634f
#define GSR_LN2 0.69314718055994531f

struct __align__(16) LdsRec {
    float4 p0;  // u, v, a2, b2      (a2 = -0.5 log2e A, b2 = -log2e B)
    float4 p1;  // c2, o, thr, -     (c2 = -0.5 log2e C, thr = log2(alpha_min / o))
    float4 p2;  // r, g, b, slot bits
};

__device__ __forceinline__ void stage_record(const RasterArgs& a, uint32_t slot, LdsRec& r)
{
    float4 gm = a.geom[slot];
    float4 co = a.conic_o[slot];
    float4 cd = a.rgb_d[slot];
    float thr = a.cfg.alpha_min > 0.0f ? __log2f(a.cfg.alpha_min / co.w) : -INFINITY;
    r.p0 = make_float4(gm.x, gm.y, -0.5f * GSR_LOG2E * co.x, -GSR_LOG2E * co.y);
    r.p1 = make_float4(-0.5f * GSR_LOG2E * co.z, co.w, thr, 0.0f);
    r.p2 = make_float4(cd.x, cd.y, cd.z, __uint_as_float(slot));
}

// power2 of a record at pixel centre (fpx, fpy); identical in both passes
__device__ __forceinline__ float eval_power2(const LdsRec& r, float fpx, float fpy, float& dx, float& dy,
                                             float& t)
{
    dx = fpx - r.p0.x;
    dy = fpy - r.p0.y;
    t = __builtin_fmaf(r.p0.z, dx, r.p0.w * dy);  // a2 dx + b2 dy
    return __builtin_fmaf(t, dx, r.p1.x * dy * dy);
}

struct TileCtx {
    int v, tx, ty, px, py;
    bool inside;
    int64_t pix;      // index into the concatenated [H][W] planes
    int64_t plane;    // H * W of the view
    int64_t rgb0;     // offset of channel 0 of this pixel
};

__device__ __forceinline__ TileCtx tile_ctx(const RasterArgs& a, int log2_tw)
{
    TileCtx c;
    const int tile = blockIdx.x;
    c.v = view_of_tile(a.views, tile);
    const ViewInfo& vw = a.views->v[c.v];
    int lt = tile - vw.tile_base;
    c.ty = lt / vw.tiles_x;
    c.tx = lt - c.ty * vw.tiles_x;
    const int tw = 1 << log2_tw;
    c.px = c.tx * tw + (threadIdx.x & (tw - 1));
    c.py = c.ty * a.cfg.tile_h + (threadIdx.x >> log2_tw);
    c.inside = c.px < vw.width && c.py < vw.height;
    c.plane = (int64_t)vw.width * vw.height;
    c.pix = (int64_t)vw.pix_base + (int64_t)c.py * vw.width + c.px;
    c.rgb0 = 3 * (int64_t)vw.pix_base + (int64_t)c.py * vw.width + c.px;
    return c;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_raster_fwd(RasterArgs a)
{
    __shared__ LdsRec rec[BLOCK];
    const TileCtx c = tile_ctx(a, a.cfg.log2_tw);
    const bool overflow = a.counters->overflow != 0u;
    const uint2 range = overflow ? make_uint2(0u, 0u) : a.ranges[blockIdx.x];
    const float fpx = (float)c.px + 0.5f, fpy = (float)c.py + 0.5f;
    const float amax = a.cfg.alpha_max, tmin = a.cfg.T_min;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    uint32_t last = 0, nb = 0;
    bool done = !c.inside;
    for (uint32_t base = range.x; base < range.y; base += BLOCK) {
        if (__syncthreads_and(done)) break;
        uint32_t j = base + threadIdx.x;
        if (j < range.y) stage_record(a, a.vals[j], rec[threadIdx.x]);
        __syncthreads();
        const int cnt = (int)min((uint32_t)BLOCK, range.y - base);
        for (int k = 0; k < cnt && !done; ++k) {
            const LdsRec r = rec[k];
            float dx, dy, t;
            float p2 = eval_power2(r, fpx, fpy, dx, dy, t);
            if (p2 < r.p1.z) continue;
            float alpha = fminf(amax, r.p1.y * __builtin_amdgcn_exp2f(p2));
            float Tn = __builtin_fmaf(-T, alpha, T);
            if (Tn < tmin) {
                done = true;
                break;
            }
            float wgt = alpha * T;
            C0 = __builtin_fmaf(r.p2.x, wgt, C0);
            C1 = __builtin_fmaf(r.p2.y, wgt, C1);
            C2 = __builtin_fmaf(r.p2.z, wgt, C2);
            T = Tn;
            last = base + (uint32_t)k - range.x + 1u;
            ++nb;
        }
    }
    if (!c.inside) return;
    if (overflow) {
        const float q = __builtin_nanf("");
        a.rgb[c.rgb0] = q;
        a.rgb[c.rgb0 + c.plane] = q;
        a.rgb[c.rgb0 + 2 * c.plane] = q;
        a.T_final[c.pix] = q;
        a.n_contrib[c.pix] = 0;
        if (a.n_blend) a.n_blend[c.pix] = 0;
        return;
    }
    a.rgb[c.rgb0] = __builtin_fmaf(T, a.cfg.bg0, C0);
    a.rgb[c.rgb0 + c.plane] = __builtin_fmaf(T, a.cfg.bg1, C1);
    a.rgb[c.rgb0 + 2 * c.plane] = __builtin_fmaf(T, a.cfg.bg2, C2);
    a.T_final[c.pix] = T;
    a.n_contrib[c.pix] = (int32_t)last;
    if (a.n_blend) a.n_blend[c.pix] = (int32_t)nb;
}

// One exchange step of the transposed reduction: keep half of 2N values,
// add the partner's copy of the kept half.
template <int N>
__device__ __forceinline__ void xchg(float* v, int lane, int mask)
{
    const bool hi = (lane & mask) != 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        float send = hi ? v[j] : v[N + j];
        float keep = hi ? v[N + j] : v[j];
        v[j] = keep + __shfl_xor(send, mask, 64);
    }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_raster_bwd(RasterArgs a)
{
    __shared__ LdsRec rec[BLOCK];
    __shared__ float acc[GSR_G2][BLOCK];
    __shared__ uint32_t smax;
    const TileCtx c = tile_ctx(a, a.cfg.log2_tw);
    if (a.counters->overflow) return;
    const uint2 range = a.ranges[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63;
    const float fpx = (float)c.px + 0.5f, fpy = (float)c.py + 0.5f;
    const float amax = a.cfg.alpha_max;

    float Tf = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, gT = 0.0f;
    uint32_t my_n = 0;
    if (c.inside) {
        Tf = a.T_final_in[c.pix];
        my_n = (uint32_t)a.n_contrib_in[c.pix];
        g0 = a.dL_drgb[c.rgb0];
        g1 = a.dL_drgb[c.rgb0 + c.plane];
        g2 = a.dL_drgb[c.rgb0 + 2 * c.plane];
        if (a.dL_dT) gT = a.dL_dT[c.pix];
    }
    if (tid == 0) smax = 0u;
    for (int f = 0; f < GSR_G2; ++f) acc[f][tid] = 0.0f;
    __syncthreads();
    atomicMax(&smax, my_n);
    __syncthreads();
    const uint32_t end = range.x + min(smax, range.y - range.x);

    float T = Tf;
    // g . (colour behind) + dL/dT_final T_final, maintained incrementally
    float gsk = __builtin_fmaf(gT, Tf, Tf * (g0 * a.cfg.bg0 + g1 * a.cfg.bg1 + g2 * a.cfg.bg2));
    const int64_t S = a.slots;

    for (uint32_t hi_ = end; hi_ > range.x;) {
        const uint32_t lo_ = hi_ - range.x > (uint32_t)BLOCK ? hi_ - BLOCK : range.x;
        const int cnt = (int)(hi_ - lo_);
        if (tid < cnt) stage_record(a, a.vals[hi_ - 1 - tid], rec[tid]);
        __syncthreads();
        for (int k = 0; k < cnt; ++k) {
            const uint32_t pos = hi_ - 1 - (uint32_t)k - range.x;
            const LdsRec r = rec[k];
            float dx, dy, t;
            float p2 = eval_power2(r, fpx, fpy, dx, dy, t);
            bool contrib = pos < my_n && p2 >= r.p1.z;
            float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            float v8 = 0.0f;
            if (contrib) {
                float G = __builtin_amdgcn_exp2f(p2);
                float a_raw = r.p1.y * G;
                bool clamped = !(a_raw < amax);
                float alpha = clamped ? amax : a_raw;
                float rcp = 1.0f / (1.0f - alpha);
                float Tb = T * rcp;
                float gcol = __builtin_fmaf(g0, r.p2.x, __builtin_fmaf(g1, r.p2.y, g2 * r.p2.z));
                float dalpha = __builtin_fmaf(Tb, gcol, -rcp * gsk);
                float wgt = alpha * Tb;
                v[6] = g0 * wgt;
                v[7] = g1 * wgt;
                v8 = g2 * wgt;
                gsk = __builtin_fmaf(wgt, gcol, gsk);
                T = Tb;
                if (!clamped) {
                    float dd = dalpha * alpha;
                    float ddx = dd * dx;
                    v[0] = dd * (t + r.p0.z * dx);                         // 2 a2 dx + b2 dy
                    v[1] = dd * __builtin_fmaf(r.p0.w, dx, 2.0f * r.p1.x * dy);  // b2 dx + 2 c2 dy
                    v[2] = ddx * dx;
                    v[3] = ddx * dy;
                    v[4] = dd * dy * dy;
                    v[5] = dalpha * G;
                }
            }
            if (__any(contrib)) {
                xchg<4>(v, lane, 32);
                xchg<2>(v, lane, 16);
                xchg<1>(v, lane, 8);
                float s = v[0];
                s += __shfl_xor(s, 4, 64);
                s += __shfl_xor(s, 2, 64);
                s += __shfl_xor(s, 1, 64);
                v8 = wave_sum(v8);
                if ((lane & 7) == 0) atomicAdd(&acc[lane >> 3][k], s);
                if (lane == 0) atomicAdd(&acc[8][k], v8);
            }
        }
        __syncthreads();
        if (tid < cnt) {
            const uint32_t slot = __float_as_uint(rec[tid].p2.w);
            // fields: du, dv, dA, dB, dC, do, dr, dg, db
            const float scale[GSR_G2] = {-GSR_LN2, -GSR_LN2, -0.5f, -1.0f, -0.5f, 1.0f, 1.0f, 1.0f, 1.0f};
#pragma unroll
            for (int f = 0; f < GSR_G2; ++f) {
                float x = acc[f][tid];
                if (x != 0.0f) atomic_add_f32(&a.grad2d[f * S + slot], x * scale[f]);
                acc[f][tid] = 0.0f;
            }
        }
        __syncthreads();
        hi_ = lo_;
    }
}

hipError_t launch_raster_fwd(const RasterArgs& a, int total_tiles, int tile_px, hipStream_t s)
{
    if (total_tiles == 0) return hipSuccess;
    switch (tile_px) {
    case 64: hipLaunchKernelGGL(k_raster_fwd<64>, dim3(total_tiles), dim3(64), 0, s, a); break;
    case 128: hipLaunchKernelGGL(k_raster_fwd<128>, dim3(total_tiles), dim3(128), 0, s, a); break;
    case 256: hipLaunchKernelGGL(k_raster_fwd<256>, dim3(total_tiles), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const RasterArgs& a, int total_tiles, int tile_px, hipStream_t s)
{
    if (total_tiles == 0) return hipSuccess;
    switch (tile_px) {
    case 64: hipLaunchKernelGGL(k_raster_bwd<64>, dim3(total_tiles), dim3(64), 0, s, a); break;
    case 128: hipLaunchKernelGGL(k_raster_bwd<128>, dim3(total_tiles), dim3(128), 0, s, a); break;
    case 256: hipLaunchKernelGGL(k_raster_bwd<256>, dim3(total_tiles), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// L1 photometric loss seed, Eq. (photometric): dL/dC = sign(C - target) / count

__global__ void k_loss_l1(LossArgs a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.count;
         i += (int64_t)gridDim.x * blockDim.x) {
        float d = a.rgb[i] - a.target[i];
        a.dL_drgb[i] = d > 0.0f ? a.scale : (d < 0.0f ? -a.scale : 0.0f);
    }
}

hipError_t launch_loss_l1(const LossArgs& a, hipStream_t s)
{
    if (a.count == 0) return hipSuccess;
    int64_t blocks = (a.count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_loss_l1, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void k_fill_nan(float* p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = __builtin_nanf("");
}

hipError_t launch_fill_nan(float* p, int64_t count, hipStream_t s)
{
    if (count == 0 || !p) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_nan, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

}  // namespace gsr
