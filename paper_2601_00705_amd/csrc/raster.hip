// raster.hip -- per-tile alpha compositing, Eq. (alpha), forward and backward.
//
// One wavefront (64 lanes) per (view, tile); each lane owns PPT = tile
// pixels / 64 pixels of one column of the tile (rows l / tile_w + k * 64 /
// tile_w).  The tile's depth-sorted pair range is walked in batches of
// BATCH (64, 128 or 256) records: every lane stages BATCH / 64 records into
// LDS in exp2 form, the quadratic form expanded around the tile centre in
// double (power2 = c0 + g . d + a2 dx^2 + b2 dx dy + c2 dy^2 for the offset d
// of a pixel from the tile centre, the conic scaled by -log2(e)/2, and the
// alpha_min test as power2 < log2(alpha_min / o)); then the lane walks the
// batch for each of its pixels, sharing the per-entry terms of its column.
//
// Forward: alpha = min(alpha_max, o 2^power2); entries below alpha_min are
// skipped; compositing stops before an entry that would take T below T_min;
// out = C + T bg, plus T_final and n_contrib (list position + 1 of the last
// blended entry) and, optionally, the number of blended entries.
//
// Backward: the range is replayed from the tile's largest n_contrib down.
// Each pixel recovers T before an entry as T / (1 - alpha) and keeps
// g . (colour behind) as a running scalar, so that
//   dL/dalpha_i = T_i g.c_i - (g.S_i + dL/dT_final T_final) / (1 - alpha_i).
// A lane sums its pixels' 9 screen-space partials of an entry, the wavefront
// reduces them on VALU cross-lane instructions (a transposed exchange of 8
// values in 7 swaps plus 3 DPP adds, and one full sum), and 9 lanes add the
// tile's totals to the slot's double accumulators with one atomic
// instruction (plus one).  Per-pixel work is branch-free (selects); an entry
// no lane of the wave needs is skipped as a whole.
#include "kernels.h"

namespace gsr {

#define GSR_LOG2E 1.4426950408889634f
#define GSR_LN2 0.69314718055994531f

struct __align__(16) LdsRec {
    float4 p0;  // c0, gx, gy, a2   (power2 at the tile centre and its gradient; a2 = k A)
    float4 p1;  // b2, c2, o, thr   (b2 = 2 k B, c2 = k C, thr = log2(alpha_min / o))
    float4 p2;  // r, g, b, slot bits
    float4 p3;  // ox, oy, 1/o, -   (tile centre - projected centre)
};

// Stages the record of `slot` for the tile centred at (xc, yc).  With
// k = -log2(e) / 2 and o = (xc, yc) - (u, v), the exp2-space power at a pixel
// offset d from the tile centre is
//   power2(d) = k (o + d)^T conic (o + d)
//             = c0 + gx dx + gy dy + a2 dx^2 + b2 dx dy + c2 dy^2,
// c0 = k o^T conic o, (gx, gy) = 2 k conic o, formed here in double: the
// quadratic form of a Gaussian whose centre lies far from the tile cancels
// heavily, and |d| is at most half a tile.
// The staged fields of a slot, from either record format: MIXED reads the
// 32-byte record (float32 centre and conic, binary16 colour).
struct Staged {
    double u, v, A, B, C;
    float o, r, g, b;
};

template <bool MIXED>
__device__ __forceinline__ Staged load_staged(const RasterArgs& a, uint32_t slot)
{
    Staged t;
    if (MIXED) {
        const StageRecM sr = static_cast<const StageRecM*>(a.stage)[slot];
        t.u = sr.u;
        t.v = sr.v;
        t.A = sr.A;
        t.B = sr.B;
        t.C = sr.C;
        t.o = sr.o;
        t.r = __half2float(sr.r);
        t.g = __half2float(sr.g);
        t.b = __half2float(sr.b);
    } else {
        const StageRec sr = static_cast<const StageRec*>(a.stage)[slot];
        t.u = sr.u;
        t.v = sr.v;
        t.A = sr.A;
        t.B = sr.B;
        t.C = sr.C;
        t.o = sr.o;
        t.r = sr.r;
        t.g = sr.g;
        t.b = sr.b;
    }
    return t;
}

template <bool MIXED>
__device__ __forceinline__ void stage_record(const RasterArgs& a, uint32_t slot, double xc, double yc,
                                             LdsRec& r)
{
    const Staged sr = load_staged<MIXED>(a, slot);
    const double k = -0.5 * 1.4426950408889634;
    const double ox = xc - sr.u, oy = yc - sr.v;
    const double qx = sr.A * ox + sr.B * oy, qy = sr.B * ox + sr.C * oy;
    const float thr = a.cfg.alpha_min > 0.0f ? log2f(a.cfg.alpha_min / sr.o) : -INFINITY;
    r.p0 = make_float4((float)(k * (ox * qx + oy * qy)), (float)(2.0 * k * qx), (float)(2.0 * k * qy),
                       (float)(k * sr.A));
    r.p1 = make_float4((float)(2.0 * k * sr.B), (float)(k * sr.C), sr.o, thr);
    r.p2 = make_float4(sr.r, sr.g, sr.b, __uint_as_float(slot));
    r.p3 = make_float4((float)ox, (float)oy, 1.0f / sr.o, 0.0f);
}

// writes one colour value of the image (float32, or binary16 when MIXED)
template <bool MIXED>
__device__ __forceinline__ void put_rgb(void* rgb, int64_t i, float x)
{
    if (MIXED) static_cast<__half*>(rgb)[i] = __float2half_rn(x);
    else static_cast<float*>(rgb)[i] = x;
}

// The terms of power2 shared by the pixels of one lane (same column offset
// dx), and power2 at row offset dy; the same operation sequence in both
// passes, so that their decisions agree bit for bit.
struct ColTerms {
    float s0;  // c0 + gx dx + a2 dx^2
    float s1;  // gy + b2 dx
};

__device__ __forceinline__ ColTerms col_terms(const LdsRec& r, float dx)
{
    ColTerms t;
    t.s0 = __builtin_fmaf(__builtin_fmaf(r.p0.w, dx, r.p0.y), dx, r.p0.x);
    t.s1 = __builtin_fmaf(r.p1.x, dx, r.p0.z);
    return t;
}

__device__ __forceinline__ float power2(const ColTerms& t, float c2, float dy)
{
    return __builtin_fmaf(__builtin_fmaf(c2, dy, t.s1), dy, t.s0);
}

template <int PPT>
struct TileCtx {
    int tile;                 // global tile of this workgroup
    int px, py0, rs;          // column, first row, row stride
    int width, height, pix_base;
    int64_t base;             // index of row py0 into the concatenated [H][W] planes
    int64_t plane;            // H * W of the view
    double xc, yc;            // tile centre in view pixel coordinates
    float dx;                 // this lane's pixel-centre offset from it (column)
    float dy[PPT];            // and its rows'
    // the lane's k-th pixel: inside the view, its [H][W] index, and its
    // channel-0 index into the concatenated [3][H][W] images (derived when
    // needed rather than held in registers)
    __device__ __forceinline__ bool inside(int k) const { return px < width && py0 + k * rs < height; }
    __device__ __forceinline__ int64_t pix(int k) const { return base + (int64_t)(k * rs) * width; }
    __device__ __forceinline__ int64_t rgb0(int k) const { return pix(k) + 2 * (int64_t)pix_base; }
};

// The lane's PPT pixels of `tile`, starting at pixel k0 of the lane's
// column in the tile (rows (lane >> log2 tw) + (k0 + k) * rs); k0 = 0 and the
// tile's full PPT for a whole tile, a sub-range for a part of a split tile.
template <int PPT>
__device__ __forceinline__ TileCtx<PPT> tile_ctx_at(const RasterArgs& a, int tile, int k0)
{
    TileCtx<PPT> c;
    c.tile = tile;
    const int v = view_of_tile(a.views, tile);
    const ViewInfo& vw = a.views->v[v];
    const int lt = tile - vw.tile_base;
    const int ty = lt / vw.tiles_x;
    const int tx = lt - ty * vw.tiles_x;
    const int lane = threadIdx.x;
    const int l2 = a.cfg.log2_tw;
    c.px = tx * a.cfg.tile_w + (lane & (a.cfg.tile_w - 1));
    c.rs = 64 >> l2;
    c.py0 = ty * a.cfg.tile_h + (lane >> l2) + k0 * c.rs;
    c.plane = (int64_t)vw.width * vw.height;
    c.xc = (double)(tx * a.cfg.tile_w) + 0.5 * a.cfg.tile_w;
    c.yc = (double)(ty * a.cfg.tile_h) + 0.5 * a.cfg.tile_h;
    c.dx = (float)(lane & (a.cfg.tile_w - 1)) + 0.5f - 0.5f * (float)a.cfg.tile_w;
    c.width = vw.width;
    c.height = vw.height;
    c.pix_base = vw.pix_base;
    c.base = (int64_t)vw.pix_base + (int64_t)c.py0 * vw.width + c.px;
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        c.dy[k] = (float)((lane >> l2) + (k0 + k) * c.rs) + 0.5f - 0.5f * (float)a.cfg.tile_h;
    return c;
}

// the workgroup's tile (processing order) and all of its pixels
template <int PPT>
__device__ __forceinline__ TileCtx<PPT> tile_ctx(const RasterArgs& a)
{
    return tile_ctx_at<PPT>(a, (int)a.order[blockIdx.x], 0);
}

// Whether an entry of opacity o can have a clamped alpha anywhere (alpha =
// o G with G <= 1): o >= alpha_max.  Both are positive floats, whose order is
// their bit patterns' order, so the test runs on the scalar unit with the
// first lane's o (the staged record is the same for every lane).
__device__ __forceinline__ bool may_clamp(float o, float amax)
{
    return __builtin_amdgcn_readfirstlane(__float_as_int(o)) >= __float_as_int(amax);
}

// Walks the batch in LDS for the lane's pixels.  A pixel that has stopped
// (or lies outside the view) carries a NaN row offset, so every later test
// power2 >= thr fails for it without a per-pixel flag.  Reaching T_min is
// rare (once per pixel at most), so the common step applies every passing
// entry and a wave-uniform branch undoes the blend of stopping pixels.
template <int PPT, bool COUNT>
__device__ __forceinline__ void fwd_batch(const LdsRec* rec, int cnt, uint32_t pos0, float amax, float tmin,
                                          float dx, float (&dy)[PPT], float (&T)[PPT], float (&C0)[PPT],
                                          float (&C1)[PPT], float (&C2)[PPT], uint32_t (&last)[PPT],
                                          uint32_t (&nb)[PPT])
{
    for (int e = 0; e < cnt; ++e) {
        if ((e & 15) == 0) {
            uint64_t live = 0;
#pragma unroll
            for (int k = 0; k < PPT; ++k) live |= __builtin_amdgcn_ballot_w64(dy[k] == dy[k]);
            if (live == 0) break;
        }
        const LdsRec r = rec[e];
        const ColTerms ct = col_terms(r, dx);
        float p2[PPT];
        bool pass[PPT];
        uint64_t any = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            p2[k] = power2(ct, r.p1.y, dy[k]);
            pass[k] = p2[k] >= r.p1.w;
            any |= __builtin_amdgcn_ballot_w64(pass[k]);
        }
        if (any == 0) continue;
        float ab[PPT], Tn[PPT];
        bool stop[PPT];
        uint64_t any_stop = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const float alpha = fminf(amax, r.p1.z * __builtin_amdgcn_exp2f(p2[k]));
            ab[k] = pass[k] ? alpha : 0.0f;
            Tn[k] = __builtin_fmaf(-T[k], ab[k], T[k]);
            stop[k] = Tn[k] < tmin;
            any_stop |= __builtin_amdgcn_ballot_w64(stop[k]);
        }
        if (any_stop != 0) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                ab[k] = stop[k] ? 0.0f : ab[k];
                Tn[k] = stop[k] ? T[k] : Tn[k];
                dy[k] = stop[k] ? __builtin_nanf("") : dy[k];
            }
        }
        const uint32_t pos1 = pos0 + (uint32_t)e + 1u;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const bool blend = pass[k] & !stop[k];
            const float wgt = ab[k] * T[k];
            C0[k] = __builtin_fmaf(r.p2.x, wgt, C0[k]);
            C1[k] = __builtin_fmaf(r.p2.y, wgt, C1[k]);
            C2[k] = __builtin_fmaf(r.p2.z, wgt, C2[k]);
            T[k] = Tn[k];
            last[k] = blend ? pos1 : last[k];
            if (COUNT) nb[k] += blend ? 1u : 0u;
        }
    }
}

// COUNT: also count the blended entries per pixel (into a.n_blend); a
// separate instantiation, so that the plain forward carries no counters
template <int PPT, int GSR_BATCH, bool COUNT, bool MIXED>
__device__ __forceinline__ void fwd_tile(const RasterArgs& a, const TileCtx<PPT>& c, LdsRec* rec)
{
    const int lane = threadIdx.x;
    const bool overflow = a.counters->overflow != 0u;
    const uint2 range = overflow ? make_uint2(0u, 0u) : a.ranges[c.tile];
    const float amax = a.cfg.alpha_max, tmin = a.cfg.T_min;
    float T[PPT], C0[PPT], C1[PPT], C2[PPT], dy[PPT];
    uint32_t last[PPT], nb[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = 0.0f;
        last[k] = nb[k] = 0u;
        dy[k] = c.inside(k) ? c.dy[k] : __builtin_nanf("");
    }
    for (uint32_t base = range.x; base < range.y; base += GSR_BATCH) {
        uint64_t live = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) live |= __builtin_amdgcn_ballot_w64(dy[k] == dy[k]);
        if (live == 0) break;
#pragma unroll
        for (int r = 0; r < GSR_BATCH / 64; ++r) {
            const uint32_t j = base + lane + 64 * r;
            if (j < range.y) stage_record<MIXED>(a, a.vals[j], c.xc, c.yc, rec[lane + 64 * r]);
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)GSR_BATCH, range.y - base);
        fwd_batch<PPT, COUNT>(rec, cnt, base - range.x, amax, tmin, c.dx, dy, T, C0, C1, C2, last, nb);
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (!c.inside(k)) continue;
        if (overflow) {
            const float q = __builtin_nanf("");
            put_rgb<MIXED>(a.rgb, c.rgb0(k), q);
            put_rgb<MIXED>(a.rgb, c.rgb0(k) + c.plane, q);
            put_rgb<MIXED>(a.rgb, c.rgb0(k) + 2 * c.plane, q);
            a.T_final[c.pix(k)] = q;
            a.n_contrib[c.pix(k)] = 0;
            if (COUNT) a.n_blend[c.pix(k)] = 0;
            continue;
        }
        put_rgb<MIXED>(a.rgb, c.rgb0(k), __builtin_fmaf(T[k], a.cfg.bg0, C0[k]));
        put_rgb<MIXED>(a.rgb, c.rgb0(k) + c.plane, __builtin_fmaf(T[k], a.cfg.bg1, C1[k]));
        put_rgb<MIXED>(a.rgb, c.rgb0(k) + 2 * c.plane, __builtin_fmaf(T[k], a.cfg.bg2, C2[k]));
        a.T_final[c.pix(k)] = T[k];
        a.n_contrib[c.pix(k)] = (int32_t)last[k];
        if (COUNT) a.n_blend[c.pix(k)] = (int32_t)nb[k];
    }
}

// The longest tiles are split: a wave's time is its tile's list, and the
// few longest lists would otherwise run alone at the end of the launch
// (measured: emptying the longest 1 % of the tiles at window-1M-10views,
// 5 % of the pairs, shortened the forward by 16 %).  A tile is long when
// its list holds at least half the pairs a resident wave would composite
// with the step's pairs spread evenly (GSR_FWD_WAVES resident waves), and
// at least GSR_FWD_LONG, rounded up to a power of two.  The processing
// order puts such tiles first (it is bucketed by floor(log2 length)), so
// they are the order's first K tiles, found by binary search.  Each is
// composited as FWD_SPLIT(PPT) parts, every part a wave with PPT / split of
// the lane's pixels and the whole list; a pixel's arithmetic is the same
// either way.  Splitting costs each part the whole list's per-entry work,
// so it pays only for the tail: where most tiles' lists are long (the
// 3M-Gaussian mapping views) the threshold rises with the pair count.
#ifndef GSR_FWD_SPLIT_MAX
#define GSR_FWD_SPLIT_MAX 4   // parts of the longest tiles (twice the threshold or more)
#endif
#ifndef GSR_FWD_LONG_PRIO
#define GSR_FWD_LONG_PRIO 2   // issue priority of the long tiles' waves (s_setprio, 0..3)
#endif

template <int PPT>
struct FwdSplit {
    static constexpr int parts = PPT < GSR_FWD_SPLIT ? PPT : GSR_FWD_SPLIT;
    static constexpr int ppt = PPT / parts;
    // tiles of twice the threshold or more: more parts, fewer pixels each
    static constexpr int parts2 = PPT < GSR_FWD_SPLIT_MAX ? PPT : (GSR_FWD_SPLIT_MAX < parts ? parts : GSR_FWD_SPLIT_MAX);
    static constexpr int ppt2 = PPT / parts2;
};

__device__ __forceinline__ uint32_t long_threshold(const RasterArgs& a)
{
    const unsigned long long even = a.counters->pairs / (2ull * GSR_FWD_WAVES);
    uint32_t t = GSR_FWD_LONG;
    while ((unsigned long long)t < even && t < (1u << 30)) t <<= 1;
    return t;
}

__device__ __forceinline__ int long_tiles(const RasterArgs& a, int total_tiles, uint32_t thr)
{
    int lo = 0, hi = total_tiles;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const uint2 r = a.ranges[a.order[mid]];
        if (r.y - r.x < thr) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <int PPT, int GSR_BATCH, bool COUNT, bool MIXED>
__global__ __launch_bounds__(64) void k_raster_fwd(RasterArgs a)
{
    __shared__ LdsRec rec[GSR_BATCH];
    const TileCtx<PPT> c = tile_ctx<PPT>(a);
    if (FwdSplit<PPT>::parts > 1) {
        const uint2 r = a.ranges[c.tile];
        if (r.y - r.x >= long_threshold(a)) return;  // composited in parts by k_raster_fwd_long
    }
    fwd_tile<PPT, GSR_BATCH, COUNT, MIXED>(a, c, rec);
}

// Persistent waves that take (long tile, part) items from a queue (zeroed
// before the launch) until the long tiles' parts are done.  The K2 tiles of
// twice the threshold or more (the order's first) come in parts2 parts, the
// others in parts; items go longest tile first.  The waves raise their issue
// priority: each carries a whole list and ends the forward, while the short
// tiles' waves beside them on the same SIMDs can wait a little.
template <int PPT, int GSR_BATCH, bool COUNT, bool MIXED>
__global__ __launch_bounds__(64) void k_raster_fwd_long(RasterArgs a, int total_tiles)
{
    using F = FwdSplit<PPT>;
    constexpr int S = F::parts, Q = F::ppt, S2 = F::parts2, Q2 = F::ppt2;
    __shared__ LdsRec rec[GSR_BATCH];
    if (GSR_FWD_LONG_PRIO) __builtin_amdgcn_s_setprio(GSR_FWD_LONG_PRIO);
    const uint32_t thr = long_threshold(a);
    const int k2 = S2 > S ? long_tiles(a, total_tiles, 2u * thr) : 0;
    const int items2 = k2 * S2;
    const int items = items2 + (long_tiles(a, total_tiles, thr) - k2) * S;
    for (;;) {
        uint32_t item = 0u;
        if (threadIdx.x == 0) item = atomicAdd(a.fwd_queue, 1u);
        item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item);
        if ((int)item >= items) break;
        if ((int)item < items2) {
            const int tile = (int)a.order[item / S2];
            const TileCtx<Q2> c = tile_ctx_at<Q2>(a, tile, (int)(item % S2) * Q2);
            fwd_tile<Q2, GSR_BATCH, COUNT, MIXED>(a, c, rec);
        } else {
            const uint32_t j = item - (uint32_t)items2;
            const int tile = (int)a.order[k2 + (int)(j / S)];
            const TileCtx<Q> c = tile_ctx_at<Q>(a, tile, (int)(j % S) * Q);
            fwd_tile<Q, GSR_BATCH, COUNT, MIXED>(a, c, rec);
        }
    }
}

__global__ void k_zero_queue(uint32_t* q)
{
    *q = 0u;
}

// scale of field f (du, dv, dA, dB, dC, -, dr, dg, db) from the reduced
// power2-space partials to the screen-space gradient (the opacity field is
// scaled by the record's 1/o)
__device__ __forceinline__ float field_scale(int f)
{
    return f < 2 ? -GSR_LN2 : (f == 3 ? -1.0f : (f < 5 ? -0.5f : 1.0f));
}

// Deterministic mode: the tile totals are added exactly, as fixed-point
// numbers, so that the sums do not depend on the order in which tiles run.
// A field is held in GSR_FIX_LIMBS signed 64-bit limbs; limb k collects the
// bits [32 k, 32 k + 32) of every addend (the lowest bit weighing
// 2^-GSR_FIX_UNIT) with its sign, without carries, which leaves 31 bits of
// headroom for the count of addends.  A float addend M 2^(E - 150) (M its
// 24-bit significand) spans at most two limbs: two integer atomics, no
// return value.  A slot's limbs are stored limb-major ([limb][field], 72
// bytes per limb), so that the 9 lanes of an entry's first atomic mostly
// hit one 72-byte block, as the FP64 path's do.  Bits below 2^-96 are
// dropped (truncation toward zero); magnitudes of 2^32 and beyond,
// infinities and NaN saturate to just below 2^32.
__device__ __forceinline__ void fixed_add(unsigned long long* limbs, int stride, float v)
{
    const uint32_t bits = __float_as_uint(v);
    const int E = (int)((bits >> 23) & 0xffu);
    if (E == 0) return;  // zero or subnormal: below the lowest bit
    uint32_t M = (bits & 0x7fffffu) | 0x800000u;
    int p = E - 150 + GSR_FIX_UNIT;  // weight 2^(p - 96) of M's lowest bit
    if (p > 32 * (GSR_FIX_LIMBS - 1) + 8) {
        M = 0xffffffu;
        p = 32 * (GSR_FIX_LIMBS - 1) + 8;
    }
    if (p < 0) {
        if (p <= -24) return;
        M >>= -p;
        p = 0;
    }
    const int k = p >> 5;
    const unsigned long long wide = (unsigned long long)M << (p & 31);
    const unsigned long long c0 = wide & 0xffffffffull, c1 = wide >> 32;
    const bool neg = (bits >> 31) != 0u;
    atomicAdd(&limbs[k * stride], neg ? 0ull - c0 : c0);
    if (c1 != 0ull && k + 1 < GSR_FIX_LIMBS) atomicAdd(&limbs[(k + 1) * stride], neg ? 0ull - c1 : c1);
}

// the value of a fixed-point field: carries propagated upwards (limbs 0..2
// end in [0, 2^32), the top limb keeps the sign); a negative total is
// negated and normalised again, so that the magnitude is summed from the
// top without cancellation
__device__ __forceinline__ double fixed_value(const unsigned long long* limbs, int stride)
{
    long long c[GSR_FIX_LIMBS];
#pragma unroll
    for (int k = 0; k < GSR_FIX_LIMBS; ++k) c[k] = (long long)limbs[k * stride];
#pragma unroll
    for (int k = 0; k + 1 < GSR_FIX_LIMBS; ++k) {
        c[k + 1] += c[k] >> 32;
        c[k] &= 0xffffffffll;
    }
    const bool neg = c[GSR_FIX_LIMBS - 1] < 0;
    if (neg) {
#pragma unroll
        for (int k = 0; k < GSR_FIX_LIMBS; ++k) c[k] = -c[k];
#pragma unroll
        for (int k = 0; k + 1 < GSR_FIX_LIMBS; ++k) {
            c[k + 1] += c[k] >> 32;
            c[k] &= 0xffffffffll;
        }
    }
    // the top limb's lowest bit weighs 2^(32 (limbs - 1) - unit) = 1
    static_assert(32 * (GSR_FIX_LIMBS - 1) == GSR_FIX_UNIT, "the top limb counts units of 1");
    double v = (double)c[0];
#pragma unroll
    for (int k = 1; k < GSR_FIX_LIMBS; ++k) v = (double)c[k] + v * 0x1p-32;
    return neg ? -v : v;
}

// Counts the tile as done for its view; the tile completing a whole
// backward of the view (the view's count reaching a multiple of its tiles:
// the count runs on across backward calls, so it needs no reset) stamps the
// view's completion time.
__device__ __forceinline__ void view_done(const RasterArgs& a, int tile, int lane)
{
    if (lane != 0) return;
    const int v = view_of_tile(a.views, tile);
    const unsigned long long tiles = (unsigned long long)(a.views->v[v].tiles_x * a.views->v[v].tiles_y);
    const unsigned long long old = atomicAdd(&a.tiles_done[v], 1ull);
    if ((old + 1ull) % tiles == 0ull) a.stamps[v] = (unsigned long long)wall_clock64();
}

// Adds a tile's total of screen-space field f to slot's accumulator: an FP64
// atomic, or (deterministic mode) the exact fixed-point limbs.
template <bool DET>
__device__ __forceinline__ void add_field(const RasterArgs& a, uint32_t slot, int f, float value)
{
    if (DET) fixed_add(a.acc + GSR_G2 * GSR_FIX_LIMBS * (int64_t)slot + f, GSR_G2, value);
    else atomic_add_f64(&a.grad2d[GSR_G2 * (int64_t)slot + f], (double)value);
}

// The ninth field (the blue colour partial) of a reduced entry waits for the
// next reduced entry's, and the two are summed over the wave in one chain
// (wave_sum_pair); slot is wave-uniform.
struct PendingField {
    bool have;
    uint32_t slot;
    float w;
};

// One entry of the backward replay for the lane's pixels, then the wave's
// reduction of the entry's nine screen-space partials and their addition to
// the slot's accumulators.  Per pixel, with rcp = 1 / (1 - alpha), T_j = T
// rcp the transmittance before the entry, gcol = g . c and gsk the running
// g . (colour behind) + dL/dT_final T_final:
//   dL/dalpha = T_j gcol - gsk rcp,
//   gsk'      = gsk + alpha T_j gcol,
//   dd        = alpha dL/dalpha = gsk' - gsk rcp   (one FMA);
// a pixel the entry does not reach takes alpha = 0, for which rcp(1) = 1
// exactly, so T, gsk and every partial stay unchanged without selects.
// CLAMP: the entry may clamp at alpha_max (o >= alpha_max), where alpha has
// no gradient (dd = 0) but still attenuates.
template <int PPT, bool CLAMP, bool DET>
__device__ __forceinline__ void bwd_entry(const RasterArgs& a, const LdsRec& r, const ColTerms& ct,
                                          const float (&p2)[PPT], const bool (&on)[PPT], float amax,
                                          const TileCtx<PPT>& c, const float (&g0)[PPT], const float (&g1)[PPT],
                                          const float (&g2)[PPT], const float (&dy2)[PPT], float (&T)[PPT],
                                          float (&gsk)[PPT], int lane, PendingField& pend)
{
    float c0s = 0.0f, c1s = 0.0f, c2s = 0.0f, D = 0.0f, Dy = 0.0f, Dyy = 0.0f;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const float a_raw = r.p1.z * __builtin_amdgcn_exp2f(p2[k]);
        const float alpha = on[k] ? (CLAMP ? fminf(a_raw, amax) : a_raw) : 0.0f;
        const float rcp = __builtin_amdgcn_rcpf(1.0f - alpha);
        const float Tb = T[k] * rcp;
        const float gcol = __builtin_fmaf(g0[k], r.p2.x, __builtin_fmaf(g1[k], r.p2.y, g2[k] * r.p2.z));
        const float wgt = alpha * Tb;
        c0s = __builtin_fmaf(g0[k], wgt, c0s);
        c1s = __builtin_fmaf(g1[k], wgt, c1s);
        c2s = __builtin_fmaf(g2[k], wgt, c2s);
        const float gsk_new = __builtin_fmaf(wgt, gcol, gsk[k]);
        float dd = __builtin_fmaf(-gsk[k], rcp, gsk_new);
        if (CLAMP) dd = a_raw < amax ? dd : 0.0f;
        gsk[k] = gsk_new;
        T[k] = Tb;
        D += dd;
        Dy = __builtin_fmaf(dd, c.dy[k], Dy);
        Dyy = __builtin_fmaf(dd, dy2[k], Dyy);
    }
    // power2 partials per pixel: d/du = -(2 a2 dx + b2 dy + gx),
    // d/dv = -(b2 dx + 2 c2 dy + gy) (d = pixel - tile centre), and
    // d/d(A, B, C) = k (fx^2, 2 fx fy, fy^2) with (fx, fy) = d + o the
    // offset from the projected centre; d alpha / d o = alpha / o
    const float fx = c.dx + r.p3.x;
    const float Fy = __builtin_fmaf(r.p3.y, D, Dy);  // sum dd fy
    float v[9];
    v[0] = __builtin_fmaf(__builtin_fmaf(2.0f * r.p0.w, c.dx, r.p0.y), D, r.p1.x * Dy);
    v[1] = __builtin_fmaf(ct.s1, D, 2.0f * r.p1.y * Dy);
    v[2] = fx * (fx * D);
    v[3] = fx * Fy;
    v[4] = __builtin_fmaf(r.p3.y, Fy + Dy, Dyy);
    v[5] = D;
    v[6] = c0s;
    v[7] = c1s;
    v[8] = c2s;
    const float s = wave_sum8_transposed(v, lane);
    const uint32_t slot = __builtin_amdgcn_readfirstlane(__float_as_uint(r.p2.w));
    if ((lane & 7) == 0) {
        const int f = lane >> 3;
        add_field<DET>(a, slot, f, s * (f == 5 ? r.p3.z : field_scale(f)));
    }
    if (pend.have) {
        const float w = wave_sum_pair(pend.w, v[8]);
        if (lane == 1) add_field<DET>(a, pend.slot, 8, w);
        if (lane == 33) add_field<DET>(a, slot, 8, w);
        pend.have = false;
    } else {
        pend.w = v[8];
        pend.slot = slot;
        pend.have = true;
    }
}

template <int PPT, int GSR_BATCH, bool DET, bool MIXED>
__global__ __launch_bounds__(64) void k_raster_bwd(RasterArgs a)
{
    __shared__ LdsRec rec[GSR_BATCH];
    const TileCtx<PPT> c = tile_ctx<PPT>(a);
    // the accumulators are in use from here on (the clearing kernel, which
    // reads the flag, has completed before this kernel starts)
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counters->grad_dirty = 1u;
    const int lane = threadIdx.x;
    if (a.counters->overflow) {
        view_done(a, c.tile, lane);
        return;
    }
    const uint2 range = a.ranges[c.tile];
    const float amax = a.cfg.alpha_max;

    float T[PPT], Tf[PPT], gsk[PPT], g0[PPT], g1[PPT], g2[PPT], dy2[PPT];
    uint32_t my_n[PPT];
    uint32_t lane_max = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        Tf[k] = 1.0f;
        g0[k] = g1[k] = g2[k] = 0.0f;
        float gT = 0.0f;
        my_n[k] = 0u;
        if (c.inside(k)) {
            Tf[k] = a.T_final_in[c.pix(k)];
            my_n[k] = (uint32_t)a.n_contrib_in[c.pix(k)];
            g0[k] = a.dL_drgb[c.rgb0(k)];
            g1[k] = a.dL_drgb[c.rgb0(k) + c.plane];
            g2[k] = a.dL_drgb[c.rgb0(k) + 2 * c.plane];
            if (a.dL_dT) gT = a.dL_dT[c.pix(k)];
        }
        T[k] = Tf[k];
        dy2[k] = c.dy[k] * c.dy[k];
        // g . (colour behind) + dL/dT_final T_final, maintained incrementally
        gsk[k] = __builtin_fmaf(gT, Tf[k], Tf[k] * (g0[k] * a.cfg.bg0 + g1[k] * a.cfg.bg1 + g2[k] * a.cfg.bg2));
        lane_max = max(lane_max, my_n[k]);
    }
    for (int off = 32; off > 0; off >>= 1) lane_max = max(lane_max, (uint32_t)__shfl_xor((int)lane_max, off, 64));
    const uint32_t end = range.x + min(lane_max, range.y - range.x);

    PendingField pend{false, 0u, 0.0f};
    for (uint32_t hi_ = end; hi_ > range.x;) {
        const uint32_t lo_ = hi_ - range.x > (uint32_t)GSR_BATCH ? hi_ - GSR_BATCH : range.x;
        const int cnt = (int)(hi_ - lo_);
#pragma unroll
        for (int r = 0; r < GSR_BATCH / 64; ++r) {
            const int t = lane + 64 * r;
            if (t < cnt) stage_record<MIXED>(a, a.vals[hi_ - 1 - t], c.xc, c.yc, rec[t]);
        }
        __syncthreads();
        for (int e = 0; e < cnt; ++e) {
            const uint32_t pos = hi_ - 1 - (uint32_t)e - range.x;
            const LdsRec r = rec[e];
            const ColTerms ct = col_terms(r, c.dx);
            float p2[PPT];
            bool on[PPT], any = false;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                p2[k] = power2(ct, r.p1.y, c.dy[k]);
                on[k] = (pos < my_n[k]) & (p2[k] >= r.p1.w);
                any |= on[k];
            }
            if (!__any(any)) continue;
            // alpha = o G <= o: only an entry with o >= alpha_max can clamp,
            // a test uniform over the wave
            if (may_clamp(r.p1.z, amax))
                bwd_entry<PPT, true, DET>(a, r, ct, p2, on, amax, c, g0, g1, g2, dy2, T, gsk, lane, pend);
            else
                bwd_entry<PPT, false, DET>(a, r, ct, p2, on, amax, c, g0, g1, g2, dy2, T, gsk, lane, pend);
        }
        __syncthreads();
        hi_ = lo_;
    }
    if (pend.have) {  // the last reduced entry's ninth field, alone
        const float w = wave_sum_pair(pend.w, 0.0f);
        if (lane == 1) add_field<DET>(a, pend.slot, 8, w);
    }
    view_done(a, c.tile, lane);
}

template <int PPT, int B, bool COUNT, bool MIXED>
static void launch_fwd_b(const RasterArgs& a, int tiles, hipStream_t s, hipStream_t side)
{
    if (FwdSplit<PPT>::parts > 1) {
        hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(1), 0, side, a.fwd_queue);
        hipLaunchKernelGGL((k_raster_fwd_long<PPT, B, COUNT, MIXED>), dim3(GSR_FWD_LONG_WAVES), dim3(64), 0, side,
                           a, tiles);
    }
    hipLaunchKernelGGL((k_raster_fwd<PPT, B, COUNT, MIXED>), dim3(tiles), dim3(64), 0, s, a);
}

template <int PPT, bool COUNT, bool MIXED>
static hipError_t launch_fwd_c(const RasterArgs& a, int tiles, int batch, hipStream_t s, hipStream_t side)
{
    switch (batch) {
    case 64: launch_fwd_b<PPT, 64, COUNT, MIXED>(a, tiles, s, side); break;
    case 128: launch_fwd_b<PPT, 128, COUNT, MIXED>(a, tiles, s, side); break;
    case 256: launch_fwd_b<PPT, 256, COUNT, MIXED>(a, tiles, s, side); break;
    default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

template <int PPT>
static hipError_t launch_fwd_t(const RasterArgs& a, int tiles, int batch, hipStream_t s, hipStream_t side)
{
    if (a.cfg.mixed)
        return a.n_blend ? launch_fwd_c<PPT, true, true>(a, tiles, batch, s, side)
                         : launch_fwd_c<PPT, false, true>(a, tiles, batch, s, side);
    return a.n_blend ? launch_fwd_c<PPT, true, false>(a, tiles, batch, s, side)
                     : launch_fwd_c<PPT, false, false>(a, tiles, batch, s, side);
}

template <int PPT, bool DET, bool MIXED>
static hipError_t launch_bwd_d(const RasterArgs& a, int tiles, int batch, hipStream_t s)
{
    switch (batch) {
    case 64: hipLaunchKernelGGL((k_raster_bwd<PPT, 64, DET, MIXED>), dim3(tiles), dim3(64), 0, s, a); break;
    case 128: hipLaunchKernelGGL((k_raster_bwd<PPT, 128, DET, MIXED>), dim3(tiles), dim3(64), 0, s, a); break;
    case 256: hipLaunchKernelGGL((k_raster_bwd<PPT, 256, DET, MIXED>), dim3(tiles), dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

template <int PPT>
static hipError_t launch_bwd_t(const RasterArgs& a, int tiles, int batch, hipStream_t s)
{
    if (a.cfg.mixed)
        return a.acc ? launch_bwd_d<PPT, true, true>(a, tiles, batch, s)
                     : launch_bwd_d<PPT, false, true>(a, tiles, batch, s);
    return a.acc ? launch_bwd_d<PPT, true, false>(a, tiles, batch, s)
                 : launch_bwd_d<PPT, false, false>(a, tiles, batch, s);
}

// The long tiles' parts run on `side`, forked from `s` and joined back (the
// fork and join are graph edges when `s` is being captured).
hipError_t launch_raster_fwd(const RasterArgs& a, int total_tiles, int tile_px, int batch, hipStream_t s,
                             hipStream_t side, hipEvent_t fork, hipEvent_t join)
{
    if (total_tiles == 0) return hipSuccess;
    hipError_t e = hipEventRecord(fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    if (e != hipSuccess) return e;
    switch (tile_px) {
    case 64: e = launch_fwd_t<1>(a, total_tiles, batch, s, side); break;
    case 128: e = launch_fwd_t<2>(a, total_tiles, batch, s, side); break;
    case 256: e = launch_fwd_t<4>(a, total_tiles, batch, s, side); break;
    case 512: e = launch_fwd_t<8>(a, total_tiles, batch, s, side); break;
    default: return hipErrorInvalidValue;
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
    return e;
}

// zero the screen-space accumulators of every projected slot (rx >= 0) when
// a backward has added to them since the projection zeroed them; the
// backward only ever adds to and reads such slots, so each backward starts
// from zero however often it is called
__global__ void k_clear_grad2d(const Counters* counters, const float4* geom, double* grad2d, int64_t slots)
{
    if (!counters->grad_dirty) return;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (geom[s].z >= 0.0f) {
#pragma unroll
            for (int f = 0; f < GSR_G2; ++f) grad2d[GSR_G2 * s + f] = 0.0;
        }
    }
}

// deterministic mode: the same for the fixed-point accumulators
__global__ void k_clear_acc(const Counters* counters, const float4* geom, unsigned long long* acc, int64_t slots)
{
    if (!counters->grad_dirty) return;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (geom[s].z >= 0.0f) {
            ulonglong2* p = reinterpret_cast<ulonglong2*>(acc + GSR_G2 * GSR_FIX_LIMBS * s);
#pragma unroll
            for (int k = 0; k < GSR_G2 * GSR_FIX_LIMBS / 2; ++k) p[k] = make_ulonglong2(0ull, 0ull);
        }
    }
}

// deterministic mode: the accumulators of every projected slot into grad2d
__global__ void k_fix_to_grad2d(const float4* geom, const unsigned long long* acc, double* grad2d, int64_t slots)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (geom[s].z >= 0.0f) {
#pragma unroll
            for (int f = 0; f < GSR_G2; ++f)
                grad2d[GSR_G2 * s + f] = fixed_value(acc + GSR_G2 * GSR_FIX_LIMBS * s + f, GSR_G2);
        }
    }
}

hipError_t launch_clear_grad2d(const RasterArgs& a, hipStream_t s)
{
    if (a.slots <= 0) return hipSuccess;
    int64_t blocks = (a.slots + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (a.acc)
        hipLaunchKernelGGL(k_clear_acc, dim3((unsigned)blocks), dim3(256), 0, s, a.counters, a.geom, a.acc,
                           a.slots);
    else
        hipLaunchKernelGGL(k_clear_grad2d, dim3((unsigned)blocks), dim3(256), 0, s, a.counters, a.geom, a.grad2d,
                           a.slots);
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const RasterArgs& a, int total_tiles, int tile_px, int batch, hipStream_t s)
{
    if (total_tiles == 0) return hipSuccess;
    hipError_t e;
    switch (tile_px) {
    case 64: e = launch_bwd_t<1>(a, total_tiles, batch, s); break;
    case 128: e = launch_bwd_t<2>(a, total_tiles, batch, s); break;
    case 256: e = launch_bwd_t<4>(a, total_tiles, batch, s); break;
    case 512: e = launch_bwd_t<8>(a, total_tiles, batch, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e == hipSuccess && a.acc && a.slots > 0) {
        int64_t blocks = (a.slots + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_fix_to_grad2d, dim3((unsigned)blocks), dim3(256), 0, s, a.geom, a.acc, a.grad2d,
                           a.slots);
    }
    return e != hipSuccess ? e : hipGetLastError();
}

// ---------------------------------------------------------------------------
// L1 photometric loss seed, Eq. (photometric): dL/dC = sign(C - target) / count

__device__ __forceinline__ float l1_sign(float x, float t, float scale)
{
    const float d = x - t;
    return d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
}

template <bool HALF>
__global__ void k_loss_l1(LossArgs a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float x = HALF ? __half2float(static_cast<const __half*>(a.rgb)[i]) : static_cast<const float*>(a.rgb)[i];
        a.dL_drgb[i] = l1_sign(x, a.target[i], a.scale);
    }
}

// the float32 image four values at a time (count a multiple of 4, the three
// buffers 16-byte aligned)
__global__ void k_loss_l1_vec(LossArgs a)
{
    const float4* rgb = static_cast<const float4*>(a.rgb);
    const float4* tgt = reinterpret_cast<const float4*>(a.target);
    float4* out = reinterpret_cast<float4*>(a.dL_drgb);
    const int64_t n4 = a.count / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 x = rgb[i], t = tgt[i];
        out[i] = make_float4(l1_sign(x.x, t.x, a.scale), l1_sign(x.y, t.y, a.scale), l1_sign(x.z, t.z, a.scale),
                             l1_sign(x.w, t.w, a.scale));
    }
}

hipError_t launch_loss_l1(const LossArgs& a, hipStream_t s)
{
    if (a.count == 0) return hipSuccess;
    int64_t blocks = (a.count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    const bool vec = !a.half_image && a.count % 4 == 0 && (((uintptr_t)a.rgb | (uintptr_t)a.target |
                                                            (uintptr_t)a.dL_drgb) & 15) == 0;
    if (vec) {
        int64_t vb = (a.count / 4 + 255) / 256;
        if (vb > 65536) vb = 65536;
        hipLaunchKernelGGL(k_loss_l1_vec, dim3((unsigned)vb), dim3(256), 0, s, a);
    } else if (a.half_image) {
        hipLaunchKernelGGL(k_loss_l1<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_loss_l1<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace gsr
