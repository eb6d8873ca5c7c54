// order.hip -- the spatial storage order of a map.
//
// The method's sums do not depend on where a Gaussian is stored (only equal
// depths in the sets N(p) of Eq. (alpha) fall back on the index), so the
// order is a layout choice.  A map kept in this order gives the projection
// waves whose Gaussians share visibility, and the binning chunks whose pairs
// fall into few tiles; the brick interleave keeps the chunks' work even.
//
//   k_order_box     least and greatest coordinates of the finite means,
//                   one partial box per block (min and max need no order)
//   k_order_codes   the box from the partials, then 10-bit cubic cells over
//                   it (FP64: the box's extent rounded up to a power of two,
//                   so the scaling is exact), their Morton code, 2^30 for a
//                   non-finite mean
//   4 radix passes  stable LSD ranking of (code, index), 8 bits a pass:
//     k_radix_hist    per-block digit counts, digit-major
//     k_radix_scan    one block per digit: exclusive scan of the digit's
//                     counts over the blocks, and the digit's total
//     k_radix_scatter each key at its digit's start (a scan of the totals)
//                     plus its block's offset plus its rank among the
//                     block's equal digits (wave ballots, then the waves in
//                     order), so the pass is stable
//   k_order_bricks  position j B + k takes rank ((j P) mod F) B + k
#include "order.h"

namespace gsr {

// float -> uint32 in the order of the floats, and back
__device__ __forceinline__ uint32_t float_ord(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float ord_float(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__device__ __forceinline__ uint32_t spread10(uint32_t x)
{
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x30000ffu;
    x = (x | (x << 8)) & 0x300f00fu;
    x = (x | (x << 4)) & 0x30c30c3u;
    x = (x | (x << 2)) & 0x9249249u;
    return x;
}

// block-wide min of lo[3] and max of hi[3] (256 threads); thread 0 ends
// with the block's values
__device__ __forceinline__ void block_box(uint32_t (&lo)[3], uint32_t (&hi)[3])
{
    __shared__ uint32_t part[4][6];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        for (int off = 32; off > 0; off >>= 1) {
            lo[k] = min(lo[k], (uint32_t)__shfl_xor((int)lo[k], off, 64));
            hi[k] = max(hi[k], (uint32_t)__shfl_xor((int)hi[k], off, 64));
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            part[w][k] = lo[k];
            part[w][3 + k] = hi[k];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; ++q) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                lo[k] = min(lo[k], part[q][k]);
                hi[k] = max(hi[k], part[q][3 + k]);
            }
        }
    }
}

// partial box of block b's stride of Gaussians at box[8 b .. 8 b + 6) (a
// block without a finite mean leaves the identities 0xffffffff and 0)
__global__ __launch_bounds__(256) void k_order_box(OrderArgs a)
{
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = a.mean[i], y = a.mean[a.n + i], z = a.mean[2 * a.n + i];
        if (__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z)) {
            const uint32_t o[3] = {float_ord(x), float_ord(y), float_ord(z)};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                lo[k] = min(lo[k], o[k]);
                hi[k] = max(hi[k], o[k]);
            }
        }
    }
    block_box(lo, hi);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            a.box[8 * blockIdx.x + k] = lo[k];
            a.box[8 * blockIdx.x + 3 + k] = hi[k];
        }
    }
}

__global__ __launch_bounds__(256) void k_order_codes(OrderArgs a)
{
    __shared__ uint32_t bx[6];
    {
        uint32_t blo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, bhi[3] = {0u, 0u, 0u};
        for (int b = threadIdx.x; b < GSR_BOX_BLOCKS; b += blockDim.x) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                blo[k] = min(blo[k], a.box[8 * b + k]);
                bhi[k] = max(bhi[k], a.box[8 * b + 3 + k]);
            }
        }
        block_box(blo, bhi);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                bx[k] = blo[k];
                bx[3 + k] = bhi[k];
            }
        }
        __syncthreads();
    }
    double lo[3], w = 0.0;
    const bool any = bx[0] != 0xffffffffu;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lo[k] = any ? (double)ord_float(bx[k]) : 0.0;
        const double hi = any ? (double)ord_float(bx[3 + k]) : 0.0;
        w = fmax(w, hi - lo[k]);
    }
    // cells of side 2^e / 1024 with w = m 2^e, m in [0.5, 1): (x - lo) 2^(10 - e)
    // is below 1024 and the scaling by a power of two is exact
    double scale = 0.0;
    if (w > 0.0) {
        int e = 0;
        (void)frexp(w, &e);
        scale = ldexp(1.0, 10 - e);
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = a.mean[i], y = a.mean[a.n + i], z = a.mean[2 * a.n + i];
        uint32_t code = 1u << 30;
        if (__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z)) {
            const float c[3] = {x, y, z};
            uint32_t q[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double t = floor(((double)c[k] - lo[k]) * scale);
                q[k] = t >= 1023.0 ? 1023u : (uint32_t)t;
            }
            code = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
        }
        a.code[0][i] = code;
        a.val[0][i] = (uint32_t)i;
    }
}

// digit counts of block b's keys, at hist[digit * blocks + b]
__global__ __launch_bounds__(256) void k_radix_hist(OrderArgs a, int src, int shift)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * GSR_RADIX_TILE;
    const uint32_t* code = a.code[src];
#pragma unroll 4
    for (int k = 0; k < GSR_RADIX_TILE / 256; ++k) {
        const int64_t i = base + k * 256 + tid;
        if (i < a.n) atomicAdd(&h[(code[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    a.hist[(int64_t)tid * a.blocks + blockIdx.x] = h[tid];
}

// block d: exclusive scan of digit d's counts over the blocks, in place, and
// the digit's total
__global__ __launch_bounds__(256) void k_radix_scan(OrderArgs a)
{
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t* row = a.hist + (int64_t)blockIdx.x * a.blocks;
    const int per = (a.blocks + 255) / 256;
    const int lo = min(tid * per, a.blocks), hi = min(lo + per, a.blocks);
    uint32_t sum = 0u;
    for (int k = lo; k < hi; ++k) sum += row[k];
    uint32_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int k = 0; k < w; ++k) run += wsum[k];
    for (int k = lo; k < hi; ++k) {
        const uint32_t c = row[k];
        row[k] = run;
        run += c;
    }
    if (tid == 0) a.tot[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Each key of block b goes to its digit's start plus the digit's keys in
// the earlier blocks plus its rank among the block's earlier keys of that
// digit.  The block takes its keys 256 at a
// time, in order; within a wave the keys of one digit are found by matching
// the digit's 8 bits with ballots, and the waves' counts are added in wave
// order, so that equal digits keep their input order.
__global__ __launch_bounds__(256) void k_radix_scatter(OrderArgs a, int src, int shift)
{
    __shared__ uint32_t goff[256], run[256], wc[4][256], wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    {
        // digit tid starts after the keys of the smaller digits
        const uint32_t t = a.tot[tid];
        uint32_t incl = t;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t start = incl - t;
        for (int k = 0; k < w; ++k) start += wsum[k];
        goff[tid] = start + a.hist[(int64_t)tid * a.blocks + blockIdx.x];
    }
    run[tid] = 0u;
    const int64_t base = (int64_t)blockIdx.x * GSR_RADIX_TILE;
    const uint32_t* code_in = a.code[src];
    const uint32_t* val_in = a.val[src];
    uint32_t* code_out = a.code[src ^ 1];
    uint32_t* val_out = a.val[src ^ 1];
    const uint64_t below = (1ull << lane) - 1ull;
    for (int k = 0; k < GSR_RADIX_TILE / 256; ++k) {
        for (int d = lane; d < 256; d += 64) wc[w][d] = 0u;
        const int64_t i = base + k * 256 + tid;
        const bool valid = i < a.n;
        const uint32_t c = valid ? code_in[i] : 0u;
        const uint32_t v = valid ? val_in[i] : 0u;
        const uint32_t d = (c >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < GSR_RADIX_BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t set = __ballot(bit);
            peers &= bit ? set : ~set;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0u) wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            const uint32_t c0 = wc[0][tid], c1 = wc[1][tid], c2 = wc[2][tid], c3 = wc[3][tid], r = run[tid];
            wc[0][tid] = r;
            wc[1][tid] = r + c0;
            wc[2][tid] = r + c0 + c1;
            wc[3][tid] = r + c0 + c1 + c2;
            run[tid] = r + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        const uint32_t pos = goff[d] + wc[w][d] + rank;
        if (valid && pos < (uint64_t)a.n) {  // always below n when the counts agree
            code_out[pos] = c;
            val_out[pos] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_order_bricks(OrderArgs a, int src)
{
    const uint32_t* by_rank = a.val[src];
    const int64_t B = a.brick, inb = a.full * B;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = j < inb ? ((j / B) * a.mult % a.full) * B + j % B : j;
        a.index[j] = (int32_t)by_rank[r];
    }
}

hipError_t launch_spatial_order(const OrderArgs& a, hipStream_t s)
{
    int64_t grid = (a.n + 255) / 256;
    if (grid > 2048) grid = 2048;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_order_box, dim3(GSR_BOX_BLOCKS), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_order_codes, dim3((unsigned)grid), dim3(256), 0, s, a);
    int src = 0;
    for (int shift = 0; shift < 32; shift += GSR_RADIX_BITS) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)a.blocks), dim3(256), 0, s, a, src, shift);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)a.blocks), dim3(256), 0, s, a, src, shift);
        src ^= 1;
    }
    hipLaunchKernelGGL(k_order_bricks, dim3((unsigned)grid), dim3(256), 0, s, a, src);
    return hipGetLastError();
}

}  // namespace gsr
