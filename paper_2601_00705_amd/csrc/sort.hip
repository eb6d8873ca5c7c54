// sort.hip -- stable LSD radix sort of (key u64, value u32) pairs, 8-bit digits.
//
// One pass = three kernels over virtual blocks of SORT_ITEMS pairs:
//   k_sort_hist    per-block digit histogram (wave64 match: each distinct
//                  digit of a 64-key round costs one LDS atomic)
//   k_sort_scan    one block per digit scans that digit's row of block counts
//   k_sort_scatter per block: stable local ranking (wave match + per-wave
//                  running counters), staging in LDS in digit order, then a
//                  coalesced store at the digit's global offset.
// Pair count and overflow flag are read from device memory, so the launch
// configuration depends only on the capacity (graph-capturable).  Items are
// ranked in index order (wave, round, lane), which makes every pass stable.
#include "kernels.h"

namespace gsr {

__device__ __forceinline__ unsigned long long match_digit(uint32_t d, bool valid)
{
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        bool bit = (d >> b) & 1u;
        unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__device__ __forceinline__ unsigned long long live_pairs(const Counters* c)
{
    return c->overflow ? 0ull : c->pairs;
}

__global__ __launch_bounds__(GSR_SORT_THREADS) void k_sort_hist(SortArgs a)
{
    __shared__ uint32_t hist[256];
    const unsigned long long M = live_pairs(a.counters);
    const int nvb = (int)((M + GSR_SORT_ITEMS - 1) / GSR_SORT_ITEMS);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        hist[tid] = 0;
        __syncthreads();
        const unsigned long long base = (unsigned long long)vb * GSR_SORT_ITEMS + w * 1024;
        for (int r = 0; r < 16; ++r) {
            unsigned long long idx = base + r * 64 + lane;
            bool valid = idx < M;
            uint32_t d = valid ? (uint32_t)(a.keys_in[idx] >> a.shift) & 255u : 0u;
            unsigned long long m = match_digit(d, valid);
            unsigned long long lt = (1ull << lane) - 1ull;
            if (valid && (m & lt) == 0ull) atomicAdd(&hist[d], (uint32_t)__popcll(m));
        }
        __syncthreads();
        a.hist[tid * a.max_blocks + vb] = hist[tid];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_sort_scan(SortArgs a)
{
    __shared__ uint32_t wsum[4];
    const unsigned long long M = live_pairs(a.counters);
    const int nvb = (int)((M + GSR_SORT_ITEMS - 1) / GSR_SORT_ITEMS);
    const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t* row = a.hist + (size_t)d * a.max_blocks;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nvb; b0 += 256) {
        int b = b0 + tid;
        uint32_t x = b < nvb ? row[b] : 0u;
        uint32_t incl = x;
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t wofs = 0;
        for (int k = 0; k < w; ++k) wofs += wsum[k];
        if (b < nvb) row[b] = carry + wofs + incl - x;
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (tid == 0) a.digit_total[d] = carry;
}

__global__ __launch_bounds__(GSR_SORT_THREADS) void k_sort_scatter(SortArgs a)
{
    __shared__ unsigned long long sk[GSR_SORT_ITEMS];
    __shared__ uint32_t sv[GSR_SORT_ITEMS];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t gdig[256];
    __shared__ uint32_t wsum[4];
    const unsigned long long M = live_pairs(a.counters);
    const int nvb = (int)((M + GSR_SORT_ITEMS - 1) / GSR_SORT_ITEMS);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;

    // exclusive scan of the digit totals: global start of each digit
    {
        uint32_t x = a.digit_total[tid];
        uint32_t incl = x;
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t wofs = 0;
        for (int k = 0; k < w; ++k) wofs += wsum[k];
        gdig[tid] = wofs + incl - x;
        __syncthreads();
    }

    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const unsigned long long base = (unsigned long long)vb * GSR_SORT_ITEMS;
        const int cnt = (int)min((unsigned long long)GSR_SORT_ITEMS, M - base);
        for (int k = tid; k < 4 * 256; k += GSR_SORT_THREADS) (&wcnt[0][0])[k] = 0;
        __syncthreads();
        unsigned long long key[16];
        uint32_t val[16];
        uint32_t rank[16];
        uint32_t dig[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int li = w * 1024 + r * 64 + lane;
            bool valid = li < cnt;
            key[r] = valid ? a.keys_in[base + li] : 0ull;
            val[r] = valid ? a.vals_in[base + li] : 0u;
            uint32_t d = (uint32_t)(key[r] >> a.shift) & 255u;
            dig[r] = valid ? d : 256u;
            unsigned long long m = match_digit(d, valid);
            uint32_t below = (uint32_t)__popcll(m & lt);
            uint32_t start = valid ? wcnt[w][d] : 0u;
            // every lane of the wave has read its counter before a leader
            // updates it (lockstep; the barrier keeps the order explicit)
            __builtin_amdgcn_wave_barrier();
            rank[r] = start + below;
            if (valid && below == 0u) wcnt[w][d] = start + (uint32_t)__popcll(m);
        }
        __syncthreads();
        // per digit (thread = digit): wave prefixes and the block's digit starts
        {
            uint32_t c0 = wcnt[0][tid], c1 = wcnt[1][tid], c2 = wcnt[2][tid], c3 = wcnt[3][tid];
            uint32_t tot = c0 + c1 + c2 + c3;
            uint32_t incl = tot;
            for (int off = 1; off < 64; off <<= 1) {
                uint32_t y = __shfl_up(incl, off, 64);
                if (lane >= off) incl += y;
            }
            if (lane == 63) wsum[w] = incl;
            __syncthreads();
            uint32_t wofs = 0;
            for (int k = 0; k < w; ++k) wofs += wsum[k];
            uint32_t ds = wofs + incl - tot;
            dstart[tid] = ds;
            wcnt[0][tid] = ds;
            wcnt[1][tid] = ds + c0;
            wcnt[2][tid] = ds + c0 + c1;
            wcnt[3][tid] = ds + c0 + c1 + c2;
            gbase[tid] = gdig[tid] + a.hist[tid * a.max_blocks + vb];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (dig[r] < 256u) {
                uint32_t pos = wcnt[w][dig[r]] + rank[r];
                sk[pos] = key[r];
                sv[pos] = val[r];
            }
        }
        __syncthreads();
        for (int i = tid; i < cnt; i += GSR_SORT_THREADS) {
            unsigned long long k = sk[i];
            uint32_t d = (uint32_t)(k >> a.shift) & 255u;
            uint32_t out = gbase[d] + (uint32_t)i - dstart[d];
            a.keys_out[out] = k;
            a.vals_out[out] = sv[i];
        }
        __syncthreads();
    }
}

hipError_t launch_sort_pass(const SortArgs& a, int grid_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_sort_hist, dim3(grid_blocks), dim3(GSR_SORT_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_sort_scan, dim3(256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sort_scatter, dim3(grid_blocks), dim3(GSR_SORT_THREADS), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// tile ranges of the sorted keys

__global__ void k_ranges_zero(RangeArgs a)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.total_tiles) a.ranges[t] = make_uint2(0u, 0u);
    if (t < 64) a.buckets[t] = 0u;
}

__global__ void k_ranges(RangeArgs a)
{
    const unsigned long long M = live_pairs(a.counters);
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        uint32_t t = (uint32_t)(a.keys[i] >> 32);
        if (i == 0 || (uint32_t)(a.keys[i - 1] >> 32) != t) a.ranges[t].x = (uint32_t)i;
        if (i == M - 1 || (uint32_t)(a.keys[i + 1] >> 32) != t) a.ranges[t].y = (uint32_t)(i + 1);
    }
}

// ---------------------------------------------------------------------------
// processing order of the tiles: descending pair count, bucketed by
// floor(log2(count)) (bucket 0 holds the longest lists); the compositing
// kernels take their tile from this order so that long lists start first

__device__ __forceinline__ uint32_t count_bucket(uint2 r)
{
    uint32_t c = r.y - r.x;
    return c == 0u ? 31u : (uint32_t)__clz(c);  // 31 - floor(log2 c)
}

__global__ void k_order_count(RangeArgs a)
{
    __shared__ uint32_t h[32];
    if (threadIdx.x < 32) h[threadIdx.x] = 0u;
    __syncthreads();
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.total_tiles) atomicAdd(&h[count_bucket(a.ranges[t])], 1u);
    __syncthreads();
    if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&a.buckets[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_order_place(RangeArgs a)
{
    __shared__ uint32_t base[32];
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int b = 0; b < 32; ++b) {
            base[b] = run;
            run += a.buckets[b];
        }
    }
    __syncthreads();
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.total_tiles) {
        uint32_t b = count_bucket(a.ranges[t]);
        a.order[base[b] + atomicAdd(&a.buckets[32 + b], 1u)] = (uint32_t)t;
    }
}

hipError_t launch_ranges(const RangeArgs& a, int grid_blocks, hipStream_t s)
{
    const int tb = (a.total_tiles + 255) / 256;
    hipLaunchKernelGGL(k_ranges_zero, dim3(tb > 0 ? tb : 1), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_ranges, dim3(grid_blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_order_count, dim3(tb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_order_place, dim3(tb), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
