// sort.hip -- per-tile ordering of the emitted pairs, and the tiles' order.
//
// k_seg_sort   one block per tile (longest first): sorts the
//              segment's unique 64-bit keys (depth bits << 32 | Gaussian
//              index) ascending with a stable LSD radix sort of 8-bit digits,
//              skipping every digit that is the same for all keys of the
//              segment.  In LDS the depth digits go first and the runs of
//              equal depth are then put in index order by odd-even
//              transposition (falling back to every digit when a run does
//              not settle in 8 rounds).  Then it writes the final pairs: key (tile << 32 | depth
//              bits), value slot = view * n + index.  Segments of up to
//              the block's LDS capacity are sorted in LDS; longer ones in
//              chunks of that size, then merged pairwise through global
//              memory.
// k_order_*    processing order of the tiles: descending pair count, bucketed
//              by floor(log2(count)), for the segment sort and compositing.
//
// Ranking inside the block is stable: items are ranked in index order (wave,
// round, lane) with wave-private digit counters; equal digits inside a round
// are found with 8 ballots.
#include "kernels.h"

#ifndef GSR_SORT_SMALL_MAIN
#define GSR_SORT_SMALL_MAIN 512  // small-class blocks also launched on the main stream (0: none)
#endif

namespace gsr {

// lanes of the wave (valid ones) holding the same 8-bit digit as this lane:
// for every bit, keep the ballot of that bit where this lane's bit is 1 and
// its complement where it is 0, i.e. m &= ~(ballot ^ sign-extended bit), on
// the two 32-bit halves
__device__ __forceinline__ unsigned long long match_digit(uint32_t d, bool valid)
{
    const unsigned long long v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint32_t s = (uint32_t)((int32_t)(d << (31 - b)) >> 31);  // 0 or ~0
        const unsigned long long bb = __ballot(s != 0u);
        lo &= ~((uint32_t)bb ^ s);
        hi &= ~((uint32_t)(bb >> 32) ^ s);
    }
    return ((unsigned long long)hi << 32) | lo;
}

template <int WAVES, int ITEMS>
struct SegLds {
    // the digit scans give one thread to each of the 256 digits
    static_assert(WAVES * 64 >= 256, "a sorting block needs at least 256 threads");
    unsigned long long sk[ITEMS];          // keys in digit order (LDS path)
    uint32_t wcnt[WAVES][256];             // per-wave digit counters, then wave offsets
    uint32_t dstart[256];                  // block-local start of each digit
    uint32_t wsum[4];
    unsigned long long red[2][WAVES];
};

// Stable ranking of the block's items by digit (key >> shift) & 255.  Item
// (r, lane) of wave w has index w * R * 64 + r * 64 + lane; on return
// pos[r] is its position in digit order (digit-major, index order within a
// digit) or ~0 for an item past m, and L.dstart[] holds the first position
// of each digit.
template <int WAVES, int ITEMS, int MAXR>
__device__ __forceinline__ void rank_items(const unsigned long long* key, int R, int m, int shift, uint32_t* pos,
                                           SegLds<WAVES, ITEMS>& L)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int k = tid; k < WAVES * 256; k += WAVES * 64) (&L.wcnt[0][0])[k] = 0u;
    __syncthreads();
    uint32_t dig[MAXR];
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        if (r >= R) break;
        const int li = w * R * 64 + r * 64 + lane;
        const bool valid = li < m;
        const uint32_t d = valid ? (uint32_t)(key[r] >> shift) & 255u : 0u;
        const unsigned long long mk = match_digit(d, valid);
        // set bits of mk in the lanes below this one
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
        const uint32_t start = valid ? L.wcnt[w][d] : 0u;
        // every lane has read its counter before a leader updates it
        __builtin_amdgcn_wave_barrier();
        pos[r] = start + below;
        dig[r] = valid ? d : 256u;
        if (valid && below == 0u) L.wcnt[w][d] = start + (uint32_t)__popcll(mk);
    }
    __syncthreads();
    // threads 0..255 (one per digit): wave offsets inside the digit and the
    // block's digit starts
    uint32_t tot = 0, incl = 0;
    if (tid < 256) {
        for (int k = 0; k < WAVES; ++k) tot += L.wcnt[k][tid];
        incl = tot;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) L.wsum[w] = incl;
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t ds = incl - tot;
        for (int k = 0; k < w; ++k) ds += L.wsum[k];
        L.dstart[tid] = ds;
        for (int k = 0; k < WAVES; ++k) {
            const uint32_t c = L.wcnt[k][tid];
            L.wcnt[k][tid] = ds;
            ds += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        if (r >= R) break;
        pos[r] = dig[r] < 256u ? L.wcnt[w][dig[r]] + pos[r] : 0xffffffffu;
    }
}

// OR and AND of the block's keys (identity for no key)
template <int WAVES, int ITEMS>
__device__ __forceinline__ void block_or_and(unsigned long long o, unsigned long long a, SegLds<WAVES, ITEMS>& L,
                                             unsigned long long& bor, unsigned long long& band)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        o |= __shfl_xor(o, off, 64);
        a &= __shfl_xor(a, off, 64);
    }
    if (lane == 0) {
        L.red[0][w] = o;
        L.red[1][w] = a;
    }
    __syncthreads();
    bor = 0ull;
    band = ~0ull;
    for (int k = 0; k < WAVES; ++k) {
        bor |= L.red[0][k];
        band &= L.red[1][k];
    }
    __syncthreads();
}

__device__ __forceinline__ void write_pair(const SegArgs& a, uint32_t at, unsigned long long k, unsigned long long tile,
                                           uint32_t vbase)
{
    a.keys[at] = (tile << 32) | (k >> 32);
    a.vals[at] = vbase + (uint32_t)k;
}

// Sorts the m <= ITEMS keys src[0, m) with the whole block in LDS; on return
// key[r] of thread (w, lane) holds the key of sorted position
// w * R * 64 + r * 64 + lane (R = ceil(m / THREADS)) when that is below m.
template <int WAVES, int ITEMS>
__device__ void lds_sort(const unsigned long long* src, int m, unsigned long long (&key)[ITEMS / (WAVES * 64)],
                         SegLds<WAVES, ITEMS>& L)
{
    constexpr int THREADS = WAVES * 64;
    constexpr int MAXR = ITEMS / THREADS;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int R = (m + THREADS - 1) / THREADS;
    uint32_t pos[MAXR];
    unsigned long long o = 0ull, an = ~0ull;
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        if (r >= R) break;
        const int li = w * R * 64 + r * 64 + lane;
        key[r] = li < m ? src[li] : 0ull;
        if (li < m) {
            o |= key[r];
            an &= key[r];
        }
    }
    unsigned long long bor, band;
    block_or_and(o, an, L, bor, band);
    const unsigned long long diff = bor ^ band;
    // depth digits first.  Keys that share a depth then stand in runs in
    // emission order; odd-even transposition inside those runs puts them in
    // index order (a few rounds: runs are short).  Runs that do not settle
    // within 8 rounds fall back to sorting every digit, LSD from the index.
    bool sorted = false, in_lds = false;
    for (int d = 4; d < 8; ++d) {
        if (((diff >> (8 * d)) & 255ull) == 0ull) continue;
        rank_items<WAVES, ITEMS, MAXR>(key, R, m, 8 * d, pos, L);
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
            if (r >= R) break;
            if (pos[r] != 0xffffffffu) L.sk[pos[r]] = key[r];
        }
        __syncthreads();
        in_lds = true;
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
            if (r >= R) break;
            const int li = w * R * 64 + r * 64 + lane;
            if (li < m) key[r] = L.sk[li];
        }
        __syncthreads();
    }
    if ((diff & 0xffffffffull) == 0ull) {
        sorted = true;  // a single key
    } else if (diff >> 32) {
        if (!in_lds) {
#pragma unroll
            for (int r = 0; r < MAXR; ++r) {
                if (r >= R) break;
                const int li = w * R * 64 + r * 64 + lane;
                if (li < m) L.sk[li] = key[r];
            }
            __syncthreads();
        }
        for (int round = 0; round < 8 && !sorted; ++round) {
            bool swapped = false;
            for (int par = 0; par < 2; ++par) {
                for (int i = par + 2 * tid; i + 1 < m; i += 2 * THREADS) {
                    const unsigned long long x = L.sk[i], y = L.sk[i + 1];
                    if ((x >> 32) == (y >> 32) && x > y) {
                        L.sk[i] = y;
                        L.sk[i + 1] = x;
                        swapped = true;
                    }
                }
                __syncthreads();
            }
            sorted = __syncthreads_or(swapped) == 0;
        }
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
            if (r >= R) break;
            const int li = w * R * 64 + r * 64 + lane;
            if (li < m) key[r] = L.sk[li];
        }
        __syncthreads();
    }
    if (!sorted) {
        for (int d = 0; d < 8; ++d) {
            if (((diff >> (8 * d)) & 255ull) == 0ull) continue;
            rank_items<WAVES, ITEMS, MAXR>(key, R, m, 8 * d, pos, L);
#pragma unroll
            for (int r = 0; r < MAXR; ++r) {
                if (r >= R) break;
                if (pos[r] != 0xffffffffu) L.sk[pos[r]] = key[r];
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < MAXR; ++r) {
                if (r >= R) break;
                const int li = w * R * 64 + r * 64 + lane;
                if (li < m) key[r] = L.sk[li];
            }
            __syncthreads();
        }
    }
}

// Merges the sorted runs A[0, na) and B[0, nb) (unique keys) with the whole
// block: thread t produces the outputs [t per, (t + 1) per), per =
// ceil((na + nb) / THREADS), finding how many of them come from A by a
// binary search along its first diagonal (merge path), then merging
// sequentially.  out(d, key) receives output position d.
template <int THREADS, class Out>
__device__ __forceinline__ void merge_runs(const unsigned long long* A, int na, const unsigned long long* B, int nb,
                                           Out&& out)
{
    const int n = na + nb;
    const int per = (n + THREADS - 1) / THREADS;
    const int d0 = min(n, (int)threadIdx.x * per), d1 = min(n, d0 + per);
    if (d0 >= d1) return;
    int lo = max(0, d0 - nb), hi = min(d0, na);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A[mid] < B[d0 - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    int i = lo, j = d0 - lo;
    for (int d = d0; d < d1; ++d) {
        const bool take_a = j >= nb || (i < na && A[i] < B[j]);
        out(d, take_a ? A[i++] : B[j++]);
    }
}

// Sorts the segment of one tile with the whole block (WAVES * 64 threads,
// ITEMS keys fit in LDS).  A longer segment is cut into chunks of ITEMS
// keys, each sorted in LDS, and the sorted chunks are merged pairwise
// (merge path) through global memory, ping-ponging between the segment's
// emission buffer and its output key array; the last merge reads the
// emission buffer and writes the final pairs.
template <int WAVES, int ITEMS, bool CHUNKED>
__device__ void sort_segment(const SegArgs& a, uint32_t tile, uint2 rg, SegLds<WAVES, ITEMS>& L)
{
    constexpr int THREADS = WAVES * 64;
    constexpr int MAXR = ITEMS / THREADS;
    const int m = (int)(rg.y - rg.x);
    const int v = view_of_tile(a.views, (int)tile);
    const uint32_t vbase = (uint32_t)((int64_t)v * a.n);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    unsigned long long key[MAXR];

    if (m <= ITEMS) {
        lds_sort<WAVES, ITEMS>(a.seg + rg.x, m, key, L);
        const int R = (m + THREADS - 1) / THREADS;
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
            if (r >= R) break;
            const int li = w * R * 64 + r * 64 + lane;
            if (li < m) write_pair(a, rg.x + (uint32_t)li, key[r], tile, vbase);
        }
        return;
    }
    if (!CHUNKED) return;  // not reached: the class's lists fit in LDS

    unsigned long long* bufA = a.seg + rg.x;
    unsigned long long* bufB = a.keys + rg.x;  // output keys double as scratch
    const int chunks = (m + ITEMS - 1) / ITEMS;
    int passes = 0;
    while ((1 << passes) < chunks) ++passes;
    // the sorted chunks go where the last merge will read from bufA
    unsigned long long* cur = (passes & 1) ? bufA : bufB;
    for (int cb = 0; cb < m; cb += ITEMS) {
        const int cm = min(ITEMS, m - cb);
        lds_sort<WAVES, ITEMS>(bufA + cb, cm, key, L);
        const int R = (cm + THREADS - 1) / THREADS;
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
            if (r >= R) break;
            const int li = w * R * 64 + r * 64 + lane;
            if (li < cm) cur[cb + li] = key[r];
        }
        __syncthreads();
    }
    for (int p = 1, width = ITEMS; p <= passes; ++p, width *= 2) {
        unsigned long long* nxt = cur == bufA ? bufB : bufA;
        for (int a0 = 0; a0 < m; a0 += 2 * width) {
            const int na = min(width, m - a0);
            const int nb = max(0, min(width, m - a0 - width));
            if (p == passes)
                merge_runs<THREADS>(cur + a0, na, cur + a0 + na, nb, [&](int d, unsigned long long k) {
                    write_pair(a, rg.x + (uint32_t)(a0 + d), k, tile, vbase);
                });
            else
                merge_runs<THREADS>(cur + a0, na, cur + a0 + na, nb,
                                    [&](int d, unsigned long long k) { nxt[a0 + d] = k; });
        }
        __syncthreads();
        cur = nxt;
    }
}

// first position of the processing order whose tile has fewer than `below`
// pairs (the order is grouped by floor(log2(count)), longest first, and
// `below` is a power of two, so the predicate is monotone along it)
__device__ __forceinline__ int first_below(const SegArgs& a, int total_tiles, uint32_t below)
{
    int lo = 0, hi = total_tiles;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const uint2 r = a.ranges[a.order[mid]];
        if (r.y - r.x < below) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Three classes of segments, each a contiguous stretch of the processing
// order (longest first).  CLASS 2, lists of GSR_SEG_ITEMS keys or more, and
// CLASS 1, from GSR_SEG_SMALL_ITEMS up to GSR_SEG_ITEMS: block b takes
// position b and returns at once if that tile belongs to another class (the
// middle class's blocks retire tile by tile, which lets the long class's
// blocks in; persistent middle blocks measured slower where long lists are
// many).  CLASS 0, below GSR_SEG_SMALL_ITEMS: persistent 256-thread blocks
// take tiles from a work queue over their stretch (found by binary search),
// so no block is spent on another class's tile; the small blocks keep more
// short lists in flight per CU.
template <int THREADS, int ITEMS, int CLASS>
__global__ __launch_bounds__(THREADS) void k_seg_sort(SegArgs a, int total_tiles)
{
    __shared__ SegLds<THREADS / 64, ITEMS> L;
    if (a.counters->overflow) return;
    if (CLASS == 2) {
        const uint32_t tile = a.order[blockIdx.x];
        const uint2 rg = a.ranges[tile];
        if (rg.y - rg.x < (uint32_t)GSR_SEG_ITEMS) return;
        sort_segment<THREADS / 64, ITEMS, true>(a, tile, rg, L);
        return;
    }
    if (CLASS == 1) {
        const uint32_t tile = a.order[blockIdx.x];
        const uint2 rg = a.ranges[tile];
        const uint32_t m = rg.y - rg.x;
        if (m < (uint32_t)GSR_SEG_SMALL_ITEMS || m >= (uint32_t)GSR_SEG_ITEMS) return;
        sort_segment<THREADS / 64, ITEMS, false>(a, tile, rg, L);
        return;
    }
    const int begin = first_below(a, total_tiles, GSR_SEG_SMALL_ITEMS);
    const int end = total_tiles;
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = begin + (int)atomicAdd(&a.queue[CLASS], 1u);
        __syncthreads();
        const int p = next;
        __syncthreads();
        if (p >= end) break;
        const uint32_t tile = a.order[p];
        const uint2 rg = a.ranges[tile];
        if (rg.y == rg.x) break;  // empty tiles end the order
        sort_segment<THREADS / 64, ITEMS, false>(a, tile, rg, L);
    }
}

// The long segments run on `side`, forked from `s` after the tile ranges,
// followed there by the short ones; the middle class runs on `s`; `side` is
// joined back before anything later on `s` (the fork and join are recorded
// into a graph when `s` is captured).
hipError_t launch_seg_sort(const SegArgs& a, int total_tiles, int64_t capacity, hipStream_t s, hipStream_t side,
                           hipEvent_t fork, hipEvent_t join)
{
    if (total_tiles == 0) return hipSuccess;
    hipError_t e = hipEventRecord(fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    if (e != hipSuccess) return e;
    // the long segments lead the processing order, and at most
    // capacity / GSR_SEG_ITEMS of them fit in the pair buffer
    const int64_t longs = capacity / GSR_SEG_ITEMS + 1;
    const unsigned long_grid = (unsigned)(longs < total_tiles ? longs : total_tiles);
    hipLaunchKernelGGL((k_seg_sort<GSR_SEG_LONG_THREADS, GSR_SEG_LONG_ITEMS, 2>), dim3(long_grid),
                       dim3(GSR_SEG_LONG_THREADS), 0, side, a, total_tiles);
    // the small class: four persistent blocks per CU (what their registers
    // allow)
    const unsigned small_grid = (unsigned)(total_tiles < 1024 ? total_tiles : 1024);
    hipLaunchKernelGGL((k_seg_sort<GSR_SEG_SMALL_THREADS, GSR_SEG_SMALL_ITEMS, 0>), dim3(small_grid),
                       dim3(GSR_SEG_SMALL_THREADS), 0, side, a, total_tiles);
    hipLaunchKernelGGL((k_seg_sort<GSR_SEG_THREADS, GSR_SEG_ITEMS, 1>), dim3((unsigned)total_tiles),
                       dim3(GSR_SEG_THREADS), 0, s, a, total_tiles);
    // more persistent small-class blocks on `s` once the middle class is
    // done: they take tiles from the same queue as those on `side`, so the
    // stream that frees up first drains the short lists
    if (GSR_SORT_SMALL_MAIN > 0) {
        const unsigned g = (unsigned)(total_tiles < GSR_SORT_SMALL_MAIN ? total_tiles : GSR_SORT_SMALL_MAIN);
        hipLaunchKernelGGL((k_seg_sort<GSR_SEG_SMALL_THREADS, GSR_SEG_SMALL_ITEMS, 0>), dim3(g),
                           dim3(GSR_SEG_SMALL_THREADS), 0, s, a, total_tiles);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
    return e;
}

// ---------------------------------------------------------------------------
// processing order of the tiles: descending pair count, bucketed by
// floor(log2(count)) (bucket 0 holds the longest lists)

__device__ __forceinline__ uint32_t count_bucket(uint2 r)
{
    uint32_t c = r.y - r.x;
    return c == 0u ? 31u : (uint32_t)__clz(c);  // 31 - floor(log2 c)
}

__global__ void k_order_zero(RangeArgs a)
{
    if (threadIdx.x < 66) a.buckets[threadIdx.x] = 0u;
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

// places each tile at its bucket's base plus a block-aggregated cursor: one
// global atomic per (block, bucket)
__global__ void k_order_place(RangeArgs a)
{
    __shared__ uint32_t base[32], cnt[32], blk[32];
    if (threadIdx.x < 32) cnt[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int b = 0; b < 32; ++b) {
            base[b] = run;
            run += a.buckets[b];
        }
    }
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t b = 0, local = 0;
    if (t < a.total_tiles) {
        b = count_bucket(a.ranges[t]);
        local = atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 32) blk[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&a.buckets[32 + threadIdx.x], cnt[threadIdx.x]) : 0u;
    __syncthreads();
    if (t < a.total_tiles) a.order[base[b] + blk[b] + local] = (uint32_t)t;
}

hipError_t launch_order(const RangeArgs& a, hipStream_t s)
{
    if (a.total_tiles == 0) return hipSuccess;
    const int tb = (a.total_tiles + 255) / 256;
    hipLaunchKernelGGL(k_order_zero, dim3(1), dim3(128), 0, s, a);
    hipLaunchKernelGGL(k_order_count, dim3(tb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_order_place, dim3(tb), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
