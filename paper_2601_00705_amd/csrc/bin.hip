// bin.hip -- the depth-ordered sets N(p) of Eq. (alpha), grouped by tile.
//
// For every live slot the conservative tile rectangle (tile_rect) gives the
// candidate tiles; a candidate is kept when the slot's ellipse reaches the
// tile's pixel-centre box (tile_hit).  Each kept (tile, slot) pair goes into
// the tile's segment of the pair array as one 64-bit key
//   (float bits of the camera depth << 32) | Gaussian index,
// which orders a segment by depth and breaks ties by index (positive floats
// order like their bit patterns).  The tile is the most significant part of
// the order, so it is resolved by counting instead of sorting.  A chunk is
// chunk_mult * GSR_BIN_CHUNK consecutive entries of one view's list of live
// Gaussians (those whose rectangle is not empty), staged GSR_BIN_CHUNK at a
// time:
//
//   k_bin_list    per view, the list of live Gaussians from the projection's
//                 liveness ballots (a block scans its words' popcounts and
//                 reserves its places with one atomic on the view's counter,
//                 so the list's order is arbitrary; every later step is exact
//                 whatever the order)
//   k_bin_count   per chunk: pairs per tile of the view, one row of the
//                 view's [chunk][tile] count matrix (LDS histogram; views
//                 with more than GSR_BIN_LDS_TILES tiles add straight into
//                 the row)
//   k_bin_colscan per tile: exclusive prefix of its column (the chunk's offset
//                 inside the tile's segment) and the tile's total, four
//                 waves to a column
//   k_bin_tiles   the tile ranges from the column scan's per-block prefixes
//                 and block sums, the pair count and the capacity flag
//   k_bin_emit    the chunk's pairs, each at its tile's cursor (LDS atomics:
//                 the order inside a chunk's group is arbitrary, and the
//                 per-tile sort of the unique keys makes it exact)
//
// The grid of the count and emit kernels covers the most chunks a view can
// have (rounded up to a multiple of GSR_XCDS); blocks past a view's list exit
// at once.  The emit pass maps blocks to chunks so that each die takes one
// contiguous range of a view's chunks: the runs that consecutive chunks
// write into a tile's segment are adjacent, and a cache line filled by
// several chunks is then filled inside one die's L2 instead of being
// written back in pieces by several (measured: 3.5x the key bytes written
// to HBM with chunks dealt round-robin).  Candidates of a staged
// group are numbered by the prefix of the rectangle areas over the group's
// owners (its slots with a non-empty rectangle, compacted); each thread
// walks a contiguous run of them, its first owner found by binary search.
// The walk has no branch per candidate: every step reloads its owner's
// 48-byte record from LDS (three 16-byte reads, the same for every lane
// wherever a lane stands in its run) and advances tile, row and owner by
// selects, so that the lanes of a wave never diverge over owner or row
// changes.
#include "kernels.h"

#include <algorithm>

#ifndef GSR_EMIT_BATCH
#define GSR_EMIT_BATCH 4
#endif

namespace gsr {

static_assert(GSR_BIN_CHUNK == 256, "one staged slot per thread");

// A staged owner: ellipse, reciprocals and rectangle (origin, width,
// height; the height's sign bit marks an ellipse with a non-finite term,
// which takes tile_hit itself).
struct __align__(16) Owner {
    float u, v, A, B;
    float C, q, iA, iC;
    int x0, y0, w, h;
};

struct ChunkLds {
    uint32_t excl[GSR_BIN_CHUNK + 1];  // prefix of the owners' rectangle areas
    Owner own[GSR_BIN_CHUNK];
    uint2 key[GSR_BIN_CHUNK];          // (depth bits, Gaussian index)
    uint32_t wsum[4], wnz[4];
};

// The records of one staged group, fetched into registers (thread t owns
// entry t).  All fields are loaded at once, so that one memory round trip
// serves the group; the next group's fetch is issued before the current
// group is walked.
struct GroupRegs {
    float4 gm, co;
    float q;
    uint32_t dbits, idx;
    bool in;
};

// entries of view v's live list
__device__ __forceinline__ uint32_t live_len(const BinArgs& a, int v)
{
    const uint32_t c = a.live_count[v * GSR_LIVE_STRIDE];
    return c < (uint64_t)a.n ? c : (uint32_t)a.n;
}

__device__ __forceinline__ int view_chunks(const BinArgs& a, int v)
{
    const uint32_t per = (uint32_t)a.chunk_mult * GSR_BIN_CHUNK;
    return (int)((live_len(a, v) + per - 1u) / per);
}

// entries base .. of view v's live list (len entries)
__device__ __forceinline__ void fetch_group(const BinArgs& a, int v, int64_t base, uint32_t len, bool want_depth,
                                            GroupRegs& R)
{
    const int64_t j = base + threadIdx.x;
    R.in = j < (int64_t)len;
    if (R.in) {
        const uint32_t i = a.live[(int64_t)v * a.n + j];
        R.idx = i;
        const int64_t slot = (int64_t)v * a.n + i;
        R.gm = a.geom[slot];
        R.co = a.conic_o[slot];
        R.q = a.qthr[slot];
        R.dbits = want_depth ? __float_as_uint(a.rgb_d[slot].w) : 0u;
    }
}

struct Staged {
    uint32_t total;   // candidates
    int owners;       // slots with a non-empty rectangle
};

// Stages a fetched group: the owners' records, compacted, and the scan of
// their rectangle areas.  Starts and ends with a block barrier.
__device__ Staged stage_group(const BinArgs& a, const ViewInfo& vw, const GroupRegs& R, bool want_key, ChunkLds& L)
{
    const float inv_tw = 1.0f / (float)a.cfg.tile_w, inv_th = 1.0f / (float)a.cfg.tile_h;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    __syncthreads();
    int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
    const bool nz = R.in && tile_rect(R.gm.x, R.gm.y, R.gm.z, R.gm.w, inv_tw, inv_th, vw.tiles_x, vw.tiles_y, x0,
                                      y0, x1, y1);
    const uint32_t area = nz ? (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1)) : 0u;
    uint32_t ia = area, in_ = nz ? 1u : 0u;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t ya = __shfl_up(ia, off, 64), yn = __shfl_up(in_, off, 64);
        if (lane >= off) {
            ia += ya;
            in_ += yn;
        }
    }
    if (lane == 63) {
        L.wsum[w] = ia;
        L.wnz[w] = in_;
    }
    __syncthreads();
    uint32_t oa = 0, on = 0;
    for (int k = 0; k < w; ++k) {
        oa += L.wsum[k];
        on += L.wnz[k];
    }
    if (nz) {
        const uint32_t c = on + in_ - 1u;
        L.excl[c] = oa + ia - area;
        Owner o;
        o.u = R.gm.x;
        o.v = R.gm.y;
        o.A = R.co.x;
        o.B = R.co.y;
        o.C = R.co.z;
        o.q = R.q;
        o.iA = 1.0f / o.A;
        o.iC = 1.0f / o.C;
        const bool fast = __builtin_isfinite(o.A) && __builtin_isfinite(o.B) && __builtin_isfinite(o.C) &&
                          __builtin_isfinite(o.iA) && __builtin_isfinite(o.iC);
        o.x0 = x0;
        o.y0 = y0;
        o.w = x1 - x0 + 1;
        o.h = (y1 - y0 + 1) | (fast ? 0 : (int)0x80000000);
        L.own[c] = o;
        if (want_key) L.key[c] = make_uint2(R.dbits, R.idx);
    }
    Staged st;
    st.total = L.wsum[0] + L.wsum[1] + L.wsum[2] + L.wsum[3];
    st.owners = (int)(L.wnz[0] + L.wnz[1] + L.wnz[2] + L.wnz[3]);
    if (tid == 0) L.excl[st.owners] = st.total;
    __syncthreads();
    return st;
}

// tile_hit on a staged owner: the same float32 operations on the same
// operands, so the same decision, with 1/A and 1/C computed once per owner.
// Tile box corners come from exact values (float)(tx tw) + 0.5 (integers
// below 2^23 plus one half; the far corner adds tw - 1 exactly), the edge
// minimiser's clamp is a median of three and the minimum over the edges a
// float minimum: both equal tile_hit's comparisons when the clamped value
// is not NaN, which holds when A, B, C, 1/A, 1/C are finite (then
// -(B X) / C is a finite or infinite number, never NaN); a q that is NaN is
// skipped by both.  Owners with a non-finite term call tile_hit.
__device__ __forceinline__ bool owner_hit(const Owner& o, bool fast, int tx, int ty, int tw, int th)
{
    if (!fast) return tile_hit(o.u, o.v, o.A, o.B, o.C, o.iA, o.iC, o.q, tx, ty, tw, th);
    const float fx = (float)(tx * tw) + 0.5f, fy = (float)(ty * th) + 0.5f;
    const float x0 = fx - o.u, x1 = (fx + (float)(tw - 1)) - o.u;
    const float y0 = fy - o.v, y1 = (fy + (float)(th - 1)) - o.v;
    if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return true;
    const float B2 = 2.0f * o.B;
    float m = INFINITY;
    {
        const float ys = __builtin_amdgcn_fmed3f(-(o.B * x0) * o.iC, y0, y1);
        m = fminf(m, (o.A * x0) * x0 + (B2 * x0) * ys + (o.C * ys) * ys);
    }
    {
        const float ys = __builtin_amdgcn_fmed3f(-(o.B * x1) * o.iC, y0, y1);
        m = fminf(m, (o.A * x1) * x1 + (B2 * x1) * ys + (o.C * ys) * ys);
    }
    {
        const float xs = __builtin_amdgcn_fmed3f(-(o.B * y0) * o.iA, x0, x1);
        m = fminf(m, (o.A * xs) * xs + (B2 * xs) * y0 + (o.C * y0) * y0);
    }
    {
        const float xs = __builtin_amdgcn_fmed3f(-(o.B * y1) * o.iA, x0, x1);
        m = fminf(m, (o.A * xs) * xs + (B2 * xs) * y1 + (o.C * y1) * y1);
    }
    return m <= o.q;
}

// Walks this thread's contiguous run of the staged group's candidates,
// BATCH at a time: batch(tt, hit, key) gets, for each, the tile within the
// view, whether the tile test keeps it and (WANT_KEY) the owner's key.
template <int BATCH, bool WANT_KEY, class Batch>
__device__ __forceinline__ void walk_group(const ChunkLds& L, const Staged& st, const BinArgs& a, const ViewInfo& vw,
                                           Batch&& batch)
{
    const uint32_t per = (st.total + 255u) / 256u;
    uint32_t j = threadIdx.x * per;
    const uint32_t j1 = min(j + per, st.total);
    if (j >= j1) return;
    const int tw = a.cfg.tile_w, th = a.cfg.tile_h;
    // first owner: the largest s with excl[s] <= j
    int lo = 0, hi = st.owners - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.excl[mid] <= j) lo = mid; else hi = mid - 1;
    }
    int s = lo;
    const uint32_t r = j - L.excl[s];
    const uint32_t w0 = (uint32_t)L.own[s].w;
    int dx = (int)(r % w0), dy = (int)(r / w0);
    while (j < j1) {
        uint32_t tt[BATCH];
        bool hit[BATCH];
        uint2 key[BATCH];
#pragma unroll
        for (int e = 0; e < BATCH; ++e) {
            const bool valid = BATCH == 1 || j < j1;
            const int sl = BATCH == 1 ? s : min(s, st.owners - 1);
            const Owner o = L.own[sl];
            key[e] = WANT_KEY ? L.key[sl] : make_uint2(0u, 0u);
            const int h = o.h & 0x7fffffff;
            const int tx = o.x0 + dx, ty = o.y0 + dy;
            tt[e] = (uint32_t)(ty * vw.tiles_x + tx);
            hit[e] = valid && owner_hit(o, o.h >= 0, tx, ty, tw, th);
            // next candidate: along the row, then the next row, then the
            // next owner
            ++dx;
            const bool row_end = dx == o.w;
            dx = row_end ? 0 : dx;
            dy += row_end ? 1 : 0;
            const bool own_end = dy == h;
            dy = own_end ? 0 : dy;
            s += own_end ? 1 : 0;
            ++j;
        }
        batch(tt, hit, key);
    }
}

#define GSR_LIST_WORDS 2  // ballot words per thread of k_bin_list

__global__ __launch_bounds__(256) void k_bin_list(BinArgs a)
{
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t base_s;
    const int v = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t w0 = ((int64_t)blockIdx.x * 256 + tid) * GSR_LIST_WORDS;
    uint64_t m[GSR_LIST_WORDS];
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < GSR_LIST_WORDS; ++k) {
        const int64_t wd = w0 + k;
        m[k] = wd < a.mask_words ? a.live_mask[wd * a.n_views + v] : 0ull;
        // no Gaussian past n
        if (wd == a.mask_words - 1 && (a.n & 63)) m[k] &= (1ull << (a.n & 63)) - 1ull;
        cnt += (uint32_t)__popcll(m[k]);
    }
    uint32_t incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    if (tid == 0) {
        const uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base_s = total ? atomicAdd(&a.live_count[v * GSR_LIVE_STRIDE], total) : 0u;
    }
    __syncthreads();
    uint32_t pos = base_s + incl - cnt;
    for (int k = 0; k < w; ++k) pos += wsum[k];
    uint32_t* list = a.live + (int64_t)v * a.n;
    // the wave writes its words' entries together, one word at a time: lane
    // l keeps bit l of the word, so the set bits go out as one coalesced run
    // (in index order, as a thread would write them)
    const uint64_t below = (1ull << lane) - 1ull;
    for (int j = 0; j < 64; ++j) {
        uint32_t at = (uint32_t)__builtin_amdgcn_readlane((int)pos, j);
#pragma unroll
        for (int k = 0; k < GSR_LIST_WORDS; ++k) {
            const uint64_t word = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(m[k] >> 32), j) << 32) |
                                  (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)m[k], j);
            if (word == 0ull) continue;
            if ((word >> lane) & 1ull) {
                const int64_t wd = (int64_t)(blockIdx.x * 256 + w * 64 + j) * GSR_LIST_WORDS + k;
                list[at + (uint32_t)__popcll(word & below)] = (uint32_t)(wd * 64 + lane);
            }
            at += (uint32_t)__popcll(word);
        }
    }
}

// row of the count matrix of (view, chunk)
__device__ __forceinline__ uint32_t* count_row(const BinArgs& a, const ViewInfo& vw, int chunk)
{
    const int64_t tiles_v = (int64_t)vw.tiles_x * vw.tiles_y;
    return a.cnt + (int64_t)a.chunks * vw.tile_base + (int64_t)chunk * tiles_v;
}

template <bool LDS_HIST>
__global__ __launch_bounds__(256) void k_bin_count(BinArgs a)
{
    HIP_DYNAMIC_SHARED(uint32_t, hist)  // [tiles of the view] when LDS_HIST
    __shared__ ChunkLds L;
    const int v = blockIdx.y;
    if ((int)blockIdx.x >= view_chunks(a, v)) return;
    const uint32_t len = live_len(a, v);
    const ViewInfo vw = a.views->v[v];
    const int tiles_v = vw.tiles_x * vw.tiles_y;
    uint32_t* row = count_row(a, vw, blockIdx.x);
    if (LDS_HIST)
        for (int t = threadIdx.x; t < tiles_v; t += 256) hist[t] = 0u;
    GroupRegs cur, nxt;
    int64_t base = (int64_t)blockIdx.x * a.chunk_mult * GSR_BIN_CHUNK;
    fetch_group(a, v, base, len, false, nxt);
    for (int sub = 0; sub < a.chunk_mult; ++sub, base += GSR_BIN_CHUNK) {
        if (base >= (int64_t)len) break;
        cur = nxt;
        if (sub + 1 < a.chunk_mult) fetch_group(a, v, base + GSR_BIN_CHUNK, len, false, nxt);
        const Staged st = stage_group(a, vw, cur, false, L);
        walk_group<1, false>(L, st, a, vw, [&](const uint32_t(&tt)[1], const bool(&hit)[1], const uint2(&)[1]) {
            // a miss adds 0: no branch
            if (LDS_HIST) atomicAdd(&hist[tt[0]], hit[0] ? 1u : 0u);
            else if (hit[0]) atomicAdd(&row[tt[0]], 1u);
        });
    }
    if (LDS_HIST) {
        __syncthreads();
        for (int t = threadIdx.x; t < tiles_v; t += 256) row[t] = hist[t];
    }
}

__global__ void k_zero_u32(uint32_t* p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Column scan: a block takes 64 consecutive global tiles; its wave s takes
// the s-th quarter of every tile's chunks (so a wave reads 64 adjacent
// counters of one row at a time).  Each wave sums its quarter of the
// column, the quarters' sums give each quarter its offset, and the wave
// rewrites its quarter as the exclusive prefix over chunks; the column's
// total goes to ranges[].y.  32 loads are in flight at a time.
__device__ __forceinline__ uint32_t colscan_run(uint32_t* col, int64_t stride, int c0, int c1, bool write,
                                                uint32_t run)
{
    constexpr int K = 32;
    int c = c0;
    for (; c + K <= c1; c += K) {
        uint32_t x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = col[(int64_t)(c + k) * stride];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (write) col[(int64_t)(c + k) * stride] = run;
            run += x[k];
        }
    }
    for (; c < c1; ++c) {
        const uint32_t x = col[(int64_t)c * stride];
        if (write) col[(int64_t)c * stride] = run;
        run += x;
    }
    return run;
}

__global__ __launch_bounds__(256) void k_bin_colscan(BinArgs a)
{
    __shared__ uint32_t part[4][64];
    const int lt = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int g = blockIdx.x * 64 + lt;
    const bool in = g < a.total_tiles;
    uint32_t* col = nullptr;
    int64_t stride = 0;
    int c0 = 0, c1 = 0;
    if (in) {
        const int v = view_of_tile(a.views, g);
        const ViewInfo& vw = a.views->v[v];
        stride = (int64_t)vw.tiles_x * vw.tiles_y;
        col = a.cnt + (int64_t)a.chunks * vw.tile_base + (g - vw.tile_base);
        const int chunks_v = view_chunks(a, v);
        const int per = (chunks_v + 3) / 4;
        c0 = min(q * per, chunks_v);
        c1 = min(c0 + per, chunks_v);
    }
    const uint32_t sum = in ? colscan_run(col, stride, c0, c1, false, 0u) : 0u;
    part[q][lt] = sum;
    __syncthreads();
    uint32_t off = 0u;
    for (int k = 0; k < q; ++k) off += part[k][lt];
    if (in) colscan_run(col, stride, c0, c1, true, off);
    if (q == 3) {
        // the last wave holds the 64 tiles' totals: their exclusive prefix
        // within the block goes to ranges[].x, the block's pairs to
        // tile_blocks (k_bin_tiles adds the earlier blocks')
        const uint32_t total = off + sum;
        unsigned long long incl = total;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl_up(incl, o, 64);
            if (lt >= o) incl += y;
        }
        if (in) a.ranges[g] = make_uint2((uint32_t)(incl - total), total);
        if (lt == 63) a.tile_blocks[blockIdx.x] = incl;
    }
}

// the tile ranges: each tile's start is the pairs of the earlier 64-tile
// blocks plus its prefix within its block; the pair count and the capacity
// flag come from the blocks' sum (every block forms it, so that all decide
// the overflow alike)
__global__ __launch_bounds__(256) void k_bin_tiles(BinArgs a)
{
    __shared__ unsigned long long red[2][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nb = (a.total_tiles + 63) / 64;
    const int b0 = (int)blockIdx.x * 4;
    unsigned long long pre = 0ull, tot = 0ull;
    for (int k = tid; k < nb; k += 256) {
        const unsigned long long x = a.tile_blocks[k];
        tot += x;
        if (k < b0) pre += x;
    }
    for (int o = 32; o > 0; o >>= 1) {
        pre += __shfl_xor(pre, o, 64);
        tot += __shfl_xor(tot, o, 64);
    }
    if (lane == 0) {
        red[0][w] = pre;
        red[1][w] = tot;
    }
    __syncthreads();
    pre = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    tot = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const bool over = tot > a.counters->capacity;
    const int g = (int)blockIdx.x * 256 + tid;
    if (g < a.total_tiles) {
        for (int k = b0; k < b0 + w; ++k) pre += a.tile_blocks[k];
        const uint2 r = a.ranges[g];
        const unsigned long long start = pre + r.x;
        // empty tiles get [0, 0); on overflow every range is empty, so that
        // no kernel reads past the capacity
        a.ranges[g] = (over || r.y == 0u) ? make_uint2(0u, 0u)
                                          : make_uint2((uint32_t)start, (uint32_t)(start + r.y));
    }
    if (blockIdx.x == 0 && tid == 0) {
        a.counters->pairs = tot;
        a.counters->overflow = over ? 1u : 0u;
    }
}

template <bool LDS_HIST>
__global__ __launch_bounds__(256) void k_bin_emit(BinArgs a)
{
    HIP_DYNAMIC_SHARED(uint32_t, cursor)  // [tiles of the view] when LDS_HIST
    __shared__ ChunkLds L;
    if (a.counters->overflow) return;
    const int v = blockIdx.y;
    // block x runs on die x % GSR_XCDS (the grid's width is a multiple of
    // GSR_XCDS); die k takes chunks [k per, (k + 1) per)
    const int nc = view_chunks(a, v);
    const int per = (nc + GSR_XCDS - 1) / GSR_XCDS;
    const int chunk = (int)(blockIdx.x % GSR_XCDS) * per + (int)(blockIdx.x / GSR_XCDS);
    if ((int)(blockIdx.x / GSR_XCDS) >= per || chunk >= nc) return;
    const uint32_t len = live_len(a, v);
    const ViewInfo vw = a.views->v[v];
    const int tiles_v = vw.tiles_x * vw.tiles_y;
    uint32_t* row = count_row(a, vw, chunk);
    const uint2* rng = a.ranges + vw.tile_base;
    if (LDS_HIST)
        for (int t = threadIdx.x; t < tiles_v; t += 256) cursor[t] = rng[t].x + row[t];
    GroupRegs cur, nxt;
    int64_t base = (int64_t)chunk * a.chunk_mult * GSR_BIN_CHUNK;
    fetch_group(a, v, base, len, true, nxt);
    for (int sub = 0; sub < a.chunk_mult; ++sub, base += GSR_BIN_CHUNK) {
        if (base >= (int64_t)len) break;
        cur = nxt;
        if (sub + 1 < a.chunk_mult) fetch_group(a, v, base + GSR_BIN_CHUNK, len, true, nxt);
        const Staged st = stage_group(a, vw, cur, true, L);
        walk_group<GSR_EMIT_BATCH, true>(L, st, a, vw, [&](const uint32_t(&tt)[GSR_EMIT_BATCH],
                                                           const bool(&hit)[GSR_EMIT_BATCH],
                                                           const uint2(&key)[GSR_EMIT_BATCH]) {
            uint32_t pos[GSR_EMIT_BATCH];
            if (LDS_HIST) {
                // a miss adds 0 (its result is unused), so that the atomics
                // issue back to back and one wait covers them
#pragma unroll
                for (int e = 0; e < GSR_EMIT_BATCH; ++e) pos[e] = atomicAdd(&cursor[tt[e]], hit[e] ? 1u : 0u);
            } else {
#pragma unroll
                for (int e = 0; e < GSR_EMIT_BATCH; ++e)
                    pos[e] = hit[e] ? rng[tt[e]].x + atomicAdd(&row[tt[e]], 1u) : 0u;
            }
#pragma unroll
            for (int e = 0; e < GSR_EMIT_BATCH; ++e)
                if (hit[e]) a.seg[pos[e]] = ((unsigned long long)key[e].x << 32) | key[e].y;
        });
    }
}

hipError_t launch_bin(const BinArgs& a, int max_tiles_view, hipStream_t s)
{
    if (a.total_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(16), dim3(256), 0, s, a.live_count, (int64_t)GSR_LIVE_STRIDE * GSR_MAX_VIEWS);
    const int64_t per_block = 256 * GSR_LIST_WORDS;
    hipLaunchKernelGGL(k_bin_list,
                       dim3((unsigned)std::max<int64_t>((a.mask_words + per_block - 1) / per_block, 1),
                            (unsigned)a.n_views),
                       dim3(256), 0, s, a);
    dim3 grid((unsigned)((a.chunks + GSR_XCDS - 1) / GSR_XCDS * GSR_XCDS), (unsigned)a.n_views);
    const bool lds = max_tiles_view <= GSR_BIN_LDS_TILES;
    const size_t dyn = lds ? sizeof(uint32_t) * (size_t)max_tiles_view : 0;
    if (lds) {
        hipLaunchKernelGGL(k_bin_count<true>, grid, dim3(256), dyn, s, a);
    } else {
        const int64_t entries = (int64_t)a.chunks * a.total_tiles;
        hipLaunchKernelGGL(k_zero_u32, dim3(2048), dim3(256), 0, s, a.cnt, entries);
        hipLaunchKernelGGL(k_bin_count<false>, grid, dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_bin_colscan, dim3((unsigned)((a.total_tiles + 63) / 64)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bin_tiles, dim3((unsigned)((a.total_tiles + 255) / 256)), dim3(256), 0, s, a);
    if (lds) hipLaunchKernelGGL(k_bin_emit<true>, grid, dim3(256), dyn, s, a);
    else hipLaunchKernelGGL(k_bin_emit<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
