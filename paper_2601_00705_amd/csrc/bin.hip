// bin.hip -- the depth-ordered sets N(p) of Eq. (alpha), grouped by tile.
//
// For every live slot the conservative tile rectangle (tile_rect) gives the
// candidate tiles; a candidate is kept when the slot's ellipse reaches the
// tile's pixel-centre box (tile_hit).  Each kept (tile, slot) pair goes into
// the tile's segment of the pair array as one 64-bit key
//   (float bits of the camera depth << 32) | Gaussian index,
// which orders a segment by depth and breaks ties by index (positive floats
// order like their bit patterns).  The tile is the most significant part of
// the order, so it is resolved by counting instead of sorting:
//
//   k_bin_count   per chunk of one view (chunk_mult * GSR_BIN_CHUNK Gaussians):
//                 pairs per tile of the view, one row of the view's
//                 [chunk][tile] count matrix (LDS histogram; views with more
//                 than GSR_BIN_LDS_TILES tiles add straight into the row)
//   k_bin_colscan per tile: exclusive prefix of its column (the chunk's offset
//                 inside the tile's segment) and the tile's total
//   k_bin_tiles   exclusive scan of the tile totals: the tile ranges, the pair
//                 count and the capacity flag
//   k_bin_emit    the chunk's pairs, each at its tile's cursor (LDS atomics:
//                 the order inside a chunk's group is arbitrary, and the
//                 per-tile sort of the unique keys makes it exact)
//
// Candidates of a staged group of Gaussians are expanded cooperatively: each
// thread walks a contiguous run of them, its first owner found by binary
// search over the rectangle-area prefix.
#include "kernels.h"

namespace gsr {

struct ChunkLds {
    uint32_t excl[GSR_BIN_CHUNK + 1];  // prefix of rectangle areas
    int rx0[GSR_BIN_CHUNK], ry0[GSR_BIN_CHUNK], rw[GSR_BIN_CHUNK];
    float u[GSR_BIN_CHUNK], v[GSR_BIN_CHUNK], A[GSR_BIN_CHUNK], B[GSR_BIN_CHUNK], C[GSR_BIN_CHUNK];
    float q[GSR_BIN_CHUNK];
    uint32_t dbits[GSR_BIN_CHUNK];
    uint32_t wsum[4];
};

// The records of one staged group, fetched into registers (thread t owns
// items IPT t .. IPT t + IPT - 1).  All fields are loaded at once, live or
// not, so that one memory round trip serves the group; the next group's
// fetch is issued before the current group is expanded.
constexpr int IPT = GSR_BIN_CHUNK / 256;

struct ChunkRegs {
    float4 gm[IPT], co[IPT];
    float q[IPT];
    uint32_t dbits[IPT];
    bool in[IPT];
};

__device__ __forceinline__ void fetch_chunk(const BinArgs& a, int v, int64_t base, bool want_depth, ChunkRegs& R)
{
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int64_t i = base + threadIdx.x * IPT + k;
        R.in[k] = i < a.n;
        if (R.in[k]) {
            const int64_t slot = (int64_t)v * a.n + i;
            R.gm[k] = a.geom[slot];
            R.co[k] = a.conic_o[slot];
            R.q[k] = a.qthr[slot];
            R.dbits[k] = want_depth ? __float_as_uint(a.rgb_d[slot].w) : 0u;
        }
    }
}

// Stages a fetched group: rectangles, ellipse data and the scan of the
// rectangle areas.  Returns the total area.  Starts and ends with a block
// barrier.
__device__ uint32_t stage_chunk(const BinArgs& a, const ViewInfo& vw, const ChunkRegs& R, ChunkLds& L)
{
    const float inv_tw = 1.0f / (float)a.cfg.tile_w, inv_th = 1.0f / (float)a.cfg.tile_h;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    __syncthreads();
    uint32_t area[IPT], tsum = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int li = tid * IPT + k;
        area[k] = 0;
        int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
        if (R.in[k] && tile_rect(R.gm[k].x, R.gm[k].y, R.gm[k].z, R.gm[k].w, inv_tw, inv_th, vw.tiles_x,
                                 vw.tiles_y, x0, y0, x1, y1)) {
            area[k] = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
            L.u[li] = R.gm[k].x;
            L.v[li] = R.gm[k].y;
            L.A[li] = R.co[k].x;
            L.B[li] = R.co[k].y;
            L.C[li] = R.co[k].z;
            L.q[li] = R.q[k];
            L.dbits[li] = R.dbits[k];
        }
        L.rx0[li] = x0;
        L.ry0[li] = y0;
        L.rw[li] = x1 - x0 + 1;
        tsum += area[k];
    }
    uint32_t incl = tsum;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) L.wsum[w] = incl;
    __syncthreads();
    uint32_t wofs = 0;
    for (int k = 0; k < w; ++k) wofs += L.wsum[k];
    uint32_t run = wofs + incl - tsum;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        L.excl[tid * IPT + k] = run;
        run += area[k];
    }
    const uint32_t total = L.wsum[0] + L.wsum[1] + L.wsum[2] + L.wsum[3];
    if (tid == 0) L.excl[GSR_BIN_CHUNK] = total;
    __syncthreads();
    return total;
}

// Walks the staged group's candidates: thread t takes the contiguous run
// [t per, (t + 1) per) of them, finds the run's first owner (largest s with
// excl[s] <= j) by one binary search, then advances tile by tile along the
// owner's rectangle and owner by owner, with no search or division per
// candidate and the owner's ellipse (with 1/A and 1/C) held in registers.  hit(s, tx, ty) is
// called for every candidate the tile test keeps.
template <class Hit>
__device__ __forceinline__ void walk_candidates(const ChunkLds& L, uint32_t total, const BinArgs& a, Hit&& hit)
{
    const uint32_t per = (total + 255u) / 256u;
    uint32_t j = threadIdx.x * per;
    const uint32_t j1 = min(j + per, total);
    if (j >= j1) return;
    int lo = 0, hi = GSR_BIN_CHUNK - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.excl[mid] <= j) lo = mid; else hi = mid - 1;
    }
    int s = lo;
    // candidates left in s's rectangle (at least 1: excl[s + 1] > j)
    uint32_t left = L.excl[s + 1] - j;
    const uint32_t r = j - L.excl[s];
    int w = L.rw[s];
    int dx = (int)(r % (uint32_t)w), dy = (int)(r / (uint32_t)w);
    float u = L.u[s], v = L.v[s], A = L.A[s], B = L.B[s], C = L.C[s], q = L.q[s];
    float iA = 1.0f / A, iC = 1.0f / C;
    int x0 = L.rx0[s], y0 = L.ry0[s];
    for (; j < j1; ++j) {
        if (left == 0u) {
            // the next owner with a non-empty rectangle (one exists: j < total)
            do {
                ++s;
                left = L.excl[s + 1] - L.excl[s];
            } while (left == 0u);
            w = L.rw[s];
            dx = dy = 0;
            u = L.u[s];
            v = L.v[s];
            A = L.A[s];
            B = L.B[s];
            C = L.C[s];
            q = L.q[s];
            iA = 1.0f / A;
            iC = 1.0f / C;
            x0 = L.rx0[s];
            y0 = L.ry0[s];
        }
        const int tx = x0 + dx, ty = y0 + dy;
        if (tile_hit(u, v, A, B, C, iA, iC, q, tx, ty, a.cfg.tile_w, a.cfg.tile_h)) hit(s, tx, ty);
        --left;
        if (++dx == w) {
            dx = 0;
            ++dy;
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
    const ViewInfo vw = a.views->v[v];
    const int tiles_v = vw.tiles_x * vw.tiles_y;
    uint32_t* row = count_row(a, vw, blockIdx.x);
    if (LDS_HIST)
        for (int t = threadIdx.x; t < tiles_v; t += 256) hist[t] = 0u;
    ChunkRegs cur, nxt;
    int64_t base = (int64_t)blockIdx.x * a.chunk_mult * GSR_BIN_CHUNK;
    fetch_chunk(a, v, base, false, nxt);
    for (int sub = 0; sub < a.chunk_mult; ++sub, base += GSR_BIN_CHUNK) {
        if (base >= a.n) break;
        cur = nxt;
        if (sub + 1 < a.chunk_mult) fetch_chunk(a, v, base + GSR_BIN_CHUNK, false, nxt);
        const uint32_t total = stage_chunk(a, vw, cur, L);
        walk_candidates(L, total, a, [&](int, int tx, int ty) {
            const int tt = ty * vw.tiles_x + tx;
            if (LDS_HIST) atomicAdd(&hist[tt], 1u);
            else atomicAdd(&row[tt], 1u);
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

// thread per global tile: the column of the tile in its view's count matrix
// becomes the exclusive prefix over chunks; the total goes to ranges[].y
__global__ __launch_bounds__(256) void k_bin_colscan(BinArgs a)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.total_tiles) return;
    const int v = view_of_tile(a.views, g);
    const ViewInfo& vw = a.views->v[v];
    const int64_t tiles_v = (int64_t)vw.tiles_x * vw.tiles_y;
    uint32_t* col = a.cnt + (int64_t)a.chunks * vw.tile_base + (g - vw.tile_base);
    uint32_t run = 0;
    int c = 0;
    for (; c + 8 <= a.chunks; c += 8) {
        uint32_t x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = col[(int64_t)(c + k) * tiles_v];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            col[(int64_t)(c + k) * tiles_v] = run;
            run += x[k];
        }
    }
    for (; c < a.chunks; ++c) {
        const uint32_t x = col[(int64_t)c * tiles_v];
        col[(int64_t)c * tiles_v] = run;
        run += x;
    }
    a.ranges[g] = make_uint2(0u, run);
}

// one block: exclusive scan of the tile totals into the ranges; pair count
// and capacity flag
__global__ __launch_bounds__(1024) void k_bin_tiles(BinArgs a)
{
    __shared__ unsigned long long part[1024];
    const int nt = a.total_tiles;
    const int per = (nt + 1023) / 1024;
    const int lo = threadIdx.x * per;
    unsigned long long s = 0;
    for (int k = 0; k < per && lo + k < nt; ++k) s += a.ranges[lo + k].y;
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned long long x = threadIdx.x >= off ? part[threadIdx.x - off] : 0ull;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned long long run = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
    const unsigned long long total = part[1023];
    const bool over = total > a.counters->capacity;
    for (int k = 0; k < per && lo + k < nt; ++k) {
        const uint32_t c = a.ranges[lo + k].y;
        // empty tiles get [0, 0); on overflow every range is empty, so that
        // no kernel reads past the capacity
        a.ranges[lo + k] = (over || c == 0u) ? make_uint2(0u, 0u) : make_uint2((uint32_t)run, (uint32_t)(run + c));
        run += c;
    }
    if (threadIdx.x == 1023) {
        a.counters->pairs = total;
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
    const ViewInfo vw = a.views->v[v];
    const int tiles_v = vw.tiles_x * vw.tiles_y;
    uint32_t* row = count_row(a, vw, blockIdx.x);
    const uint2* rng = a.ranges + vw.tile_base;
    if (LDS_HIST)
        for (int t = threadIdx.x; t < tiles_v; t += 256) cursor[t] = rng[t].x + row[t];
    ChunkRegs cur, nxt;
    int64_t base = (int64_t)blockIdx.x * a.chunk_mult * GSR_BIN_CHUNK;
    fetch_chunk(a, v, base, true, nxt);
    for (int sub = 0; sub < a.chunk_mult; ++sub, base += GSR_BIN_CHUNK) {
        if (base >= a.n) break;
        cur = nxt;
        if (sub + 1 < a.chunk_mult) fetch_chunk(a, v, base + GSR_BIN_CHUNK, true, nxt);
        const uint32_t total = stage_chunk(a, vw, cur, L);
        walk_candidates(L, total, a, [&](int s, int tx, int ty) {
            const int tt = ty * vw.tiles_x + tx;
            const uint32_t pos = LDS_HIST ? atomicAdd(&cursor[tt], 1u) : rng[tt].x + atomicAdd(&row[tt], 1u);
            a.seg[pos] = ((unsigned long long)L.dbits[s] << 32) | (unsigned long long)(base + s);
        });
    }
}

hipError_t launch_bin(const BinArgs& a, int max_tiles_view, hipStream_t s)
{
    if (a.total_tiles == 0) return hipSuccess;
    dim3 grid((unsigned)a.chunks, (unsigned)a.n_views);
    const bool lds = max_tiles_view <= GSR_BIN_LDS_TILES;
    const size_t dyn = lds ? sizeof(uint32_t) * (size_t)max_tiles_view : 0;
    if (lds) {
        hipLaunchKernelGGL(k_bin_count<true>, grid, dim3(256), dyn, s, a);
    } else {
        const int64_t entries = (int64_t)a.chunks * a.total_tiles;
        hipLaunchKernelGGL(k_zero_u32, dim3(2048), dim3(256), 0, s, a.cnt, entries);
        hipLaunchKernelGGL(k_bin_count<false>, grid, dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_bin_colscan, dim3((unsigned)((a.total_tiles + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bin_tiles, dim3(1), dim3(1024), 0, s, a);
    if (lds) hipLaunchKernelGGL(k_bin_emit<true>, grid, dim3(256), dyn, s, a);
    else hipLaunchKernelGGL(k_bin_emit<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
