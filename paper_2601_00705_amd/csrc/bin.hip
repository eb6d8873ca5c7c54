// bin.hip -- pair emission for the depth-ordered sets N(p) of Eq. (alpha).
//
// For every live slot the conservative tile rectangle (tile_rect) gives the
// candidate tiles; a candidate is kept when the slot's ellipse reaches the
// tile's pixel-centre box (tile_hit).  Each kept tile yields one
// (key, value) pair: key = (global tile << 32) | float bits of the camera
// depth (positive floats order like their bit patterns), value = slot.
// Emission is in slot order, rectangle tiles row by row, so that a stable
// sort breaks depth ties by slot, i.e. by Gaussian index.
//
//   k_bin_count : per chunk of BIN_CHUNK Gaussians of one view, the number of
//                 kept tiles (the chunk's rectangles are expanded
//                 cooperatively: one candidate per thread and step, owner
//                 found by binary search over the rectangle-area prefix)
//   k_bin_scan  : exclusive scan of the chunk counts, total, capacity check
//   k_bin_emit  : the same expansion; kept candidates are compacted in order
//                 (wave ballots + a block prefix) so that stores are coalesced
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

// Loads the chunk's slots (thread t owns chunk items 4t .. 4t+3, which keeps
// slot order), their rectangles and ellipse data, and scans the areas.
// Returns the chunk's total rectangle area.
__device__ uint32_t load_chunk(const BinArgs& a, const ViewInfo& vw, int v, int64_t base, bool want_depth,
                               ChunkLds& L)
{
    const float inv_tw = 1.0f / (float)a.cfg.tile_w, inv_th = 1.0f / (float)a.cfg.tile_h;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t area[4], tsum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int li = tid * 4 + k;
        const int64_t i = base + li;
        area[k] = 0;
        int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
        if (i < a.n) {
            const int64_t slot = (int64_t)v * a.n + i;
            const float4 gm = a.geom[slot];
            if (tile_rect(gm.x, gm.y, gm.z, gm.w, inv_tw, inv_th, vw.tiles_x, vw.tiles_y, x0, y0, x1, y1)) {
                area[k] = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
                const float4 co = a.conic_o[slot];
                L.u[li] = gm.x;
                L.v[li] = gm.y;
                L.A[li] = co.x;
                L.B[li] = co.y;
                L.C[li] = co.z;
                L.q[li] = a.qthr[slot];
                if (want_depth) L.dbits[li] = __float_as_uint(a.rgb_d[slot].w);
            }
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
    for (int k = 0; k < 4; ++k) {
        L.excl[tid * 4 + k] = run;
        run += area[k];
    }
    const uint32_t total = L.wsum[0] + L.wsum[1] + L.wsum[2] + L.wsum[3];
    if (tid == 0) L.excl[GSR_BIN_CHUNK] = total;
    __syncthreads();
    return total;
}

// candidate j of the chunk: owner slot (largest s with excl[s] <= j) and tile
__device__ __forceinline__ bool candidate(const ChunkLds& L, uint32_t j, const BinArgs& a, int& s, int& tx,
                                          int& ty)
{
    int lo = 0, hi = GSR_BIN_CHUNK - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.excl[mid] <= j) lo = mid; else hi = mid - 1;
    }
    s = lo;
    const uint32_t r = j - L.excl[lo];
    const uint32_t wdt = (uint32_t)L.rw[lo];
    ty = L.ry0[lo] + (int)(r / wdt);
    tx = L.rx0[lo] + (int)(r % wdt);
    return tile_hit(L.u[lo], L.v[lo], L.A[lo], L.B[lo], L.C[lo], L.q[lo], tx, ty, a.cfg.tile_w, a.cfg.tile_h);
}

__global__ __launch_bounds__(256) void k_bin_count(BinArgs a)
{
    __shared__ ChunkLds L;
    __shared__ uint32_t red[4];
    const int v = blockIdx.y;
    const ViewInfo vw = a.views->v[v];
    const int64_t base = (int64_t)blockIdx.x * GSR_BIN_CHUNK;
    const uint32_t total = load_chunk(a, vw, v, base, false, L);
    uint32_t c = 0;
    for (uint32_t j = threadIdx.x; j < total; j += 256) {
        int s, tx, ty;
        c += candidate(L, j, a, s, tx, ty) ? 1u : 0u;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) a.block_sums[v * a.chunks + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(1024) void k_bin_scan(BinArgs a)
{
    __shared__ unsigned long long part[1024];
    const int nb = a.n_views * a.chunks;
    const int per = (nb + 1023) / 1024;
    const int lo = threadIdx.x * per;
    unsigned long long s = 0;
    for (int k = 0; k < per && lo + k < nb; ++k) s += a.block_sums[lo + k];
    part[threadIdx.x] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan of the 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned long long x = threadIdx.x >= off ? part[threadIdx.x - off] : 0ull;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned long long run = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
    for (int k = 0; k < per && lo + k < nb; ++k) {
        a.block_offs[lo + k] = run;
        run += a.block_sums[lo + k];
    }
    if (threadIdx.x == 1023) {
        unsigned long long total = part[1023];
        a.counters->pairs = total;
        a.counters->overflow = total > a.counters->capacity ? 1u : 0u;
    }
}

__global__ __launch_bounds__(256) void k_bin_emit(BinArgs a)
{
    __shared__ ChunkLds L;
    __shared__ uint32_t wcount[4];
    if (a.counters->overflow) return;
    const int v = blockIdx.y;
    const ViewInfo vw = a.views->v[v];
    const int64_t base = (int64_t)blockIdx.x * GSR_BIN_CHUNK;
    const uint32_t total = load_chunk(a, vw, v, base, true, L);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    unsigned long long out = a.block_offs[v * a.chunks + blockIdx.x];
    for (uint32_t j0 = 0; j0 < total; j0 += 256) {
        const uint32_t j = j0 + tid;
        int s = 0, tx = 0, ty = 0;
        const bool hit = j < total && candidate(L, j, a, s, tx, ty);
        const unsigned long long m = __ballot(hit);
        if (lane == 0) wcount[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0;
        for (int k = 0; k < w; ++k) before += wcount[k];
        if (hit) {
            const unsigned long long pos = out + before + (uint32_t)__popcll(m & lt);
            const unsigned long long tile = (unsigned long long)(vw.tile_base + ty * vw.tiles_x + tx);
            a.keys[pos] = (tile << 32) | L.dbits[s];
            a.vals[pos] = (uint32_t)((int64_t)v * a.n + base + s);
        }
        out += wcount[0] + wcount[1] + wcount[2] + wcount[3];
        __syncthreads();
    }
}

hipError_t launch_bin(const BinArgs& a, hipStream_t s)
{
    dim3 grid((unsigned)a.chunks, (unsigned)a.n_views);
    hipLaunchKernelGGL(k_bin_count, grid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_bin_emit, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
