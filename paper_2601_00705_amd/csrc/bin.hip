// bin.hip -- pair emission for the depth-ordered sets N(p) of Eq. (alpha).
//
// For every live slot the conservative tile rectangle (tile_rect, the
// binning contract) is expanded into one (key, value) pair per covered tile:
// key = (global tile << 32) | float bits of the camera depth (positive floats
// order like their bit patterns), value = slot.  Emission is in slot order so
// that a stable sort breaks depth ties by slot, i.e. by Gaussian index.
//
//   k_bin_count : per chunk of BIN_CHUNK Gaussians of one view, the pair count
//   k_bin_scan  : exclusive scan of the chunk counts, total, capacity check
//   k_bin_emit  : per chunk, a block scan of per-slot counts, then a
//                 cooperative expansion (one output pair per thread and step,
//                 owner found by binary search) so that stores are coalesced.
#include "kernels.h"

namespace gsr {

struct SlotRect {
    int x0, y0, w, h;
};

__device__ __forceinline__ uint32_t slot_count(const BinArgs& a, const ViewInfo& vw, int64_t i,
                                               int v, SlotRect& r, float inv_tw, float inv_th)
{
    if (i >= a.n) return 0;
    float4 gm = a.geom[(int64_t)v * a.n + i];
    int x0, y0, x1, y1;
    if (!tile_rect(gm.x, gm.y, gm.z, gm.w, inv_tw, inv_th, vw.tiles_x, vw.tiles_y, x0, y0, x1, y1))
        return 0;
    r.x0 = x0;
    r.y0 = y0;
    r.w = x1 - x0 + 1;
    r.h = y1 - y0 + 1;
    return (uint32_t)(r.w * r.h);
}

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t x, uint32_t* red)
{
    // 256 threads = 4 waves
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[w] = x;
    __syncthreads();
    uint32_t t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void k_bin_count(BinArgs a)
{
    __shared__ uint32_t red[4];
    const int v = blockIdx.y;
    const ViewInfo vw = a.views->v[v];
    const float inv_tw = 1.0f / (float)a.cfg.tile_w, inv_th = 1.0f / (float)a.cfg.tile_h;
    int64_t base = (int64_t)blockIdx.x * GSR_BIN_CHUNK;
    uint32_t c = 0;
    for (int k = 0; k < GSR_BIN_CHUNK / 256; ++k) {
        SlotRect r;
        c += slot_count(a, vw, base + k * 256 + threadIdx.x, v, r, inv_tw, inv_th);
    }
    uint32_t t = block_sum_u32(c, red);
    if (threadIdx.x == 0) a.block_sums[v * a.chunks + blockIdx.x] = t;
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
    __shared__ uint32_t excl[GSR_BIN_CHUNK + 1];
    __shared__ int rx0[GSR_BIN_CHUNK], ry0[GSR_BIN_CHUNK], rw[GSR_BIN_CHUNK];
    __shared__ uint32_t dbits[GSR_BIN_CHUNK];
    __shared__ uint32_t wsum[4];
    if (a.counters->overflow) return;
    const int v = blockIdx.y;
    const ViewInfo vw = a.views->v[v];
    const float inv_tw = 1.0f / (float)a.cfg.tile_w, inv_th = 1.0f / (float)a.cfg.tile_h;
    const int64_t base = (int64_t)blockIdx.x * GSR_BIN_CHUNK;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // blocked layout: thread t owns chunk items 4t .. 4t+3 (keeps slot order)
    uint32_t cnt[4], tsum = 0;
    for (int k = 0; k < 4; ++k) {
        int li = tid * 4 + k;
        SlotRect r{0, 0, 0, 0};
        cnt[k] = slot_count(a, vw, base + li, v, r, inv_tw, inv_th);
        rx0[li] = r.x0;
        ry0[li] = r.y0;
        rw[li] = r.w;
        if (cnt[k]) {
            float d = a.rgb_d[(int64_t)v * a.n + base + li].w;
            dbits[li] = __float_as_uint(d);
        }
        tsum += cnt[k];
    }
    // block exclusive scan of the per-thread sums
    uint32_t incl = tsum;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t wofs = 0;
    for (int k = 0; k < w; ++k) wofs += wsum[k];
    uint32_t run = wofs + incl - tsum;
    for (int k = 0; k < 4; ++k) {
        excl[tid * 4 + k] = run;
        run += cnt[k];
    }
    const uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (tid == 0) excl[GSR_BIN_CHUNK] = total;
    __syncthreads();
    const unsigned long long out0 = a.block_offs[v * a.chunks + blockIdx.x];
    for (uint32_t j = tid; j < total; j += 256) {
        // owner: largest s with excl[s] <= j
        int lo = 0, hi = GSR_BIN_CHUNK - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (excl[mid] <= j) lo = mid; else hi = mid - 1;
        }
        uint32_t r = j - excl[lo];
        int wdt = rw[lo];
        int ty = ry0[lo] + (int)(r / (uint32_t)wdt);
        int tx = rx0[lo] + (int)(r % (uint32_t)wdt);
        unsigned long long tile = (unsigned long long)(vw.tile_base + ty * vw.tiles_x + tx);
        a.keys[out0 + j] = (tile << 32) | dbits[lo];
        a.vals[out0 + j] = (uint32_t)((int64_t)v * a.n + base + lo);
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
