// maintain.hip -- map maintenance: the optimiser step of the appendix's
// optimisation settings with the anchor of Eq. (app-ema), the co-visibility
// score of Eq. (iou), and the pruning and merging of Sec. "Insertion,
// Lightweight Merging, and Pruning".  All are bound by memory traffic.
//
// Adam step (Kingma and Ba, Algorithm 1) over the five parameter planes,
// each with its own learning rate, after clipping the global L2 norm of all
// gradients:
//   k_adam_norm    per block, the sum of g^2 (double) over a fixed set of
//                  elements of every plane, into the block's slot;
//   k_adam_clip    one block: the slots in a fixed order, the norm and the
//                  clip factor min(1, max_norm / (norm + 1e-6));
//   k_adam_update  per element: g' = c g, m = b1 m + (1 - b1) g',
//                  v = b2 v + (1 - b2) g'^2,
//                  p -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps),
//                  and for the means the anchor (1 - eta) a + eta p.
// Four floats of a plane per thread (one 16-byte access per array) where the
// plane allows it.
//
// Co-visibility: per frame, the pixels whose accumulated opacity 1 - T
// exceeds tau in the key frame and in the frame, counted per block and added
// with one 64-bit integer atomic per block and counter (exact, order-free).
//
// Pruning: a Gaussian is dropped when m < m_min, v < v_min,
// sum_k exp(2 log_scale_k) > sigma_max^2 (the trace of R diag(s^2) R^T) or
// sigmoid(opacity_logit) < alpha_min, decided in double; the kept indices are
// listed in order by a three-pass scan (block counts, one-block scan of the
// counts, block-local ranks).  The same scan lists the entries of a caller's
// keep mask (after merging).
//
// Merging: the planes are copied to the output in 16-byte vectors
// (k_merge_copy); then one thread per Gaussian (k_merge) reads its nearest
// neighbour j and j's; for a mutual pair the thread of the lower index
// decides for both (centre distance within radius times the smaller
// geometric-mean scale, first three colour rows within colour_tol, in
// double), writes both keep flags and, when they merge, the merged column:
// visibility-weighted means of mean, colour rows and opacity (as sigmoid),
// and of the two world covariances, split back by a cyclic Jacobi
// eigen-decomposition (double) into a unit quaternion of the eigenvector
// rotation and the log-scales.
#include "kernels.h"
#include "mat3.h"

namespace gsr {

#define ADAM_THREADS 256

__device__ __forceinline__ double mt_wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__global__ __launch_bounds__(ADAM_THREADS) void k_adam_norm(AdamArgs a)
{
    __shared__ double red[ADAM_THREADS / 64];
    const int64_t stride = (int64_t)gridDim.x * ADAM_THREADS;
    const int64_t t0 = (int64_t)blockIdx.x * ADAM_THREADS + threadIdx.x;
    double s = 0.0;
    for (int k = 0; k < 5; ++k) {
        const float* g = a.g[k];
        for (int64_t i = t0; i < a.len[k]; i += stride) {
            const double x = (double)g[i];
            s = __builtin_fma(x, x, s);
        }
    }
    s = mt_wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < ADAM_THREADS / 64; ++w) t += red[w];
        a.part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(ADAM_THREADS) void k_adam_clip(AdamArgs a)
{
    __shared__ double red[ADAM_THREADS / 64];
    double s = 0.0;
    for (int j = threadIdx.x; j < GSR_ADAM_BLOCKS; j += ADAM_THREADS) s += a.part[j];
    s = mt_wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < ADAM_THREADS / 64; ++w) t += red[w];
        const double norm = sqrt(t);
        const double c = a.max_norm > 0.0f ? fmin(1.0, (double)a.max_norm / (norm + 1e-6)) : 1.0;
        a.part[GSR_ADAM_BLOCKS] = c;
        if (a.norm) a.norm[0] = norm;
    }
}

__device__ __forceinline__ void adam_one(float& p, float& m, float& v, float g, float c, float b1, float b2,
                                         float omb1, float omb2, float step_size, float inv_sqrt_bc2, float eps)
{
    const float gc = c * g;
    m = __builtin_fmaf(b1, m, omb1 * gc);
    v = __builtin_fmaf(b2, v, omb2 * gc * gc);
    const float denom = __builtin_sqrtf(v) * inv_sqrt_bc2 + eps;
    p -= step_size * (m / denom);
}

template <bool VEC>
__global__ __launch_bounds__(ADAM_THREADS) void k_adam_update(AdamArgs a)
{
    const int k = blockIdx.y;
    const float c = (float)a.part[GSR_ADAM_BLOCKS];
    const float b1 = a.beta1, b2 = a.beta2, o1 = a.omb1, o2 = a.omb2, eps = a.eps, ss = a.step_size[k];
    const float ib = a.inv_sqrt_bc2;
    const bool anchor = k == 0 && a.anchor != nullptr;
    const float eta = a.ema;
    float* P = a.p[k];
    float* M = a.m[k];
    float* V = a.v[k];
    const float* G = a.g[k];
    const int64_t stride = (int64_t)gridDim.x * ADAM_THREADS;
    const int64_t t0 = (int64_t)blockIdx.x * ADAM_THREADS + threadIdx.x;
    if (VEC) {
        const int64_t len4 = a.len[k] / 4;
        for (int64_t i = t0; i < len4; i += stride) {
            float4 p = reinterpret_cast<float4*>(P)[i], m = reinterpret_cast<float4*>(M)[i];
            float4 v = reinterpret_cast<float4*>(V)[i];
            const float4 g = reinterpret_cast<const float4*>(G)[i];
            adam_one(p.x, m.x, v.x, g.x, c, b1, b2, o1, o2, ss, ib, eps);
            adam_one(p.y, m.y, v.y, g.y, c, b1, b2, o1, o2, ss, ib, eps);
            adam_one(p.z, m.z, v.z, g.z, c, b1, b2, o1, o2, ss, ib, eps);
            adam_one(p.w, m.w, v.w, g.w, c, b1, b2, o1, o2, ss, ib, eps);
            reinterpret_cast<float4*>(P)[i] = p;
            reinterpret_cast<float4*>(M)[i] = m;
            reinterpret_cast<float4*>(V)[i] = v;
            if (anchor) {
                float4 q = reinterpret_cast<float4*>(a.anchor)[i];
                q.x = __builtin_fmaf(eta, p.x - q.x, q.x);
                q.y = __builtin_fmaf(eta, p.y - q.y, q.y);
                q.z = __builtin_fmaf(eta, p.z - q.z, q.z);
                q.w = __builtin_fmaf(eta, p.w - q.w, q.w);
                reinterpret_cast<float4*>(a.anchor)[i] = q;
            }
        }
    } else {
        for (int64_t i = t0; i < a.len[k]; i += stride) {
            float p = P[i], m = M[i], v = V[i];
            adam_one(p, m, v, G[i], c, b1, b2, o1, o2, ss, ib, eps);
            P[i] = p;
            M[i] = m;
            V[i] = v;
            if (anchor) a.anchor[i] = __builtin_fmaf(eta, p - a.anchor[i], a.anchor[i]);
        }
    }
}

hipError_t launch_adam(const AdamArgs& a, bool vec, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam_norm, dim3(GSR_ADAM_BLOCKS), dim3(ADAM_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_adam_clip, dim3(1), dim3(ADAM_THREADS), 0, s, a);
    int64_t longest = 0;
    for (int k = 0; k < 5; ++k) longest = a.len[k] > longest ? a.len[k] : longest;
    int64_t blocks = ((vec ? longest / 4 : longest) + ADAM_THREADS - 1) / ADAM_THREADS;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (vec) hipLaunchKernelGGL(k_adam_update<true>, dim3((unsigned)blocks, 5), dim3(ADAM_THREADS), 0, s, a);
    else hipLaunchKernelGGL(k_adam_update<false>, dim3((unsigned)blocks, 5), dim3(ADAM_THREADS), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// co-visibility

__global__ void k_covis_zero(CovisArgs a)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * a.frames; i += gridDim.x * blockDim.x)
        a.counts[i] = 0ull;
}

__global__ __launch_bounds__(256) void k_covis_count(CovisArgs a)
{
    __shared__ unsigned long long red[2][4];
    const int f = blockIdx.y;
    const float* T = a.T_frames + (int64_t)f * a.pixels;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t inter = 0, uni = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.pixels; i += stride) {
        const bool va = (1.0f - a.T_key[i]) > a.tau, vb = (1.0f - T[i]) > a.tau;
        inter += (va & vb) ? 1u : 0u;
        uni += (va | vb) ? 1u : 0u;
    }
    unsigned long long si = inter, su = uni;
    for (int off = 32; off > 0; off >>= 1) {
        si += __shfl_xor(si, off, 64);
        su += __shfl_xor(su, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = si;
        red[1][threadIdx.x >> 6] = su;
    }
    __syncthreads();
    // one atomic per block and counter: few blocks per frame, so that the
    // adds to the frame's two counters do not queue up in L2
    if (threadIdx.x < 2) {
        const unsigned long long t = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] +
                                     red[threadIdx.x][3];
        if (t) atomicAdd(&a.counts[2 * f + threadIdx.x], t);
    }
}

__global__ void k_covis_iou(CovisArgs a)
{
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < a.frames; f += gridDim.x * blockDim.x) {
        const unsigned long long i = a.counts[2 * f], u = a.counts[2 * f + 1];
        a.iou[f] = u ? (double)i / (double)u : 0.0;
    }
}

hipError_t launch_covis(const CovisArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_covis_zero, dim3(1), dim3(256), 0, s, a);
    // 64 pixels per thread and at most 64 blocks per frame
    int64_t blocks = (a.pixels + 16383) / 16384;
    if (blocks > 64) blocks = 64;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_covis_count, dim3((unsigned)blocks, (unsigned)a.frames), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_covis_iou, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pruning

__device__ __forceinline__ bool prune_keep(const PruneArgs& a, int64_t i)
{
    if (a.mask) return a.mask[i] != 0;
    const double tr = exp(2.0 * (double)a.log_scale[i]) + exp(2.0 * (double)a.log_scale[a.n + i]) +
                      exp(2.0 * (double)a.log_scale[2 * a.n + i]);
    const double alpha = 1.0 / (1.0 + exp(-(double)a.opacity_logit[i]));
    const bool drop = a.m_obs[i] < a.m_min || (double)a.v_vis[i] < a.v_min || tr > a.sigma_max2 ||
                      alpha < a.alpha_min;
    return !drop;
}

// per block of GSR_PRUNE_CHUNK Gaussians: the number kept
__global__ __launch_bounds__(256) void k_prune_count(PruneArgs a)
{
    __shared__ uint32_t red[4];
    const int64_t base = (int64_t)blockIdx.x * GSR_PRUNE_CHUNK;
    uint32_t c = 0;
    for (int j = threadIdx.x; j < GSR_PRUNE_CHUNK; j += 256) {
        const int64_t i = base + j;
        if (i < a.n && prune_keep(a, i)) ++c;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) a.block_count[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// one block: exclusive scan of the block counts (each thread a contiguous
// run of blocks), and the total
__global__ __launch_bounds__(1024) void k_prune_scan(PruneArgs a)
{
    __shared__ unsigned long long part[1024];
    const int nb = a.blocks;
    const int per = (nb + 1023) / 1024;
    const int lo = threadIdx.x * per;
    unsigned long long s = 0;
    for (int k = 0; k < per && lo + k < nb; ++k) s += a.block_count[lo + k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long x = threadIdx.x >= off ? part[threadIdx.x - off] : 0ull;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned long long run = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
    for (int k = 0; k < per && lo + k < nb; ++k) {
        const uint32_t c = a.block_count[lo + k];
        a.block_count[lo + k] = (uint32_t)run;
        run += c;
    }
    if (threadIdx.x == 1023) a.kept[0] = (long long)part[1023];
}

// per block: the kept indices at their ranks (a block-local scan of the
// flags in index order)
__global__ __launch_bounds__(256) void k_prune_emit(PruneArgs a)
{
    __shared__ uint32_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * GSR_PRUNE_CHUNK;
    uint32_t run = a.block_count[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j0 = 0; j0 < GSR_PRUNE_CHUNK; j0 += 256) {
        const int64_t i = base + j0 + threadIdx.x;
        const bool keep = i < a.n && prune_keep(a, i);
        const unsigned long long bal = __ballot(keep);
        const uint32_t below = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t wofs = 0;
        for (int k = 0; k < w; ++k) wofs += wsum[k];
        if (keep) a.keep_index[run + wofs + below] = (int32_t)i;
        run += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

hipError_t launch_prune(const PruneArgs& a, hipStream_t s)
{
    if (a.blocks <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_prune_count, dim3((unsigned)a.blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_prune_emit, dim3((unsigned)a.blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// dst[r][j] = src[r][keep_index[j]] for the kept columns j < kept
__global__ __launch_bounds__(256) void k_compact(CompactArgs a)
{
    const long long kept = a.kept[0];
    const int r = blockIdx.y;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < kept; j += (int64_t)gridDim.x * blockDim.x)
        a.dst[(int64_t)r * a.n + j] = a.src[(int64_t)r * a.n + a.keep_index[j]];
}

hipError_t launch_compact(const CompactArgs& a, hipStream_t s)
{
    int64_t blocks = (a.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)blocks, (unsigned)a.rows), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// merging: mutual nearest neighbours with overlapping footprints and similar
// colours become one Gaussian (at the lower index) carrying the
// visibility-weighted mean of mean, colour, opacity (as alpha) and world
// covariance, the covariance split back into rotation and scales by a
// cyclic Jacobi eigen-decomposition; all in double

__device__ __forceinline__ void quat_rot(double w, double x, double y, double z, double (&R)[3][3])
{
    const double s = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= s;
    x *= s;
    y *= s;
    z *= s;
    R[0][0] = 1 - 2 * (y * y + z * z);
    R[0][1] = 2 * (x * y - w * z);
    R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);
    R[1][1] = 1 - 2 * (x * x + z * z);
    R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);
    R[2][1] = 2 * (y * z + w * x);
    R[2][2] = 1 - 2 * (x * x + y * y);
}

// world covariance of Gaussian i of the input planes, weighted, added to S
__device__ __forceinline__ void add_cov(const MergeArgs& a, int64_t i, double wgt, double (&S)[3][3])
{
    double R[3][3];
    quat_rot(a.in[1][i], a.in[1][a.n + i], a.in[1][2 * a.n + i], a.in[1][3 * a.n + i], R);
    double s2[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) s2[k] = exp(2.0 * (double)a.in[2][(int64_t)k * a.n + i]);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            S[r][c] += wgt * (R[r][0] * s2[0] * R[c][0] + R[r][1] * s2[1] * R[c][1] + R[r][2] * s2[2] * R[c][2]);
}

// whether the mutual pair (lo, hi) merges
__device__ __forceinline__ bool merge_test(const MergeArgs& a, int64_t lo, int64_t hi)
{
    double d2 = 0.0, sl = 0.0, sh = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double e = (double)a.in[0][(int64_t)k * a.n + lo] - (double)a.in[0][(int64_t)k * a.n + hi];
        d2 += e * e;
        sl += (double)a.in[2][(int64_t)k * a.n + lo];
        sh += (double)a.in[2][(int64_t)k * a.n + hi];
    }
    const double sbar = fmin(exp(sl / 3.0), exp(sh / 3.0));
    if (!(sqrt(d2) <= a.radius * sbar)) return false;
    double cd = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        cd = fmax(cd, fabs((double)a.in[4][(int64_t)k * a.n + lo] - (double)a.in[4][(int64_t)k * a.n + hi]));
    return cd <= a.colour_tol;
}

// out = in, plane blockIdx.y, in 16-byte vectors where both planes allow
__global__ __launch_bounds__(256) void k_merge_copy(MergeArgs a)
{
    const int k = blockIdx.y;
    const int rows = k == 0 || k == 2 ? 3 : k == 1 ? 4 : k == 3 ? 1 : a.colour_rows;
    const float* src = a.in[k];
    float* dst = a.out[k];
    const int64_t len = (int64_t)rows * a.n;
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t done = 0;
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) {
        const int64_t len4 = len / 4;
        for (int64_t q = t; q < len4; q += stride)
            reinterpret_cast<float4*>(dst)[q] = reinterpret_cast<const float4*>(src)[q];
        done = len4 * 4;
    }
    for (int64_t q = done + t; q < len; q += stride) dst[q] = src[q];
}

// log(exp(x) + exp(y)), -inf when both are -inf
__device__ __forceinline__ double log_add_exp(double x, double y)
{
    const double hi = fmax(x, y), lo = fmin(x, y);
    return hi == -INFINITY ? hi : hi + log1p(exp(lo - hi));
}

// log sigmoid(x) = -log(1 + exp(-x)), without overflow for large |x|
__device__ __forceinline__ double log_sigmoid(double x)
{
    return -(fmax(-x, 0.0) + log1p(exp(-fabs(x))));
}

// logit of the weighted mean a = (wi sigmoid(xi) + wj sigmoid(xj)) / (wi + wj):
// a and 1 - a are both weighted sums of sigmoids (1 - sigmoid(x) =
// sigmoid(-x)), summed in the log domain, so that saturated opacities keep a
// finite logit where a itself rounds to 1
__device__ __forceinline__ double merged_logit(double xi, double xj, double wi, double wj)
{
    const double li = wi > 0.0 ? log(wi) : -INFINITY, lj = wj > 0.0 ? log(wj) : -INFINITY;
    return log_add_exp(li + log_sigmoid(xi), lj + log_sigmoid(xj)) -
           log_add_exp(li + log_sigmoid(-xi), lj + log_sigmoid(-xj));
}

// the merge proper, after k_merge_copy: keep flags, and the merged columns
// of the survivors
__global__ __launch_bounds__(256) void k_merge(MergeArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int64_t j = a.nn[i];
    const bool mutual = j >= 0 && j < a.n && j != i && (int64_t)a.nn[j] == i;
    if (!mutual) {
        a.keep[i] = 1;
        return;
    }
    if (j < i) return;  // the lower index of the pair decides and writes both flags
    const bool merged = merge_test(a, i, j);
    a.keep[i] = 1;
    a.keep[j] = merged ? 0 : 1;
    if (!merged) return;
    double wi = (double)a.v_vis[i], wj = (double)a.v_vis[j];
    if (!(wi + wj > 0.0)) wi = wj = 1.0;
    const double W = wi + wj;
#pragma unroll
    for (int r = 0; r < 3; ++r)
        a.out[0][(int64_t)r * a.n + i] =
            (float)((wi * (double)a.in[0][(int64_t)r * a.n + i] + wj * (double)a.in[0][(int64_t)r * a.n + j]) / W);
    for (int r = 0; r < a.colour_rows; ++r)
        a.out[4][(int64_t)r * a.n + i] =
            (float)((wi * (double)a.in[4][(int64_t)r * a.n + i] + wj * (double)a.in[4][(int64_t)r * a.n + j]) / W);
    a.out[3][i] = (float)merged_logit((double)a.in[3][i], (double)a.in[3][j], wi, wj);
    double S[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    add_cov(a, i, wi / W, S);
    add_cov(a, j, wj / W, S);
    double V[3][3], lam[3];
    eig3(S, V, lam);
    const double det = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) -
                       V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
                       V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
    if (det < 0.0)
#pragma unroll
        for (int r = 0; r < 3; ++r) V[r][0] = -V[r][0];
    double q[4];
    rot_quat(V, q);
#pragma unroll
    for (int k = 0; k < 4; ++k) a.out[1][(int64_t)k * a.n + i] = (float)q[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) a.out[2][(int64_t)k * a.n + i] = (float)(0.5 * log(fmax(lam[k], 1e-300)));
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    int64_t blocks = ((int64_t)a.colour_rows * a.n / 4 + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_merge_copy, dim3((unsigned)blocks, 5), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_merge, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
