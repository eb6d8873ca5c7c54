// track.hip -- the tracking loss of the appendix (Tracking and Camera Pose
// Optimization) over all views of a plan, and its gradient seed for the
// compositing backward.
//
// Per view, with I_hat the render, I the observation and x running over the
// view's pixels and colour channels:
//   (g, b) = argmin sum (I - g I_hat - b)^2                       Eq. (app-ls)
//   L = sum_pixels w sum_channels |I - g I_hat - b|                Eqs. (app-bright), (app-trackloss)
//   w = clip((1 - T_final) / tau_alpha, 0, 1)
//       * clip(||grad I||_2 / tau_grad, 0, 1)                      Eq. (app-weight)
// (g, b) is the least-squares solution as a function of the render, and the
// gradient dL/dI_hat includes that dependence; dL/dT_final comes from the
// opacity weight.  ||grad I||_2 is the Frobenius norm over the channels of the
// observation's central differences (one-sided at the border, zero along an
// axis of extent 1).  A render without variance takes g = 1 and
// b = mean(I) - mean(I_hat).
//
// Three launches over a (GSR_TRACK_BLOCKS, views) grid, each block striding
// over its view's pixels, all arithmetic in double.  Double division and
// square root take tens of instructions at half the float rate, so the
// per-view reciprocals are formed once and the pixel's column and row are
// stepped, not divided out:
//   k_track_sums   sum I_hat, sum I, sum I_hat^2, sum I_hat I per block;
//   k_track_signs  (g, b) from those partials, then per block
//                  sum w |r|, sum w sign(r), sum w sign(r) I_hat;
//   k_track_grad   the gradient; block 0 of each view writes the loss and
//                  (g, b).
// Every partial goes to its own workspace slot and is summed in a fixed
// order, so the results do not depend on scheduling.
#include "kernels.h"

namespace gsr {

#define GSR_TRACK_THREADS 256
// relative variance below which the render counts as constant
#define GSR_TRACK_DEGENERATE 1e-12

__device__ __forceinline__ double wave_sum_d(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// block-wide sums of K doubles, in a fixed order; every thread gets them
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*lds)[GSR_TRACK_THREADS / 64])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s = wave_sum_d(v[k]);
        if (lane == 0) lds[k][w] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int j = 0; j < GSR_TRACK_THREADS / 64; ++j) s += lds[k][j];
        v[k] = s;
    }
    __syncthreads();
}

// the sums of the view's partial slots [first, first + K) over its blocks,
// in a fixed order: lane j of one wave adds the slots of blocks j, j + 64,
// ..., then a shuffle tree
template <int K>
__device__ __forceinline__ void view_totals(const double* part, int v, int first, double (&tot)[K],
                                            double (*lds)[GSR_TRACK_THREADS / 64])
{
    const int tid = threadIdx.x;
    double x[K];
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = 0.0;
    if (tid < 64) {
        for (int j = tid; j < GSR_TRACK_BLOCKS; j += 64) {
            const double* p = part + ((int64_t)v * GSR_TRACK_BLOCKS + j) * GSR_TRACK_SLOTS + first;
#pragma unroll
            for (int k = 0; k < K; ++k) x[k] += p[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = wave_sum_d(x[k]);
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) lds[k][0] = x[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) tot[k] = lds[k][0];
    __syncthreads();
}

struct Exposure {
    double N, Sx, Sy, D, g, b;
    bool degenerate;
};

__device__ __forceinline__ Exposure exposure_of(const double (&s)[4], double N)
{
    Exposure e;
    e.N = N;
    e.Sx = s[0];
    e.Sy = s[1];
    e.D = N * s[2] - s[0] * s[0];
    e.degenerate = !(e.D > GSR_TRACK_DEGENERATE * N * s[2]);
    if (e.degenerate) {
        e.g = 1.0;
        e.b = (s[1] - s[0]) / N;
    } else {
        e.g = (N * s[3] - s[0] * s[1]) / e.D;
        e.b = (s[1] - e.g * s[0]) / N;
    }
    return e;
}

// the observation's gradient norm at (x, y) of a [3][H][W] image
__device__ __forceinline__ double grad_norm_at(const float* img, int W, int H, int x, int y)
{
    const int plane = W * H;
    const int at = y * W + x;
    const int xl = x > 0 ? x - 1 : x, xr = x < W - 1 ? x + 1 : x;
    const int yu = y > 0 ? y - 1 : y, yd = y < H - 1 ? y + 1 : y;
    const double hx = (xr - xl) == 2 ? 0.5 : 1.0, hy = (yd - yu) == 2 ? 0.5 : 1.0;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float* p = img + c * plane;
        const double gx = W > 1 ? ((double)p[at - x + xr] - (double)p[at - x + xl]) * hx : 0.0;
        const double gy = H > 1 ? ((double)p[yd * W + x] - (double)p[yu * W + x]) * hy : 0.0;
        s += gx * gx + gy * gy;
    }
    return sqrt(s);
}

// A thread's pixels i = i0, i0 + S, ... (S = GSR_TRACK_BLOCKS x threads) of
// a W-wide view with their column and row, advanced without a division.
struct PixelWalk {
    int i, x, y, dx, dy;
    __device__ PixelWalk(int W)
    {
        constexpr int S = GSR_TRACK_BLOCKS * GSR_TRACK_THREADS;
        i = (int)blockIdx.x * GSR_TRACK_THREADS + (int)threadIdx.x;
        y = i / W;
        x = i - y * W;
        dy = S / W;
        dx = S - dy * W;
    }
    __device__ void next(int W)
    {
        i += GSR_TRACK_BLOCKS * GSR_TRACK_THREADS;
        x += dx;
        y += dy;
        if (x >= W) {
            x -= W;
            ++y;
        }
    }
};

__device__ __forceinline__ double clip01(double z) { return fmin(fmax(z, 0.0), 1.0); }

__device__ __forceinline__ double sgn(double r) { return r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0); }

__global__ __launch_bounds__(GSR_TRACK_THREADS) void k_track_sums(TrackArgs a)
{
    __shared__ double lds[8][GSR_TRACK_THREADS / 64];
    const int v = blockIdx.y;
    const ViewInfo& vw = a.views->v[v];
    const int64_t hw = (int64_t)vw.width * vw.height;
    const float* Ih = a.rgb + 3 * (int64_t)vw.pix_base;
    const float* I = a.target + 3 * (int64_t)vw.pix_base;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = (int)blockIdx.x * GSR_TRACK_THREADS + (int)threadIdx.x; i < (int)hw;
         i += GSR_TRACK_BLOCKS * GSR_TRACK_THREADS) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double x = Ih[c * hw + i], y = I[c * hw + i];
            s[0] += x;
            s[1] += y;
            s[2] += x * x;
            s[3] += x * y;
        }
    }
    block_sum<4>(s, lds);
    if (threadIdx.x < 4)
        a.part[((int64_t)v * GSR_TRACK_BLOCKS + blockIdx.x) * GSR_TRACK_SLOTS + threadIdx.x] = s[threadIdx.x];
}

__global__ __launch_bounds__(GSR_TRACK_THREADS) void k_track_signs(TrackArgs a)
{
    __shared__ double lds[8][GSR_TRACK_THREADS / 64];
    const int v = blockIdx.y;
    const ViewInfo& vw = a.views->v[v];
    const int W = vw.width, H = vw.height;
    const int64_t hw = (int64_t)W * H;
    double st[4];
    view_totals<4>(a.part, v, 0, st, lds);
    const Exposure e = exposure_of(st, 3.0 * (double)hw);
    const float* Ih = a.rgb + 3 * (int64_t)vw.pix_base;
    const float* I = a.target + 3 * (int64_t)vw.pix_base;
    const float* T = a.T_final + vw.pix_base;
    const double inv_tg = 1.0 / a.tau_grad;
    double q[3] = {0.0, 0.0, 0.0};  // sum w |r|, sum w s, sum w s I_hat
    for (PixelWalk p(W); p.i < (int)hw; p.next(W)) {
        const int i = p.i;
        const double w = clip01((1.0 - (double)T[i]) / a.tau_alpha) *
                         clip01(grad_norm_at(I, W, H, p.x, p.y) * inv_tg);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double xh = Ih[c * hw + i];
            const double r = (double)I[c * hw + i] - (e.g * xh + e.b);
            const double s = sgn(r);
            q[0] += w * fabs(r);
            q[1] += w * s;
            q[2] += w * s * xh;
        }
    }
    block_sum<3>(q, lds);
    if (threadIdx.x < 3)
        a.part[((int64_t)v * GSR_TRACK_BLOCKS + blockIdx.x) * GSR_TRACK_SLOTS + 4 + threadIdx.x] = q[threadIdx.x];
}

__global__ __launch_bounds__(GSR_TRACK_THREADS) void k_track_grad(TrackArgs a)
{
    __shared__ double lds[8][GSR_TRACK_THREADS / 64];
    const int v = blockIdx.y;
    const ViewInfo& vw = a.views->v[v];
    const int W = vw.width, H = vw.height;
    const int64_t hw = (int64_t)W * H;
    double st[4], q[3];
    view_totals<4>(a.part, v, 0, st, lds);
    view_totals<3>(a.part, v, 4, q, lds);
    const Exposure e = exposure_of(st, 3.0 * (double)hw);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.loss[v] = q[0];
        a.exposure[2 * v] = e.g;
        a.exposure[2 * v + 1] = e.b;
    }
    // dL/dI_hat_k = -w s g + dL/dg dg/dI_hat_k + dL/db db/dI_hat_k with
    // dL/dg = -Q1, dL/db = -Q0, and from the normal equations
    // dg/dI_hat_k = (N I_k - Sy - 2 g (N I_hat_k - Sx)) / D,
    // db/dI_hat_k = -(Sx dg/dI_hat_k + g) / N (g fixed at 1 when degenerate)
    const double Q0 = q[1], Q1 = q[2];
    const double inv_N = 1.0 / e.N, inv_D = e.degenerate ? 0.0 : 1.0 / e.D, inv_tg = 1.0 / a.tau_grad;
    const double inv_ta = 1.0 / a.tau_alpha;
    const float* Ih = a.rgb + 3 * (int64_t)vw.pix_base;
    const float* I = a.target + 3 * (int64_t)vw.pix_base;
    const float* T = a.T_final + vw.pix_base;
    float* dI = a.dL_drgb + 3 * (int64_t)vw.pix_base;
    float* dT = a.dL_dT ? a.dL_dT + vw.pix_base : nullptr;
    for (PixelWalk p(W); p.i < (int)hw; p.next(W)) {
        const int i = p.i;
        // the one division kept: za decides whether dL/dT_final is zero
        const double za = (1.0 - (double)T[i]) / a.tau_alpha;
        const double wg = clip01(grad_norm_at(I, W, H, p.x, p.y) * inv_tg);
        const double w = clip01(za) * wg;
        double abs_sum = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double xh = Ih[c * hw + i], yo = I[c * hw + i];
            const double r = yo - (e.g * xh + e.b);
            double d = -w * sgn(r) * e.g;
            if (e.degenerate) {
                d += Q0 * inv_N;
            } else {
                const double dg = (e.N * yo - e.Sy - 2.0 * e.g * (e.N * xh - e.Sx)) * inv_D;
                const double db = -(e.Sx * dg + e.g) * inv_N;
                d -= Q1 * dg + Q0 * db;
            }
            dI[c * hw + i] = (float)d;
            abs_sum += fabs(r);
        }
        if (dT) dT[i] = (float)((za > 0.0 && za < 1.0) ? -(wg * inv_ta) * abs_sum : 0.0);
    }
}

hipError_t launch_loss_track(const TrackArgs& a, int n_views, hipStream_t s)
{
    if (n_views <= 0) return hipSuccess;
    const dim3 grid(GSR_TRACK_BLOCKS, (unsigned)n_views);
    hipLaunchKernelGGL(k_track_sums, grid, dim3(GSR_TRACK_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_track_signs, grid, dim3(GSR_TRACK_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_track_grad, grid, dim3(GSR_TRACK_THREADS), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
