// project_bwd.hip -- from screen-space gradients to Gaussian parameters and
// the SE(3) pose tangent.
//
// One thread per Gaussian loops over the views; for each slot the
// projection marked live (its liveness ballots: one 64-bit word per wave
// and view, read through the scalar cache) it recomputes the forward
// projection (project_math.h, in double) and applies the chain rule of
// Eq. (proj):
//   conic (A, B, C) = Sigma_I^-1:   dSigma_I = -Sigma_I^-1 dconic Sigma_I^-1
//   Sigma_I = M Sigma_W M^T, M = J R:  dSigma_W = M^T G M, dM = 2 G M Sigma_W
//   dJ = dM R^T, dR_cam = J^T dM;  J(mu_C), (u, v)(mu_C) -> d mu_C
// and of the pose tangent, Eqs. (muCjac), (muIjac), (sigmaIjac):
//   d rho += d mu_C,  d omega += mu_C x d mu_C + vee(P - P^T), P = dR_cam R^T
//   (SH colour: the camera centre moves by -R^T rho, so d rho += R dd).
// The arithmetic is double: near the near plane the Jacobians grow like
// 1/z^2 and would amplify float rounding of the accumulated gradients (the
// FP64 vector rate of the chip equals its unpacked FP32 rate, and this kernel
// is a small part of the step).  Per view each wave reduces its 6 tangent
// partials (transposed wave exchange) into LDS; after the last view the
// block sums its waves' partials into a per-block slot of each view; a
// second kernel sums the slots in a fixed order, so the pose gradient is
// deterministic given the accumulators.  Parameter gradients are summed over
// the views not flagged pose-only and written once (overwrite).
#include "kernels.h"
#include "project_math.h"

namespace gsr {

template <int N>
__device__ __forceinline__ void xchg_d(double* v, int lane, int mask)
{
    const bool hi = (lane & mask) != 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double send = hi ? v[j] : v[N + j];
        double keep = hi ? v[N + j] : v[j];
        v[j] = keep + __shfl_xor(send, mask, 64);
    }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(ProjectBwdArgs a)
{
    typedef double T;
    __shared__ double red[GSR_MAX_VIEWS][4][6];  // per view and wave: the 6 tangent partials
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n = a.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
    const bool live_thread = i < n;
    const int64_t S = (int64_t)a.views->n * n;
    // one colour row here (RGB, or the single coefficient of SH degree 0);
    // SH of degree 1-3 is differentiated by k_sh_bwd (its own registers), and
    // the geometry chain here then carries no colour state
    constexpr int K = 1;

    Activated<T> g;
    T col[K][3];
    if (live_thread) {
        activate<T>(a.mean, a.quat, a.log_scale, a.opacity_logit, n, i, g);
        extent_factor<T>(g, a.cfg);
        if (DEG == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) col[k][c] = (T)a.colour[(k * 3 + c) * n + i];
        }
    }
    T dmw[3] = {0, 0, 0}, dSw[6] = {0, 0, 0, 0, 0, 0}, d_o = 0;
    T dcol[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) dcol[k][0] = dcol[k][1] = dcol[k][2] = 0;

    // the wave's liveness words, one per view (bit = lane): the projection's
    // ballots of the same slots; a wave wholly past n (the grid's last block,
    // or n = 0) has none and reads none
    const int64_t wword = __builtin_amdgcn_readfirstlane((int)(i >> 6));
    const bool wave_in = wword < (n + 63) / 64;
    const uint64_t* lm = a.live_mask + (wave_in ? wword : 0) * a.views->n;
    for (int v = 0; v < a.views->n; ++v) {
        const ViewInfo vw = a.views->v[v];
        const float* pose = a.poses + 12 * v;
        T R[9];
        for (int k = 0; k < 9; ++k) R[k] = (T)pose[k];
        const bool params = ((a.pose_only >> v) & 1ull) == 0ull;
        T xi[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int64_t slot = (int64_t)v * n + i;
        const uint64_t word = wave_in ? lm[v] : 0ull;
        bool live = live_thread && ((word >> lane) & 1ull);
        Projected<T> p;
        if (live) {
            project_gaussian<T>(g, pose, vw, a.cfg, p);
            live = p.valid;
        }
        if (live) {
            const double* g2 = a.grad2d + GSR_G2 * slot;
            T gu = g2[0], gv = g2[1];
            T gA = g2[2], gB = g2[3], gC = g2[4];
            T go = g2[5];
            T gc[3] = {g2[6], g2[7], g2[8]};
            // conic -> Sigma_I entries (a, b, c): dSigma = -Sigma^-1 dConic Sigma^-1
            const T A = p.A, B = p.B, C = p.C;
            T da = -(A * A * gA + A * B * gB + B * B * gC);
            T db = -((T)2 * A * B * gA + (A * C + B * B) * gB + (T)2 * B * C * gC);
            T dc = -(B * B * gA + B * C * gB + C * C * gC);
            T G00 = da, G01 = (T)0.5 * db, G11 = dc;
            const T* M = p.M;
            // GM = G M (2 x 3)
            T GM0[3], GM1[3];
            for (int k = 0; k < 3; ++k) {
                GM0[k] = G00 * M[k] + G01 * M[3 + k];
                GM1[k] = G01 * M[k] + G11 * M[3 + k];
            }
            // dM = 2 GM Sigma_W
            const T* Sw = g.Sw;
            T Sfull[9] = {Sw[0], Sw[1], Sw[2], Sw[1], Sw[3], Sw[4], Sw[2], Sw[4], Sw[5]};
            T dM0[3], dM1[3];
            for (int k = 0; k < 3; ++k) {
                dM0[k] = (T)2 * (GM0[0] * Sfull[k] + GM0[1] * Sfull[3 + k] + GM0[2] * Sfull[6 + k]);
                dM1[k] = (T)2 * (GM1[0] * Sfull[k] + GM1[1] * Sfull[3 + k] + GM1[2] * Sfull[6 + k]);
            }
            // M = J R
            T dJ00 = dM0[0] * R[0] + dM0[1] * R[1] + dM0[2] * R[2];
            T dJ02 = dM0[0] * R[6] + dM0[1] * R[7] + dM0[2] * R[8];
            T dJ11 = dM1[0] * R[3] + dM1[1] * R[4] + dM1[2] * R[5];
            T dJ12 = dM1[0] * R[6] + dM1[1] * R[7] + dM1[2] * R[8];
            T dRc[9];
            for (int k = 0; k < 3; ++k) {
                dRc[k] = p.J00 * dM0[k];
                dRc[3 + k] = p.J11 * dM1[k];
                dRc[6 + k] = p.J02 * dM0[k] + p.J12 * dM1[k];
            }
            // J and (u, v) as functions of mu_C
            const T x = p.mc[0], y = p.mc[1], iz = p.iz;
            const T fx = (T)vw.fx, fy = (T)vw.fy, iz2 = iz * iz, iz3 = iz2 * iz;
            T dmc0 = dJ02 * (-fx * iz2) + gu * fx * iz;
            T dmc1 = dJ12 * (-fy * iz2) + gv * fy * iz;
            T dmc2 = dJ00 * (-fx * iz2) + dJ02 * ((T)2 * fx * x * iz3) + dJ11 * (-fy * iz2) +
                     dJ12 * ((T)2 * fy * y * iz3) - gu * fx * x * iz2 - gv * fy * y * iz2;
            // pose tangent
            T P[9];
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q)
                    P[r * 3 + q] = dRc[r * 3] * R[q * 3] + dRc[r * 3 + 1] * R[q * 3 + 1] + dRc[r * 3 + 2] * R[q * 3 + 2];
            const T z = p.mc[2];
            xi[0] = dmc0;
            xi[1] = dmc1;
            xi[2] = dmc2;
            xi[3] = y * dmc2 - z * dmc1 + (P[7] - P[5]);
            xi[4] = z * dmc0 - x * dmc2 + (P[2] - P[6]);
            xi[5] = x * dmc1 - y * dmc0 + (P[3] - P[1]);
            T dm[3];
            for (int q = 0; q < 3; ++q) dm[q] = R[q] * dmc0 + R[3 + q] * dmc1 + R[6 + q] * dmc2;
            if (DEG == 0) {
                T oc[3];
                camera_centre<T>(pose, oc);
                T ddv[3] = {g.mw[0] - oc[0], g.mw[1] - oc[1], g.mw[2] - oc[2]};
                T inv = (T)1 / sqrt(ddv[0] * ddv[0] + ddv[1] * ddv[1] + ddv[2] * ddv[2]);
                T nx = ddv[0] * inv, ny = ddv[1] * inv, nz = ddv[2] * inv;
                T Y[16];
                sh_eval<DEG < 0 ? 0 : DEG, T>(nx, ny, nz, Y);
                T wk[16];
#pragma unroll
                for (int k = 0; k < K; ++k) wk[k] = gc[0] * col[k][0] + gc[1] * col[k][1] + gc[2] * col[k][2];
                T gx = 0, gy = 0, gz = 0;
                sh_grad_acc<DEG < 0 ? 0 : DEG, T>(nx, ny, nz, wk, gx, gy, gz);
                T dot = gx * nx + gy * ny + gz * nz;
                T e0 = (gx - nx * dot) * inv, e1 = (gy - ny * dot) * inv, e2 = (gz - nz * dot) * inv;
                dm[0] += e0;
                dm[1] += e1;
                dm[2] += e2;
                xi[0] += R[0] * e0 + R[1] * e1 + R[2] * e2;
                xi[1] += R[3] * e0 + R[4] * e1 + R[5] * e2;
                xi[2] += R[6] * e0 + R[7] * e1 + R[8] * e2;
                if (params) {
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) dcol[k][c] += gc[c] * Y[k];
                }
            } else if (DEG < 0 && params) {
                dcol[0][0] += gc[0];
                dcol[0][1] += gc[1];
                dcol[0][2] += gc[2];
            }
            if (params) {
                dmw[0] += dm[0];
                dmw[1] += dm[1];
                dmw[2] += dm[2];
                d_o += go;
                // dSigma_W = M^T G M (symmetric)
                dSw[0] += M[0] * GM0[0] + M[3] * GM1[0];
                dSw[1] += M[0] * GM0[1] + M[3] * GM1[1];
                dSw[2] += M[0] * GM0[2] + M[3] * GM1[2];
                dSw[3] += M[1] * GM0[1] + M[4] * GM1[1];
                dSw[4] += M[1] * GM0[2] + M[4] * GM1[2];
                dSw[5] += M[2] * GM0[2] + M[5] * GM1[2];
            }
        }
        // the wave's sums of the 6 tangent partials (uniform control flow),
        // kept per view: the waves run through the views without waiting for
        // each other
        xchg_d<4>(xi, lane, 32);
        xchg_d<2>(xi, lane, 16);
        xchg_d<1>(xi, lane, 8);
        T s = xi[0];
        s += __shfl_xor(s, 4, 64);
        s += __shfl_xor(s, 2, 64);
        s += __shfl_xor(s, 1, 64);
        if ((lane & 7) == 0 && (lane >> 3) < 6) red[v][wv][lane >> 3] = s;
    }
    // the block's partials of every view, the waves summed in a fixed order
    __syncthreads();
    for (int e = tid; e < a.views->n * 6; e += blockDim.x) {
        const int v = e / 6, f = e - 6 * (e / 6);
        const T t = red[v][0][f] + red[v][1][f] + red[v][2][f] + red[v][3][f];
        a.xi_partial[((int64_t)v * a.blocks + blockIdx.x) * 6 + f] = t;
    }
    if (!live_thread || !a.d_mean) return;

    // Sigma_W = R_q diag(s2) R_q^T  ->  log-scales and quaternion
    const T* Rq = g.Rq;
    T dS[9] = {dSw[0], dSw[1], dSw[2], dSw[1], dSw[3], dSw[4], dSw[2], dSw[4], dSw[5]};
    T dRq[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            dRq[r * 3 + k] = (T)2 * g.s2[k] * (dS[r * 3] * Rq[k] + dS[r * 3 + 1] * Rq[3 + k] + dS[r * 3 + 2] * Rq[6 + k]);
    for (int k = 0; k < 3; ++k) {
        // 2 s_k^2 (R_q^T dS R_q)_kk = sum_r R_q[r][k] dRq[r][k]
        T acc = Rq[k] * dRq[k] + Rq[3 + k] * dRq[3 + k] + Rq[6 + k] * dRq[6 + k];
        a.d_log_scale[k * n + i] = (float)acc;
    }
    const T w = g.qh[0], x = g.qh[1], y = g.qh[2], z = g.qh[3];
    T dqw = (T)2 * (-z * dRq[1] + y * dRq[2] + z * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
    T dqx = (T)2 * (y * dRq[1] + z * dRq[2] + y * dRq[3] - (T)2 * x * dRq[4] - w * dRq[5] + z * dRq[6] +
                    w * dRq[7] - (T)2 * x * dRq[8]);
    T dqy = (T)2 * (-(T)2 * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + z * dRq[5] - w * dRq[6] +
                    z * dRq[7] - (T)2 * y * dRq[8]);
    T dqz = (T)2 * (-(T)2 * z * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - (T)2 * z * dRq[4] +
                    y * dRq[5] + x * dRq[6] + y * dRq[7]);
    T dot = dqw * w + dqx * x + dqy * y + dqz * z;
    T iq = g.ok ? (T)1 / g.qn : (T)0;
    a.d_quat[i] = (float)((dqw - w * dot) * iq);
    a.d_quat[n + i] = (float)((dqx - x * dot) * iq);
    a.d_quat[2 * n + i] = (float)((dqy - y * dot) * iq);
    a.d_quat[3 * n + i] = (float)((dqz - z * dot) * iq);
    a.d_mean[i] = (float)dmw[0];
    a.d_mean[n + i] = (float)dmw[1];
    a.d_mean[2 * n + i] = (float)dmw[2];
    a.d_opacity_logit[i] = (float)(d_o * g.o * ((T)1 - g.o));
    if (DEG <= 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) a.d_colour[(k * 3 + c) * n + i] = (float)dcol[k][c];
    }
}

// SH colour of degree DEG >= 1, after k_project_bwd: the colour gradients
// (dL/dc_k = sum over the parameter views of dL/dcolour Y_k(n)), and the
// view-direction term: with n = (mu_W - o_c) / |mu_W - o_c|, the colour's
// gradient in n projected off n and divided by the distance is added to
// dL/dmu_W (parameter views) and, through the camera centre o_c = -R^T t
// (which moves by -R^T rho under the left update), R times it to d rho of
// every view.  This chain is well conditioned (no 1/z), so it runs in FP32.
template <int DEG>
__global__ __launch_bounds__(256) void k_sh_bwd(ProjectBwdArgs a)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    __shared__ double red[GSR_MAX_VIEWS][4][3];  // per view and wave: the 3 rho partials
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n = a.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
    const bool live_thread = i < n;
    float col[K][3], dcol[K][3], mw[3] = {0.0f, 0.0f, 0.0f}, dm[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            col[k][c] = live_thread ? a.colour[(k * 3 + c) * n + i] : 0.0f;
            dcol[k][c] = 0.0f;
        }
    if (live_thread)
        for (int c = 0; c < 3; ++c) mw[c] = a.mean[c * n + i];
    // the wave's liveness words, one per view (bit = lane): the projection's
    // ballots of the same slots; a wave wholly past n (the grid's last block,
    // or n = 0) has none and reads none
    const int64_t wword = __builtin_amdgcn_readfirstlane((int)(i >> 6));
    const bool wave_in = wword < (n + 63) / 64;
    const uint64_t* lm = a.live_mask + (wave_in ? wword : 0) * a.views->n;
    for (int v = 0; v < a.views->n; ++v) {
        const ViewInfo vw = a.views->v[v];
        const float* pose = a.poses + 12 * v;
        const bool params = ((a.pose_only >> v) & 1ull) == 0ull;
        double xe[3] = {0.0, 0.0, 0.0};
        const int64_t slot = (int64_t)v * n + i;
        const uint64_t word = wave_in ? lm[v] : 0ull;
        const bool live = live_thread && ((word >> lane) & 1ull);
        if (live) {
            const double* g2 = a.grad2d + GSR_G2 * slot;
            const float gc[3] = {(float)g2[6], (float)g2[7], (float)g2[8]};
            float oc[3];
            camera_centre<float>(pose, oc);
            const float d0 = mw[0] - oc[0], d1 = mw[1] - oc[1], d2 = mw[2] - oc[2];
            const float inv = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
            const float nx = d0 * inv, ny = d1 * inv, nz = d2 * inv;
            float Y[16], wk[16];
            sh_eval<DEG, float>(nx, ny, nz, Y);
#pragma unroll
            for (int k = 0; k < K; ++k) wk[k] = gc[0] * col[k][0] + gc[1] * col[k][1] + gc[2] * col[k][2];
            float gx = 0.0f, gy = 0.0f, gz = 0.0f;
            sh_grad_acc<DEG, float>(nx, ny, nz, wk, gx, gy, gz);
            const float dot = gx * nx + gy * ny + gz * nz;
            const float e0 = (gx - nx * dot) * inv, e1 = (gy - ny * dot) * inv, e2 = (gz - nz * dot) * inv;
            xe[0] = (double)(pose[0] * e0 + pose[1] * e1 + pose[2] * e2);
            xe[1] = (double)(pose[3] * e0 + pose[4] * e1 + pose[5] * e2);
            xe[2] = (double)(pose[6] * e0 + pose[7] * e1 + pose[8] * e2);
            if (params) {
                dm[0] += e0;
                dm[1] += e1;
                dm[2] += e2;
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) dcol[k][c] += gc[c] * Y[k];
            }
        }
        // the wave's sums of the three rho partials (a transposed exchange
        // of four values, the fourth zero, then a sum over 16 lanes), kept
        // per view (uniform control flow)
        double x4[4] = {xe[0], xe[1], xe[2], 0.0};
        xchg_d<2>(x4, lane, 32);
        xchg_d<1>(x4, lane, 16);
        double t = x4[0];
        t += __shfl_xor(t, 8, 64);
        t += __shfl_xor(t, 4, 64);
        t += __shfl_xor(t, 2, 64);
        t += __shfl_xor(t, 1, 64);
        if ((lane & 15) == 0 && (lane >> 4) < 3) red[v][wv][lane >> 4] = t;
    }
    // the block's partials of every view, the waves summed in a fixed order
    __syncthreads();
    for (int e = tid; e < a.views->n * 6; e += blockDim.x) {
        const int v = e / 6, f = e - 6 * (e / 6);
        const double t = f < 3 ? red[v][0][f] + red[v][1][f] + red[v][2][f] + red[v][3][f] : 0.0;
        a.xi_partial_sh[((int64_t)v * a.blocks + blockIdx.x) * 6 + f] = t;
    }
    if (!live_thread || !a.d_mean) return;
    for (int c = 0; c < 3; ++c) a.d_mean[c * n + i] += dm[c];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) a.d_colour[(k * 3 + c) * n + i] = dcol[k][c];
}

// sum of the per-block tangent partials (and those of the SH chain, when
// given), fixed order: one 1,024-thread block per view (a view's partials
// number one per 256 Gaussians, so the loads of many threads hide each
// other's latency)
#define GSR_XI_THREADS 1024
__global__ __launch_bounds__(GSR_XI_THREADS) void k_xi_reduce(const double* partial, const double* partial_sh,
                                                              int blocks, float* d_xi)
{
    __shared__ double red[6][GSR_XI_THREADS];
    const int v = blockIdx.x, tid = threadIdx.x;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = tid; b < blocks; b += GSR_XI_THREADS)
        for (int k = 0; k < 6; ++k) {
            s[k] += partial[((int64_t)v * blocks + b) * 6 + k];
            if (partial_sh) s[k] += partial_sh[((int64_t)v * blocks + b) * 6 + k];
        }
    for (int k = 0; k < 6; ++k) red[k][tid] = s[k];
    __syncthreads();
    for (int off = GSR_XI_THREADS / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < 6; ++k) red[k][tid] += red[k][tid + off];
        __syncthreads();
    }
    if (tid < 6) d_xi[v * 6 + tid] = (float)red[tid][0];
}

hipError_t launch_project_bwd(const ProjectBwdArgs& a, int sh_degree, float* d_xi, int n_views,
                              hipStream_t s)
{
    {
        dim3 grid((unsigned)a.blocks), block(256);
        switch (sh_degree) {
        case -1: hipLaunchKernelGGL(k_project_bwd<-1>, grid, block, 0, s, a); break;
        case 0: hipLaunchKernelGGL(k_project_bwd<0>, grid, block, 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_project_bwd<1>, grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_project_bwd<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_project_bwd<3>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
        switch (sh_degree) {
        case 1: hipLaunchKernelGGL(k_sh_bwd<1>, grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_sh_bwd<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_sh_bwd<3>, grid, block, 0, s, a); break;
        default: break;
        }
    }
    if (d_xi && n_views > 0)
        hipLaunchKernelGGL(k_xi_reduce, dim3(n_views), dim3(GSR_XI_THREADS), 0, s, a.xi_partial,
                           sh_degree >= 1 ? a.xi_partial_sh : (const double*)nullptr, a.blocks, d_xi);
    return hipGetLastError();
}

}  // namespace gsr
