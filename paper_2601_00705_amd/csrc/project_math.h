// project_math.h -- per-(Gaussian, view) projection on the device.
//
// Sec. "Gaussian Splatting Representation", Eq. (proj): mu_I = pi(R mu_W + t),
// Sigma_I = J R Sigma_W R^T J^T with J the pinhole Jacobian at mu_C, plus a
// dilation eps I; appendix: Sigma_W = R_q diag(s^2) R_q^T from a unit
// quaternion and log-scales; opacity o = sigmoid(logit); colour RGB or real SH
// of degree <= 3 (Eq. app-sh) at the direction from the camera centre.
// Templated on the scalar type: the forward projection runs in float (it
// produces the float records the compositing reads); the projection backward
// recomputes the same quantities in double, because its chain rule multiplies
// accumulated screen-space gradients by Jacobians that grow like 1/z^2 near
// the near plane.
#pragma once
#include "gsr_device.h"

namespace gsr {

// Real spherical harmonics, index l*l + l + m, no Condon-Shortley phase.
#define GSR_SH_C0 0.28209479177387814
#define GSR_SH_C1 0.48860251190291992
#define GSR_SH_C2A 1.0925484305920792   // xy, yz, xz
#define GSR_SH_C2B 0.31539156525252005  // 3z^2 - 1
#define GSR_SH_C2C 0.54627421529603959  // x^2 - y^2
#define GSR_SH_C3A 0.59004358992664352  // m = +-3
#define GSR_SH_C3B 2.8906114426405538   // xyz
#define GSR_SH_C3C 0.45704579946446572  // m = +-1
#define GSR_SH_C3D 0.37317633259011546  // m = 0
#define GSR_SH_C3E 1.4453057213202769   // z(x^2 - y^2)

template <int DEG, class T>
__device__ __forceinline__ void sh_eval(T x, T y, T z, T* Y)
{
    Y[0] = (T)GSR_SH_C0;
    if (DEG >= 1) {
        Y[1] = (T)GSR_SH_C1 * y;
        Y[2] = (T)GSR_SH_C1 * z;
        Y[3] = (T)GSR_SH_C1 * x;
    }
    if (DEG >= 2) {
        Y[4] = (T)GSR_SH_C2A * x * y;
        Y[5] = (T)GSR_SH_C2A * y * z;
        Y[6] = (T)GSR_SH_C2B * ((T)3 * z * z - (T)1);
        Y[7] = (T)GSR_SH_C2A * x * z;
        Y[8] = (T)GSR_SH_C2C * (x * x - y * y);
    }
    if (DEG >= 3) {
        Y[9] = (T)GSR_SH_C3A * y * ((T)3 * x * x - y * y);
        Y[10] = (T)GSR_SH_C3B * x * y * z;
        Y[11] = (T)GSR_SH_C3C * y * ((T)5 * z * z - (T)1);
        Y[12] = (T)GSR_SH_C3D * z * ((T)5 * z * z - (T)3);
        Y[13] = (T)GSR_SH_C3C * x * ((T)5 * z * z - (T)1);
        Y[14] = (T)GSR_SH_C3E * z * (x * x - y * y);
        Y[15] = (T)GSR_SH_C3A * x * (x * x - (T)3 * y * y);
    }
}

// gradient of the polynomial forms above w.r.t. (x, y, z), accumulated as
// g += sum_k w[k] * grad Y_k
template <int DEG, class T>
__device__ __forceinline__ void sh_grad_acc(T x, T y, T z, const T* w, T& gx, T& gy, T& gz)
{
    if (DEG >= 1) {
        gy += (T)GSR_SH_C1 * w[1];
        gz += (T)GSR_SH_C1 * w[2];
        gx += (T)GSR_SH_C1 * w[3];
    }
    if (DEG >= 2) {
        gx += (T)GSR_SH_C2A * (w[4] * y + w[7] * z) + (T)GSR_SH_C2C * (T)2 * x * w[8];
        gy += (T)GSR_SH_C2A * (w[4] * x + w[5] * z) - (T)GSR_SH_C2C * (T)2 * y * w[8];
        gz += (T)GSR_SH_C2A * (w[5] * y + w[7] * x) + (T)GSR_SH_C2B * (T)6 * z * w[6];
    }
    if (DEG >= 3) {
        T zz5 = (T)5 * z * z - (T)1;
        gx += w[9] * (T)GSR_SH_C3A * (T)6 * x * y + w[10] * (T)GSR_SH_C3B * y * z + w[13] * (T)GSR_SH_C3C * zz5 +
              w[14] * (T)GSR_SH_C3E * (T)2 * x * z + w[15] * (T)GSR_SH_C3A * (T)3 * (x * x - y * y);
        gy += w[9] * (T)GSR_SH_C3A * (T)3 * (x * x - y * y) + w[10] * (T)GSR_SH_C3B * x * z +
              w[11] * (T)GSR_SH_C3C * zz5 - w[14] * (T)GSR_SH_C3E * (T)2 * y * z -
              w[15] * (T)GSR_SH_C3A * (T)6 * x * y;
        gz += w[10] * (T)GSR_SH_C3B * x * y + w[11] * (T)GSR_SH_C3C * (T)10 * y * z +
              w[12] * (T)GSR_SH_C3D * ((T)15 * z * z - (T)3) + w[13] * (T)GSR_SH_C3C * (T)10 * x * z +
              w[14] * (T)GSR_SH_C3E * (x * x - y * y);
    }
}

// View-independent activation of one Gaussian.
template <class T>
struct Activated {
    T mw[3];          // world mean
    T qh[4], qn;      // unit quaternion, |q|
    T Rq[9];          // rotation of the Gaussian
    T s2[3];          // squared scales
    T Sw[6];          // Sigma_W: xx, xy, xz, yy, yz, zz
    T o;              // opacity
    T kext;           // sqrt(2 ln(o / alpha_min)): the extent factor, the same in every view
    bool ok;
};

// the Gaussian's extent factor, once for all views
template <class T>
__device__ __forceinline__ void extent_factor(Activated<T>& g, const DevCfg& cfg)
{
    g.kext = (cfg.alpha_min > 0.0f && g.o >= (T)cfg.alpha_min) ? sqrt((T)2 * log(g.o / (T)cfg.alpha_min)) : (T)0;
}

template <class T>
__device__ __forceinline__ void activate(const float* mean, const float* quat, const float* log_scale,
                                         const float* logit, int64_t n, int64_t i, Activated<T>& a)
{
    a.mw[0] = (T)mean[i];
    a.mw[1] = (T)mean[n + i];
    a.mw[2] = (T)mean[2 * n + i];
    T q0 = (T)quat[i], q1 = (T)quat[n + i], q2 = (T)quat[2 * n + i], q3 = (T)quat[3 * n + i];
    T qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    a.ok = qn > (T)0 && qn < (T)INFINITY;
    T iq = a.ok ? (T)1 / qn : (T)0;
    T w = q0 * iq, x = q1 * iq, y = q2 * iq, z = q3 * iq;
    a.qh[0] = w; a.qh[1] = x; a.qh[2] = y; a.qh[3] = z;
    a.qn = qn;
    T* R = a.Rq;
    R[0] = (T)1 - (T)2 * (y * y + z * z); R[1] = (T)2 * (x * y - w * z); R[2] = (T)2 * (x * z + w * y);
    R[3] = (T)2 * (x * y + w * z); R[4] = (T)1 - (T)2 * (x * x + z * z); R[5] = (T)2 * (y * z - w * x);
    R[6] = (T)2 * (x * z - w * y); R[7] = (T)2 * (y * z + w * x); R[8] = (T)1 - (T)2 * (x * x + y * y);
    for (int k = 0; k < 3; ++k) {
        T s = exp((T)log_scale[k * n + i]);
        a.s2[k] = s * s;
    }
    // Sigma_W = R diag(s2) R^T
    a.Sw[0] = R[0] * R[0] * a.s2[0] + R[1] * R[1] * a.s2[1] + R[2] * R[2] * a.s2[2];
    a.Sw[1] = R[0] * R[3] * a.s2[0] + R[1] * R[4] * a.s2[1] + R[2] * R[5] * a.s2[2];
    a.Sw[2] = R[0] * R[6] * a.s2[0] + R[1] * R[7] * a.s2[1] + R[2] * R[8] * a.s2[2];
    a.Sw[3] = R[3] * R[3] * a.s2[0] + R[4] * R[4] * a.s2[1] + R[5] * R[5] * a.s2[2];
    a.Sw[4] = R[3] * R[6] * a.s2[0] + R[4] * R[7] * a.s2[1] + R[5] * R[8] * a.s2[2];
    a.Sw[5] = R[6] * R[6] * a.s2[0] + R[7] * R[7] * a.s2[1] + R[8] * R[8] * a.s2[2];
    a.o = (T)1 / ((T)1 + exp(-(T)logit[i]));
}

// Per-view projection of an activated Gaussian.
template <class T>
struct Projected {
    bool valid;
    T mc[3];      // camera-space mean
    T iz;         // 1 / z
    T J00, J02, J11, J12;
    T M[6];       // J R (2 x 3)
    T a, b, c;    // Sigma_I incl. dilation
    T det;
    T A, B, C;    // conic
    T u, v, rx, ry;
};

// ac - b^2 with one rounding for the products (compensated difference)
template <class T>
__device__ __forceinline__ T det2(T a, T b, T c)
{
    T w = b * b;
    T e = fma(-b, b, w);
    T f = fma(a, c, -w);
    return f + e;
}

template <class T>
__device__ __forceinline__ void project_gaussian(const Activated<T>& g, const float* pose, const ViewInfo& vw,
                                                 const DevCfg& cfg, Projected<T>& p)
{
    T R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = (T)pose[k];
    for (int k = 0; k < 3; ++k) t[k] = (T)pose[9 + k];
    p.valid = false;
    // Camera-space mean from double products (a float32 product is exact in
    // double), rounded once: R mu + t cancels when the camera is close to the
    // Gaussian, and the rounded depth is the key that orders the tile lists.
    for (int r = 0; r < 3; ++r) {
        double acc = (double)pose[9 + r];
        acc = fma((double)pose[3 * r], (double)g.mw[0], acc);
        acc = fma((double)pose[3 * r + 1], (double)g.mw[1], acc);
        acc = fma((double)pose[3 * r + 2], (double)g.mw[2], acc);
        p.mc[r] = (T)acc;
    }
    T x = p.mc[0], y = p.mc[1], z = p.mc[2];
    if (!g.ok || !(z > (T)cfg.z_near) || !(z < (T)INFINITY)) return;
    const T fx = (T)vw.fx, fy = (T)vw.fy;
    T iz = (T)1 / z;
    p.iz = iz;
    p.u = fx * x * iz + (T)vw.cx;
    p.v = fy * y * iz + (T)vw.cy;
    p.J00 = fx * iz;
    p.J02 = -fx * x * iz * iz;
    p.J11 = fy * iz;
    p.J12 = -fy * y * iz * iz;
    // M = J R
    for (int k = 0; k < 3; ++k) {
        p.M[k] = p.J00 * R[k] + p.J02 * R[6 + k];
        p.M[3 + k] = p.J11 * R[3 + k] + p.J12 * R[6 + k];
    }
    // Sigma_I = M Sigma_W M^T
    const T* S = g.Sw;
    T t0x = p.M[0] * S[0] + p.M[1] * S[1] + p.M[2] * S[2];
    T t0y = p.M[0] * S[1] + p.M[1] * S[3] + p.M[2] * S[4];
    T t0z = p.M[0] * S[2] + p.M[1] * S[4] + p.M[2] * S[5];
    T t1x = p.M[3] * S[0] + p.M[4] * S[1] + p.M[5] * S[2];
    T t1y = p.M[3] * S[1] + p.M[4] * S[3] + p.M[5] * S[4];
    T t1z = p.M[3] * S[2] + p.M[4] * S[4] + p.M[5] * S[5];
    p.a = t0x * p.M[0] + t0y * p.M[1] + t0z * p.M[2] + (T)cfg.dilation;
    p.b = t0x * p.M[3] + t0y * p.M[4] + t0z * p.M[5];
    p.c = t1x * p.M[3] + t1y * p.M[4] + t1z * p.M[5] + (T)cfg.dilation;
    p.det = det2(p.a, p.b, p.c);
    if (!(p.det > (T)0) || !(p.det < (T)INFINITY)) return;
    T id = (T)1 / p.det;
    p.A = p.c * id;
    p.B = -p.b * id;
    p.C = p.a * id;
    // extent: alpha >= alpha_min inside d^T Sigma_I^-1 d <= 2 ln(o / alpha_min)
    if (cfg.alpha_min > 0.0f) {
        if (!(g.o >= (T)cfg.alpha_min)) return;
        const T k = g.kext;
        p.rx = k * sqrt(p.a);
        p.ry = k * sqrt(p.c);
    } else {
        p.rx = (T)INFINITY;
        p.ry = (T)INFINITY;
    }
    if (!(p.u == p.u) || !(p.v == p.v) || !(fabs(p.u) < (T)INFINITY) || !(fabs(p.v) < (T)INFINITY)) return;
    p.valid = true;
}

// camera centre o_c = -R^T t
template <class T>
__device__ __forceinline__ void camera_centre(const float* pose, T* oc)
{
    for (int k = 0; k < 3; ++k)
        oc[k] = -((T)pose[k] * (T)pose[9] + (T)pose[3 + k] * (T)pose[10] + (T)pose[6 + k] * (T)pose[11]);
}

}  // namespace gsr
