// project_math.h -- per-(Gaussian, view) projection in FP32 on the device.
//
// Sec. "Gaussian Splatting Representation", Eq. (proj): mu_I = pi(R mu_W + t),
// Sigma_I = J R Sigma_W R^T J^T with J the pinhole Jacobian at mu_C, plus a
// dilation eps I; appendix: Sigma_W = R_q diag(s^2) R_q^T from a unit
// quaternion and log-scales; opacity o = sigmoid(logit); colour RGB or real SH
// of degree <= 3 (Eq. app-sh) at the direction from the camera centre.
// The forward projection kernel and the projection backward both call
// project_gaussian(), so the backward sees the forward's values exactly.
#pragma once
#include "gsr_device.h"

namespace gsr {

// Real spherical harmonics, index l*l + l + m, no Condon-Shortley phase.
#define GSR_SH_C0 0.28209479177387814f
#define GSR_SH_C1 0.48860251190291992f
#define GSR_SH_C2A 1.0925484305920792f   // xy, yz, xz
#define GSR_SH_C2B 0.31539156525252005f  // 3z^2 - 1
#define GSR_SH_C2C 0.54627421529603959f  // x^2 - y^2
#define GSR_SH_C3A 0.59004358992664352f  // m = +-3
#define GSR_SH_C3B 2.8906114426405538f   // xyz
#define GSR_SH_C3C 0.45704579946446572f  // m = +-1
#define GSR_SH_C3D 0.37317633259011546f  // m = 0
#define GSR_SH_C3E 1.4453057213202769f   // z(x^2 - y^2)

template <int DEG>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float* Y)
{
    Y[0] = GSR_SH_C0;
    if (DEG >= 1) {
        Y[1] = GSR_SH_C1 * y;
        Y[2] = GSR_SH_C1 * z;
        Y[3] = GSR_SH_C1 * x;
    }
    if (DEG >= 2) {
        Y[4] = GSR_SH_C2A * x * y;
        Y[5] = GSR_SH_C2A * y * z;
        Y[6] = GSR_SH_C2B * (3.0f * z * z - 1.0f);
        Y[7] = GSR_SH_C2A * x * z;
        Y[8] = GSR_SH_C2C * (x * x - y * y);
    }
    if (DEG >= 3) {
        Y[9] = GSR_SH_C3A * y * (3.0f * x * x - y * y);
        Y[10] = GSR_SH_C3B * x * y * z;
        Y[11] = GSR_SH_C3C * y * (5.0f * z * z - 1.0f);
        Y[12] = GSR_SH_C3D * z * (5.0f * z * z - 3.0f);
        Y[13] = GSR_SH_C3C * x * (5.0f * z * z - 1.0f);
        Y[14] = GSR_SH_C3E * z * (x * x - y * y);
        Y[15] = GSR_SH_C3A * x * (x * x - 3.0f * y * y);
    }
}

// gradient of the polynomial forms above w.r.t. (x, y, z), accumulated as
// g += sum_k w[k] * grad Y_k
template <int DEG>
__device__ __forceinline__ void sh_grad_acc(float x, float y, float z, const float* w, float& gx,
                                            float& gy, float& gz)
{
    if (DEG >= 1) {
        gy += GSR_SH_C1 * w[1];
        gz += GSR_SH_C1 * w[2];
        gx += GSR_SH_C1 * w[3];
    }
    if (DEG >= 2) {
        gx += GSR_SH_C2A * (w[4] * y + w[7] * z) + GSR_SH_C2C * 2.0f * x * w[8];
        gy += GSR_SH_C2A * (w[4] * x + w[5] * z) - GSR_SH_C2C * 2.0f * y * w[8];
        gz += GSR_SH_C2A * (w[5] * y + w[7] * x) + GSR_SH_C2B * 6.0f * z * w[6];
    }
    if (DEG >= 3) {
        float zz5 = 5.0f * z * z - 1.0f;
        gx += w[9] * GSR_SH_C3A * 6.0f * x * y + w[10] * GSR_SH_C3B * y * z + w[13] * GSR_SH_C3C * zz5 +
              w[14] * GSR_SH_C3E * 2.0f * x * z + w[15] * GSR_SH_C3A * 3.0f * (x * x - y * y);
        gy += w[9] * GSR_SH_C3A * 3.0f * (x * x - y * y) + w[10] * GSR_SH_C3B * x * z +
              w[11] * GSR_SH_C3C * zz5 - w[14] * GSR_SH_C3E * 2.0f * y * z -
              w[15] * GSR_SH_C3A * 6.0f * x * y;
        gz += w[10] * GSR_SH_C3B * x * y + w[11] * GSR_SH_C3C * 10.0f * y * z +
              w[12] * GSR_SH_C3D * (15.0f * z * z - 3.0f) + w[13] * GSR_SH_C3C * 10.0f * x * z +
              w[14] * GSR_SH_C3E * (x * x - y * y);
    }
}

// View-independent activation of one Gaussian.
struct Activated {
    float mw[3];          // world mean
    float qh[4], qn;      // unit quaternion, |q|
    float Rq[9];          // rotation of the Gaussian
    float s2[3];          // squared scales
    float Sw[6];          // Sigma_W: xx, xy, xz, yy, yz, zz
    float o;              // opacity
    bool ok;
};

__device__ __forceinline__ void activate(const float* mean, const float* quat, const float* log_scale,
                                         const float* logit, int64_t n, int64_t i, Activated& a)
{
    a.mw[0] = mean[i];
    a.mw[1] = mean[n + i];
    a.mw[2] = mean[2 * n + i];
    float q0 = quat[i], q1 = quat[n + i], q2 = quat[2 * n + i], q3 = quat[3 * n + i];
    float qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    a.ok = qn > 0.0f && qn < INFINITY;
    float iq = a.ok ? 1.0f / qn : 0.0f;
    float w = q0 * iq, x = q1 * iq, y = q2 * iq, z = q3 * iq;
    a.qh[0] = w; a.qh[1] = x; a.qh[2] = y; a.qh[3] = z;
    a.qn = qn;
    float* R = a.Rq;
    R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
    for (int k = 0; k < 3; ++k) {
        float s = expf(log_scale[k * n + i]);
        a.s2[k] = s * s;
    }
    // Sigma_W = R diag(s2) R^T
    a.Sw[0] = R[0] * R[0] * a.s2[0] + R[1] * R[1] * a.s2[1] + R[2] * R[2] * a.s2[2];
    a.Sw[1] = R[0] * R[3] * a.s2[0] + R[1] * R[4] * a.s2[1] + R[2] * R[5] * a.s2[2];
    a.Sw[2] = R[0] * R[6] * a.s2[0] + R[1] * R[7] * a.s2[1] + R[2] * R[8] * a.s2[2];
    a.Sw[3] = R[3] * R[3] * a.s2[0] + R[4] * R[4] * a.s2[1] + R[5] * R[5] * a.s2[2];
    a.Sw[4] = R[3] * R[6] * a.s2[0] + R[4] * R[7] * a.s2[1] + R[5] * R[8] * a.s2[2];
    a.Sw[5] = R[6] * R[6] * a.s2[0] + R[7] * R[7] * a.s2[1] + R[8] * R[8] * a.s2[2];
    a.o = 1.0f / (1.0f + expf(-logit[i]));
}

// Per-view projection of an activated Gaussian.
struct Projected {
    bool valid;
    float mc[3];      // camera-space mean
    float iz;         // 1 / z
    float J00, J02, J11, J12;
    float M[6];       // J R (2 x 3)
    float a, b, c;    // Sigma_I incl. dilation
    float det;
    float A, B, C;    // conic
    float u, v, rx, ry;
};

// ac - b^2 with one rounding for the products (compensated difference)
__device__ __forceinline__ float det2(float a, float b, float c)
{
    float w = b * b;
    float e = __builtin_fmaf(-b, b, w);
    float f = __builtin_fmaf(a, c, -w);
    return f + e;
}

__device__ __forceinline__ void project_gaussian(const Activated& g, const float* pose, const ViewInfo& vw,
                                                 const DevCfg& cfg, Projected& p)
{
    const float* R = pose;
    const float* t = pose + 9;
    p.valid = false;
    p.mc[0] = R[0] * g.mw[0] + R[1] * g.mw[1] + R[2] * g.mw[2] + t[0];
    p.mc[1] = R[3] * g.mw[0] + R[4] * g.mw[1] + R[5] * g.mw[2] + t[1];
    p.mc[2] = R[6] * g.mw[0] + R[7] * g.mw[1] + R[8] * g.mw[2] + t[2];
    float x = p.mc[0], y = p.mc[1], z = p.mc[2];
    if (!g.ok || !(z > cfg.z_near) || !(z < INFINITY)) return;
    float iz = 1.0f / z;
    p.iz = iz;
    p.u = vw.fx * x * iz + vw.cx;
    p.v = vw.fy * y * iz + vw.cy;
    p.J00 = vw.fx * iz;
    p.J02 = -vw.fx * x * iz * iz;
    p.J11 = vw.fy * iz;
    p.J12 = -vw.fy * y * iz * iz;
    // M = J R
    for (int k = 0; k < 3; ++k) {
        p.M[k] = p.J00 * R[k] + p.J02 * R[6 + k];
        p.M[3 + k] = p.J11 * R[3 + k] + p.J12 * R[6 + k];
    }
    // Sigma_I = M Sigma_W M^T
    const float* S = g.Sw;
    float t0x = p.M[0] * S[0] + p.M[1] * S[1] + p.M[2] * S[2];
    float t0y = p.M[0] * S[1] + p.M[1] * S[3] + p.M[2] * S[4];
    float t0z = p.M[0] * S[2] + p.M[1] * S[4] + p.M[2] * S[5];
    float t1x = p.M[3] * S[0] + p.M[4] * S[1] + p.M[5] * S[2];
    float t1y = p.M[3] * S[1] + p.M[4] * S[3] + p.M[5] * S[4];
    float t1z = p.M[3] * S[2] + p.M[4] * S[4] + p.M[5] * S[5];
    p.a = t0x * p.M[0] + t0y * p.M[1] + t0z * p.M[2] + cfg.dilation;
    p.b = t0x * p.M[3] + t0y * p.M[4] + t0z * p.M[5];
    p.c = t1x * p.M[3] + t1y * p.M[4] + t1z * p.M[5] + cfg.dilation;
    p.det = det2(p.a, p.b, p.c);
    if (!(p.det > 0.0f) || !(p.det < INFINITY)) return;
    float id = 1.0f / p.det;
    p.A = p.c * id;
    p.B = -p.b * id;
    p.C = p.a * id;
    // extent: alpha >= alpha_min inside d^T Sigma_I^-1 d <= 2 ln(o / alpha_min)
    if (cfg.alpha_min > 0.0f) {
        if (!(g.o >= cfg.alpha_min)) return;
        float k = sqrtf(2.0f * logf(g.o / cfg.alpha_min));
        p.rx = k * sqrtf(p.a);
        p.ry = k * sqrtf(p.c);
    } else {
        p.rx = INFINITY;
        p.ry = INFINITY;
    }
    if (!(p.u == p.u) || !(p.v == p.v) || !(fabsf(p.u) < INFINITY) || !(fabsf(p.v) < INFINITY)) return;
    p.valid = true;
}

// camera centre o_c = -R^T t
__device__ __forceinline__ void camera_centre(const float* pose, float* oc)
{
    const float* R = pose;
    const float* t = pose + 9;
    for (int k = 0; k < 3; ++k) oc[k] = -(R[k] * t[0] + R[3 + k] * t[1] + R[6 + k] * t[2]);
}

}  // namespace gsr
