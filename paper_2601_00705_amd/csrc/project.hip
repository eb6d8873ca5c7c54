// project.hip -- forward projection, one thread per Gaussian looping over views.
//
// Eq. (proj) with the appendix's parameterisation (see project_math.h).  The
// Gaussian's parameters are read once (coalesced SoA planes) and kept in
// registers for every view of the batch; the per-view pose is read from
// device memory so that a captured graph sees pose updates.  For every slot
// (view, Gaussian) the kernel writes geom/conic_o/rgb_d; a culled slot gets
// rx = ry = -1.
#include "kernels.h"
#include "project_math.h"

namespace gsr {

template <int DEG>
__global__ __launch_bounds__(256) void k_project(ProjectArgs a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int64_t n = a.n;
    Activated<float> g;
    activate<float>(a.mean, a.quat, a.log_scale, a.opacity_logit, n, i, g);
    constexpr int K = DEG < 0 ? 1 : (DEG + 1) * (DEG + 1);
    float col[K][3];
    if (DEG < 0) {
        for (int c = 0; c < 3; ++c) col[0][c] = a.colour[c * n + i];
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) col[k][c] = a.colour[(k * 3 + c) * n + i];
    }
    const ViewTable* vt = a.views;
    const float inv_tw = 1.0f / (float)a.cfg.tile_w, inv_th = 1.0f / (float)a.cfg.tile_h;
    for (int v = 0; v < vt->n; ++v) {
        const ViewInfo vw = vt->v[v];
        const float* pose = a.poses + 12 * v;
        Projected<float> p;
        project_gaussian<float>(g, pose, vw, a.cfg, p);
        int64_t slot = (int64_t)v * n + i;
        int x0, y0, x1, y1;
        bool live = p.valid && tile_rect(p.u, p.v, p.rx, p.ry, inv_tw, inv_th, vw.tiles_x, vw.tiles_y,
                                         x0, y0, x1, y1);
        if (!live) {
            a.geom[slot] = make_float4(0.0f, 0.0f, -1.0f, -1.0f);
            continue;
        }
        float rgb[3];
        if (DEG < 0) {
            rgb[0] = col[0][0];
            rgb[1] = col[0][1];
            rgb[2] = col[0][2];
        } else {
            float oc[3];
            camera_centre<float>(pose, oc);
            float dx = g.mw[0] - oc[0], dy = g.mw[1] - oc[1], dz = g.mw[2] - oc[2];
            float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
            float Y[16];
            sh_eval<DEG < 0 ? 0 : DEG, float>(dx * inv, dy * inv, dz * inv, Y);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < K; ++k) acc += col[k][c] * Y[k];
                rgb[c] = acc;
            }
        }
        a.geom[slot] = make_float4(p.u, p.v, p.rx, p.ry);
        a.conic_o[slot] = make_float4(p.A, p.B, p.C, g.o);
        a.rgb_d[slot] = make_float4(rgb[0], rgb[1], rgb[2], p.mc[2]);
        // binning level of d^T conic d: the alpha_min ellipse 2 ln(o / alpha_min)
        // widened by 5% + 0.01 so that rounding never drops a tile the
        // compositing would reach
        a.qthr[slot] = a.cfg.alpha_min > 0.0f ? 1.05f * (2.0f * logf(g.o / a.cfg.alpha_min)) + 0.01f : INFINITY;
    }
}

hipError_t launch_project(const ProjectArgs& a, int sh_degree, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    switch (sh_degree) {
    case -1: hipLaunchKernelGGL(k_project<-1>, grid, block, 0, s, a); break;
    case 0: hipLaunchKernelGGL(k_project<0>, grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_project<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_project<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_project<3>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gsr
