// project.hip -- forward projection, one thread per Gaussian looping over views.
//
// Eq. (proj) with the appendix's parameterisation (see project_math.h).  The
// Gaussian's parameters are read once (coalesced SoA planes) and kept in
// registers for every view of the batch; the per-view pose is read from
// device memory so that a captured graph sees pose updates.  For every live
// slot (view, Gaussian) the kernel writes geom/conic_o/rgb_d/qthr (float),
// the staging record (double centre and conic) and zeroes the slot's
// screen-space gradient accumulators; a culled slot keeps or gets a culled
// marker (rx = ry = -1 where it was live before, NaN from the plan's set-up
// otherwise).  A
// slot is live when its tile rectangle is not empty; per view, each wave
// also stores the ballot of its slots' liveness (word [w][v], bit k:
// Gaussian 64 w + k; lanes past n have left and add 0), from which the
// binning lists the live slots.
#include "kernels.h"
#include "project_math.h"

namespace gsr {

template <int DEG>
__global__ __launch_bounds__(256, 3) void k_project(ProjectArgs a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the accumulators of the live slots are zeroed below: the next backward
    // needs no clearing pass
    if (i == 0) {
        a.counters->grad_dirty = 0u;
        a.stamps[a.views->n] = (unsigned long long)wall_clock64();
    }
    if (i >= a.n) return;
    const int64_t n = a.n;
    // the wave's ballots go to LDS, one per view, and are stored together
    // after the last view
    __shared__ uint64_t ballots[4][GSR_MAX_VIEWS];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wave_word = (int64_t)blockIdx.x * 4 + wave;
    uint64_t* wave_ballots = ballots[wave];
    const int lane = threadIdx.x & 63;
    // the geometry is computed in double (the chip's FP64 vector rate equals
    // its FP32 rate and this kernel is bound by memory), so that every float
    // record below is the correctly rounded value of the exact projection
    Activated<double> g;
    activate<double>(a.mean, a.quat, a.log_scale, a.opacity_logit, n, i, g);
    extent_factor<double>(g, a.cfg);
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
    // the wave's ballot words of the previous projection (a bound plan
    // starts with all clear and every slot culled); read before this
    // projection's words replace them below
    const uint64_t* old_words = a.live_mask + wave_word * vt->n;
    const float inv_tw = 1.0f / (float)a.cfg.tile_w, inv_th = 1.0f / (float)a.cfg.tile_h;
    const float o = (float)g.o;
    // binning level of d^T conic d, the same in every view: the alpha_min
    // ellipse 2 ln(o / alpha_min) widened by 5% + 0.01 so that rounding
    // never drops a tile the compositing would reach
    const float qthr = a.cfg.alpha_min > 0.0f ? 1.05f * (2.0f * logf(o / a.cfg.alpha_min)) + 0.01f : INFINITY;
    for (int v = 0; v < vt->n; ++v) {
        const ViewInfo vw = vt->v[v];
        const float* pose = a.poses + 12 * v;
        Projected<double> p;
        project_gaussian<double>(g, pose, vw, a.cfg, p);
        int64_t slot = (int64_t)v * n + i;
        const float u = (float)p.u, vv = (float)p.v, rx = (float)p.rx, ry = (float)p.ry;
        int x0, y0, x1, y1;
        bool live = p.valid && tile_rect(u, vv, rx, ry, inv_tw, inv_th, vw.tiles_x, vw.tiles_y, x0, y0, x1, y1);
        const uint64_t ballot = __ballot(live);
        if (!live) {
            // a slot culled at the previous projection too (its old ballot
            // bit clear) already holds a culled marker
            if ((old_words[v] >> lane) & 1ull) a.geom[slot] = make_float4(0.0f, 0.0f, -1.0f, -1.0f);
        } else {
            float rgb[3];
            if (DEG < 0) {
                rgb[0] = col[0][0];
                rgb[1] = col[0][1];
                rgb[2] = col[0][2];
            } else {
                double oc[3];
                camera_centre<double>(pose, oc);
                double dx = g.mw[0] - oc[0], dy = g.mw[1] - oc[1], dz = g.mw[2] - oc[2];
                double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
                float Y[16];
                sh_eval<DEG < 0 ? 0 : DEG, float>((float)(dx * inv), (float)(dy * inv), (float)(dz * inv), Y);
    #pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float acc = 0.0f;
    #pragma unroll
                    for (int k = 0; k < K; ++k) acc += col[k][c] * Y[k];
                    rgb[c] = acc;
                }
            }
            a.geom[slot] = make_float4(u, vv, rx, ry);
            a.conic_o[slot] = make_float4((float)p.A, (float)p.B, (float)p.C, o);
            a.rgb_d[slot] = make_float4(rgb[0], rgb[1], rgb[2], (float)p.mc[2]);
            if (a.cfg.mixed) {
                StageRecM sr;
                sr.u = (float)p.u;
                sr.v = (float)p.v;
                sr.A = (float)p.A;
                sr.B = (float)p.B;
                sr.C = (float)p.C;
                sr.o = o;
                sr.r = __float2half_rn(rgb[0]);
                sr.g = __float2half_rn(rgb[1]);
                sr.b = __float2half_rn(rgb[2]);
                sr.pad = 0;
                static_cast<StageRecM*>(a.stage)[slot] = sr;
            } else {
                StageRec sr;
                sr.u = p.u;
                sr.v = p.v;
                sr.A = p.A;
                sr.B = p.B;
                sr.C = p.C;
                sr.o = o;
                sr.r = rgb[0];
                sr.g = rgb[1];
                sr.b = rgb[2];
                sr.pad[0] = sr.pad[1] = 0.0f;
                static_cast<StageRec*>(a.stage)[slot] = sr;
            }
    #pragma unroll
            for (int f = 0; f < GSR_G2; ++f) a.grad2d[GSR_G2 * slot + f] = 0.0;
            if (a.acc) {
                ulonglong2* z = reinterpret_cast<ulonglong2*>(a.acc + GSR_G2 * GSR_FIX_LIMBS * slot);
    #pragma unroll
                for (int k = 0; k < GSR_G2 * GSR_FIX_LIMBS / 2; ++k) z[k] = make_ulonglong2(0ull, 0ull);
            }
            a.qthr[slot] = qthr;
        }
        // after the slot's stores, so that no register of a load in flight
        // is taken for it
        if (lane == 0) wave_ballots[v] = ballot;
    }
    // lane v stores view v's word; in a wave cut short by n, the lanes past
    // n have left, so lane 0 stores them all
    __builtin_amdgcn_wave_barrier();
    uint64_t* out = a.live_mask + wave_word * vt->n;
    if ((wave_word + 1) * 64 <= n) {
        if (lane < vt->n) out[lane] = wave_ballots[lane];
    } else if (lane == 0) {
        for (int v = 0; v < vt->n; ++v) out[v] = wave_ballots[v];
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
