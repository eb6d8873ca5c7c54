// ssim.hip -- the mapping loss of the appendix's optimisation settings,
//   L = (1 - lambda) mean |x - y| + lambda (1 - mean SSIM(x, y)),
// the means over every pixel and channel of every view (x the render, y the
// target), and its gradient dL/dx for the compositing backward.
//
// SSIM per channel (Wang et al. 2004): an 11 x 11 Gaussian window (sigma
// 1.5, weights summing to 1), C1 = 0.01^2, C2 = 0.03^2, zeros outside the
// image.  With the local moments m = w * x, mxx = w * x^2, mxy = w * (x y)
// and those of y,
//   SSIM(p) = A1 A2 / (B1 B2),  A1 = 2 m my + C1,  A2 = 2 (mxy - m my) + C2,
//             B1 = m^2 + my^2 + C1,  B2 = (mxx - m^2) + (myy - my^2) + C2,
//   d sum_p SSIM(p) / dx(q) = (w * S1)(q) + 2 x(q) (w * Sxx)(q) + y(q) (w * Sxy)(q),
// S1, Sxx, Sxy the partials of SSIM(p) in m, mxx, mxy, zero outside the
// image (the sum runs over the image's pixels; the window is symmetric, so
// the adjoint of a zero-padded window sum is the same window sum).  The same
// holds with x and y replaced by x - kx and y - ky for constants kx, ky (the
// zero padding becoming -kx, -ky): the kernel works with shifted moments.
//
// One kernel, one block per (32 x 32 output tile, view); nothing but the
// gradient and two partial sums per block reaches HBM.  Per channel the block
//   1. loads x and y over the tile plus a 10-pixel apron (52 x 52) into LDS;
//   2. filters the five products x, y, x^2, y^2, x y along rows, over the
//      tile plus a 5-pixel apron (52 rows x 42 columns);
//   3. filters those along columns (42 x 42), forms SSIM and its three
//      partials there;
//   4. filters the partials along rows (42 rows x 32 columns);
//   5. filters those along columns and writes the tile's gradient.
// The next channel's inputs are fetched into registers while the current
// one is filtered.  Every pass slides the 11-tap window along a run of outputs kept in
// registers, so each LDS value is read once per run.  SSIM and |x - y| of
// the tile's own pixels go to the block's partial slots, which a second
// launch sums in a fixed order (the loss does not depend on scheduling).
#include "kernels.h"

namespace gsr {

#define MAP_R 5
#define MAP_TAPS (2 * MAP_R + 1)
#define MAP_T 32                   // output tile edge
#define MAP_P (MAP_T + 2 * MAP_R)  // 42: where SSIM and its partials are formed
#define MAP_I (MAP_P + 2 * MAP_R)  // 52: where the inputs are read
#define MAP_THREADS 256
// run lengths of the four filtering passes
#define MAP_RUN2 7                 // 6 runs per row of 42
#define MAP_RUN3 7                 // 6 runs per column of 42
#define MAP_RUN4 8                 // 4 runs per row of 32
#define MAP_RUN5 4                 // 8 runs per column of 32
#define MAP_LOADS ((MAP_I * MAP_I + MAP_THREADS - 1) / MAP_THREADS)

static_assert(MAP_P % MAP_RUN2 == 0 && MAP_P % MAP_RUN3 == 0, "runs tile the apron region");
static_assert(MAP_T % MAP_RUN4 == 0 && (MAP_T / MAP_RUN5) * MAP_T == MAP_THREADS, "runs tile the output");
static_assert(MAP_P * (MAP_P / MAP_RUN3) <= MAP_THREADS && MAP_P * (MAP_T / MAP_RUN4) <= MAP_THREADS,
              "one run per thread in passes 3 and 4");

struct MapLds {
    union {
        struct {
            float x[MAP_I][MAP_I];
            float y[MAP_I][MAP_I];
        } in;                            // passes 1-2
        float pm[3][MAP_P][MAP_P];       // passes 3-4: S1, Sxx, Sxy
    } a;
    union {
        float h[5][MAP_I][MAP_P];        // passes 2-3: row-filtered products
        float hp[3][MAP_P][MAP_T];       // passes 4-5: row-filtered partials
    } b;
    double red[2][MAP_THREADS / 64];
};

__device__ __forceinline__ double map_wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__global__ __launch_bounds__(MAP_THREADS) void k_map_loss(MapLossArgs a)
{
    __shared__ MapLds L;
    const int v = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
    const ViewInfo vw = a.views->v[v];
    const int W = vw.width, H = vw.height;
    const int ntx = (W + MAP_T - 1) / MAP_T, nty = (H + MAP_T - 1) / MAP_T;
    double* slot = a.part + ((int64_t)v * a.max_tiles + b) * 2;
    if (b >= ntx * nty) {
        if (tid == 0) slot[0] = slot[1] = 0.0;
        return;
    }
    const int ox = (b % ntx) * MAP_T, oy = (b / ntx) * MAP_T;
    const int64_t plane = (int64_t)W * H;
    const int64_t base = 3 * (int64_t)vw.pix_base;
    // the pixels this thread writes in pass 5: column qc, rows 4 qr .. 4 qr + 3
    const int qc = tid % MAP_T, qr = (tid / MAP_T) * MAP_RUN5;
    float ssum = 0.0f, l1sum = 0.0f;
    // the inputs of a channel over the 52 x 52 region (zero outside the
    // image), fetched into registers one channel ahead so that the loads are
    // in flight while the previous channel is filtered
    float px[MAP_LOADS], py[MAP_LOADS];
    auto fetch = [&](int ch) {
        const float* X = a.rgb + base + ch * plane;
        const float* Y = a.target + base + ch * plane;
#pragma unroll
        for (int k = 0; k < MAP_LOADS; ++k) {
            const int i = tid + k * MAP_THREADS;
            const int r = i / MAP_I, c = i - r * MAP_I;
            const int gx = ox - 2 * MAP_R + c, gy = oy - 2 * MAP_R + r;
            const bool in = i < MAP_I * MAP_I && gx >= 0 && gx < W && gy >= 0 && gy < H;
            const int64_t off = in ? (int64_t)gy * W + gx : 0;
            px[k] = in ? X[off] : 0.0f;
            py[k] = in ? Y[off] : 0.0f;
        }
    };
    fetch(0);

    for (int ch = 0; ch < 3; ++ch) {
        // 1. the fetched inputs into LDS
#pragma unroll
        for (int k = 0; k < MAP_LOADS; ++k) {
            const int i = tid + k * MAP_THREADS;
            if (i < MAP_I * MAP_I) {
                (&L.a.in.x[0][0])[i] = px[k];
                (&L.a.in.y[0][0])[i] = py[k];
            }
        }
        __syncthreads();
        float xo[MAP_RUN5], yo[MAP_RUN5];
#pragma unroll
        for (int o = 0; o < MAP_RUN5; ++o) {
            xo[o] = L.a.in.x[qr + o + 2 * MAP_R][qc + 2 * MAP_R];
            yo[o] = L.a.in.y[qr + o + 2 * MAP_R][qc + 2 * MAP_R];
        }
        // the products are formed of x - kx and y - ky, kx and ky the values
        // at the tile's centre pixel (clamped into the image; the apron's
        // zeros become -kx and -ky): the moments are shift-invariant, and the
        // variance w * x^2 - m^2 then cancels little where the image is
        // nearly flat
        const int kc = min(ox + MAP_T / 2, W - 1) - ox + 2 * MAP_R, kr = min(oy + MAP_T / 2, H - 1) - oy + 2 * MAP_R;
        const float kx = L.a.in.x[kr][kc], ky = L.a.in.y[kr][kc];
        if (ch + 1 < 3) fetch(ch + 1);
        // 2. rows: the five products over 52 rows x 42 columns
        for (int i = tid; i < MAP_I * (MAP_P / MAP_RUN2); i += MAP_THREADS) {
            const int r = i / (MAP_P / MAP_RUN2), c0 = (i % (MAP_P / MAP_RUN2)) * MAP_RUN2;
            float xv[MAP_RUN2 + 2 * MAP_R], yv[MAP_RUN2 + 2 * MAP_R];
#pragma unroll
            for (int j = 0; j < MAP_RUN2 + 2 * MAP_R; ++j) {
                xv[j] = L.a.in.x[r][c0 + j] - kx;
                yv[j] = L.a.in.y[r][c0 + j] - ky;
            }
#pragma unroll
            for (int o = 0; o < MAP_RUN2; ++o) {
                float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, s4 = 0.0f;
#pragma unroll
                for (int t = 0; t < MAP_TAPS; ++t) {
                    const float xx = xv[o + t], yy = yv[o + t];
                    const float wx = a.w[t] * xx, wy = a.w[t] * yy;
                    s0 += wx;
                    s1 += wy;
                    s2 = __builtin_fmaf(wx, xx, s2);
                    s3 = __builtin_fmaf(wy, yy, s3);
                    s4 = __builtin_fmaf(wx, yy, s4);
                }
                L.b.h[0][r][c0 + o] = s0;
                L.b.h[1][r][c0 + o] = s1;
                L.b.h[2][r][c0 + o] = s2;
                L.b.h[3][r][c0 + o] = s3;
                L.b.h[4][r][c0 + o] = s4;
            }
        }
        __syncthreads();
        // 3. columns: the moments over 42 x 42, then SSIM and its partials
        if (tid < MAP_P * (MAP_P / MAP_RUN3)) {
            const int c = tid % MAP_P, r0 = (tid / MAP_P) * MAP_RUN3;
            float m[5][MAP_RUN3];
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int o = 0; o < MAP_RUN3; ++o) m[k][o] = 0.0f;
#pragma unroll
            for (int j = 0; j < MAP_RUN3 + 2 * MAP_R; ++j) {
                float hv[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) hv[k] = L.b.h[k][r0 + j][c];
#pragma unroll
                for (int o = 0; o < MAP_RUN3; ++o) {
                    const int t = j - o;
                    if (t >= 0 && t < MAP_TAPS)
#pragma unroll
                        for (int k = 0; k < 5; ++k) m[k][o] = __builtin_fmaf(a.w[t], hv[k], m[k][o]);
                }
            }
            const int gx = ox - MAP_R + c;
            const bool col_in = gx >= 0 && gx < W, col_own = c >= MAP_R && c < MAP_R + MAP_T;
#pragma unroll
            for (int o = 0; o < MAP_RUN3; ++o) {
                const int pr = r0 + o, gy = oy - MAP_R + pr;
                float d1 = 0.0f, dxx = 0.0f, dxy = 0.0f;
                if (col_in && gy >= 0 && gy < H) {
                    // shifted means ms and the means mu = ms + k
                    const float msx = m[0][o], msy = m[1][o], mux = msx + kx, muy = msy + ky;
                    const float A1 = __builtin_fmaf(2.0f * mux, muy, a.c1);
                    const float A2 = __builtin_fmaf(2.0f, m[4][o] - msx * msy, a.c2);
                    const float B1 = __builtin_fmaf(mux, mux, __builtin_fmaf(muy, muy, a.c1));
                    const float B2 = (m[2][o] - msx * msx) + (m[3][o] - msy * msy) + a.c2;
                    const float i1 = 1.0f / B1, i2 = 1.0f / B2, inv = i1 * i2;
                    const float S = A1 * A2 * inv;
                    // the partial in the shifted mean: mu_x enters A1 and B1,
                    // the shifted mean enters A2 and B2
                    d1 = 2.0f * (muy * A2 - msy * A1) * inv - 2.0f * S * (mux * i1 - msx * i2);
                    dxx = -S * i2;
                    dxy = 2.0f * A1 * inv;
                    if (col_own && pr >= MAP_R && pr < MAP_R + MAP_T) ssum += S;
                }
                L.a.pm[0][pr][c] = d1;
                L.a.pm[1][pr][c] = dxx;
                L.a.pm[2][pr][c] = dxy;
            }
        }
        __syncthreads();
        // 4. rows: the partials over 42 rows x 32 columns
        if (tid < MAP_P * (MAP_T / MAP_RUN4)) {
            const int r = tid % MAP_P, c0 = (tid / MAP_P) * MAP_RUN4;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float pv[MAP_RUN4 + 2 * MAP_R];
#pragma unroll
                for (int j = 0; j < MAP_RUN4 + 2 * MAP_R; ++j) pv[j] = L.a.pm[k][r][c0 + j];
#pragma unroll
                for (int o = 0; o < MAP_RUN4; ++o) {
                    float s = 0.0f;
#pragma unroll
                    for (int t = 0; t < MAP_TAPS; ++t) s = __builtin_fmaf(a.w[t], pv[o + t], s);
                    L.b.hp[k][r][c0 + o] = s;
                }
            }
        }
        __syncthreads();
        // 5. columns: the filtered partials at the tile's pixels, the gradient
        {
            float f[3][MAP_RUN5];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int o = 0; o < MAP_RUN5; ++o) f[k][o] = 0.0f;
#pragma unroll
            for (int j = 0; j < MAP_RUN5 + 2 * MAP_R; ++j) {
                float hv[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) hv[k] = L.b.hp[k][qr + j][qc];
#pragma unroll
                for (int o = 0; o < MAP_RUN5; ++o) {
                    const int t = j - o;
                    if (t >= 0 && t < MAP_TAPS)
#pragma unroll
                        for (int k = 0; k < 3; ++k) f[k][o] = __builtin_fmaf(a.w[t], hv[k], f[k][o]);
                }
            }
            float* G = a.dL_drgb + base + ch * plane;
#pragma unroll
            for (int o = 0; o < MAP_RUN5; ++o) {
                const int gx = ox + qc, gy = oy + qr + o;
                if (gx < W && gy < H) {
                    const float r = xo[o] - yo[o];
                    const float sg = r > 0.0f ? a.scale_l1 : (r < 0.0f ? -a.scale_l1 : 0.0f);
                    const float ds = __builtin_fmaf(2.0f * (xo[o] - kx), f[1][o],
                                                    __builtin_fmaf(yo[o] - ky, f[2][o], f[0][o]));
                    G[(int64_t)gy * W + gx] = __builtin_fmaf(a.scale_ssim, ds, sg);
                    l1sum += fabsf(r);
                }
            }
        }
        // the next channel's pass 1 overwrites the partials (read in pass 4,
        // behind the barrier above) and its barrier orders pass 2's writes
        // after this pass's reads
    }
    // the block's partial sums, in a fixed order
    double s[2] = {(double)ssum, (double)l1sum};
    const int lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double t = map_wave_sum(s[k]);
        if (lane == 0) L.red[k][w] = t;
    }
    __syncthreads();
    if (tid == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int j = 0; j < MAP_THREADS / 64; ++j) {
            t0 += L.red[0][j];
            t1 += L.red[1][j];
        }
        slot[0] = t0;
        slot[1] = t1;
    }
}

// one block: the slots in a fixed order, then the loss
__global__ __launch_bounds__(MAP_THREADS) void k_map_loss_total(MapLossArgs a, int64_t slots)
{
    __shared__ double red[2][MAP_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = tid; i < slots; i += MAP_THREADS) {
        s0 += a.part[2 * i];
        s1 += a.part[2 * i + 1];
    }
    s0 = map_wave_sum(s0);
    s1 = map_wave_sum(s1);
    if (lane == 0) {
        red[0][w] = s0;
        red[1][w] = s1;
    }
    __syncthreads();
    if (tid == 0) {
        double ss = 0.0, l1 = 0.0;
        for (int j = 0; j < MAP_THREADS / 64; ++j) {
            ss += red[0][j];
            l1 += red[1][j];
        }
        a.loss[0] = (1.0 - a.lambda) * l1 * a.inv_n + a.lambda * (1.0 - ss * a.inv_n);
    }
}

hipError_t launch_loss_mapping(const MapLossArgs& a, int n_views, hipStream_t s)
{
    if (n_views <= 0 || a.max_tiles <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_map_loss, dim3((unsigned)a.max_tiles, (unsigned)n_views), dim3(MAP_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_map_loss_total, dim3(1), dim3(MAP_THREADS), 0, s, a,
                       (int64_t)n_views * a.max_tiles);
    return hipGetLastError();
}

}  // namespace gsr
