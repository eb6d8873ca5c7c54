// seed.hip -- the one-shot Gaussian seeding from dense correspondences (Sec.
// "Dense Feature Matching" and the appendix's initialisation), one thread per
// reference pixel.
//
// k_seed_triangulate: for every neighbour n of the reference keyframe, the
//   two-view linear system A X = 0 (rows x P^3 - P^1, y P^3 - P^2 of both
//   views) is solved in double by a one-sided Jacobi SVD of the 4x4 A: plane
//   rotations orthogonalise A's columns and accumulate V; the column of V
//   whose rotated column of A has the smallest norm is the right singular
//   vector of the smallest singular value.  Among the neighbours the
//   hypothesis with the smallest reprojection error (RMS of the two
//   reprojection distances, in front of both cameras) is kept, ties going to
//   the larger baseline angle; it is rejected when its error reaches
//   max_reproj or its angle is below min_parallax.  Eq. (conf) gives
//   kappa_bar, Eq. (app-alpha-init) the opacity; the colour is the median of
//   the exposure-corrected bilinear samples over the supporting views (the
//   reference, and every neighbour whose match lies within max_reproj of the
//   kept point's projection).
//
// k_seed_bbox .. k_seed_knn: isotropic scale from the mean distance to the 3
//   nearest other kept seeds, on two uniform grids.  The coarse grid covers
//   the seeds' bounding box (cell size from its volume and the seed count, at
//   most ~4 cells per seed).  Seeds concentrate on surfaces, and a few far
//   seeds inflate the box, so when a seed shares its coarse cell with more
//   than 8 others on average, a fine grid refines the cell size towards ~4
//   seeds per cell, with GSR_KNN_LEVELS - 1 levels of 2x coarser cells above
//   it for sparser regions; their cells are spatially hashed into a table of ~2
//   slots per seed per level (a bucket may hold several cells; a candidate
//   counts only for its own cell).  All are counting sorts by cell.  A query
//   searches cubic shells of cells around its own until the third distance
//   found cannot be beaten by a farther shell (a seed beyond shell r lies at
//   least r + its distance to its own cell's nearer face, in cells, away):
//   up to 2 shells on each fine level, from the level whose cells match the
//   spacing its coarse cell's count suggests upwards, then up to 2 shells on
//   the coarse grid.  The few
//   queries still unsettled (seeds far from all others), or that would
//   examine more than GSR_KNN_BUDGET candidates on one lane (seeds beside
//   much denser regions), are listed and each is answered exactly by a whole
//   block scanning every valid seed.
#include "kernels.h"
#include "mat3.h"

namespace gsr {

#define GSR_SEED_THREADS 256

// ---------------------------------------------------------------------------
// triangulation

// right singular vector of the smallest singular value of the 4x4 A (rows)
__device__ void smallest_right_singular(double A[4][4], double out[4])
{
    double V[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        bool rotated = false;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
#pragma unroll
            for (int q = p + 1; q < 4; ++q) {
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    al += A[i][p] * A[i][p];
                    be += A[i][q] * A[i][q];
                    ga += A[i][p] * A[i][q];
                }
                // a pair counts as orthogonal at ~4.5 machine epsilons of
                // its norms: below that the rounding of the dot products
                // themselves dominates, and a stricter test never settles
                // (every system would run to the sweep cap)
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                rotated = true;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double ap = A[i][p], aq = A[i][q];
                    A[i][p] = c * ap - s * aq;
                    A[i][q] = s * ap + c * aq;
                    const double vp = V[i][p], vq = V[i][q];
                    V[i][p] = c * vp - s * vq;
                    V[i][q] = s * vp + c * vq;
                }
            }
        }
        if (!rotated) break;
    }
    int best = 0;
    double bn = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double nrm = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) nrm += A[i][j] * A[i][j];
        if (j == 0 || nrm < bn) {
            bn = nrm;
            best = j;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = V[i][best];
}

__device__ __forceinline__ void project_px(const double* P, const double X[3], double& u, double& v, double& z)
{
    const double y0 = P[0] * X[0] + P[1] * X[1] + P[2] * X[2] + P[3];
    const double y1 = P[4] * X[0] + P[5] * X[1] + P[6] * X[2] + P[7];
    z = P[8] * X[0] + P[9] * X[1] + P[10] * X[2] + P[11];
    u = y0 / z;
    v = y1 / z;
}

// bilinear sample of channel c, pixel centres at +1/2, clamped to the border
__device__ __forceinline__ double bilinear(const SeedView& vw, int c, double x, double y)
{
    const int W = vw.width, H = vw.height;
    const double fx = fmin(fmax(x - 0.5, 0.0), (double)(W - 1));
    const double fy = fmin(fmax(y - 0.5, 0.0), (double)(H - 1));
    const int x0 = (int)floor(fx), y0 = (int)floor(fy);
    const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
    const double ax = fx - x0, ay = fy - y0;
    const float* p = vw.image + (int64_t)c * W * H;
    return (double)p[y0 * W + x0] * (1.0 - ax) * (1.0 - ay) + (double)p[y0 * W + x1] * ax * (1.0 - ay) +
           (double)p[y1 * W + x0] * (1.0 - ax) * ay + (double)p[y1 * W + x1] * ax * ay;
}

__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_triangulate(SeedArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x;
    if (i >= a.n) return;
    const int K = a.K;
    const double xr[2] = {(double)a.x_ref[i], (double)a.x_ref[a.n + i]};
    const SeedView& R = a.views[0];

    // Eq. (conf) and Eq. (app-alpha-init)
    double ks = 0.0;
    for (int k = 0; k < K; ++k) ks += (double)a.kappa[(int64_t)k * a.n + i];
    const double kbar = ks / (double)K;
    const double alpha = a.alpha_lo + (a.alpha_hi - a.alpha_lo) * kbar;
    if (a.kappa_bar) a.kappa_bar[i] = (float)kbar;
    a.opacity_logit[i] = (float)log(alpha / (1.0 - alpha));

    double best_err = INFINITY, best_ang = -1.0, bX[3] = {0.0, 0.0, 0.0};
    int best = -1;
    for (int k = 0; k < K; ++k) {
        const SeedView& N = a.views[1 + k];
        const double xn[2] = {(double)a.x_nb[(int64_t)(2 * k) * a.n + i], (double)a.x_nb[(int64_t)(2 * k + 1) * a.n + i]};
        double A[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            A[0][j] = xr[0] * R.P[8 + j] - R.P[j];
            A[1][j] = xr[1] * R.P[8 + j] - R.P[4 + j];
            A[2][j] = xn[0] * N.P[8 + j] - N.P[j];
            A[3][j] = xn[1] * N.P[8 + j] - N.P[4 + j];
        }
        double h[4];
        smallest_right_singular(A, h);
        if (h[3] == 0.0) continue;
        const double X[3] = {h[0] / h[3], h[1] / h[3], h[2] / h[3]};
        double ur, vr, zr, un, vn, zn;
        project_px(R.P, X, ur, vr, zr);
        project_px(N.P, X, un, vn, zn);
        if (!(zr > 0.0 && zn > 0.0)) continue;
        const double e0 = ur - xr[0], e1 = vr - xr[1], e2 = un - xn[0], e3 = vn - xn[1];
        const double err = sqrt(0.5 * ((e0 * e0 + e1 * e1) + (e2 * e2 + e3 * e3)));
        const double ra[3] = {X[0] - R.centre[0], X[1] - R.centre[1], X[2] - R.centre[2]};
        const double rb[3] = {X[0] - N.centre[0], X[1] - N.centre[1], X[2] - N.centre[2]};
        const double dot = ra[0] * rb[0] + ra[1] * rb[1] + ra[2] * rb[2];
        const double na = sqrt(ra[0] * ra[0] + ra[1] * ra[1] + ra[2] * ra[2]);
        const double nb = sqrt(rb[0] * rb[0] + rb[1] * rb[1] + rb[2] * rb[2]);
        const double ang = acos(fmin(fmax(dot / (na * nb), -1.0), 1.0));
        if (best < 0 || err < best_err || (err == best_err && ang > best_ang)) {
            best_err = err;
            best_ang = ang;
            best = k;
            bX[0] = X[0];
            bX[1] = X[1];
            bX[2] = X[2];
        }
    }
    // a point whose float32 position overflows is no usable Gaussian
    const bool finite = isfinite((float)bX[0]) && isfinite((float)bX[1]) && isfinite((float)bX[2]);
    const bool ok = best >= 0 && best_err < a.max_reproj && best_ang >= a.min_parallax && finite;
    a.valid[i] = ok ? 1 : 0;
    if (a.best) a.best[i] = best;
    if (a.err) a.err[i] = (float)best_err;
    if (a.angle) a.angle[i] = best >= 0 ? (float)best_ang : 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) a.mean[(int64_t)c * a.n + i] = (float)bX[c];

    // colour: median of the corrected samples over the supporting views.
    // The supporting views form a bit mask; per channel the samples sit in a
    // fixed register array (absent views as +inf), sorted by an unrolled
    // odd-even transposition network, and the median is picked by index
    // compares, so that nothing is indexed dynamically (no scratch memory).
    uint32_t support = 0u;
    if (ok) {
        support = 1u;
#pragma unroll
        for (int v = 1; v <= GSR_SEED_MAX_NEIGHBOURS; ++v) {
            if (v > K) break;
            const double xn0 = (double)a.x_nb[(int64_t)(2 * (v - 1)) * a.n + i];
            const double xn1 = (double)a.x_nb[(int64_t)(2 * (v - 1) + 1) * a.n + i];
            double u, w, z;
            project_px(a.views[v].P, bX, u, w, z);
            const double du = u - xn0, dv = w - xn1;
            if (sqrt(du * du + dv * dv) < a.max_reproj) support |= 1u << v;
        }
    }
    const int m = __popc(support);
    constexpr int NS = GSR_SEED_MAX_NEIGHBOURS + 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double smp[NS];
#pragma unroll
        for (int v = 0; v < NS; ++v) {
            smp[v] = INFINITY;
            if ((support >> v) & 1u) {
                const double px = v == 0 ? xr[0] : (double)a.x_nb[(int64_t)(2 * (v - 1)) * a.n + i];
                const double py = v == 0 ? xr[1] : (double)a.x_nb[(int64_t)(2 * (v - 1) + 1) * a.n + i];
                const SeedView& vw = a.views[v];
                smp[v] = (bilinear(vw, c, px, py) - vw.bias) / vw.gain;
            }
        }
#pragma unroll
        for (int round = 0; round < NS; ++round) {
#pragma unroll
            for (int j = round & 1; j + 1 < NS; j += 2) {
                const double lo = fmin(smp[j], smp[j + 1]), hi = fmax(smp[j], smp[j + 1]);
                smp[j] = lo;
                smp[j + 1] = hi;
            }
        }
        double lo_mid = 0.0, hi_mid = 0.0;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            if (j == (m - 1) / 2) lo_mid = smp[j];
            if (j == m / 2) hi_mid = smp[j];
        }
        const double med = m == 0 ? 0.0 : ((m & 1) ? hi_mid : (lo_mid + hi_mid) / 2.0);
        a.colour[(int64_t)c * a.n + i] = (float)med;
    }
}

hipError_t launch_seed_triangulate(const SeedArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const int64_t blocks = (a.n + GSR_SEED_THREADS - 1) / GSR_SEED_THREADS;
    hipLaunchKernelGGL(k_seed_triangulate, dim3((unsigned)blocks), dim3(GSR_SEED_THREADS), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// nearest-neighbour scale

// per-block bounds of the kept seeds and their count
__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_bbox(KnnArgs a)
{
    __shared__ float red[7][GSR_SEED_THREADS / 64];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float cnt = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x; i < a.n;
         i += (int64_t)GSR_KNN_BLOCKS * GSR_SEED_THREADS) {
        if (!a.valid[i]) continue;
        cnt += 1.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float x = a.mean[(int64_t)c * a.n + i];
            lo[c] = fminf(lo[c], x);
            hi[c] = fmaxf(hi[c], x);
        }
    }
    // counts reach at most n / GSR_KNN_BLOCKS per block: exact in float for
    // any n below 2^24 * GSR_KNN_BLOCKS
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], __shfl_xor(lo[c], off, 64));
            hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], off, 64));
        }
        cnt += __shfl_xor(cnt, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            red[c][w] = lo[c];
            red[3 + c][w] = hi[c];
        }
        red[6][w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        const int k = threadIdx.x;
        float r = red[k][0];
        for (int j = 1; j < GSR_SEED_THREADS / 64; ++j)
            r = k < 3 ? fminf(r, red[k][j]) : (k < 6 ? fmaxf(r, red[k][j]) : r + red[k][j]);
        a.bpart[(int64_t)blockIdx.x * 8 + k] = r;
    }
}

// the coarse grid: origin, cell size and dimensions from the blocks' bounds
__global__ void k_seed_grid(KnnArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double cnt = 0.0;
    for (int b = 0; b < GSR_KNN_BLOCKS; ++b) {
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], a.bpart[b * 8 + c]);
            hi[c] = fmaxf(hi[c], a.bpart[b * 8 + 3 + c]);
        }
        cnt += a.bpart[b * 8 + 6];
    }
    *a.bf_count = 0u;
    KnnGrid g{};
    g.count = (int64_t)cnt;
    g.fine = 0;
    g.h1 = 1.0;
    g.inv_h1 = 1.0;
    if (g.count == 0) {
        g.dims[0] = g.dims[1] = g.dims[2] = 1;
        g.cells = 1;
        g.h = 1.0;
        *a.grid = g;
        return;
    }
    double ext[3], vol = 1.0;
    for (int c = 0; c < 3; ++c) {
        ext[c] = fmax((double)hi[c] - (double)lo[c], 0.0);
        g.origin[c] = (double)lo[c];
    }
    const double maxext = fmax(ext[0], fmax(ext[1], ext[2]));
    double h = maxext > 0.0 ? maxext : 1.0;
    for (int c = 0; c < 3; ++c) vol *= fmax(ext[c], 1e-6 * h);
    h = fmax(cbrt(vol / (double)g.count), 1e-6 * h);
    // coarsen until the grid fits; non-finite extents (the caller's means
    // must be finite) end in a single cell
    g.cells = 0;
    for (int it = 0; it < 256 && isfinite(h); ++it) {
        int64_t cells = 1;
        for (int c = 0; c < 3; ++c) {
            g.dims[c] = (int)fmin(fmax(floor(ext[c] / h) + 1.0, 1.0), 1e6);
            cells *= g.dims[c];
        }
        if (cells <= a.max_cells) {
            g.cells = cells;
            break;
        }
        h *= 1.25;
    }
    if (g.cells == 0) {
        g.dims[0] = g.dims[1] = g.dims[2] = 1;
        g.cells = 1;
        h = 1.0;
    }
    g.h = h;
    *a.grid = g;
}

__device__ __forceinline__ int cell_coord(const KnnGrid& g, int c, float x)
{
    const double k = floor(((double)x - g.origin[c]) / g.h);
    if (!(k > 0.0)) return 0;  // also NaN
    return k >= (double)(g.dims[c] - 1) ? g.dims[c] - 1 : (int)k;
}

// cell coordinate on fine level l (unbounded grid, clamped to +-2^30); the
// level's inverse cell size is inv_h1 / 2^l, exact in binary
__device__ __forceinline__ int fine_coord(const KnnGrid& g, int l, int c, float x)
{
    const double k = floor(((double)x - g.origin[c]) * (g.inv_h1 * ldexp(1.0, -l)));
    if (!(k > -1073741824.0)) return -1073741824;  // also NaN
    return k < 1073741824.0 ? (int)k : 1073741824;
}

__device__ __forceinline__ uint32_t fine_bucket(int x, int y, int z, uint32_t mask)
{
    return (((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349663u) ^ ((uint32_t)z * 83492791u)) & mask;
}

__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_zero(KnnArgs a)
{
    const KnnGrid g = *a.grid;
    const int64_t T1 = ((int64_t)1 << a.table_bits) + 1;
    for (int64_t c = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x; c <= g.cells || c < GSR_KNN_LEVELS * T1;
         c += (int64_t)gridDim.x * GSR_SEED_THREADS) {
        if (c <= g.cells) a.cell_count[c] = 0u;
        if (c < GSR_KNN_LEVELS * T1) a.fine_count[c] = 0u;
    }
}

// rank of this lane's entry in counters[key], with one atomic per distinct
// key of the wave (its lanes of equal key take consecutive ranks): many
// seeds share a cell of a coarse level, and one atomic each would serialise
// on its counter
__device__ __forceinline__ uint32_t wave_rank_add(uint32_t* counters, uint32_t key)
{
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(1);
    uint32_t rank = 0u;
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const uint32_t lead_key = __shfl(key, leader, 64);
        const uint64_t same = __ballot(key == lead_key);
        uint32_t base = 0u;
        if (lane == leader) base = atomicAdd(&counters[lead_key], (uint32_t)__popcll(same));
        base = __shfl(base, leader, 64);
        if (key == lead_key) rank = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
        pending &= ~same;
    }
    return rank;
}

__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_count(KnnArgs a)
{
    const KnnGrid g = *a.grid;
    const int64_t i = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x;
    if (i >= a.n || !a.valid[i]) return;
    int cc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) cc[c] = cell_coord(g, c, a.mean[(int64_t)c * a.n + i]);
    const uint32_t cell = (uint32_t)(((int64_t)cc[2] * g.dims[1] + cc[1]) * g.dims[0] + cc[0]);
    a.cell_of[i] = cell;
    a.rank[i] = wave_rank_add(a.cell_count, cell);
}

// sum over coarse cells of count^2 (per block), the seeds' mean cell sharing
__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_occ(KnnArgs a)
{
    __shared__ double red[GSR_SEED_THREADS / 64];
    const KnnGrid g = *a.grid;
    double s = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x; c < g.cells;
         c += (int64_t)GSR_KNN_BLOCKS * GSR_SEED_THREADS) {
        const double k = (double)a.cell_count[c];
        s += k * k;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int j = 0; j < GSR_SEED_THREADS / 64; ++j) t += red[j];
        a.opart[blockIdx.x] = t;
    }
}

// the fine grid's cell size (or none), one thread
__global__ void k_seed_fine_grid(KnnArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    KnnGrid g = *a.grid;
    double s = 0.0;
    for (int b = 0; b < GSR_KNN_BLOCKS; ++b) s += a.opart[b];
    const double occ = g.count > 0 ? s / (double)g.count : 0.0;
    if (g.count >= 8 && occ > 8.0) {
        g.fine = 1;
        g.h1 = fmax(g.h * sqrt(4.0 / occ), 1e-3 * g.h);
        g.inv_h1 = 1.0 / g.h1;
    }
    *a.grid = g;
}

__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_fcount(KnnArgs a)
{
    const KnnGrid g = *a.grid;
    const int64_t i = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x;
    if (!g.fine || i >= a.n || !a.valid[i]) return;
    const int64_t T1 = ((int64_t)1 << a.table_bits) + 1;
    const uint32_t mask = ((uint32_t)1 << a.table_bits) - 1u;
    const int levels = a.fine_levels > 0 ? a.fine_levels : GSR_KNN_LEVELS;
    for (int l = 0; l < levels; ++l) {
        const uint32_t b = fine_bucket(fine_coord(g, l, 0, a.mean[i]), fine_coord(g, l, 1, a.mean[a.n + i]),
                                       fine_coord(g, l, 2, a.mean[2 * a.n + i]), mask);
        a.fine_of[l * a.n + i] = b;
        a.fine_rank[l * a.n + i] = wave_rank_add(a.fine_count + l * T1, b);
    }
}

// exclusive scan of len counts (len = coarse cells + 1, or table size + 1):
// per 1024-entry block, then the block totals, then their offsets
__device__ __forceinline__ int64_t scan_len(const KnnArgs& a, int which)
{
    return which == 0 ? a.grid->cells + 1 : ((int64_t)1 << a.table_bits) + 1;
}

__device__ __forceinline__ const uint32_t* scan_in(const KnnArgs& a, int which)
{
    return which == 0 ? a.cell_count : a.fine_count + (int64_t)(which - 1) * (((int64_t)1 << a.table_bits) + 1);
}

__device__ __forceinline__ uint32_t* scan_out(const KnnArgs& a, int which)
{
    return which == 0 ? a.cell_start : a.fine_start + (int64_t)(which - 1) * (((int64_t)1 << a.table_bits) + 1);
}

__global__ __launch_bounds__(1024) void k_scan_local(KnnArgs a, int which)
{
    __shared__ uint32_t wsum[16];
    const int64_t len = scan_len(a, which);
    if (which > 0 && !a.grid->fine) return;
    const int64_t base = (int64_t)blockIdx.x * 1024;
    if (base >= len) return;
    const uint32_t* cnt = scan_in(a, which);
    uint32_t* out = scan_out(a, which);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t c = base + tid;
    const uint32_t x = c < len ? cnt[c] : 0u;
    uint32_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t wofs = 0;
    for (int k = 0; k < w; ++k) wofs += wsum[k];
    if (c < len) out[c] = wofs + incl - x;
    if (tid == 1023) a.scan_tot[blockIdx.x] = wofs + incl;
}

__global__ __launch_bounds__(1024) void k_scan_totals(KnnArgs a, int which)
{
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry;
    if (which > 0 && !a.grid->fine) return;
    const int64_t nb = (scan_len(a, which) + 1023) / 1024;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry = 0u;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t c = base + tid;
        const uint32_t x = c < nb ? a.scan_tot[c] : 0u;
        uint32_t incl = x;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t wofs = 0;
        for (int k = 0; k < w; ++k) wofs += wsum[k];
        const uint32_t start = carry + wofs + incl - x;
        if (c < nb) a.scan_tot[c] = start;
        __syncthreads();
        if (tid == 1023) carry = start + x;
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_scan_add(KnnArgs a, int which)
{
    if (which > 0 && !a.grid->fine) return;
    const int64_t len = scan_len(a, which);
    const int64_t c = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (c >= len) return;
    uint32_t* out = scan_out(a, which);
    out[c] += a.scan_tot[blockIdx.x];
}

__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_place(KnnArgs a)
{
    const KnnGrid g = *a.grid;
    const int64_t i = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x;
    if (i >= a.n) return;
    if (!a.valid[i]) {
        if (a.log_scale)
#pragma unroll
            for (int c = 0; c < 3; ++c) a.log_scale[(int64_t)c * a.n + i] = 0.0f;
        if (a.nn_index) a.nn_index[i] = -1;
        return;
    }
    // the seed's position travels with its index, so that a query reads one
    // 16-byte record per candidate, in bucket order
    const float4 q = make_float4(a.mean[i], a.mean[a.n + i], a.mean[2 * a.n + i], __uint_as_float((uint32_t)i));
    const int64_t pos = a.cell_start[a.cell_of[i]] + a.rank[i];
    a.sorted[pos] = (uint32_t)i;
    a.cell_pts[pos] = q;
    if (g.fine) {
        const int64_t T1 = ((int64_t)1 << a.table_bits) + 1;
        const int levels = a.fine_levels > 0 ? a.fine_levels : GSR_KNN_LEVELS;
        for (int l = 0; l < levels; ++l)
            a.fine_pts[l * a.n + a.fine_start[l * T1 + a.fine_of[l * a.n + i]] + a.fine_rank[l * a.n + i]] = q;
    }
}

// (distance, index) pairs ordered by distance, then index: the 3 nearest
// are unique even among equal distances
__device__ __forceinline__ bool knn_before(double d, uint32_t j, double bd, uint32_t bj)
{
    return d < bd || (d == bd && j < bj);
}

__device__ __forceinline__ void knn_insert(double d, uint32_t idx, double (&best)[3], uint32_t (&bidx)[3],
                                           int& found)
{
    int j;
    if (found < 3) {
        j = found++;
    } else if (knn_before(d, idx, best[2], bidx[2])) {
        j = 2;
    } else {
        return;
    }
    while (j > 0 && knn_before(d, idx, best[j - 1], bidx[j - 1])) {
        best[j] = best[j - 1];
        bidx[j] = bidx[j - 1];
        --j;
    }
    best[j] = d;
    bidx[j] = idx;
}

__device__ __forceinline__ void knn_candidate(const float4& q, int64_t i, float px, float py, float pz,
                                              double (&best)[3], uint32_t (&bidx)[3], int& found)
{
    const uint32_t j = __float_as_uint(q.w);
    if ((int64_t)j == i) return;
    if (found == 3) {
        // FP32 prefilter: its squared distance is within 3e-7 relative of
        // the double one, so beyond the third-best by 1e-5 relative it is
        // strictly farther in double and could not be inserted
        const float fx = q.x - px, fy = q.y - py, fz = q.z - pz;
        if (fx * fx + fy * fy + fz * fz > (float)best[2] * 1.00001f) return;
    }
    const double ex = (double)q.x - (double)px;
    const double ey = (double)q.y - (double)py;
    const double ez = (double)q.z - (double)pz;
    knn_insert(ex * ex + ey * ey + ez * ez, j, best, bidx, found);
}

// the query's outputs: its log-scale (when asked for) and its nearest
// other seed (when asked for; -1 for none)
__device__ __forceinline__ void knn_write(const KnnArgs& a, int64_t i, const double (&best)[3],
                                          const uint32_t (&bidx)[3], int found)
{
    if (a.log_scale) {
        double mean_d = 0.0;
        for (int k = 0; k < found; ++k) mean_d += sqrt(best[k]);
        const double sc = found ? fmax(mean_d / (double)found, (double)a.floor_scale) : (double)a.floor_scale;
        const float ls = (float)log(sc);
#pragma unroll
        for (int c = 0; c < 3; ++c) a.log_scale[(int64_t)c * a.n + i] = ls;
    }
    if (a.nn_index) a.nn_index[i] = found ? (int32_t)bidx[0] : -1;
}

#define GSR_KNN_FINE_SHELLS 2
#define GSR_KNN_COARSE_SHELLS 2
#define GSR_KNN_BUDGET 2048

// one thread per valid seed, taken in coarse-cell order so that a wave's
// queries are spatial neighbours with similar search costs
__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_knn(KnnArgs a)
{
    const KnnGrid g = *a.grid;
    const int64_t t = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x;
    if (t >= g.count) return;
    const int64_t i = a.sorted[t];
    const float px = a.mean[i], py = a.mean[a.n + i], pz = a.mean[2 * a.n + i];
    double best[3] = {INFINITY, INFINITY, INFINITY};  // squared distances, ascending
    uint32_t bidx[3] = {0u, 0u, 0u};
    int found = 0;
    bool settled = false;
    uint32_t work = 0;  // candidates examined on this lane
    if (g.fine) {
        // shells of each fine level, finest first; a bucket's entries count
        // only for their own cell
        const uint32_t mask = ((uint32_t)1 << a.table_bits) - 1u;
        const int64_t T1 = ((int64_t)1 << a.table_bits) + 1;
        // seeds of the coarse cell spread over a surface: spacing ~ h / sqrt(count)
        const double cnt = (double)a.cell_count[a.cell_of[i]];
        const double lv = floor(log2(g.h / sqrt(fmax(cnt, 1.0)) * g.inv_h1));
        const int l0 = lv > 0.0 ? (int)fmin(lv, (double)(GSR_KNN_LEVELS - 1)) : 0;
        for (int l = l0; l < GSR_KNN_LEVELS && !settled; ++l) {
            found = 0;
            best[0] = best[1] = best[2] = INFINITY;
            const uint32_t* start = a.fine_start + l * T1;
            const float4* pts = a.fine_pts + l * a.n;
            const double hl = g.h1 * ldexp(1.0, l);
            const int fx = fine_coord(g, l, 0, px), fy = fine_coord(g, l, 1, py), fz = fine_coord(g, l, 2, pz);
            // shells 0 and 1 together (shell 0 alone never settles): the 27
            // cells around the seed's, a z-slab of 9 at a time with their
            // bucket bounds loaded together, so that the loads overlap
            // instead of forming a chain of dependent round trips
            for (int dz = -1; dz <= 1; ++dz) {
                uint32_t lo[9], hi[9];
#pragma unroll
                for (int c = 0; c < 9; ++c) {
                    const uint32_t b = fine_bucket(fx + c % 3 - 1, fy + c / 3 - 1, fz + dz, mask);
                    lo[c] = start[b];
                    hi[c] = start[b + 1];
                }
#pragma unroll
                for (int c = 0; c < 9; ++c) {
                    const int x = fx + c % 3 - 1, y = fy + c / 3 - 1, z = fz + dz;
                    work += hi[c] - lo[c];
                    if (work > GSR_KNN_BUDGET) goto exhaustive;
                    for (uint32_t s = lo[c]; s < hi[c]; ++s) {
                        const float4 q = pts[s];
                        if (fine_coord(g, l, 0, q.x) != x || fine_coord(g, l, 1, q.y) != y ||
                            fine_coord(g, l, 2, q.z) != z)
                            continue;
                        knn_candidate(q, i, px, py, pz, best, bidx, found);
                    }
                }
            }
            // a seed beyond shell r lies, along some axis, at least
            // (r + the query's distance to its own cell's nearer face, in
            // cells) cell sizes away
            double mrg = 0.5;
            {
                const float pc[3] = {px, py, pz};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double t = ((double)pc[c] - g.origin[c]) * (g.inv_h1 * ldexp(1.0, -l));
                    const double f = t - floor(t);
                    mrg = fmin(mrg, fmin(f, 1.0 - f));
                }
                const double lim = (1.0 + mrg) * hl * (1.0 - 1e-12);
                settled = found == 3 && best[2] <= lim * lim;
            }
            for (int r = 2; r <= GSR_KNN_FINE_SHELLS && !settled; ++r) {
                for (int dz = -r; dz <= r; ++dz) {
                    for (int dy = -r; dy <= r; ++dy) {
                        const bool face = dz == -r || dz == r || dy == -r || dy == r;
                        for (int dx = -r; dx <= r; dx += face ? 1 : max(2 * r, 1)) {
                            const int x = fx + dx, y = fy + dy, z = fz + dz;
                            const uint32_t b = fine_bucket(x, y, z, mask);
                            const uint32_t s0 = start[b], s1 = start[b + 1];
                            work += s1 - s0;
                            if (work > GSR_KNN_BUDGET) goto exhaustive;
                            for (uint32_t s = s0; s < s1; ++s) {
                                const float4 q = pts[s];
                                if (fine_coord(g, l, 0, q.x) != x || fine_coord(g, l, 1, q.y) != y ||
                                    fine_coord(g, l, 2, q.z) != z)
                                    continue;
                                knn_candidate(q, i, px, py, pz, best, bidx, found);
                            }
                        }
                    }
                }
                const double lim = ((double)r + mrg) * hl * (1.0 - 1e-12);
                settled = found == 3 && best[2] <= lim * lim;
            }
        }
        if (!settled) {
            found = 0;
            best[0] = best[1] = best[2] = INFINITY;
        }
    }
    if (!settled) {
        const int cx = cell_coord(g, 0, px), cy = cell_coord(g, 1, py), cz = cell_coord(g, 2, pz);
        const int rmax = max(g.dims[0], max(g.dims[1], g.dims[2]));
        for (int r = 0; r <= min(rmax, GSR_KNN_COARSE_SHELLS) && !settled; ++r) {
            // the cells of the shell at Chebyshev distance r that lie in the grid
            const int z0 = max(-r, -cz), z1 = min(r, g.dims[2] - 1 - cz);
            const int y0 = max(-r, -cy), y1 = min(r, g.dims[1] - 1 - cy);
            const int x0 = max(-r, -cx), x1 = min(r, g.dims[0] - 1 - cx);
            for (int dz = z0; dz <= z1; ++dz) {
                for (int dy = y0; dy <= y1; ++dy) {
                    const bool face = dz == -r || dz == r || dy == -r || dy == r;
                    // on a face every dx, otherwise only the two ends dx = -r, r
                    for (int dx = face ? x0 : -r; dx <= (face ? x1 : r); dx += face ? 1 : max(2 * r, 1)) {
                        if (dx < x0 || dx > x1) continue;
                        const uint32_t cell =
                            (uint32_t)(((int64_t)(cz + dz) * g.dims[1] + (cy + dy)) * g.dims[0] + (cx + dx));
                        const uint32_t s0 = a.cell_start[cell], s1 = a.cell_start[cell + 1];
                        work += s1 - s0;
                        if (work > GSR_KNN_BUDGET) goto exhaustive;
                        for (uint32_t s = s0; s < s1; ++s)
                            knn_candidate(a.cell_pts[s], i, px, py, pz, best, bidx, found);
                    }
                }
            }
            // every seed in a farther shell lies at least r * h away; shell
            // rmax has covered the whole grid
            settled = r >= rmax || (found == 3 && best[2] <= ((double)r * g.h) * ((double)r * g.h));
        }
        if (!settled) goto exhaustive;
    }
    knn_write(a, i, best, bidx, found);
    return;
exhaustive:
    a.bf_list[atomicAdd(a.bf_count, 1u)] = (uint32_t)i;
}

// the listed queries, one block each (grid-stride over the list): every
// thread keeps the 3 nearest of its share of the valid seeds, then thread 0
// merges the block's candidates
__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_brute(KnnArgs a)
{
    __shared__ double cand[GSR_SEED_THREADS * 3];
    __shared__ uint32_t cand_i[GSR_SEED_THREADS * 3];
    const KnnGrid g = *a.grid;
    const uint32_t nq = *a.bf_count;
    for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int64_t i = a.bf_list[q];
        const float px = a.mean[i], py = a.mean[a.n + i], pz = a.mean[2 * a.n + i];
        double best[3] = {INFINITY, INFINITY, INFINITY};
        uint32_t bidx[3] = {0u, 0u, 0u};
        int found = 0;
        for (int64_t t = threadIdx.x; t < g.count; t += GSR_SEED_THREADS)
            knn_candidate(a.cell_pts[t], i, px, py, pz, best, bidx, found);
        for (int k = 0; k < 3; ++k) {
            cand[threadIdx.x * 3 + k] = k < found ? best[k] : INFINITY;
            cand_i[threadIdx.x * 3 + k] = bidx[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double b[3] = {INFINITY, INFINITY, INFINITY};
            uint32_t bi[3] = {0u, 0u, 0u};
            int f = 0;
            for (int k = 0; k < GSR_SEED_THREADS * 3; ++k)
                if (cand[k] < INFINITY) knn_insert(cand[k], cand_i[k], b, bi, f);
            knn_write(a, i, b, bi, f);
        }
        __syncthreads();
    }
}

// ---- anisotropic initialisation, Eq. (app-sigma-init) ----------------------
// One thread per seed.  The seeds are hashed by cells of exactly `radius`
// (the first level of the fine grid, unbounded), so the seeds within the
// radius lie in the 3 x 3 x 3 cells around the seed's own, whose distinct
// buckets are scanned once each.
// Their first and second moments about the seed (double) give
// the scatter about their mean; its eigenvector of the smallest eigenvalue
// is the plane normal v, that of the largest t1, and t2 = v x t1 (with fewer
// than three seeds: v the reference viewing ray, t1 any perpendicular).
// s_perp = det(J J^T)^(-1/4), J the reference projection's 2 x 3 Jacobian
// at the seed (the equal-area radius of the back-projected one-pixel
// footprint); s_par = c_par s_perp max(1, err) / max(sin angle, 1e-6); both
// floored.  Output: the unit quaternion of [t1 t2 v] and the log-scales
// (s_perp, s_perp, s_par).  The neighbour moments and the fit run in two
// kernels, so that the latency-bound search keeps few registers.

// the frame's hash grid: fine cells of exactly the radius
__global__ void k_seed_frame_grid(KnnArgs a, double radius)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    KnnGrid g = *a.grid;
    if (g.count > 0) {
        g.fine = 1;
        g.h1 = radius;
        g.inv_h1 = 1.0 / radius;
    }
    *a.grid = g;
}

static_assert(16 * (GSR_KNN_LEVELS - 1) >= 80, "the frame's moments need 80 bytes per seed in fine levels 1..");

__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_frame(KnnArgs a, FrameArgs f)
{
    const int64_t t = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x;
    const int64_t n = a.n;
    if (t < n && !a.valid[t]) {
        f.quat[t] = 1.0f;
#pragma unroll
        for (int k = 1; k < 4; ++k) f.quat[k * n + t] = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) f.log_scale[k * n + t] = 0.0f;
    }
    // thread t takes the t-th valid seed in cell order: the lanes of a wave
    // read the same buckets and have neighbourhoods of similar size
    const KnnGrid g = *a.grid;
    if (t >= g.count) return;
    const float4 self = a.fine_pts[t];
    const float p[3] = {self.x, self.y, self.z};
    const double r2 = f.radius * f.radius;
    const uint32_t mask = ((uint32_t)1 << a.table_bits) - 1u;
    int c0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) c0[c] = fine_coord(g, 0, c, p[c]);
    double cnt = 0.0, m1[3] = {0.0, 0.0, 0.0}, m2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // the buckets of the 27 cells, each visited once: a seed within the
    // radius lies in one of the cells, and seeds of other cells that share
    // a bucket fail the distance test
    uint32_t bk[27];
#pragma unroll
    for (int c = 0; c < 27; ++c) bk[c] = fine_bucket(c0[0] + c % 3 - 1, c0[1] + (c / 3) % 3 - 1, c0[2] + c / 9 - 1, mask);
    // FP32 prefilter: its squared distance is within 3e-7 relative of the
    // double one, so a candidate beyond r^2 (1 + 1e-5) in FP32 is beyond r^2
    const float cut = (float)(r2 * (1.0 + 1e-5));
#pragma unroll
    for (int c = 0; c < 27; ++c) {
        bool dup = false;
#pragma unroll
        for (int j = 0; j < c; ++j) dup |= bk[j] == bk[c];
        if (dup) continue;
        const uint32_t e = a.fine_start[bk[c] + 1];
        for (uint32_t k = a.fine_start[bk[c]]; k < e; ++k) {
            const float4 q = a.fine_pts[k];
            const float fx = q.x - p[0], fy = q.y - p[1], fz = q.z - p[2];
            if (fx * fx + fy * fy + fz * fz > cut) continue;
            const double ex = (double)q.x - (double)p[0];
            const double ey = (double)q.y - (double)p[1];
            const double ez = (double)q.z - (double)p[2];
            if (ex * ex + ey * ey + ez * ez <= r2) {
                cnt += 1.0;
                m1[0] += ex;
                m1[1] += ey;
                m1[2] += ez;
                m2[0] += ex * ex;
                m2[1] += ex * ey;
                m2[2] += ex * ez;
                m2[3] += ey * ey;
                m2[4] += ey * ez;
                m2[5] += ez * ez;
            }
        }
    }
    // the moments go to the unused fine levels 1.. of the record buffer
    // ([10][count] doubles; levels 1 to 7 hold 112 bytes per seed)
    double* mom = reinterpret_cast<double*>(a.fine_pts + a.n);
    const int64_t cnt_all = g.count;
    mom[t] = cnt;
#pragma unroll
    for (int c = 0; c < 3; ++c) mom[(1 + c) * cnt_all + t] = m1[c];
#pragma unroll
    for (int c = 0; c < 6; ++c) mom[(4 + c) * cnt_all + t] = m2[c];
}

// the plane fit and the scales of the t-th valid seed in cell order, from
// the moments k_seed_frame left
__global__ __launch_bounds__(GSR_SEED_THREADS) void k_seed_frame_fit(KnnArgs a, FrameArgs f)
{
    const int64_t t = (int64_t)blockIdx.x * GSR_SEED_THREADS + threadIdx.x;
    const int64_t n = a.n;
    const KnnGrid g = *a.grid;
    if (t >= g.count) return;
    const float4 self = a.fine_pts[t];
    const int64_t i = (int64_t)__float_as_uint(self.w);
    const float p[3] = {self.x, self.y, self.z};
    const double* mom = reinterpret_cast<const double*>(a.fine_pts + a.n);
    const int64_t cnt_all = g.count;
    const double cnt = mom[t];
    double m1[3], m2[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) m1[c] = mom[(1 + c) * cnt_all + t];
#pragma unroll
    for (int c = 0; c < 6; ++c) m2[c] = mom[(4 + c) * cnt_all + t];
    double v[3], t1[3];
    if (cnt >= 3.0) {
        const double ic = 1.0 / cnt;
        double S[3][3], V[3][3], lam[3];
        S[0][0] = m2[0] - m1[0] * m1[0] * ic;
        S[0][1] = S[1][0] = m2[1] - m1[0] * m1[1] * ic;
        S[0][2] = S[2][0] = m2[2] - m1[0] * m1[2] * ic;
        S[1][1] = m2[3] - m1[1] * m1[1] * ic;
        S[1][2] = S[2][1] = m2[4] - m1[1] * m1[2] * ic;
        S[2][2] = m2[5] - m1[2] * m1[2] * ic;
        eig3(S, V, lam);
        int kmin = 0, kmax = 1;
        if (lam[1] < lam[kmin]) kmin = 1;
        if (lam[2] < lam[kmin]) kmin = 2;
        kmax = kmin == 0 ? 1 : 0;
        for (int k = 0; k < 3; ++k)
            if (k != kmin && lam[k] > lam[kmax]) kmax = k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = V[c][kmin];
            t1[c] = V[c][kmax];
        }
    } else {
        double nv = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = (double)p[c] - f.centre[c];
            nv += v[c] * v[c];
        }
        nv = 1.0 / sqrt(nv);
        int am = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] *= nv;
            if (fabs(v[c]) < fabs(v[am])) am = c;
        }
        // t1 = v x e_am, normalised
        double e[3] = {0.0, 0.0, 0.0};
        e[am] = 1.0;
        t1[0] = v[1] * e[2] - v[2] * e[1];
        t1[1] = v[2] * e[0] - v[0] * e[2];
        t1[2] = v[0] * e[1] - v[1] * e[0];
        const double nt = 1.0 / sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) t1[c] *= nt;
    }
    const double t2[3] = {v[1] * t1[2] - v[2] * t1[1], v[2] * t1[0] - v[0] * t1[2], v[0] * t1[1] - v[1] * t1[0]};
    double U[3][3], q[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        U[c][0] = t1[c];
        U[c][1] = t2[c];
        U[c][2] = v[c];
    }
    rot_quat(U, q);
    // tangential scale from the reference projection's Jacobian
    const double X[3] = {(double)p[0], (double)p[1], (double)p[2]};
    const double* P = f.P;
    const double w = P[8] * X[0] + P[9] * X[1] + P[10] * X[2] + P[11];
    const double u = (P[0] * X[0] + P[1] * X[1] + P[2] * X[2] + P[3]) / w;
    const double vv = (P[4] * X[0] + P[5] * X[1] + P[6] * X[2] + P[7]) / w;
    double j1[3], j2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        j1[c] = (P[c] - u * P[8 + c]) / w;
        j2[c] = (P[4 + c] - vv * P[8 + c]) / w;
    }
    const double A = j1[0] * j1[0] + j1[1] * j1[1] + j1[2] * j1[2];
    const double B = j1[0] * j2[0] + j1[1] * j2[1] + j1[2] * j2[2];
    const double D = j2[0] * j2[0] + j2[1] * j2[1] + j2[2] * j2[2];
    const double s_perp = fmax(pow(A * D - B * B, -0.25), f.floor_scale);
    const double s_par =
        fmax(f.c_par * s_perp * fmax(1.0, (double)f.err[i]) / fmax(sin((double)f.angle[i]), 1e-6), f.floor_scale);
#pragma unroll
    for (int k = 0; k < 4; ++k) f.quat[k * n + i] = (float)q[k];
    f.log_scale[i] = (float)log(s_perp);
    f.log_scale[n + i] = (float)log(s_perp);
    f.log_scale[2 * n + i] = (float)log(s_par);
}

hipError_t launch_seed_frame(const KnnArgs& a, const FrameArgs& f, hipStream_t s)
{
    if (a.n == 0 || a.fine_levels != 1) return a.n == 0 ? hipSuccess : hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((a.n + GSR_SEED_THREADS - 1) / GSR_SEED_THREADS);
    const unsigned coarse_scan = (unsigned)((a.max_cells + 1 + 1023) / 1024);
    const unsigned fine_scan = (unsigned)((((int64_t)1 << a.table_bits) + 1 + 1023) / 1024);
    // the grid build of the nearest-neighbour search, with the fine levels
    // set to cells of the radius instead of the occupancy rule
    hipLaunchKernelGGL(k_seed_bbox, dim3(GSR_KNN_BLOCKS), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_grid, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_seed_zero, dim3(1024), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_count, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_frame_grid, dim3(1), dim3(64), 0, s, a, f.radius);
    hipLaunchKernelGGL(k_seed_fcount, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a);
    for (int which = 0; which <= 1; ++which) {
        const unsigned nb = which == 0 ? coarse_scan : fine_scan;
        hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(1024), 0, s, a, which);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, s, a, which);
        hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, a, which);
    }
    hipLaunchKernelGGL(k_seed_place, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_frame, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a, f);
    hipLaunchKernelGGL(k_seed_frame_fit, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a, f);
    return hipGetLastError();
}

hipError_t launch_seed_scale(const KnnArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.n + GSR_SEED_THREADS - 1) / GSR_SEED_THREADS);
    const unsigned coarse_scan = (unsigned)((a.max_cells + 1 + 1023) / 1024);
    const unsigned fine_scan = (unsigned)((((int64_t)1 << a.table_bits) + 1 + 1023) / 1024);
    hipLaunchKernelGGL(k_seed_bbox, dim3(GSR_KNN_BLOCKS), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_grid, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_seed_zero, dim3(1024), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_count, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_occ, dim3(GSR_KNN_BLOCKS), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_fine_grid, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_seed_fcount, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a);
    for (int which = 0; which <= GSR_KNN_LEVELS; ++which) {
        const unsigned nb = which == 0 ? coarse_scan : fine_scan;
        hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(1024), 0, s, a, which);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, s, a, which);
        hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, a, which);
    }
    hipLaunchKernelGGL(k_seed_place, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_knn, dim3(blocks), dim3(GSR_SEED_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_seed_brute, dim3(1024), dim3(GSR_SEED_THREADS), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
