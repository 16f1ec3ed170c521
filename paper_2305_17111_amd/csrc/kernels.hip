// gfx950 kernels of the list-mode multi-energy-window OSEM (arXiv 2305.17111).
//
// Layout in HBM (all float32 unless noted):
//   pix_xy  [Qp]          support pixels (compacted, padded to a multiple of 64)
//   g_qa    [na][Qp]      attenuation integral pixel -> detector plane at mu_ref
//   g_qs    [nsc][Qp]     attenuation integral pixel -> scatter point at mu_ref
//   sa      [na][nsc]     scatter points as seen from each angle, sorted by u
//   A       [rows][Qp]    per-subset scratch: a_jq for the subset's sorted events
//   part/comp [chunks][Qp] compensated partial backprojections
#include <hip/hip_runtime.h>

#include <cmath>

#include <type_traits>

#include "internal.h"

namespace lmmew {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Complementary error function by the Chebyshev-fitted formula of Numerical
// Recipes (Press et al., 2nd ed., Sec. 6.2, erfcc): erfc(z) = t exp(-z^2 +
// P(t)), t = 1 / (1 + z/2), for z >= 0, and 2 - erfc(-z) below; fractional
// error below 1.2e-7 in exact arithmetic, about 3e-6 when evaluated in FP32
// for |z| < 5.3.  No branches, so lanes of a wavefront never diverge on it.
__device__ __forceinline__ float erfc_cheb(float x)
{
    const float z = fabsf(x);
    const float t = fast_rcp(fmaf(0.5f, z, 1.f));
    float p = 0.17087277f;
    p = fmaf(t, p, -0.82215223f);
    p = fmaf(t, p, 1.48851587f);
    p = fmaf(t, p, -1.13520398f);
    p = fmaf(t, p, 0.27886807f);
    p = fmaf(t, p, -0.18628806f);
    p = fmaf(t, p, 0.09678418f);
    p = fmaf(t, p, 0.37409196f);
    p = fmaf(t, p, 1.00002368f);
    const float arg = fmaf(t, p, fmaf(-z, z, -1.26551223f));
    const float r = t * fast_exp2(arg * kLog2e);
    return x >= 0.f ? r : 2.f - r;
}

// Phi(zhi) - Phi(zlo) for the standard normal CDF = (erfc(zlo/sqrt2) -
// erfc(zhi/sqrt2)) / 2.  When both edges lie below the centre the mirrored
// form (erfc(-zhi/sqrt2) - erfc(-zlo/sqrt2)) / 2 avoids subtracting two values
// near 2; otherwise (both above, or straddling) the direct form is exact up to
// rounding.  A select, not a branch.
__device__ __forceinline__ float phi_diff(float zhi, float zlo)
{
    const float r2 = 0.70710678118654752f;
    const bool below = zhi <= 0.f;
    const float a = (below ? -zhi : zlo) * r2;
    const float b = (below ? -zlo : zhi) * r2;
    return 0.5f * (erfc_cheb(a) - erfc_cheb(b));
}

// Collimator-response probability of a bin whose edges are zhi, zlo standard
// deviations from the projected point; exactly 0 when the whole bin lies
// beyond kPsfCut standard deviations.
__device__ __forceinline__ float psf_cut(float zhi, float zlo)
{
    const float p = phi_diff(zhi, zlo);
    return (zlo >= kPsfCut || zhi <= -kPsfCut) ? 0.f : p;
}

// Collimator-response density per mm at a continuous position whose
// deviation from the projected point is z standard deviations (isig = 1 /
// sigma); exactly 0 beyond kPsfCut standard deviations.
__device__ __forceinline__ float pdf_cut(float z, float isig)
{
    const float g = (0.39894228040143268f * isig) * fast_exp2(-0.5f * kLog2e * z * z);
    return (z >= kPsfCut || z <= -kPsfCut) ? 0.f : g;
}

__device__ __forceinline__ float uniform_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// ---------------------------------------------------------------------------
// attenuation line integrals (Eq. (6)), double precision, Amanatides-Woo walk
// ---------------------------------------------------------------------------

// Integral of the pixel map over the segment (x0,y0)->(x1,y1), walking the
// cells the segment crosses in order.
__device__ double walk_segment(const double *mu, int n, double pix, double R, double x0,
                               double y0, double x1, double y1)
{
    const double dx = x1 - x0, dy = y1 - y0;
    const double L = sqrt(dx * dx + dy * dy);
    if (L == 0.0) return 0.0;
    double tmin = 0.0, tmax = 1.0;
    if (dx != 0.0) {
        double ta = (-R - x0) / dx, tb = (R - x0) / dx;
        tmin = fmax(tmin, fmin(ta, tb));
        tmax = fmin(tmax, fmax(ta, tb));
    } else if (x0 < -R || x0 > R) {
        return 0.0;
    }
    if (dy != 0.0) {
        double ta = (-R - y0) / dy, tb = (R - y0) / dy;
        tmin = fmax(tmin, fmin(ta, tb));
        tmax = fmin(tmax, fmax(ta, tb));
    } else if (y0 < -R || y0 > R) {
        return 0.0;
    }
    if (!(tmax > tmin)) return 0.0;
    const double xs = x0 + tmin * dx, ys = y0 + tmin * dy;
    const double fx = (xs + R) / pix, fy = (ys + R) / pix;
    // cell entered in the direction of travel
    int ix = (dx >= 0.0) ? (int)floor(fx) : (int)ceil(fx) - 1;
    int iy = (dy >= 0.0) ? (int)floor(fy) : (int)ceil(fy) - 1;
    ix = min(max(ix, 0), n - 1);
    iy = min(max(iy, 0), n - 1);
    const int sx = dx > 0.0 ? 1 : -1, sy = dy > 0.0 ? 1 : -1;
    double tX = INFINITY, tY = INFINITY, dX = INFINITY, dY = INFINITY;
    if (dx != 0.0) {
        double xb = (dx > 0.0 ? (ix + 1) : ix) * pix - R;
        tX = (xb - x0) / dx;
        dX = pix / fabs(dx);
    }
    if (dy != 0.0) {
        double yb = (dy > 0.0 ? (iy + 1) : iy) * pix - R;
        tY = (yb - y0) / dy;
        dY = pix / fabs(dy);
    }
    double t = tmin, sum = 0.0;
    for (int guard = 0; guard < 4 * n + 4; ++guard) {
        double tn = fmin(fmin(tX, tY), tmax);
        if (tn > t) sum += mu[iy * n + ix] * (tn - t);
        t = tn;
        if (t >= tmax) break;
        if (tX <= tn) { ix += sx; tX += dX; }
        if (tY <= tn) { iy += sy; tY += dY; }
        if (ix < 0 || iy < 0 || ix >= n || iy >= n) break;
    }
    return sum * L;
}

// A segment lying exactly on a grid line sees the mean of the two pixel
// columns (rows) that share the line; the walk along each neighbouring
// column centre gives each of them.
__device__ double seg_integral(const double *mu, int n, double pix, double R, double x0,
                               double y0, double x1, double y1)
{
    if (x0 == x1) {
        double f = (x0 + R) / pix, k = rint(f);
        if (fabs(f - k) < 1e-9) {
            double h = 0.5 * pix;
            return 0.5 * (walk_segment(mu, n, pix, R, x0 - h, y0, x1 - h, y1) +
                          walk_segment(mu, n, pix, R, x0 + h, y0, x1 + h, y1));
        }
    }
    if (y0 == y1) {
        double f = (y0 + R) / pix, k = rint(f);
        if (fabs(f - k) < 1e-9) {
            double h = 0.5 * pix;
            return 0.5 * (walk_segment(mu, n, pix, R, x0, y0 - h, x1, y1 - h) +
                          walk_segment(mu, n, pix, R, x0, y0 + h, x1, y1 + h));
        }
    }
    return walk_segment(mu, n, pix, R, x0, y0, x1, y1);
}

struct TabArgsD {
    const double *mu;
    const double2 *pix;     // [Qp]
    const double2 *dirs;    // [na]
    const double2 *sc;      // [nsc]
    float *g_qa, *g_qs;
    ScatA *sa;
    const double *pixz;     // 3-D: [Qp] voxel z
    const double *scz;      // 3-D: [nsc] scatter-point z
};

// ---- 3-D: voxel maps of nz slices of n x n, flat index (iz*n + iy)*n + ix ----

// Integral of the voxel map over a segment, walking the voxels it crosses in
// order (the segments from voxel centres to scatter points never lie in a
// grid plane: both sit at different offsets from the planes).
__device__ double walk_segment3(const double *mu, int n, int nz, double pix, double R, double Zh,
                                double x0, double y0, double z0, double x1, double y1,
                                double z1)
{
    const double d[3] = {x1 - x0, y1 - y0, z1 - z0};
    const double o[3] = {x0, y0, z0};
    const double lo[3] = {-R, -R, -Zh}, hi[3] = {R, R, Zh};
    const int cells[3] = {n, n, nz};
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (L == 0.0) return 0.0;
    double tmin = 0.0, tmax = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (d[k] != 0.0) {
            const double ta = (lo[k] - o[k]) / d[k], tb = (hi[k] - o[k]) / d[k];
            tmin = fmax(tmin, fmin(ta, tb));
            tmax = fmin(tmax, fmax(ta, tb));
        } else if (o[k] < lo[k] || o[k] > hi[k]) {
            return 0.0;
        }
    }
    if (!(tmax > tmin)) return 0.0;
    int idx[3], step[3];
    double tn[3], dt[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double f = (o[k] + tmin * d[k] - lo[k]) / pix;
        int c = (d[k] >= 0.0) ? (int)floor(f) : (int)ceil(f) - 1;   // cell entered
        c = min(max(c, 0), cells[k] - 1);
        idx[k] = c;
        step[k] = d[k] > 0.0 ? 1 : -1;
        if (d[k] != 0.0) {
            const double b = (d[k] > 0.0 ? c + 1 : c) * pix + lo[k];
            tn[k] = (b - o[k]) / d[k];
            dt[k] = pix / fabs(d[k]);
        } else {
            tn[k] = INFINITY;
            dt[k] = INFINITY;
        }
    }
    double t = tmin, sum = 0.0;
    for (int guard = 0; guard < 2 * (2 * n + nz) + 4; ++guard) {
        const double tnx = fmin(fmin(tn[0], tn[1]), fmin(tn[2], tmax));
        if (tnx > t) sum += mu[((size_t)idx[2] * n + idx[1]) * n + idx[0]] * (tnx - t);
        t = tnx;
        if (t >= tmax) break;
        bool out = false;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (tn[k] <= tnx) {
                idx[k] += step[k];
                tn[k] += dt[k];
                out |= idx[k] < 0 || idx[k] >= cells[k];
            }
        }
        if (out) break;
    }
    return sum * L;
}

__global__ __launch_bounds__(256) void k_tab_qa(const DevSys S, const TabArgsD t, double pix,
                                                double R)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int a = blockIdx.y;
    if (i >= S.Qp) return;
    float v = 0.f;
    if (i < S.Qm) {
        double2 p = t.pix[i], d = t.dirs[a];
        double depth = R - (p.x * d.x + p.y * d.y);
        v = (float)seg_integral(t.mu, S.n, pix, R, p.x, p.y, p.x + depth * d.x, p.y + depth * d.y);
    }
    t.g_qa[(size_t)a * S.Qp + i] = v;
}

__global__ __launch_bounds__(256) void k_tab_qs(const DevSys S, const TabArgsD t, double pix,
                                                double R)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int s = blockIdx.y;
    if (i >= S.Qp) return;
    float v = 0.f;
    if (i < S.Qm) {
        double2 p = t.pix[i], q = t.sc[s];
        v = (float)seg_integral(t.mu, S.n, pix, R, p.x, p.y, q.x, q.y);
    }
    t.g_qs[(size_t)s * S.Qp + i] = v;
}

__global__ __launch_bounds__(256) void k_tab_sa(const DevSys S, const TabArgsD t, double pix,
                                                double R)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int a = blockIdx.y;
    if (k >= S.nsc) return;
    ScatA &e = t.sa[(size_t)a * S.nsc + k];
    double2 q = t.sc[e.sidx], d = t.dirs[a];
    double depth = R - (q.x * d.x + q.y * d.y);
    e.gsa = (float)seg_integral(t.mu, S.n, pix, R, q.x, q.y, q.x + depth * d.x, q.y + depth * d.y);
    double u = -q.x * d.y + q.y * d.x;
    double isig = (double)e.isig;
    double zhi = (R - u) * isig, zlo = (-R - u) * isig;
    const double r2 = 0.70710678118654752;
    double D;
    if (zlo >= 0.0) D = 0.5 * (erfc(zlo * r2) - erfc(zhi * r2));
    else if (zhi <= 0.0) D = 0.5 * (erfc(-zhi * r2) - erfc(-zlo * r2));
    else D = 1.0 - 0.5 * erfc(zhi * r2) - 0.5 * erfc(-zlo * r2);
    e.D = (float)D;
}

// Detector probability of a Gaussian of 1/sigma isig about (u, z) on
// [-R, R] x [-Zh, Zh], in double precision.
__device__ double detector_prob3(double u, double z, double isig, double R, double Zh)
{
    const double r2 = 0.70710678118654752;
    auto pd = [&](double zhi, double zlo) {
        if (zlo >= 0.0) return 0.5 * (erfc(zlo * r2) - erfc(zhi * r2));
        if (zhi <= 0.0) return 0.5 * (erfc(-zhi * r2) - erfc(-zlo * r2));
        return 1.0 - 0.5 * erfc(zhi * r2) - 0.5 * erfc(-zlo * r2);
    };
    return pd((R - u) * isig, (-R - u) * isig) * pd((Zh - z) * isig, (-Zh - z) * isig);
}

// 3-D: voxel -> detector plane, a horizontal segment inside the voxel's slice
__global__ __launch_bounds__(256) void k_tab3_qa(const DevSys S, const TabArgsD t, double pix,
                                                 double R)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int a = blockIdx.y;
    if (i >= S.Qp) return;
    float v = 0.f;
    if (i < S.Qm) {
        const double2 p = t.pix[i], d = t.dirs[a];
        const int iz = (int)floor((t.pixz[i] + (double)S.nz * 0.5 * pix) / pix);
        const double depth = R - (p.x * d.x + p.y * d.y);
        v = (float)seg_integral(t.mu + (size_t)iz * S.n * S.n, S.n, pix, R, p.x, p.y,
                                p.x + depth * d.x, p.y + depth * d.y);
    }
    t.g_qa[(size_t)a * S.Qp + i] = v;
}

// 3-D: voxel -> scatter point
__global__ __launch_bounds__(256) void k_tab3_qs(const DevSys S, const TabArgsD t, double pix,
                                                 double R)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int s = blockIdx.y;
    if (i >= S.Qp) return;
    float v = 0.f;
    if (i < S.Qm) {
        const double2 p = t.pix[i], q = t.sc[s];
        const double Zh = (double)S.nz * 0.5 * pix;
        v = (float)walk_segment3(t.mu, S.n, S.nz, pix, R, Zh, p.x, p.y, t.pixz[i], q.x, q.y,
                                 t.scz[s]);
    }
    t.g_qs[(size_t)s * S.Qp + i] = v;
}

// 3-D: scatter point -> detector plane, a horizontal segment at the point's z.
// A point on a slice boundary sees the mean of the two slices that share it
// (the limit of segments displaced by +-delta; a slice outside the grid
// contributes zero).  Also the point's probability of landing on the detector.
__global__ __launch_bounds__(256) void k_tab3_sa(const DevSys S, const TabArgsD t, double pix,
                                                 double R)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int a = blockIdx.y;
    if (k >= S.nsc) return;
    ScatA &e = t.sa[(size_t)a * S.nsc + k];
    const double2 q = t.sc[e.sidx], d = t.dirs[a];
    const double z = t.scz[e.sidx];
    const double Zh = (double)S.nz * 0.5 * pix;
    const double depth = R - (q.x * d.x + q.y * d.y);
    const double x1 = q.x + depth * d.x, y1 = q.y + depth * d.y;
    const double f = (z + Zh) / pix, kz = rint(f);
    auto slice = [&](int iz) {
        if (iz < 0 || iz >= S.nz) return 0.0;
        return seg_integral(t.mu + (size_t)iz * S.n * S.n, S.n, pix, R, q.x, q.y, x1, y1);
    };
    double g;
    if (fabs(f - kz) < 1e-9)
        g = 0.5 * (slice((int)kz - 1) + slice((int)kz));
    else
        g = slice((int)floor(f));
    e.gsa = (float)g;
    const double u = -q.x * d.y + q.y * d.x;
    e.D = (float)detector_prob3(u, z, (double)e.isig, R, Zh);
}

// ---------------------------------------------------------------------------
// scatter-path parameters of one (pixel, scatter point, angle)
// ---------------------------------------------------------------------------

// For each line w: log2 of the path weight (with or without the energy
// Gaussian's normalisation), the scaled Compton energy sw*E' and sw =
// sqrt(log2(e) / (2 sigma'^2)), so that the energy factor of an event with
// measured energy E is exp2(-(sw*E - Fw)^2).  The planar model's cell
// interaction probability falls as 1/r, the 3-D model's (D3) as 1/r^2.
template <int NW, bool NORM, bool D3 = false, unsigned LM = 0xFFu>
__device__ __forceinline__ void scatter_params(const DevSys &S, float dx, float dy, float dz,
                                               float c, float s, float lc, float gqs, float gsa,
                                               float *Aw, float *sw, float *Fw, float *Ep)
{
    const float r2 = D3 ? fmaf(dz, dz, fmaf(dx, dx, dy * dy)) : dx * dx + dy * dy;
    const float rinv = fast_rsq(r2);
    const float r = r2 * rinv;
    const float reff = fmaxf(r, S.rmin);
    const float cosphi = (dx * c + dy * s) * rinv;
    const float omc = 1.f - cosphi;
    const float sin2 = omc * (1.f + cosphi);
    const float base = D3 ? lc - 2.f * fast_log2(reff) : lc - fast_log2(reff);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (NW == LMMEW_MAX_LINES && w >= S.nw) break;
        if (!((LM >> w) & 1u)) continue;                  // line not needed
        // invP = E_w / E' = 1 + eps (1 - cos phi); rs = invP^(-1/2)
        const float invP = fmaf(S.eps[w], omc, 1.f);
        const float rs = fast_rsq(invP);
        const float P = rs * rs;
        const float l2i = fast_log2(invP);
        // Klein-Nishina: log2(P + 1/P - sin^2) - 2 log2(invP), the normalised
        // Gaussian's 0.5 log2(invP) folded into the same FMA
        const float lkn = fast_log2(fmaf(rs, rs, invP) - sin2);
        // attenuation (log2 units): f_w log2(e) gqs on the way in, and on the
        // way out f(E') log2(e) gsa with f(E') = f_w invP^p, as one exp2 whose
        // exponent carries log2(f_w log2(e)) (the same for every point)
        const float ea = fast_exp2(fmaf(S.mu_pow, l2i, fast_log2(S.f[w] * kLog2e)));
        float A = fmaf(l2i, NORM ? -1.5f : -2.f, base + (NORM ? S.lsc[w] + S.nc[w] : S.lsc[w]));
        A += lkn;
        A = fmaf(-(S.f[w] * kLog2e), gqs, A);
        A = fmaf(-ea, gsa, A);
        Aw[w] = A;
        Ep[w] = S.E[w] * P;
        // sqrt(c0 * invP) = sqc0 * invP * rs ;  F = sqrt(c) * E' = sqc0 * E_w * rs
        sw[w] = S.sqc0[w] * invP * rs;
        Fw[w] = (S.sqc0[w] * S.E[w]) * rs;
    }
}

// Global-address-space views of device pointers.  For generic (flat) loads
// the compiler waits for every outstanding load before it uses any of them;
// for global loads it waits only for those a value depends on.
template <class T> using GPtr = const T __attribute__((address_space(1))) *;
template <class T> __device__ __forceinline__ GPtr<T> global_ptr(const T *p)
{
    return (GPtr<T>)p;
}

__device__ __forceinline__ ScatA load_scat(GPtr<ScatA> p)
{
    ScatA v;
    v.x = p->x;
    v.y = p->y;
    v.u = p->u;
    v.isig = p->isig;
    v.gsa = p->gsa;
    v.lc = p->lc;
    v.D = p->D;
    v.sidx = p->sidx;
    return v;
}

// ---------------------------------------------------------------------------
// per-event system model (the hot path)
//
// One wavefront per work item: 64 support pixels (one per lane) x one tile of
// up to JT events of a single angle, with JT accumulators a_jq per lane in
// registers.  The tile carries the list of scatter points whose collimator
// response reaches at least one of its events, each with the mask of its
// groups of 16 events that the response reaches.  The response factors of
// the listed (point, event) pairs come from the plan's table (k_pv_table)
// through scalar loads, so they sit in scalar registers: a zero factor skips
// the pair's exponentials with a uniform branch, and a group the point does
// not reach is skipped whole.  For each listed point every lane reads or
// derives its pixel's path parameters once and reuses them for all of the
// tile's events.  A tile's events keep the same emission lines (the line
// mask of the plan's line cut): the point loop is compiled once per mask,
// so a tile evaluates, reads and exponentiates only its kept lines.
// ---------------------------------------------------------------------------
template <int JT, int NW, bool TAB, bool D3>
__global__ __launch_bounds__(64) void k_row(const DevSys S, const RowArgs r)
{
    // Work item p = (case, pixel block, tile of the case): case-major, then
    // block-major.  Workgroups go to the 8 XCDs round-robin by id, so XCD k
    // runs ids k, k+8, ...: mapping them to the k-th contiguous eighth of the
    // items gives every XCD an equal share made of few cases and pixel blocks,
    // so the tiles an XCD runs at one time read one map's tables for few
    // pixel blocks, which then stay in its L2.
    const int nb = S.Qp / kWave;
    const int W = nb * r.ntiles;
    const int per = (W + 7) >> 3;
    int p = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (p >= W) return;
    int t0 = 0, nt = r.ntiles;
    if (r.case_tiles) {
        // The items of case c are [nb * case_tiles[c], nb * case_tiles[c+1]),
        // so item p belongs to the case of tile p / nb (tiles are grouped by
        // case): three dependent loads, whatever the number of cases.
        const int c = r.tiles[p / nb].ncase;
        t0 = r.case_tiles[c];
        nt = r.case_tiles[c + 1] - t0;
        p -= nb * t0;
    }
    const int bx = p / nt;
    const Tile T = r.tiles[t0 + p - bx * nt];
    const int lane = threadIdx.x;
    const int i = bx * kWave + lane;
    const int a = T.angle;
    // attenuation tables of the tile's case
    const float *g_qa = r.g_qa, *g_qs_ = r.g_qs, *ptab_ = r.ptab, *resp = r.resp;
    const float *respz = r.respz, *szs_ = r.sz;
    const ScatA *sab_ = r.sa;
    int nsc = S.nsc;
    if (r.maps) {
        const MapTab m = r.maps[T.ncase];
        g_qa = m.g_qa;
        g_qs_ = m.g_qs;
        sab_ = m.sa;
        ptab_ = m.ptab;
        resp = m.resp;
        respz = m.respz;
        szs_ = m.sz;
        nsc = m.nsc;
    }
    // Device tables are global memory: loads through global pointers let the
    // compiler wait for the current point's loads only, not for the next
    // point's as well (it must wait for every outstanding generic load).
    const GPtr<float> g_qs = global_ptr(g_qs_), ptab = global_ptr(ptab_), szs = global_ptr(szs_);
    const GPtr<ScatA> sab = global_ptr(sab_);
    const float2 dir = r.dirs[a];
    const float c = dir.x, s = dir.y;
    const bool valid = i < S.Qm;
    const int last = T.cnt - 1;

    // unscattered energy factor of event `lane` for every line
    float gq[NW];
    {
        const float E = r.ev_E[T.e0 + min(lane, last)];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if (NW == LMMEW_MAX_LINES && w >= S.nw) break;
            const float d = E - S.E[w];
            gq[w] = S.gnorm[w] * __expf(-d * d / (2.f * S.eres_k * S.E[w]));
        }
    }

    const float2 xy = r.pix_xy[i];
    const float xq = xy.x, yq = xy.y;
    const float zq = D3 ? r.pix_z[i] : 0.f;

    // Unscattered paths of event j at this lane's pixel (each row element is
    // written once, at the end).  Tiles of 16 stage them in LDS before the
    // scatter loop; larger tiles form them at the end, which keeps the LDS
    // from limiting how many waves a SIMD holds.
    const float dq = S.R - (xq * c + yq * s);
    const float uq = -xq * s + yq * c;
    const float isq = 1.f / ((S.fwhm0 + S.fslope * dq) * S.inv_fwhm_to_sigma);
    auto prim_of = [&](int j, const float *Pp) {
        float ps = 0.f;
        if (r.mode != 1) {
            if (!D3 && r.psft && !r.ev_u) {
                ps = r.psft[((size_t)a * S.nb + r.ev_bin[T.e0 + j]) * S.Qp + i];
            } else if (r.ev_u) {
                ps = pdf_cut((r.ev_u[T.e0 + j] - uq) * isq, isq);
            } else {
                const float lo = -S.R + (float)r.ev_bin[T.e0 + j] * S.db;
                ps = psf_cut((lo + S.db - uq) * isq, (lo - uq) * isq);
                if (D3) {
                    const float lz = -S.Zh + (float)r.ev_binz[T.e0 + j] * S.dbz;
                    ps *= psf_cut((lz + S.dbz - zq) * isq, (lz - zq) * isq);
                }
            }
        }
        float g = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if (NW == LMMEW_MAX_LINES && w >= S.nw) break;
            g = fmaf(Pp[w], __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gq[w]), j)), g);
        }
        return __fmul_rn(ps, g);
    };
    auto path_weights = [&](float *Pp) {
        const float gqa = g_qa[(size_t)a * S.Qp + i];
#pragma unroll
        for (int w = 0; w < NW; ++w) Pp[w] = S.pp[w] * fast_exp2(-S.f[w] * gqa * kLog2e);
    };
    constexpr bool kStage = JT <= 16;
    __shared__ float prim[kStage ? JT * kWave : 1];
    if (kStage) {
        float Pp[NW];
        path_weights(Pp);
        for (int j = 0; j < T.cnt; ++j) prim[j * kWave + lane] = prim_of(j, Pp);
    }

    float Ej[JT];
#pragma unroll
    for (int j = 0; j < JT; ++j) {
        Ej[j] = r.ev_E[T.e0 + min(j, last)];
    }

    float acc[JT];
#pragma unroll
    for (int j = 0; j < JT; ++j) acc[j] = 0.f;

    const GPtr<ScatA> sa = sab + (size_t)a * nsc;
    // ptab: [angle][point][line][pixel][2] -- a lane's 2 values of a line are
    // contiguous, and a tile reads only the lines its events keep.  A line's
    // address is a uniform base (scalar registers) plus the lane's fixed 32-bit
    // byte offset, so the loads need no per-point vector address arithmetic.
    const size_t lstride = (size_t)S.Qp * 2;                   // one line of a point
    const GPtr<float> pbase = TAB ? ptab + (size_t)a * nsc * S.nw * lstride : nullptr;
    const unsigned pboff = (unsigned)i * (unsigned)sizeof(float2);
    const float sqck2 = S.sqck * S.sqck;
    // A listed point's inputs: its response factors for the tile's events
    // (scalar registers), and its path parameters from the table or what the
    // kernel derives them from.  Two buffers alternate, so the next point's
    // loads are in flight while the current one is evaluated, with no copies.
    // The response factors are read as integer bits: their zero test is then a
    // scalar compare (as a float test it becomes a vector class check per pair).
    const int *pvb = reinterpret_cast<const int *>(r.pvt);
    struct Pt {
        int l;                         // scatter-list entry
        unsigned gm;                   // groups of 16 events its response reaches
        int pf[16];                    // response factors of the first 16 events (bits)
        float A[NW], sw[NW];           // table values
        ScatA sp;                      // or: the point, its pixel path, its z
        float gqs, zs;
    };
    auto load_pt = [&](int l, Pt &d, auto lmc) {
        constexpr unsigned LM = decltype(lmc)::value;
        const int2 e = r.slist[l];
        d.l = l;
        d.gm = (unsigned)e.x >> kSlistGroupShift;
#pragma unroll
        for (int j = 0; j < 16; ++j) d.pf[j] = pvb[(size_t)l * JT + j];
        const int k = e.x & kSlistPoint;
        if (TAB) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (NW == LMMEW_MAX_LINES && w >= S.nw) break;
                if (!((LM >> w) & 1u)) continue;
                // the line's base stays opaque in scalar registers and the lane's
                // 32-bit offset is widened at the load, so the compiler emits a
                // scalar-base load instead of 64-bit vector address arithmetic
                unsigned long long tb = (unsigned long long)(pbase + ((size_t)k * S.nw + w) * lstride);
                unsigned off = pboff;
                asm("" : "+s"(tb));
                asm("" : "+v"(off));
                const GPtr<float> v = (GPtr<float>)((GPtr<char>)tb + off);
                d.A[w] = v[0];
                d.sw[w] = v[1];
            }
        } else {
            d.sp = load_scat(sa + k);
            d.gqs = g_qs[(size_t)e.y * S.Qp + i];
            d.zs = D3 ? szs[e.y] : 0.f;
        }
    };
    auto run_pt = [&](const Pt &d, auto lmc) {
        constexpr unsigned LM = decltype(lmc)::value;
        float Aw[NW], sw[NW], Fw[NW];
        if (TAB) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (!((LM >> w) & 1u)) continue;
                // s_w = sqrt(log2(e) / (2 k E')), F_w = s_w E' = (log2(e) / (2 k)) / s_w
                Aw[w] = d.A[w];
                sw[w] = d.sw[w];
                Fw[w] = sqck2 * fast_rcp(d.sw[w]);
            }
        } else {
            float Ep[NW];
            scatter_params<NW, true, D3, LM>(S, d.sp.x - xq, d.sp.y - yq, d.zs - zq, c, s,
                                             d.sp.lc, d.gqs, d.sp.gsa, Aw, sw, Fw, Ep);
        }
#pragma unroll
        for (int g = 0; g < JT / 16; ++g) {
            if (JT > 16 && !((d.gm >> g) & 1u)) continue;
            int pg[16];
#pragma unroll
            for (int t = 0; t < 16; ++t)
                pg[t] = g == 0 ? d.pf[t] : pvb[(size_t)d.l * JT + 16 * g + t];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = 16 * g + t;
                // a zero factor (response cut) skips the pair on a scalar compare
                if (pg[t] != 0) {
                    constexpr int w0 = __builtin_ctz(LM);        // first kept line
                    float u = fmaf(sw[w0], Ej[j], -Fw[w0]);
                    float e = fast_exp2(fmaf(-u, u, Aw[w0]));
#pragma unroll
                    for (int w = w0 + 1; w < NW; ++w) {
                        if (NW == LMMEW_MAX_LINES && w >= S.nw) break;
                        if (!((LM >> w) & 1u)) continue;
                        u = fmaf(sw[w], Ej[j], -Fw[w]);
                        e += fast_exp2(fmaf(-u, u, Aw[w]));
                    }
                    acc[j] = fmaf(__int_as_float(pg[t]), e, acc[j]);
                }
            }
        }
    };
    const int kend = (r.mode == 2) ? T.k0 : T.k1;     // unscattered only: no scatter loop
    auto point_loop = [&](auto lmc) {
        Pt d0, d1;
        load_pt(T.k0, d0, lmc);
        for (int l = T.k0; l < kend; l += 2) {
            load_pt(min(l + 1, kend - 1), d1, lmc);
            run_pt(d0, lmc);
            if (l + 1 >= kend) break;
            load_pt(min(l + 2, kend - 1), d0, lmc);
            run_pt(d1, lmc);
        }
    };
    if (T.k0 < kend && T.lmask != 0) {
        // one specialisation per line mask: the tile's events keep the same lines
        constexpr unsigned kAll = (1u << NW) - 1u;
        if constexpr (NW <= kMaskedLines) {
            switch (T.lmask) {
            case 1: if constexpr (kAll >= 1) point_loop(std::integral_constant<unsigned, 1>{}); break;
            case 2: if constexpr (kAll >= 3) point_loop(std::integral_constant<unsigned, 2>{}); break;
            case 3: if constexpr (kAll >= 3) point_loop(std::integral_constant<unsigned, 3>{}); break;
            case 4: if constexpr (kAll >= 7) point_loop(std::integral_constant<unsigned, 4>{}); break;
            case 5: if constexpr (kAll >= 7) point_loop(std::integral_constant<unsigned, 5>{}); break;
            case 6: if constexpr (kAll >= 7) point_loop(std::integral_constant<unsigned, 6>{}); break;
            default: point_loop(std::integral_constant<unsigned, kAll>{}); break;
            }
        } else {
            point_loop(std::integral_constant<unsigned, 0xFFu>{});
        }
    }

    if (kStage) {
#pragma unroll
        for (int j = 0; j < JT; ++j) {
            if (j < T.cnt)
                r.A[(size_t)(T.e0 + j) * S.Qp + i] = valid ? prim[j * kWave + lane] + acc[j] : 0.f;
        }
    } else {
        float Pp[NW];
        path_weights(Pp);
#pragma unroll
        for (int j = 0; j < JT; ++j) {
            if (j < T.cnt)
                r.A[(size_t)(T.e0 + j) * S.Qp + i] = valid ? prim_of(j, Pp) + acc[j] : 0.f;
        }
    }
}

// Bin probability of the unscattered path of every (angle, bin, support
// pixel), the arithmetic of k_row's in-kernel formation: one lane per pixel.
__global__ __launch_bounds__(64) void k_psf_table(const DevSys S, const float2 *pix_xy,
                                                  const float2 *dirs, float *psft)
{
    const int i = blockIdx.x * kWave + threadIdx.x;
    const int b = blockIdx.y, a = blockIdx.z;
    const float2 xy = pix_xy[i], dir = dirs[a];
    const float xq = xy.x, yq = xy.y, c = dir.x, s = dir.y;
    const float dq = S.R - (xq * c + yq * s);
    const float uq = -xq * s + yq * c;
    const float isq = 1.f / ((S.fwhm0 + S.fslope * dq) * S.inv_fwhm_to_sigma);
    const float lo = -S.R + (float)b * S.db;
    psft[((size_t)a * S.nb + b) * S.Qp + i] = psf_cut((lo + S.db - uq) * isq, (lo - uq) * isq);
}

hipError_t launch_psf_table(const DevSys &S, const float2 *pix_xy, const float2 *dirs,
                            float *psft, hipStream_t st)
{
    hipLaunchKernelGGL(k_psf_table, dim3(S.Qp / kWave, S.nb, S.na), dim3(kWave), 0, st, S, pix_xy,
                       dirs, psft);
    return hipGetLastError();
}

// Response factors of every (listed point, event) pair of each tile, built
// with the tiles: the [angle][point][bin] table entry of binned events (times
// the axial one in 3-D), the Gaussian density at a continuous position.  One
// workgroup per tile.
template <bool D3>
__global__ __launch_bounds__(64) void k_pv_table(const DevSys S, const RowArgs r, int JT,
                                                 float *pvt)
{
    const Tile T = r.tiles[blockIdx.x];
    const float *resp = r.resp, *respz = r.respz;
    const ScatA *sab = r.sa;
    int nsc = S.nsc;
    if (r.maps) {
        const MapTab m = r.maps[T.ncase];
        resp = m.resp;
        respz = m.respz;
        sab = m.sa;
        nsc = m.nsc;
    }
    const int a = T.angle, last = T.cnt - 1;
    const ScatA *sa = sab + (size_t)a * nsc;
    const int n = (T.k1 - T.k0) * JT;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int l = T.k0 + t / JT, j = t % JT;
        const int k = r.slist[l].x & kSlistPoint;
        float v = 0.f;
        if (r.ev_u) {
            const ScatA sp = sa[k];
            const float z = (r.ev_u[T.e0 + min(j, last)] - sp.u) * sp.isig;
            v = j < T.cnt ? pdf_cut(z, sp.isig) : 0.f;
        } else {
            const float *rrow = resp + ((size_t)a * nsc + k) * S.nb;
            v = j < T.cnt ? rrow[r.ev_bin[T.e0 + min(j, last)]] : 0.f;
            if (D3) {
                const float *zrow = respz + ((size_t)a * nsc + k) * S.nbz;
                v *= zrow[r.ev_binz[T.e0 + min(j, last)]];
            }
        }
        pvt[(size_t)l * JT + j] = v;
    }
}

hipError_t launch_pv_table(const DevSys &S, const RowArgs &r, int event_tile, float *pvt,
                           hipStream_t st)
{
    if (r.ntiles == 0) return hipSuccess;
    if (S.nz > 0)
        hipLaunchKernelGGL(k_pv_table<true>, dim3(r.ntiles), dim3(64), 0, st, S, r, event_tile, pvt);
    else
        hipLaunchKernelGGL(k_pv_table<false>, dim3(r.ntiles), dim3(64), 0, st, S, r, event_tile,
                           pvt);
    return hipGetLastError();
}

template <int JT, bool TAB, bool D3>
static hipError_t launch_row_jt(const DevSys &S, const RowArgs &r, hipStream_t st)
{
    // one workgroup per (pixel block, tile), remapped per XCD inside the kernel
    const long W = (long)(S.Qp / kWave) * r.ntiles;
    dim3 grid((unsigned)((W + 7) / 8 * 8));
    switch (S.nw) {
    case 1: hipLaunchKernelGGL((k_row<JT, 1, TAB, D3>), grid, dim3(kWave), 0, st, S, r); break;
    case 2: hipLaunchKernelGGL((k_row<JT, 2, TAB, D3>), grid, dim3(kWave), 0, st, S, r); break;
    case 3: hipLaunchKernelGGL((k_row<JT, 3, TAB, D3>), grid, dim3(kWave), 0, st, S, r); break;
    case 4: hipLaunchKernelGGL((k_row<JT, 4, TAB, D3>), grid, dim3(kWave), 0, st, S, r); break;
    default:
        hipLaunchKernelGGL((k_row<JT, LMMEW_MAX_LINES, TAB, D3>), grid, dim3(kWave), 0, st, S, r);
        break;
    }
    return hipGetLastError();
}

// the response-factor table: one thread per (angle, scatter point, bin); the
// same expression as the per-event kernel's unscattered term
__global__ __launch_bounds__(256) void k_resp_table(const DevSys S, const ScatA *sa, float *resp)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)S.na * S.nsc * S.nb) return;
    const int b = (int)(t % S.nb);
    const long ak = t / S.nb;                       // a * nsc + k
    const ScatA sp = sa[ak];
    const float lo = -S.R + (float)b * S.db;
    resp[t] = psf_cut((lo + S.db - sp.u) * sp.isig, (lo - sp.u) * sp.isig);
}

// 3-D: the axial factors, one thread per (angle, scatter point, axial bin)
__global__ __launch_bounds__(256) void k_resp_table_z(const DevSys S, const ScatA *sa,
                                                      const float *sz, float *respz)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)S.na * S.nsc * S.nbz) return;
    const int b = (int)(t % S.nbz);
    const ScatA sp = sa[t / S.nbz];
    const float z = sz[sp.sidx];
    const float lo = -S.Zh + (float)b * S.dbz;
    respz[t] = psf_cut((lo + S.dbz - z) * sp.isig, (lo - z) * sp.isig);
}

hipError_t launch_resp_table(const DevSys &S, const ScatA *sa, float *resp, const float *sz,
                             float *respz, hipStream_t st)
{
    const long n = (long)S.na * S.nsc * S.nb;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_resp_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S, sa,
                       resp);
    if (S.nz > 0) {
        const long nz = (long)S.na * S.nsc * S.nbz;
        hipLaunchKernelGGL(k_resp_table_z, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st,
                           S, sa, sz, respz);
    }
    return hipGetLastError();
}

// the path-parameter table: one workgroup per (64 pixels, scatter point, angle)
template <int NW, bool D3>
__global__ __launch_bounds__(64) void k_path_table(const DevSys S, const float2 *pix_xy,
                                                   const float *pix_z, const float2 *dirs,
                                                   const float *g_qs, const ScatA *sa,
                                                   const float *sz, float *ptab)
{
    const int i = blockIdx.x * kWave + threadIdx.x;
    const int k = blockIdx.y, a = blockIdx.z;
    const ScatA sp = sa[(size_t)a * S.nsc + k];
    const float2 xy = pix_xy[i], dir = dirs[a];
    const float gqs = g_qs[(size_t)sp.sidx * S.Qp + i];
    const float dz = D3 ? sz[sp.sidx] - pix_z[i] : 0.f;
    float Aw[NW], sw[NW], Fw[NW], Ep[NW];
    scatter_params<NW, true, D3>(S, sp.x - xy.x, sp.y - xy.y, dz, dir.x, dir.y, sp.lc, gqs,
                                 sp.gsa, Aw, sw, Fw, Ep);
    // [angle][point][line][pixel][2]: the log2 weight and s_w = sqrt(log2(e) / (2 k E'))
    // of the scattered energy E' (the model's energy resolution, sigma'^2 = k E')
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (NW == LMMEW_MAX_LINES && w >= S.nw) break;
        float *tp = ptab + ((((size_t)a * S.nsc + k) * S.nw + w) * S.Qp + i) * 2;
        tp[0] = Aw[w];
        tp[1] = S.sqck * rsqrtf(Ep[w]);
    }
}

template <bool D3>
static void launch_path_table_d(const DevSys &S, const float2 *pix_xy, const float *pix_z,
                                const float2 *dirs, const float *g_qs, const ScatA *sa,
                                const float *sz, float *ptab, hipStream_t st)
{
    const dim3 grid(S.Qp / kWave, S.nsc, S.na);
#define PT(NWV) hipLaunchKernelGGL((k_path_table<NWV, D3>), grid, dim3(kWave), 0, st, S, pix_xy, \
                                   pix_z, dirs, g_qs, sa, sz, ptab)
    switch (S.nw) {
    case 1: PT(1); break;
    case 2: PT(2); break;
    case 3: PT(3); break;
    case 4: PT(4); break;
    default: PT(LMMEW_MAX_LINES); break;
    }
#undef PT
}

hipError_t launch_path_table(const DevSys &S, const float2 *pix_xy, const float *pix_z,
                             const float2 *dirs, const float *g_qs, const ScatA *sa,
                             const float *sz, float *ptab, hipStream_t st)
{
    if (S.nsc == 0) return hipSuccess;
    if (S.nz > 0)
        launch_path_table_d<true>(S, pix_xy, pix_z, dirs, g_qs, sa, sz, ptab, st);
    else
        launch_path_table_d<false>(S, pix_xy, pix_z, dirs, g_qs, sa, sz, ptab, st);
    return hipGetLastError();
}

hipError_t launch_row(const DevSys &S, const RowArgs &r, int event_tile, hipStream_t st)
{
    if (r.ntiles == 0) return hipSuccess;
    // the table is used when the tiles' cases all have one (see the plan)
    const bool tab = r.ptab != nullptr;
    if (S.nz > 0) {
        switch (event_tile) {
        case 16: return tab ? launch_row_jt<16, true, true>(S, r, st)
                            : launch_row_jt<16, false, true>(S, r, st);
        case 32: return tab ? launch_row_jt<32, true, true>(S, r, st)
                            : launch_row_jt<32, false, true>(S, r, st);
        default: return tab ? launch_row_jt<64, true, true>(S, r, st)
                            : launch_row_jt<64, false, true>(S, r, st);
        }
    }
    switch (event_tile) {
    case 16: return tab ? launch_row_jt<16, true, false>(S, r, st)
                        : launch_row_jt<16, false, false>(S, r, st);
    case 32: return tab ? launch_row_jt<32, true, false>(S, r, st)
                        : launch_row_jt<32, false, false>(S, r, st);
    default: return tab ? launch_row_jt<64, true, false>(S, r, st)
                        : launch_row_jt<64, false, false>(S, r, st);
    }
}

// ---------------------------------------------------------------------------
// forward projection: p_j = sum_q lambda_q a_jq, one wavefront per event row
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_forward(const DevSys S, const FwdArgs f)
{
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= f.rows) return;
    // a contiguous dot product: the row and the support copy of the image,
    // both padded with zeros to Qp (a multiple of 64), 16 bytes per load
    const float4 *A = reinterpret_cast<const float4 *>(f.A + (size_t)e * S.Qp);
    const float4 *L = reinterpret_cast<const float4 *>(f.lamc + (size_t)f.row_case[e] * S.Qp);
    float sum = 0.f;
#pragma unroll 4
    for (int k = lane; k < S.Qp / 4; k += kWave) {
        const float4 a = A[k], l = L[k];
        sum = fmaf(l.x, a.x, sum);
        sum = fmaf(l.y, a.y, sum);
        sum = fmaf(l.z, a.z, sum);
        sum = fmaf(l.w, a.w, sum);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, kWave);
    if (lane == 0) {
        f.p[e] = sum;
        f.wt[e] = sum > 0.f ? 1.f / sum : 0.f;
        if (f.logp) f.logp[e] = sum > 0.f ? log((double)sum) : 0.0;
        if (f.nskip && !(sum > 0.f)) atomicAdd(f.nskip, 1ull);
    }
}

__global__ __launch_bounds__(256) void k_compact(const DevSys S, const float *lambda, int Q,
                                                 const int *pixq, float *lamc)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= S.Qp) return;
    const int q = pixq[i];
    lamc[(size_t)c * S.Qp + i] = (i < S.Qm) ? lambda[(size_t)c * Q + q] : 0.f;
}

// Neumaier step: adds v to (sum, cmp)
__device__ __forceinline__ void neumaier(float &sum, float &cmp, float v)
{
    const float t = sum + v;
    cmp += (fabsf(sum) >= fabsf(v)) ? (sum - t) + v : (v - t) + sum;
    sum = t;
}

// One workgroup per (64 pixels, chunk of rows): wavefront k of 4 sums the
// chunk's rows r0 + k, r0 + k + 4, ... for its lane's pixel, loading four rows
// ahead; the four compensated partials are combined in a fixed order.
__global__ __launch_bounds__(256) void k_back(const DevSys S, const BackArgs b)
{
    // Four consecutive pixels per lane (16-byte row loads), 256 per
    // workgroup; each pixel's rows are summed in the same order as with one
    // pixel per lane: wave wv takes rows r0 + wv, r0 + wv + 4, ... and the
    // four partials are combined in wave order.
    __shared__ float4 ps[4][kWave], pc[4][kWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = (blockIdx.x * kWave + lane) * 4;
    const bool act = i < S.Qp;                 // Qp is a multiple of 64, not of 256
    const Chunk ch = b.chunks[blockIdx.y];
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f), cmp = sum;
    auto add = [&](const float4 &v, float w) {
        neumaier(sum.x, cmp.x, v.x * w);
        neumaier(sum.y, cmp.y, v.y * w);
        neumaier(sum.z, cmp.z, v.z * w);
        neumaier(sum.w, cmp.w, v.w * w);
    };
    auto row = [&](int e) {
        return act ? *reinterpret_cast<const float4 *>(b.A + (size_t)e * S.Qp + i)
                   : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    int e = ch.r0 + wv;
    for (; e + 12 < ch.r1; e += 16) {
        float4 v[4];
        float w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w[k] = b.wt[e + 4 * k];
            v[k] = row(e + 4 * k);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (w[k] != 0.f) add(v[k], w[k]);
    }
    for (; e < ch.r1; e += 4) {
        const float w = b.wt[e];
        if (w != 0.f) add(row(e), w);
    }
    ps[wv][lane] = sum;
    pc[wv][lane] = cmp;
    __syncthreads();
    if (wv == 0 && act) {
        float4 s0 = ps[0][lane], c0 = pc[0][lane];
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            const float4 s1 = ps[k][lane], c1 = pc[k][lane];
            neumaier(s0.x, c0.x, s1.x);
            neumaier(s0.y, c0.y, s1.y);
            neumaier(s0.z, c0.z, s1.z);
            neumaier(s0.w, c0.w, s1.w);
            c0.x += c1.x;
            c0.y += c1.y;
            c0.z += c1.z;
            c0.w += c1.w;
        }
        *reinterpret_cast<float4 *>(b.part + (size_t)blockIdx.y * S.Qp + i) = s0;
        *reinterpret_cast<float4 *>(b.comp + (size_t)blockIdx.y * S.Qp + i) = c0;
    }
}

// ---------------------------------------------------------------------------
// EM update (Eq. (18)): lambda_q <- lambda_q * B_q / sens_q, or the plain
// backprojection B_q when no sensitivity is given
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_update(const DevSys S, const UpdArgs u)
{
    // 64 pixels per workgroup; wave k of 4 sums chunks k, k + 4, ... of the
    // case, and the four compensated partials are combined in a fixed order
    __shared__ float ps[4][kWave], pc[4][kWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * kWave + lane;
    const int c = blockIdx.y;
    float sum = 0.f, cmp = 0.f;
    const int c1 = u.case_chunk[c + 1];
    for (int ch = u.case_chunk[c] + wv; ch < c1; ch += 4) {
        cmp += u.comp[(size_t)ch * S.Qp + i];
        neumaier(sum, cmp, u.part[(size_t)ch * S.Qp + i]);
    }
    ps[wv][lane] = sum;
    pc[wv][lane] = cmp;
    __syncthreads();
    if (wv != 0 || i >= S.Qm) return;
    float s0 = ps[0][lane], c0 = pc[0][lane];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        neumaier(s0, c0, ps[k][lane]);
        c0 += pc[k][lane];
    }
    const float B = s0 + c0;
    const int q = u.pixq[i];
    float *lam = u.lambda + (size_t)c * u.Q;
    float v;
    if (u.sens) {
        const float d = u.sens[(size_t)c * u.sens_stride + q];
        v = lam[q];
        if (d > 0.f) v = v * B / d;
    } else {
        v = B;
    }
    lam[q] = v;
    if (u.lamc) u.lamc[(size_t)c * S.Qp + i] = v;
}

// ---------------------------------------------------------------------------
// sensitivity: per (pixel, angle) detection probability, then per subset
// ---------------------------------------------------------------------------
template <int NW, bool D3>
__global__ __launch_bounds__(64) void k_sens(const DevSys S, const SensArgs g)
{
    const int i = blockIdx.x * kWave + threadIdx.x;
    const int a = blockIdx.y;
    const float2 dir = g.dirs[a];
    const float c = dir.x, s = dir.y;
    const float2 xy = g.pix_xy[i];
    const float xq = xy.x, yq = xy.y;
    const float zq = D3 ? g.pix_z[i] : 0.f;
    const float dq = S.R - (xq * c + yq * s);
    const float uq = -xq * s + yq * c;
    const float isq = 1.f / ((S.fwhm0 + S.fslope * dq) * S.inv_fwhm_to_sigma);
    float Dq = phi_diff((S.R - uq) * isq, (-S.R - uq) * isq);
    if (D3) Dq *= phi_diff((S.Zh - zq) * isq, (-S.Zh - zq) * isq);
    const float gqa = g.g_qa[(size_t)a * S.Qp + i];

    auto acceptance = [&](float E) {
        const float isg = fast_rsq(S.eres_k * E);
        float acc = 0.f;
        for (int k = 0; k < S.nwin; ++k) acc += phi_diff((S.whi[k] - E) * isg, (S.wlo[k] - E) * isg);
        return acc;
    };

    float tot = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (NW == LMMEW_MAX_LINES && w >= S.nw) break;
        tot += S.pp[w] * expf(-S.f[w] * gqa) * Dq * acceptance(S.E[w]);
    }
    const ScatA *sa = g.sa + (size_t)a * S.nsc;
    float scat = 0.f;
    for (int k = 0; k < S.nsc; ++k) {
        const ScatA sp = sa[k];
        const float gqs = g.g_qs[(size_t)sp.sidx * S.Qp + i];
        const float dz = D3 ? g.sz[sp.sidx] - zq : 0.f;
        float Aw[NW], sw[NW], Fw[NW], Ep[NW];
        scatter_params<NW, false, D3>(S, sp.x - xq, sp.y - yq, dz, c, s, sp.lc, gqs, sp.gsa, Aw,
                                      sw, Fw, Ep);
        float t = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if (NW == LMMEW_MAX_LINES && w >= S.nw) break;
            t = fmaf(fast_exp2(Aw[w]), acceptance(Ep[w]), t);
        }
        scat = fmaf(sp.D, t, scat);
    }
    g.Sqa[(size_t)a * S.Qp + i] = (i < S.Qm) ? tot + scat : 0.f;
}

__global__ __launch_bounds__(256) void k_sens_subsets(const DevSys S, const SensArgs g)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int sub = blockIdx.y;
    if (i >= S.Qm) return;
    float acc = 0.f;
    for (int a = sub; a < S.na; a += g.nsub) acc += g.Sqa[(size_t)a * S.Qp + i];
    g.sens[(size_t)sub * g.Q + g.pixq[i]] = S.T * acc;
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loglik(const ReduceArgs r)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int e = threadIdx.x; e < r.rows; e += 256) acc += r.logp[e];
    for (int c = 0; c < r.ncases; ++c)
        for (int q = threadIdx.x; q < r.Q; q += 256)
            acc -= (double)r.sens[(size_t)c * r.sens_stride + q] *
                   (double)r.lambda[(size_t)c * r.Q + q];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) r.out[0] = red[0];
}

__global__ __launch_bounds__(256) void k_scatter_out(const float *src, const int64_t *perm,
                                                     int64_t n, float *dst)
{
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) dst[perm[e]] = src[e];
}

// out[perm[e]][pixq[i]] = A[e][i] for the rows of one subset (full-grid rows)
__global__ __launch_bounds__(256) void k_rows_out(const DevSys S, const float *A, int rows,
                                                  const int64_t *perm, const int *pixq, int Q,
                                                  float *out)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)rows * S.Qm) return;
    const int e = (int)(t / S.Qm), i = (int)(t % S.Qm);
    out[perm[e] * Q + pixq[i]] = A[(long)e * S.Qp + i];
}

__global__ __launch_bounds__(256) void k_rows_pick(const DevSys S, const float *A, const int *ridx,
                                                   int n, const int *pixq, int Q, float *out)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)n * S.Qm) return;
    const int k = (int)(t / S.Qm), i = (int)(t % S.Qm);
    out[(long)k * Q + pixq[i]] = A[(long)ridx[k] * S.Qp + i];
}

__global__ __launch_bounds__(256) void k_gather_w(const float *w, const int64_t *perm, int64_t n,
                                                  float *dst)
{
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) dst[e] = w[perm[e]];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_tables_d(const DevSys &S, const double *mu, const double2 *pix,
                           const double *pixz, const double2 *dirs, const double2 *sc,
                           const double *scz, float *g_qa, float *g_qs, ScatA *sa, double pixmm,
                           double R, hipStream_t st)
{
    TabArgsD d{mu, pix, dirs, sc, g_qa, g_qs, sa, pixz, scz};
    if (S.nz > 0) {
        hipLaunchKernelGGL(k_tab3_qa, dim3((S.Qp + 255) / 256, S.na), dim3(256), 0, st, S, d,
                           pixmm, R);
        if (S.nsc > 0) {
            hipLaunchKernelGGL(k_tab3_qs, dim3((S.Qp + 255) / 256, S.nsc), dim3(256), 0, st, S,
                               d, pixmm, R);
            hipLaunchKernelGGL(k_tab3_sa, dim3((S.nsc + 255) / 256, S.na), dim3(256), 0, st, S,
                               d, pixmm, R);
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_tab_qa, dim3((S.Qp + 255) / 256, S.na), dim3(256), 0, st, S, d, pixmm,
                       R);
    if (S.nsc > 0) {
        hipLaunchKernelGGL(k_tab_qs, dim3((S.Qp + 255) / 256, S.nsc), dim3(256), 0, st, S, d,
                           pixmm, R);
        hipLaunchKernelGGL(k_tab_sa, dim3((S.nsc + 255) / 256, S.na), dim3(256), 0, st, S, d,
                           pixmm, R);
    }
    return hipGetLastError();
}

hipError_t launch_forward(const DevSys &S, const FwdArgs &f, hipStream_t st)
{
    if (f.rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_forward, dim3((f.rows + 3) / 4), dim3(256), 0, st, S, f);
    return hipGetLastError();
}

hipError_t launch_back(const DevSys &S, const BackArgs &b, hipStream_t st)
{
    if (b.nchunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_back, dim3((S.Qp + 4 * kWave - 1) / (4 * kWave), b.nchunks), dim3(256), 0,
                       st, S, b);
    return hipGetLastError();
}

hipError_t launch_update(const DevSys &S, const UpdArgs &u, hipStream_t st)
{
    hipLaunchKernelGGL(k_update, dim3(S.Qp / kWave, u.ncases), dim3(256), 0, st, S, u);
    return hipGetLastError();
}

hipError_t launch_sens(const DevSys &S, const SensArgs &g, hipStream_t st)
{
    dim3 grid(S.Qp / kWave, S.na);
#define SENS(NWV)                                                                          \
    do {                                                                                   \
        if (S.nz > 0)                                                                      \
            hipLaunchKernelGGL((k_sens<NWV, true>), grid, dim3(kWave), 0, st, S, g);       \
        else                                                                               \
            hipLaunchKernelGGL((k_sens<NWV, false>), grid, dim3(kWave), 0, st, S, g);      \
    } while (0)
    switch (S.nw) {
    case 1: SENS(1); break;
    case 2: SENS(2); break;
    case 3: SENS(3); break;
    case 4: SENS(4); break;
    default: SENS(LMMEW_MAX_LINES); break;
    }
#undef SENS
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sens_subsets, dim3((S.Qm + 255) / 256, g.nsub), dim3(256), 0, st, S, g);
    return hipGetLastError();
}

hipError_t launch_loglik(const ReduceArgs &r, hipStream_t st)
{
    hipLaunchKernelGGL(k_loglik, dim3(1), dim3(256), 0, st, r);
    return hipGetLastError();
}

hipError_t launch_scatter_out(const float *src, const int64_t *perm, int64_t n, float *dst,
                              hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src,
                       perm, n, dst);
    return hipGetLastError();
}

hipError_t launch_rows_out(const DevSys &S, const float *A, int rows, const int64_t *perm,
                           const int *pixq, int Q, float *out, hipStream_t st)
{
    const long n = (long)rows * S.Qm;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rows_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S, A, rows,
                       perm, pixq, Q, out);
    return hipGetLastError();
}

hipError_t launch_rows_pick(const DevSys &S, const float *A, const int *ridx, int n,
                            const int *pixq, int Q, float *out, hipStream_t st)
{
    const long m = (long)n * S.Qm;
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rows_pick, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, S, A,
                       ridx, n, pixq, Q, out);
    return hipGetLastError();
}

hipError_t launch_compact(const DevSys &S, const float *lambda, int ncases, int Q, const int *pixq,
                          float *lamc, hipStream_t st)
{
    if (ncases == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3((S.Qp + 255) / 256, ncases), dim3(256), 0, st, S, lambda,
                       Q, pixq, lamc);
    return hipGetLastError();
}

hipError_t launch_gather_w(const float *w, const int64_t *perm, int64_t n, float *dst,
                           hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_w, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, perm,
                       n, dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ROI uptake (Sec. 3.1.4): sum of an image over a region, per (case, region).
// One workgroup per (case, region); FP64 partial sums combined in a fixed
// tree, so the result is deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_roi_sums(const float *lam, int Q, const uint8_t *masks,
                                                  int K, double *out)
{
    __shared__ double red[256];
    const int c = blockIdx.y, k = blockIdx.x;
    const float *l = lam + (size_t)c * Q;
    const uint8_t *m = masks + (size_t)k * Q;
    double acc = 0.0;
    for (int q = threadIdx.x; q < Q; q += 256)
        if (m[q]) acc += (double)l[q];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)c * K + k] = red[0];
}

// FP64 sum of n floats by one workgroup in a fixed order (setup-time use).
__global__ __launch_bounds__(1024) void k_sum_f64(const float *x, long n, double *out)
{
    __shared__ double red[1024];
    double acc = 0.0;
    for (long i = threadIdx.x; i < n; i += 1024) acc += (double)x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_sum(const float *x, long n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(1024), 0, st, x, n, out);
    return hipGetLastError();
}

// FP64 sum of every row of A [rows][Qp]: one wavefront per row, the lanes'
// strided partial sums, then a butterfly over the wavefront (a fixed order).
__global__ __launch_bounds__(256) void k_row_sums(const float *A, int rows, int Qp, double *out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int r = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (r >= rows) return;
    const float *row = A + (size_t)r * Qp;
    double acc = 0.0;
    for (int q = lane; q < Qp; q += kWave) acc += (double)row[q];
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) out[r] = acc;
}

hipError_t launch_row_sums(const float *A, int rows, int Qp, double *out, hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_sums, dim3((rows + 3) / 4), dim3(256), 0, st, A, rows, Qp, out);
    return hipGetLastError();
}

hipError_t launch_roi_sums(const float *lam, int C, int Q, const uint8_t *masks, int K,
                           double *out, hipStream_t st)
{
    if (C == 0 || K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_roi_sums, dim3(K, C), dim3(256), 0, st, lam, Q, masks, K, out);
    return hipGetLastError();
}

}  // namespace lmmew
