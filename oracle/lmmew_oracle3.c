/*
 * FP64 CPU oracle, 3-D single-scatter model.  TEST INFRASTRUCTURE ONLY: see
 * lmmew_oracle3.h for the geometry.
 *
 * The path weights follow Eq. (5) in three dimensions, as the paper writes
 * it, for paths with no or one scatter; the scatter locations are the points
 * of a grid coarser than the image (the lower-resolution scatter modelling
 * the paper's appendix on 3-D requirements proposes).  Each function names
 * the passage it follows and the reading it takes.
 */
#include "lmmew_oracle3.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

static int near_int(double f, long *k)
{
    double r = floor(f + 0.5);
    if (fabs(f - r) < 1e-9) { *k = (long)r; return 1; }
    return 0;
}

static double voxel_mu(const double *mu, int n, int nz, long ix, long iy, long iz)
{
    if (ix < 0 || iy < 0 || iz < 0 || ix >= n || iy >= n || iz >= nz) return 0.0;
    return mu[((size_t)iz * n + (size_t)iy) * n + (size_t)ix];
}

/* Attenuation value seen at (xm,ym,zm) by a segment along which the
 * coordinates flagged in `fixed` do not change.  A fixed coordinate that lies
 * on a cell boundary sees the mean of the two cells sharing it (the limit of
 * segments displaced by +-delta); several such coordinates give the mean over
 * all combinations. */
static double mu3_seen(const double *mu, int n, int nz, double pix, double xm, double ym,
                       double zm, const int fixed[3])
{
    double R = 0.5 * n * pix, Zh = 0.5 * nz * pix;
    double f[3] = {(xm + R) / pix, (ym + R) / pix, (zm + Zh) / pix};
    long lo[3];
    int cnt[3];
    for (int d = 0; d < 3; ++d) {
        long k;
        if (fixed[d] && near_int(f[d], &k)) {
            lo[d] = k - 1;
            cnt[d] = 2;
        } else {
            lo[d] = (long)floor(f[d]);
            cnt[d] = 1;
        }
    }
    double s = 0.0;
    int m = 0;
    for (int i = 0; i < cnt[0]; ++i)
        for (int j = 0; j < cnt[1]; ++j)
            for (int k = 0; k < cnt[2]; ++k) {
                s += voxel_mu(mu, n, nz, lo[0] + i, lo[1] + j, lo[2] + k);
                ++m;
            }
    return s / m;
}

static int cmp_d(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Eq. (6) in 3-D: the integral of the voxelised map along the segment
 * (x0,y0,z0) -> (x1,y1,z1), as the sum over the pieces between successive
 * crossings of the grid planes of (value at the piece's midpoint) x (piece
 * length).  The map is zero outside the grid. */
double or3_segment_integral(const double *mu, int n, int nz, double pix, double x0,
                            double y0, double z0, double x1, double y1, double z1)
{
    double R = 0.5 * n * pix, Zh = 0.5 * nz * pix;
    double d[3] = {x1 - x0, y1 - y0, z1 - z0};
    double o[3] = {x0, y0, z0};
    double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (L == 0.0) return 0.0;
    double *ts = (double *)malloc(sizeof(double) * (size_t)(2 * (n + 1) + (nz + 1) + 2));
    int m = 0;
    ts[m++] = 0.0;
    ts[m++] = 1.0;
    for (int ax = 0; ax < 3; ++ax) {
        if (d[ax] == 0.0) continue;
        int cells = ax < 2 ? n : nz;
        double lo = ax < 2 ? -R : -Zh;
        for (int k = 0; k <= cells; ++k) {
            double t = (lo + k * pix - o[ax]) / d[ax];
            if (t > 0.0 && t < 1.0) ts[m++] = t;
        }
    }
    qsort(ts, (size_t)m, sizeof(double), cmp_d);
    int fixed[3] = {d[0] == 0.0, d[1] == 0.0, d[2] == 0.0};
    double sum = 0.0;
    for (int i = 0; i + 1 < m; ++i) {
        double t0 = ts[i], t1 = ts[i + 1];
        if (t1 <= t0) continue;
        double tm = 0.5 * (t0 + t1);
        sum += mu3_seen(mu, n, nz, pix, x0 + tm * d[0], y0 + tm * d[1], z0 + tm * d[2], fixed) *
               (t1 - t0) * L;
    }
    free(ts);
    return sum;
}

/* Normaliser of the Klein-Nishina angular density over the sphere:
 * Z3(E) = 2 pi * integral over cos(phi) in [-1, 1] of K, so that K / Z3 is
 * the probability per steradian of the scattered direction (the K of
 * Eq. (5) as a normalised density).  Composite Simpson on 4096 intervals of
 * a smooth rational integrand. */
double or3_kn_Z(double E, double me)
{
    const int N = 4096;
    double h = 2.0 / N, s = 0.0;
    for (int i = 0; i <= N; ++i) {
        double c = -1.0 + i * h;
        double wgt = (i == 0 || i == N) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        s += wgt * or_kn_K(c, E, me);
    }
    return 2.0 * OR_PI * s * h / 3.0;
}

void or3_voxel_centre(const or3_geom *G, int q, double *x, double *y, double *z)
{
    int n = G->S3.S.n;
    double pix = G->S3.S.pix;
    int ix = q % n, iy = (q / n) % n, iz = q / (n * n);
    *x = (ix + 0.5) * pix - G->R;
    *y = (iy + 0.5) * pix - G->R;
    *z = (iz + 0.5) * pix - G->Zh;
}

/* Precomputation of Algorithm 1 in 3-D: voxel set, scatter points and the
 * radiological paths (Eq. (6)) voxel -> detector, voxel -> scatter point and
 * scatter point -> detector.  Returns 0, or -1 for an unsupported grid. */
int or3_geom_build(or3_geom *G, const or3_sys *S3, const double *mu85, const uint8_t *mask)
{
    memset(G, 0, sizeof(*G));
    G->S3 = *S3;
    const or_sys *S = &S3->S;
    int n = S->n, nz = S3->nz, ns = S->ns, nsz = S3->nsz;
    if (n <= 0 || nz <= 0 || ns <= 0 || nsz <= 0 || n % ns || nz % nsz) return -1;
    int m = n / ns, mz = nz / nsz;
    if (m % 2 || mz % 2) return -1;
    G->R = 0.5 * n * S->pix;
    G->Zh = 0.5 * nz * S->pix;
    G->hs = 2.0 * G->R / ns;
    G->hz = 2.0 * G->Zh / nsz;
    G->db = 2.0 * G->R / S->nb;
    G->dbz = 2.0 * G->Zh / S3->nbz;
    G->Q = n * n * nz;
    G->mu = (double *)malloc(sizeof(double) * G->Q);
    memcpy(G->mu, mu85, sizeof(double) * G->Q);
    G->support = (uint8_t *)malloc(G->Q);
    for (int q = 0; q < G->Q; ++q) {
        double x, y, z;
        or3_voxel_centre(G, q, &x, &y, &z);
        G->support[q] = (x * x + y * y <= G->R * G->R) && (!mask || mask[q]);
    }
    int cells = ns * ns * nsz;
    G->sx = (double *)malloc(sizeof(double) * cells);
    G->sy = (double *)malloc(sizeof(double) * cells);
    G->sz = (double *)malloc(sizeof(double) * cells);
    G->smu = (double *)malloc(sizeof(double) * cells);
    for (int kz = 0; kz < nsz; ++kz)
        for (int ky = 0; ky < ns; ++ky)
            for (int kx = 0; kx < ns; ++kx) {
                double x = (kx + 0.5) * G->hs - G->R;
                double y = (ky + 0.5) * G->hs - G->R;
                double z = (kz + 0.5) * G->hz - G->Zh;
                double acc = 0.0;
                for (int k = 0; k < mz; ++k)
                    for (int j = 0; j < m; ++j)
                        for (int i = 0; i < m; ++i)
                            acc += voxel_mu(mu85, n, nz, kx * m + i, ky * m + j, kz * mz + k);
                acc /= (double)(m * m * mz);
                if (x * x + y * y <= G->R * G->R && acc > 0.0) {
                    G->sx[G->nsc] = x;
                    G->sy[G->nsc] = y;
                    G->sz[G->nsc] = z;
                    G->smu[G->nsc] = acc;
                    G->nsc++;
                }
            }
    int na = S->na, nsc = G->nsc > 0 ? G->nsc : 1;
    G->g_qa = (double *)calloc((size_t)na * G->Q, sizeof(double));
    G->g_qs = (double *)calloc((size_t)G->Q * nsc, sizeof(double));
    G->g_sa = (double *)calloc((size_t)na * nsc, sizeof(double));
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < G->Q; ++q) {
        if (!G->support[q]) continue;
        double x, y, z;
        or3_voxel_centre(G, q, &x, &y, &z);
        for (int a = 0; a < na; ++a) {
            double c, s;
            or_angle_dir(a, na, &c, &s);
            double d = G->R - (x * c + y * s);
            G->g_qa[(size_t)a * G->Q + q] =
                or3_segment_integral(mu85, n, nz, S->pix, x, y, z, x + d * c, y + d * s, z);
        }
        for (int si = 0; si < G->nsc; ++si)
            G->g_qs[(size_t)q * G->nsc + si] = or3_segment_integral(
                mu85, n, nz, S->pix, x, y, z, G->sx[si], G->sy[si], G->sz[si]);
    }
    for (int a = 0; a < na; ++a) {
        double c, s;
        or_angle_dir(a, na, &c, &s);
        for (int si = 0; si < G->nsc; ++si) {
            double x = G->sx[si], y = G->sy[si], z = G->sz[si];
            double d = G->R - (x * c + y * s);
            G->g_sa[(size_t)a * G->nsc + si] =
                or3_segment_integral(mu85, n, nz, S->pix, x, y, z, x + d * c, y + d * s, z);
        }
    }
    for (int w = 0; w < S->nw; ++w) G->Zw[w] = or3_kn_Z(S->E[w], S->me);
    return 0;
}

void or3_geom_free(or3_geom *G)
{
    free(G->mu); free(G->support);
    free(G->sx); free(G->sy); free(G->sz); free(G->smu);
    free(G->g_qa); free(G->g_qs); free(G->g_sa);
    memset(G, 0, sizeof(*G));
}

/* Unscattered path of Eq. (5) (n = 0): alpha_w * (Delta Omega / 4 pi) *
 * exp(-gamma(q -> detector, E_w)), Delta Omega the collimator's acceptance
 * solid angle (the t of Eq. (5) read as a constant acceptance). */
double or3_Pp(const or3_geom *G, int q, int a, int w)
{
    const or_sys *S = &G->S3.S;
    double fw = or_mu_scale(S, S->E[w]);
    return S->alpha[w] * G->S3.domega / (4.0 * OR_PI) *
           exp(-fw * G->g_qa[(size_t)a * G->Q + q]);
}

/* Once-scattered path of Eq. (5) (n = 1) through scatter point si:
 *   alpha_w * V mu_s f_w / (4 pi r^2) * exp(-gamma(q -> s, E_w))
 *   * K(phi; E_w) / Z3(E_w) * Delta Omega * exp(-gamma(s -> detector, E'))
 * V/(4 pi r^2) * mu_s is the probability that the isotropically emitted
 * photon interacts in the cell of volume V = hs^2 hz at distance r (the
 * Delta Omega / 4 pi and the intersection length of Eq. (5)), K/Z3 * Delta
 * Omega the probability of scattering into the collimator's acceptance, and
 * E' = E_w P(phi).  r is clamped below at a/sqrt(3), a = (3V / 4 pi)^(1/3):
 * the radius at which 1/r^2 equals its mean over a ball of volume V centred
 * on the emitter. */
double or3_Ps(const or3_geom *G, int q, int si, int a, int w, double *Eprime)
{
    const or_sys *S = &G->S3.S;
    double xq, yq, zq, c, s;
    or3_voxel_centre(G, q, &xq, &yq, &zq);
    or_angle_dir(a, S->na, &c, &s);
    double dx = G->sx[si] - xq, dy = G->sy[si] - yq, dz = G->sz[si] - zq;
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double V = G->hs * G->hs * G->hz;
    double rmin = cbrt(3.0 * V / (4.0 * OR_PI)) / sqrt(3.0);
    double reff = fmax(r, rmin);
    double cosphi = (dx * c + dy * s) / r;
    double E = S->E[w];
    double P = 1.0 / (1.0 + (E / S->me) * (1.0 - cosphi));
    double Ep = E * P;
    double fw = or_mu_scale(S, E), fp = or_mu_scale(S, Ep);
    double v = S->alpha[w] * V * G->smu[si] * fw / (4.0 * OR_PI * reff * reff) *
               exp(-fw * G->g_qs[(size_t)q * G->nsc + si]) *
               or_kn_K(cosphi, E, S->me) / G->Zw[w] * G->S3.domega *
               exp(-fp * G->g_sa[(size_t)a * G->nsc + si]);
    if (Eprime) *Eprime = Ep;
    return v;
}

/* Position attribute of Eq. (3) on a 2-D detector: the depth-dependent
 * Gaussian response, separable in u and v with one sigma. */
double or3_psf_bin(const or3_geom *G, int b, int bz, double x, double y, double z, int a)
{
    double c, s;
    or_angle_dir(a, G->S3.S.na, &c, &s);
    double u = -x * s + y * c;
    double sig = or_psf_sigma(&G->S3.S, G->R - (x * c + y * s));
    double lo = -G->R + b * G->db, hi = lo + G->db;
    double lz = -G->Zh + bz * G->dbz, hz = lz + G->dbz;
    return or_Phi_diff((hi - u) / sig, (lo - u) / sig) *
           or_Phi_diff((hz - z) / sig, (lz - z) / sig);
}

/* Probability of landing anywhere on the detector [-R, R) x [-Zh, Zh). */
double or3_psf_total(const or3_geom *G, double x, double y, double z, int a)
{
    double c, s;
    or_angle_dir(a, G->S3.S.na, &c, &s);
    double u = -x * s + y * c;
    double sig = or_psf_sigma(&G->S3.S, G->R - (x * c + y * s));
    return or_Phi_diff((G->R - u) / sig, (-G->R - u) / sig) *
           or_Phi_diff((G->Zh - z) / sig, (-G->Zh - z) / sig);
}

/* Per-event row (Eq. (3) with Eq. (4)'s numerator, per unit activity), as in
 * the planar model with the 3-D path weights and the 2-D detector. */
static void row3(const or3_geom *G, int b, int bz, int a, double Ehat, int primary,
                 double *row)
{
    const or_sys *S = &G->S3.S;
    for (int q = 0; q < G->Q; ++q) {
        row[q] = 0.0;
        if (!G->support[q]) continue;
        double xq, yq, zq;
        or3_voxel_centre(G, q, &xq, &yq, &zq);
        double psf_q = primary ? or3_psf_bin(G, b, bz, xq, yq, zq, a) : 0.0;
        double acc = 0.0;
        for (int w = 0; w < S->nw; ++w) {
            if (primary)
                acc += or3_Pp(G, q, a, w) * psf_q *
                       or_gauss(Ehat, S->E[w], or_sigmaE(S, S->E[w]));
            for (int si = 0; si < G->nsc; ++si) {
                double Ep;
                double ps = or3_Ps(G, q, si, a, w, &Ep);
                acc += ps * or3_psf_bin(G, b, bz, G->sx[si], G->sy[si], G->sz[si], a) *
                       or_gauss(Ehat, Ep, or_sigmaE(S, Ep));
            }
        }
        row[q] = acc;
    }
}

void or3_event_row(const or3_geom *G, int b, int bz, int a, double Ehat, double *row)
{
    row3(G, b, bz, a, Ehat, 1, row);
}

void or3_event_row_scatter(const or3_geom *G, int b, int bz, int a, double Ehat, double *row)
{
    row3(G, b, bz, a, Ehat, 0, row);
}

/* Detection probability per unit activity of voxel q at angle a (Eq. (7)
 * for one voxel and one angle): landing on the detector and inside a
 * window. */
double or3_sens_qa(const or3_geom *G, int q, int a)
{
    const or_sys *S = &G->S3.S;
    double xq, yq, zq;
    or3_voxel_centre(G, q, &xq, &yq, &zq);
    double Dq = or3_psf_total(G, xq, yq, zq, a);
    double acc = 0.0;
    for (int w = 0; w < S->nw; ++w) {
        acc += or3_Pp(G, q, a, w) * Dq * or_acc(S, S->E[w]);
        for (int si = 0; si < G->nsc; ++si) {
            double Ep;
            double ps = or3_Ps(G, q, si, a, w, &Ep);
            acc += ps * or3_psf_total(G, G->sx[si], G->sy[si], G->sz[si], a) * or_acc(S, Ep);
        }
    }
    return acc;
}

/* Denominator of Eq. (18) per subset (a mod nsub == s). */
void or3_sensitivity(const or3_geom *G, int nsub, double *sens)
{
    int na = G->S3.S.na;
    memset(sens, 0, sizeof(double) * (size_t)nsub * G->Q);
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < G->Q; ++q) {
        if (!G->support[q]) continue;
        for (int a = 0; a < na; ++a)
            sens[(size_t)(a % nsub) * G->Q + q] += G->S3.S.T * or3_sens_qa(G, q, a);
    }
}

/* Index of the first event with a bin, axial bin or angle out of range or an
 * energy outside every window, or -1. */
int or3_check_events(const or3_geom *G, long nev, const int *bin, const int *binz,
                     const int *ang, const double *E)
{
    const or_sys *S = &G->S3.S;
    for (long j = 0; j < nev; ++j) {
        if (bin[j] < 0 || bin[j] >= S->nb || binz[j] < 0 || binz[j] >= G->S3.nbz ||
            ang[j] < 0 || ang[j] >= S->na)
            return (int)j;
        int in = 0;
        for (int k = 0; k < S->nwin; ++k)
            if (E[j] >= S->wlo[k] && E[j] <= S->whi[k]) in = 1;
        if (!in || !isfinite(E[j])) return (int)j;
    }
    return -1;
}

typedef struct {
    const or3_geom *G;
    const int *bin, *binz, *ang;
    const double *E;
} list3d;

static void list3d_row(const void *ctx, long j, double *row)
{
    const list3d *L = (const list3d *)ctx;
    or3_event_row(L->G, L->bin[j], L->binz[j], L->ang[j], L->E[j], row);
}

/* p_j = sum_q a_jq lambda_q. */
void or3_forward(const or3_geom *G, long nev, const int *bin, const int *binz,
                 const int *ang, const double *E, const double *lambda, double *p)
{
#pragma omp parallel
    {
        double *row = (double *)malloc(sizeof(double) * G->Q);
#pragma omp for schedule(dynamic)
        for (long j = 0; j < nev; ++j) {
            or3_event_row(G, bin[j], binz[j], ang[j], E[j], row);
            double s = 0.0;
            for (int q = 0; q < G->Q; ++q) s += row[q] * lambda[q];
            p[j] = s;
        }
        free(row);
    }
}

/* LM-OSEM (Eq. (18)-(20)) on the 3-D rows: the loop of or_osem_rows. */
int or3_osem(const or3_geom *G, long nev, const int *bin, const int *binz,
             const int *ang, const double *E, int nsub, int niter, const double *sens,
             double *lambda, double *hist, double *ll, long *skipped)
{
    list3d L = {G, bin, binz, ang, E};
    return or_osem_rows(nev, ang, G->Q, nsub, niter, sens, lambda, hist, ll, skipped,
                        list3d_row, &L);
}
