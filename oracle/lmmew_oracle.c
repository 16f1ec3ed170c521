/*
 * FP64 CPU oracle for list-mode multi-energy-window OSEM SPECT
 * (arXiv 2305.17111).  TEST INFRASTRUCTURE ONLY: see lmmew_oracle.h.
 *
 * Each function states the passage of the paper it follows.  Where the paper
 * leaves a quantity open, the reading used is stated beside the code.
 */
#include "lmmew_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* Threads the OpenMP loops of this library will use. */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads the OpenMP loops of this library use (n >= 1). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* FWHM of a Gaussian in units of its standard deviation: 2 sqrt(2 ln 2). */
static double fwhm_per_sigma(void) { return 2.0 * sqrt(2.0 * log(2.0)); }

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

/* Detector angle a of na evenly spaced angles over 360 degrees (Sec. 3.1.2).
 * Multiples of 90 degrees get exact unit vectors so that rays along the grid
 * axes are recognised as such. */
void or_angle_dir(int a, int na, double *c, double *s)
{
    if ((4 * a) % na == 0) {
        static const double cs[4] = {1.0, 0.0, -1.0, 0.0};
        static const double sn[4] = {0.0, 1.0, 0.0, -1.0};
        int k = ((4 * a) / na) % 4;
        *c = cs[k];
        *s = sn[k];
        return;
    }
    double th = 2.0 * OR_PI * (double)a / (double)na;
    *c = cos(th);
    *s = sin(th);
}

static double pixel_mu(const double *mu, int n, int ix, int iy)
{
    if (ix < 0 || iy < 0 || ix >= n || iy >= n) return 0.0;
    return mu[iy * n + ix];
}

static int near_integer(double f, long *k)
{
    double r = floor(f + 0.5);
    if (fabs(f - r) < 1e-9) { *k = (long)r; return 1; }
    return 0;
}

/* Attenuation value seen by a segment at point (xm, ym).  A segment lying
 * exactly on a grid line (only possible for an axis-parallel segment) sees
 * the mean of the two pixels that share the line: the limit of segments
 * displaced by +-delta. */
static double mu_seen(const double *mu, int n, double pix, double xm,
                      double ym, int vertical, int horizontal)
{
    double R = 0.5 * n * pix;
    double fx = (xm + R) / pix, fy = (ym + R) / pix;
    long k;
    if (vertical && near_integer(fx, &k)) {
        int iy = (int)floor(fy);
        return 0.5 * (pixel_mu(mu, n, (int)k - 1, iy) + pixel_mu(mu, n, (int)k, iy));
    }
    if (horizontal && near_integer(fy, &k)) {
        int ix = (int)floor(fx);
        return 0.5 * (pixel_mu(mu, n, ix, (int)k - 1) + pixel_mu(mu, n, ix, (int)k));
    }
    return pixel_mu(mu, n, (int)floor(fx), (int)floor(fy));
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Eq. (6): the radiological path, the integral of the attenuation map along
 * the straight segment from (x0,y0) to (x1,y1).  The map is piecewise
 * constant on pixels and zero outside the grid, so the integral is the sum
 * over the pieces between successive grid-line crossings of (value at the
 * piece's midpoint) x (piece length). */
double or_segment_integral(const double *mu, int n, double pix,
                           double x0, double y0, double x1, double y1)
{
    double R = 0.5 * n * pix;
    double dx = x1 - x0, dy = y1 - y0;
    double L = sqrt(dx * dx + dy * dy);
    if (L == 0.0) return 0.0;
    double *ts = (double *)malloc(sizeof(double) * (size_t)(2 * (n + 1) + 2));
    int m = 0;
    ts[m++] = 0.0;
    ts[m++] = 1.0;
    for (int k = 0; k <= n; ++k) {
        double g = -R + k * pix;
        if (dx != 0.0) {
            double t = (g - x0) / dx;
            if (t > 0.0 && t < 1.0) ts[m++] = t;
        }
        if (dy != 0.0) {
            double t = (g - y0) / dy;
            if (t > 0.0 && t < 1.0) ts[m++] = t;
        }
    }
    qsort(ts, (size_t)m, sizeof(double), cmp_double);
    double sum = 0.0;
    for (int i = 0; i + 1 < m; ++i) {
        double t0 = ts[i], t1 = ts[i + 1];
        if (t1 <= t0) continue;
        double tm = 0.5 * (t0 + t1);
        double v = mu_seen(mu, n, pix, x0 + tm * dx, y0 + tm * dy,
                           dx == 0.0, dy == 0.0);
        sum += v * (t1 - t0) * L;
    }
    free(ts);
    return sum;
}

/* Phi(zhi) - Phi(zlo) for the standard normal CDF, evaluated with erfc on
 * the side where it does not cancel. */
double or_Phi_diff(double zhi, double zlo)
{
    const double r2 = sqrt(0.5);
    if (zlo >= 0.0) return 0.5 * (erfc(zlo * r2) - erfc(zhi * r2));
    if (zhi <= 0.0) return 0.5 * (erfc(-zhi * r2) - erfc(-zlo * r2));
    return 1.0 - 0.5 * erfc(zhi * r2) - 0.5 * erfc(-zlo * r2);
}

/* ------------------------------------------------------------------------ */
/* Physics                                                                   */
/* ------------------------------------------------------------------------ */

/* Klein-Nishina differential cross-section (the K of Eq. (5)) up to the
 * constant r_e^2/2: P^2 (P + 1/P - sin^2 phi), P = E'/E = 1/(1+eps(1-cos phi)),
 * eps = E / (m_e c^2). */
double or_kn_K(double cosphi, double E, double me)
{
    double eps = E / me;
    double P = 1.0 / (1.0 + eps * (1.0 - cosphi));
    double sin2 = 1.0 - cosphi * cosphi;
    return P * P * (P + 1.0 / P - sin2);
}

/* Normaliser of the Klein-Nishina weight restricted to the 2-D plane
 * (Sec. 3.2.1): Z(E) = integral over phi in [0, 2pi) of K.  The integrand is
 * smooth and periodic, so the trapezoid rule on 4096 nodes is exact to
 * rounding. */
double or_kn_Z(double E, double me)
{
    const int N = 4096;
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
        double phi = 2.0 * OR_PI * (double)i / (double)N;
        s += or_kn_K(cos(phi), E, me);
    }
    return s * (2.0 * OR_PI / (double)N);
}

/* Energy resolution (Sec. 3.1.2): FWHM = frac * ref at the reference energy,
 * the relative FWHM falling as 1/sqrt(E), so the absolute FWHM grows as
 * sqrt(E).  Evaluated at the photon's true energy. */
double or_sigmaE(const or_sys *S, double E)
{
    return S->eres_frac * S->eres_ref * sqrt(E / S->eres_ref) / fwhm_per_sigma();
}

double or_gauss(double x, double mean, double sigma)
{
    double z = (x - mean) / sigma;
    return exp(-0.5 * z * z) / (sigma * sqrt(2.0 * OR_PI));
}

/* Probability that a photon of true energy E is recorded inside one of the
 * energy windows (Sec. 3.2.2 windows). */
double or_acc(const or_sys *S, double E)
{
    double sig = or_sigmaE(S, E), a = 0.0;
    for (int k = 0; k < S->nwin; ++k)
        a += or_Phi_diff((S->whi[k] - E) / sig, (S->wlo[k] - E) / sig);
    return a;
}

/* Energy dependence of attenuation.  Sec. 3.1.1 fits water's attenuation
 * with a bilinear curve in energy but prints no coefficients; this oracle
 * reads it as a power law mu(E) = mu(E_ref) (E/E_ref)^(-p) with the exponent
 * a system parameter. */
double or_mu_scale(const or_sys *S, double E)
{
    return pow(E / S->mu_ref, -S->mu_pow);
}

/* Collimator-detector response: Gaussian with FWHM = fwhm0 + slope*depth. */
double or_psf_sigma(const or_sys *S, double depth)
{
    return (S->fwhm0 + S->fwhm_slope * depth) / fwhm_per_sigma();
}

/* Probability that a photon leaving (x,y) along n_a is recorded in bin b:
 * the position attribute of pr(A_hat | P, E) in Eq. (3). */
double or_psf_bin(const or_geom *G, int b, double x, double y, int a)
{
    double c, s;
    or_angle_dir(a, G->S.na, &c, &s);
    double u = -x * s + y * c;
    double depth = G->R - (x * c + y * s);
    double sig = or_psf_sigma(&G->S, depth);
    double lo = -G->R + b * G->db, hi = lo + G->db;
    return or_Phi_diff((hi - u) / sig, (lo - u) / sig);
}

/* Density per mm of the lateral position u at which a photon leaving (x,y)
 * along n_a is recorded, for a detector that reports a continuous position
 * instead of a bin: the position attribute of pr(A_hat | P, E) in Eq. (3)
 * as a density.  Its integral over bin b is or_psf_bin, and over [-R, R]
 * or_psf_total. */
double or_psf_density(const or_geom *G, double u, double x, double y, int a)
{
    double c, s;
    or_angle_dir(a, G->S.na, &c, &s);
    double u0 = -x * s + y * c;
    double depth = G->R - (x * c + y * s);
    return or_gauss(u, u0, or_psf_sigma(&G->S, depth));
}

/* Probability that the photon lands anywhere on the detector [-R, R]. */
double or_psf_total(const or_geom *G, double x, double y, int a)
{
    double c, s;
    or_angle_dir(a, G->S.na, &c, &s);
    double u = -x * s + y * c;
    double depth = G->R - (x * c + y * s);
    double sig = or_psf_sigma(&G->S, depth);
    return or_Phi_diff((G->R - u) / sig, (-G->R - u) / sig);
}

/* ------------------------------------------------------------------------ */
/* Precomputation (Algorithm 1: radiological paths and voxel set)            */
/* ------------------------------------------------------------------------ */

static void pixel_centre(const or_geom *G, int q, double *x, double *y)
{
    int n = G->S.n;
    *x = ((q % n) + 0.5) * G->S.pix - G->R;
    *y = ((q / n) + 0.5) * G->S.pix - G->R;
}

int or_geom_build(or_geom *G, const or_sys *S, const double *mu85,
                  const uint8_t *mask)
{
    memset(G, 0, sizeof(*G));
    G->S = *S;
    int n = S->n;
    if (n <= 0 || S->ns <= 0 || n % S->ns != 0 || ((n / S->ns) % 2) != 0)
        return -1;
    G->Q = n * n;
    G->R = 0.5 * n * S->pix;
    G->hs = 2.0 * G->R / S->ns;
    G->db = 2.0 * G->R / S->nb;
    G->mu = (double *)malloc(sizeof(double) * G->Q);
    G->support = (uint8_t *)malloc((size_t)G->Q);
    memcpy(G->mu, mu85, sizeof(double) * G->Q);
    for (int q = 0; q < G->Q; ++q) {
        double x, y;
        pixel_centre(G, q, &x, &y);
        int in = (x * x + y * y <= G->R * G->R);
        if (mask) in = in && mask[q];
        G->support[q] = (uint8_t)in;
    }
    /* scatter points: cell centres, mean attenuation of covered pixels */
    int m = n / S->ns;
    G->sx = (double *)malloc(sizeof(double) * S->ns * S->ns);
    G->sy = (double *)malloc(sizeof(double) * S->ns * S->ns);
    G->smu = (double *)malloc(sizeof(double) * S->ns * S->ns);
    G->nsc = 0;
    for (int ky = 0; ky < S->ns; ++ky)
        for (int kx = 0; kx < S->ns; ++kx) {
            double x = (kx + 0.5) * G->hs - G->R, y = (ky + 0.5) * G->hs - G->R;
            double acc = 0.0;
            for (int j = 0; j < m; ++j)
                for (int i = 0; i < m; ++i)
                    acc += mu85[(ky * m + j) * n + (kx * m + i)];
            acc /= (double)(m * m);
            if (x * x + y * y <= G->R * G->R && acc > 0.0) {
                G->sx[G->nsc] = x;
                G->sy[G->nsc] = y;
                G->smu[G->nsc] = acc;
                G->nsc++;
            }
        }
    /* attenuation line integrals at mu_ref (Eq. (6)) */
    int na = S->na;
    G->g_qa = (double *)calloc((size_t)na * G->Q, sizeof(double));
    G->g_qs = (double *)calloc((size_t)G->Q * (G->nsc > 0 ? G->nsc : 1), sizeof(double));
    G->g_sa = (double *)calloc((size_t)na * (G->nsc > 0 ? G->nsc : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < G->Q; ++q) {
        if (!G->support[q]) continue;
        double x, y;
        pixel_centre(G, q, &x, &y);
        for (int a = 0; a < na; ++a) {
            double c, s;
            or_angle_dir(a, na, &c, &s);
            double d = G->R - (x * c + y * s);
            G->g_qa[(size_t)a * G->Q + q] =
                or_segment_integral(mu85, n, S->pix, x, y, x + d * c, y + d * s);
        }
        for (int si = 0; si < G->nsc; ++si)
            G->g_qs[(size_t)q * G->nsc + si] =
                or_segment_integral(mu85, n, S->pix, x, y, G->sx[si], G->sy[si]);
    }
    for (int a = 0; a < na; ++a) {
        double c, s;
        or_angle_dir(a, na, &c, &s);
        for (int si = 0; si < G->nsc; ++si) {
            double x = G->sx[si], y = G->sy[si];
            double d = G->R - (x * c + y * s);
            G->g_sa[(size_t)a * G->nsc + si] =
                or_segment_integral(mu85, n, S->pix, x, y, x + d * c, y + d * s);
        }
    }
    for (int w = 0; w < S->nw; ++w) G->Zw[w] = or_kn_Z(S->E[w], S->me);
    return 0;
}

void or_geom_free(or_geom *G)
{
    free(G->mu); free(G->support);
    free(G->sx); free(G->sy); free(G->smu);
    free(G->g_qa); free(G->g_qs); free(G->g_sa);
    memset(G, 0, sizeof(*G));
}

/* ------------------------------------------------------------------------ */
/* Path sensitivities: Eq. (4)-(5) times the emission yield of Sec. 2.3      */
/* ------------------------------------------------------------------------ */

/* Unscattered path from pixel q to detector angle a at line w:
 * alpha_w * (collimator acceptance / 2 pi) * exp(-gamma(q -> detector, E_w)).
 * In 2-D an isotropic emitter sends a fraction dtheta/(2 pi) of its photons
 * into the collimator's acceptance (the Delta Omega / 4 pi of Eq. (5) read in
 * the plane). */
double or_Pp(const or_geom *G, int q, int a, int w)
{
    const or_sys *S = &G->S;
    double fw = or_mu_scale(S, S->E[w]);
    return S->alpha[w] * S->dtheta / (2.0 * OR_PI) *
           exp(-fw * G->g_qa[(size_t)a * G->Q + q]);
}

/* Once-scattered path pixel q -> scatter point si -> detector angle a at
 * line w (Eq. (5) with n = 1, read in the plane on a grid of scatter points):
 *   alpha_w * hs^2 / (2 pi r) * mu(s, E_w) * exp(-gamma(q -> s, E_w))
 *   * p_KN(phi; E_w) * dtheta * exp(-gamma(s -> detector, E'))
 * hs^2/(2 pi r) * mu is the probability that the isotropically emitted
 * photon interacts in the scatter cell at distance r, p_KN dtheta the
 * probability of leaving it into the collimator's acceptance, and
 * E' = E_w P(phi) the Compton energy.  r is clamped below at hs/(2 sqrt(pi)),
 * the exact mean of 1/r over a disk of area hs^2 centred on the emitter. */
double or_Ps(const or_geom *G, int q, int si, int a, int w, double *Eprime)
{
    const or_sys *S = &G->S;
    double xq, yq, c, s;
    pixel_centre(G, q, &xq, &yq);
    or_angle_dir(a, S->na, &c, &s);
    double dx = G->sx[si] - xq, dy = G->sy[si] - yq;
    double r = sqrt(dx * dx + dy * dy);
    double reff = fmax(r, G->hs / (2.0 * sqrt(OR_PI)));
    double cosphi = (dx * c + dy * s) / r;
    double E = S->E[w];
    double P = 1.0 / (1.0 + (E / S->me) * (1.0 - cosphi));
    double Ep = E * P;
    double pkn = or_kn_K(cosphi, E, S->me) / G->Zw[w];
    double fw = or_mu_scale(S, E), fp = or_mu_scale(S, Ep);
    double v = S->alpha[w] * G->hs * G->hs / (2.0 * OR_PI * reff) *
               G->smu[si] * fw *
               exp(-fw * G->g_qs[(size_t)q * G->nsc + si]) *
               pkn * S->dtheta *
               exp(-fp * G->g_sa[(size_t)a * G->nsc + si]);
    if (Eprime) *Eprime = Ep;
    return v;
}

/* Position factor of an event for a photon leaving (x,y) along n_a: the bin
 * probability when the event carries detector bin b (pos == NULL), the
 * density at *pos when it carries a continuous position. */
static double pos_factor(const or_geom *G, int b, const double *pos, double x,
                         double y, int a)
{
    return pos ? or_psf_density(G, *pos, x, y, a) : or_psf_bin(G, b, x, y, a);
}

/* Per-event system row (Eq. (3) with Eq. (4)'s numerator, per unit
 * activity): for every pixel q,
 *   a_q = sum_w [ Pp(q,a,w) psf(b | x_q, a) G(E_hat; E_w)
 *               + sum_s Ps(q,s,a,w) psf(b | x_s, a) G(E_hat; E'_{qsaw}) ]
 * with the energy Gaussian evaluated at the photon's true energy.  Pixels
 * outside the support get 0.  With primary == 0 only the scattered terms
 * are summed. */
static void event_row(const or_geom *G, int b, const double *pos, int a,
                      double Ehat, int primary, double *row)
{
    const or_sys *S = &G->S;
    for (int q = 0; q < G->Q; ++q) {
        row[q] = 0.0;
        if (!G->support[q]) continue;
        double xq, yq;
        pixel_centre(G, q, &xq, &yq);
        double psf_q = primary ? pos_factor(G, b, pos, xq, yq, a) : 0.0;
        double acc = 0.0;
        for (int w = 0; w < S->nw; ++w) {
            if (primary)
                acc += or_Pp(G, q, a, w) * psf_q *
                       or_gauss(Ehat, S->E[w], or_sigmaE(S, S->E[w]));
            for (int si = 0; si < G->nsc; ++si) {
                double Ep;
                double ps = or_Ps(G, q, si, a, w, &Ep);
                acc += ps * pos_factor(G, b, pos, G->sx[si], G->sy[si], a) *
                       or_gauss(Ehat, Ep, or_sigmaE(S, Ep));
            }
        }
        row[q] = acc;
    }
}

void or_event_row(const or_geom *G, int b, int a, double Ehat, double *row)
{
    event_row(G, b, NULL, a, Ehat, 1, row);
}

/* The row of an event recorded at continuous lateral position u (mm): the
 * same sum with the bin probability replaced by the density. */
void or_event_row_pos(const or_geom *G, double u, int a, double Ehat, double *row)
{
    event_row(G, 0, &u, a, Ehat, 1, row);
}

/* The once-scattered part of or_event_row alone (the quantity the scatter
 * surrogate learns): sum over lines and scatter points of the scattered
 * path terms. */
void or_event_row_scatter(const or_geom *G, int b, int a, double Ehat, double *row)
{
    event_row(G, b, NULL, a, Ehat, 0, row);
}

/* Row of event j of a list whose position attribute is bin[j], or pos[j]
 * when pos is not NULL. */
static void list_row(const or_geom *G, const int *bin, const double *pos, long j,
                     const int *ang, const double *E, double *row)
{
    event_row(G, pos ? 0 : bin[j], pos ? pos + j : NULL, ang[j], E[j], 1, row);
}

/* Detection probability per unit activity of pixel q at angle a (Eq. (7)
 * restricted to one pixel and one angle, counting only photons that land on
 * the detector and inside an energy window). */
double or_sens_qa(const or_geom *G, int q, int a)
{
    const or_sys *S = &G->S;
    double xq, yq;
    pixel_centre(G, q, &xq, &yq);
    double Dq = or_psf_total(G, xq, yq, a);
    double acc = 0.0;
    for (int w = 0; w < S->nw; ++w) {
        acc += or_Pp(G, q, a, w) * Dq * or_acc(S, S->E[w]);
        for (int si = 0; si < G->nsc; ++si) {
            double Ep;
            double ps = or_Ps(G, q, si, a, w, &Ep);
            acc += ps * or_psf_total(G, G->sx[si], G->sy[si], a) * or_acc(S, Ep);
        }
    }
    return acc;
}

/* Denominator of Eq. (18): T * sum over the subset's angles of the pixel
 * sensitivity.  Subset s holds the angles a with a mod nsub == s. */
void or_sensitivity(const or_geom *G, int nsub, double *sens)
{
    int na = G->S.na;
    memset(sens, 0, sizeof(double) * (size_t)nsub * G->Q);
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < G->Q; ++q) {
        if (!G->support[q]) continue;
        for (int a = 0; a < na; ++a)
            sens[(size_t)(a % nsub) * G->Q + q] += G->S.T * or_sens_qa(G, q, a);
    }
}

/* One subset's row of or_sensitivity: T * sum over the angles a with
 * a mod nsub == s of the pixel sensitivity (the denominator of Eq. (18) for
 * that subset alone). */
void or_sensitivity_subset(const or_geom *G, int nsub, int s, double *sens_s)
{
    int na = G->S.na;
    memset(sens_s, 0, sizeof(double) * (size_t)G->Q);
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < G->Q; ++q) {
        if (!G->support[q]) continue;
        for (int a = s; a < na; a += nsub)
            sens_s[q] += G->S.T * or_sens_qa(G, q, a);
    }
}

/* Masses of the categorical over (support pixel, angle, line, component)
 * from which the exact-model sampler draws: lambda_q * path sensitivity *
 * probability of landing on the detector * window acceptance.  Component 0
 * is the unscattered path, component 1+si the path through scatter point si.
 * Layout: ((qi*na + a)*nw + w)*(1+nsc) + comp, qi = rank of q in the support.
 * Returns the number of entries written. */
long or_sample_masses(const or_geom *G, const double *lambda, double *mass)
{
    const or_sys *S = &G->S;
    int na = S->na, nw = S->nw, nc = 1 + G->nsc;
    int *qs = (int *)malloc(sizeof(int) * G->Q);
    int Qm = 0;
    for (int q = 0; q < G->Q; ++q)
        if (G->support[q]) qs[Qm++] = q;
#pragma omp parallel for schedule(dynamic)
    for (int qi = 0; qi < Qm; ++qi) {
        int q = qs[qi];
        double xq, yq;
        pixel_centre(G, q, &xq, &yq);
        for (int a = 0; a < na; ++a) {
            double Dq = or_psf_total(G, xq, yq, a);
            for (int w = 0; w < nw; ++w) {
                double *m = mass + (((size_t)qi * na + a) * nw + w) * nc;
                m[0] = lambda[q] * or_Pp(G, q, a, w) * Dq * or_acc(S, S->E[w]);
                for (int si = 0; si < G->nsc; ++si) {
                    double Ep;
                    double ps = or_Ps(G, q, si, a, w, &Ep);
                    m[1 + si] = lambda[q] * ps *
                                or_psf_total(G, G->sx[si], G->sy[si], a) *
                                or_acc(S, Ep);
                }
            }
        }
    }
    free(qs);
    return (long)Qm * na * nw * nc;
}

/* ------------------------------------------------------------------------ */
/* List-mode OSEM (Sec. 2.4, Eq. (18)-(20); Algorithm 1)                     */
/* ------------------------------------------------------------------------ */

/* Event lists carry either detector bins (bin, with pos == NULL) or
 * continuous lateral positions in mm (pos, with bin unused).
 * Returns the index of the first event with a bin, position or angle out of
 * range (positions must lie in [-R, R)) or an energy outside every window,
 * or -1 when all are valid. */
int or_check_events(const or_geom *G, long nev, const int *bin,
                    const double *pos, const int *ang, const double *E)
{
    const or_sys *S = &G->S;
    for (long j = 0; j < nev; ++j) {
        if (ang[j] < 0 || ang[j] >= S->na) return (int)j;
        if (pos ? !(pos[j] >= -G->R && pos[j] < G->R)
                : (bin[j] < 0 || bin[j] >= S->nb))
            return (int)j;
        int in = 0;
        for (int k = 0; k < S->nwin; ++k)
            if (E[j] >= S->wlo[k] && E[j] <= S->whi[k]) in = 1;
        if (!in || !isfinite(E[j])) return (int)j;
    }
    return -1;
}

/* p_j = sum_q a_jq lambda_q: the denominator of Eq. (19). */
void or_forward(const or_geom *G, long nev, const int *bin, const double *pos,
                const int *ang, const double *E, const double *lambda, double *p)
{
#pragma omp parallel
    {
        double *row = (double *)malloc(sizeof(double) * G->Q);
#pragma omp for schedule(static)
        for (long j = 0; j < nev; ++j) {
            list_row(G, bin, pos, j, ang, E, row);
            double s = 0.0;
            for (int q = 0; q < G->Q; ++q) s += row[q] * lambda[q];
            p[j] = s;
        }
        free(row);
    }
}

/* out_q = sum_j a_jq w_j, events in input order. */
void or_backproject(const or_geom *G, long nev, const int *bin,
                    const double *pos, const int *ang, const double *E,
                    const double *wj, double *out)
{
    double *rows = (double *)malloc(sizeof(double) * (size_t)nev * G->Q);
#pragma omp parallel for schedule(static)
    for (long j = 0; j < nev; ++j)
        list_row(G, bin, pos, j, ang, E, rows + (size_t)j * G->Q);
    for (int q = 0; q < G->Q; ++q) out[q] = 0.0;
    for (long j = 0; j < nev; ++j) {
        if (wj[j] == 0.0) continue;
        for (int q = 0; q < G->Q; ++q) out[q] += rows[(size_t)j * G->Q + q] * wj[j];
    }
    free(rows);
}

/* LM-OSEM: for each iteration and each angle subset s (in order 0..nsub-1),
 * with the current image (the eta schedule of Eq. (20)):
 *   p_j = sum_q a_jq lambda_q                  for events j of subset s
 *   B_q = sum_{j in s, p_j > 0} a_jq / p_j
 *   lambda_q <- lambda_q B_q / sens_s[q]        where sens_s[q] > 0
 * which is Eq. (18) with z_bar of Eq. (19) summed over the paths of pixel q.
 * Events with p_j = 0 carry no information about the image and are skipped
 * and counted.  hist (optional) receives the image after every
 * sub-iteration; ll (optional) receives sum_j log p_j - sum_q sens_s[q]
 * lambda_q evaluated before the update (with one subset this is the
 * log-likelihood of Eq. (8) up to a constant); skipped (optional) receives
 * the number of skipped events.  The rows come from row(ctx, j, out), so the
 * loop serves every system model. */
int or_osem_rows(long nev, const int *ang, int Q, int nsub, int niter,
                 const double *sens, double *lambda, double *hist, double *ll,
                 long *skipped, or_row_fn row, const void *ctx)
{
    long *idx = (long *)malloc(sizeof(long) * (nev > 0 ? nev : 1));
    double *rows = NULL;
    double *p = (double *)malloc(sizeof(double) * (nev > 0 ? nev : 1));
    double *B = (double *)malloc(sizeof(double) * Q);
    int k = 0;
    for (int it = 0; it < niter; ++it) {
        for (int s = 0; s < nsub; ++s, ++k) {
            long ns = 0;
            for (long j = 0; j < nev; ++j)
                if (ang[j] % nsub == s) idx[ns++] = j;
            free(rows);
            rows = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1) * Q);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < ns; ++i)
                row(ctx, idx[i], rows + (size_t)i * Q);
            long skip = 0;
            double llv = 0.0;
            for (long i = 0; i < ns; ++i) {
                double acc = 0.0;
                for (int q = 0; q < Q; ++q) acc += rows[(size_t)i * Q + q] * lambda[q];
                p[i] = acc;
                if (acc > 0.0) llv += log(acc);
                else skip++;
            }
            for (int q = 0; q < Q; ++q) llv -= sens[(size_t)s * Q + q] * lambda[q];
            for (int q = 0; q < Q; ++q) B[q] = 0.0;
            for (long i = 0; i < ns; ++i) {
                if (!(p[i] > 0.0)) continue;
                for (int q = 0; q < Q; ++q) B[q] += rows[(size_t)i * Q + q] / p[i];
            }
            for (int q = 0; q < Q; ++q) {
                double d = sens[(size_t)s * Q + q];
                if (d > 0.0) lambda[q] = lambda[q] * B[q] / d;
            }
            if (hist) memcpy(hist + (size_t)k * Q, lambda, sizeof(double) * Q);
            if (ll) ll[k] = llv;
            if (skipped) skipped[k] = skip;
        }
    }
    free(idx); free(rows); free(p); free(B);
    return 0;
}

/* Event list of the planar model, for the row callback. */
typedef struct {
    const or_geom *G;
    const int *bin, *ang;
    const double *pos, *E;
} list2d;

static void list2d_row(const void *ctx, long j, double *row)
{
    const list2d *L = (const list2d *)ctx;
    list_row(L->G, L->bin, L->pos, j, L->ang, L->E, row);
}

int or_osem(const or_geom *G, long nev, const int *bin, const double *pos,
            const int *ang, const double *E, int nsub, int niter, const double *sens,
            double *lambda, double *hist, double *ll, long *skipped)
{
    list2d L = {G, bin, ang, pos, E};
    return or_osem_rows(nev, ang, G->Q, nsub, niter, sens, lambda, hist, ll, skipped,
                        list2d_row, &L);
}
