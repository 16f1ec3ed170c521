/*
 * FP64 CPU oracle for list-mode multi-energy-window OSEM SPECT
 * (Rahman, Li, Yu, Laforest, Thorek, Jha, arXiv 2305.17111).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * shares no code, header or table with it.
 *
 * Everything here is plain, slow and written to be read against the paper:
 * one function per quantity, double precision throughout, no blocking, no
 * caching beyond the attenuation line integrals that the paper's Algorithm 1
 * itself precomputes.
 *
 * Geometry conventions (readings of a paper that fixes only the symbolic
 * model; each is listed with its reason in the design notes):
 *   - square grid n x n, pixel size pix (mm); FOV = n*pix centred on (0,0);
 *     pixel (ix,iy) has centre ((ix+1/2)pix - R, (iy+1/2)pix - R), R = FOV/2,
 *     and flat index q = iy*n + ix;
 *   - support: pixel centres with |x| <= R (the circular field of view of
 *     Sec. 3.1.2) that are also set in the optional caller mask;
 *   - scatter grid ns x ns, cell side hs = FOV/ns, point at the cell centre,
 *     mu_s = mean of the pixels the cell covers; a point is used when
 *     |x_s| <= R and mu_s > 0;
 *   - angle a has direction n_a = (cos th, sin th), th = 2 pi a / na, exact at
 *     multiples of 90 degrees; lateral axis t_a = (-sin th, cos th); the
 *     detector plane is x.n_a = R and bin b covers
 *     u in [-R + b*db, -R + (b+1)*db), db = FOV/nb.
 */
#ifndef LMMEW_ORACLE_H
#define LMMEW_ORACLE_H

#include <stdint.h>

#define OR_MAX_LINES 8
#define OR_MAX_WIN 8

typedef struct {
    int n;              /* pixels per side */
    double pix;         /* pixel size, mm */
    int ns;             /* scatter points per side (n/ns even) */
    int nb, na;         /* detector bins, angles over 360 degrees */
    double fwhm0;       /* collimator-detector PSF FWHM at depth 0, mm */
    double fwhm_slope;  /* PSF FWHM growth per mm of depth */
    double dtheta;      /* collimator angular acceptance, rad */
    int nw;             /* emission lines */
    double E[OR_MAX_LINES];      /* line energies, keV */
    double alpha[OR_MAX_LINES];  /* photons per decay for each line */
    int nwin;           /* energy windows */
    double wlo[OR_MAX_WIN], whi[OR_MAX_WIN];
    double eres_frac;   /* energy FWHM as a fraction at eres_ref */
    double eres_ref;    /* keV */
    double mu_ref;      /* keV at which the attenuation map is given */
    double mu_pow;      /* mu(E) = mu_ref_map * (E/mu_ref)^(-mu_pow) */
    double T;           /* acquisition time */
    double me;          /* electron rest energy, keV */
} or_sys;

typedef struct {
    or_sys S;
    double R, hs, db;
    int Q;                 /* n*n */
    double *mu;            /* [Q] attenuation at mu_ref, 1/mm */
    uint8_t *support;      /* [Q] 1 where lambda may be non-zero */
    int nsc;               /* scatter points in use */
    double *sx, *sy, *smu; /* [nsc] position and mean attenuation */
    double *g_qa;          /* [na][Q]   pixel centre -> detector plane */
    double *g_qs;          /* [Q][nsc]  pixel centre -> scatter point */
    double *g_sa;          /* [na][nsc] scatter point -> detector plane */
    double Zw[OR_MAX_LINES];  /* 2-D Klein-Nishina normaliser per line */
} or_geom;

int    or_threads(void);
void   or_set_threads(int n);

/* ---- physics and geometry primitives ---------------------------------- */
void   or_angle_dir(int a, int na, double *c, double *s);
double or_segment_integral(const double *mu, int n, double pix,
                           double x0, double y0, double x1, double y1);
double or_Phi_diff(double zhi, double zlo);
double or_kn_K(double cosphi, double E, double me);
double or_kn_Z(double E, double me);
double or_sigmaE(const or_sys *S, double E);
double or_gauss(double x, double mean, double sigma);
double or_acc(const or_sys *S, double E);
double or_mu_scale(const or_sys *S, double E);
double or_psf_sigma(const or_sys *S, double depth);
double or_psf_bin(const or_geom *G, int b, double x, double y, int a);
double or_psf_total(const or_geom *G, double x, double y, int a);
double or_psf_density(const or_geom *G, double u, double x, double y, int a);

/* ---- model ------------------------------------------------------------- */
int    or_geom_build(or_geom *G, const or_sys *S, const double *mu85,
                     const uint8_t *mask);
void   or_geom_free(or_geom *G);
double or_Pp(const or_geom *G, int q, int a, int w);
double or_Ps(const or_geom *G, int q, int si, int a, int w, double *Eprime);
void   or_event_row(const or_geom *G, int b, int a, double Ehat, double *row);
void   or_event_row_pos(const or_geom *G, double u, int a, double Ehat, double *row);
void   or_event_row_scatter(const or_geom *G, int b, int a, double Ehat, double *row);
double or_sens_qa(const or_geom *G, int q, int a);
void   or_sensitivity(const or_geom *G, int nsub, double *sens);
void   or_sensitivity_subset(const or_geom *G, int nsub, int s, double *sens_s);
long   or_sample_masses(const or_geom *G, const double *lambda, double *mass);

/* ---- list-mode OSEM ----------------------------------------------------- */
/* Event lists: bin[j] (detector bin) when pos is NULL, else pos[j] (lateral
 * position in mm, continuous); ang[j] angle index; E[j] energy in keV. */
int  or_check_events(const or_geom *G, long nev, const int *bin,
                     const double *pos, const int *ang, const double *E);
void or_forward(const or_geom *G, long nev, const int *bin, const double *pos,
                const int *ang, const double *E, const double *lambda, double *p);
void or_backproject(const or_geom *G, long nev, const int *bin,
                    const double *pos, const int *ang, const double *E,
                    const double *wj, double *out);
/* Row a_j of event j (Q values) for the OSEM loop below. */
typedef void (*or_row_fn)(const void *ctx, long j, double *row);
int  or_osem_rows(long nev, const int *ang, int Q, int nsub, int niter,
                  const double *sens, double *lambda, double *hist, double *ll,
                  long *skipped, or_row_fn row, const void *ctx);
int  or_osem(const or_geom *G, long nev, const int *bin, const double *pos,
             const int *ang, const double *E, int nsub, int niter, const double *sens,
             double *lambda, double *hist, double *ll, long *skipped);

#endif
