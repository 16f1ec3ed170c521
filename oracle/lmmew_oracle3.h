/*
 * FP64 CPU oracle, 3-D single-scatter model (the extension the paper's
 * Discussion, Sec. 5, and its appendix on 3-D computational requirements name
 * as the next step, with the scatter modelled at a lower resolution).
 *
 * TEST INFRASTRUCTURE ONLY, like the planar oracle (lmmew_oracle.h).
 *
 * Geometry (readings; the planar conventions extended along z):
 *   - voxel grid n x n x nz of cubes of side pix; voxel (ix,iy,iz) has centre
 *     ((ix+1/2)pix - R, (iy+1/2)pix - R, (iz+1/2)pix - Zh), R = n pix / 2,
 *     Zh = nz pix / 2, flat index q = (iz*n + iy)*n + ix;
 *   - support: voxel centres with x^2 + y^2 <= R^2 (a cylindrical field of
 *     view), also set in the optional caller mask;
 *   - the camera rotates about z: angle a has n_a = (cos th, sin th, 0), the
 *     detector plane is x.n_a = R, the detector coordinates are
 *     u = x.t_a (t_a = (-sin th, cos th, 0)) and v = z; bin (b, bz) covers
 *     u in [-R + b db, -R + (b+1) db), v in [-Zh + bz dbz, -Zh + (bz+1) dbz);
 *   - scatter grid ns x ns x nsz of cells hs x hs x hz (n/ns and nz/nsz
 *     even), point at the cell centre, mu_s = mean of the covered voxels,
 *     used when x_s^2 + y_s^2 <= R^2 and mu_s > 0.
 */
#ifndef LMMEW_ORACLE3_H
#define LMMEW_ORACLE3_H

#include "lmmew_oracle.h"

typedef struct {
    or_sys S;          /* transaxial grid, lines, windows, resolutions */
    int nz;            /* slices */
    int nsz;           /* scatter points along z */
    int nbz;           /* axial detector bins */
    double domega;     /* collimator acceptance solid angle, sr */
} or3_sys;

typedef struct {
    or3_sys S3;
    double R, Zh, hs, hz, db, dbz;
    int Q;                 /* n*n*nz */
    double *mu;            /* [Q] attenuation at mu_ref, 1/mm */
    uint8_t *support;      /* [Q] */
    int nsc;
    double *sx, *sy, *sz, *smu;   /* [nsc] */
    double *g_qa;          /* [na][Q]   voxel centre -> detector plane */
    double *g_qs;          /* [Q][nsc]  voxel centre -> scatter point */
    double *g_sa;          /* [na][nsc] scatter point -> detector plane */
    double Zw[OR_MAX_LINES];   /* Klein-Nishina normaliser over the sphere */
} or3_geom;

double or3_segment_integral(const double *mu, int n, int nz, double pix, double x0,
                            double y0, double z0, double x1, double y1, double z1);
double or3_kn_Z(double E, double me);
int    or3_geom_build(or3_geom *G, const or3_sys *S, const double *mu85,
                      const uint8_t *mask);
void   or3_geom_free(or3_geom *G);
void   or3_voxel_centre(const or3_geom *G, int q, double *x, double *y, double *z);
double or3_Pp(const or3_geom *G, int q, int a, int w);
double or3_Ps(const or3_geom *G, int q, int si, int a, int w, double *Eprime);
double or3_psf_bin(const or3_geom *G, int b, int bz, double x, double y, double z, int a);
double or3_psf_total(const or3_geom *G, double x, double y, double z, int a);
void   or3_event_row(const or3_geom *G, int b, int bz, int a, double Ehat, double *row);
void   or3_event_row_scatter(const or3_geom *G, int b, int bz, int a, double Ehat,
                             double *row);
double or3_sens_qa(const or3_geom *G, int q, int a);
void   or3_sensitivity(const or3_geom *G, int nsub, double *sens);
int    or3_check_events(const or3_geom *G, long nev, const int *bin, const int *binz,
                        const int *ang, const double *E);
void   or3_forward(const or3_geom *G, long nev, const int *bin, const int *binz,
                   const int *ang, const double *E, const double *lambda, double *p);
int    or3_osem(const or3_geom *G, long nev, const int *bin, const int *binz,
                const int *ang, const double *E, int nsub, int niter,
                const double *sens, double *lambda, double *hist, double *ll,
                long *skipped);

#endif
