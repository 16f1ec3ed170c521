// Internal structures shared by the host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lmmew.h"

namespace lmmew {

constexpr int kWave = 64;          // CDNA wavefront
constexpr float kLog2e = 1.4426950408889634f;
constexpr double kPi = 3.14159265358979323846;
// scatter-list entry .x: the point's index in its angle's list (low bits) and
// the mask of the tile's groups of 16 events that its response reaches
constexpr int kSlistGroupShift = 24;
constexpr int kSlistPoint = (1 << kSlistGroupShift) - 1;
// An event drops a line's scattered terms when their energy factor is below
// 2^-kLineCutBits for every energy the scattered photon can have.  Tiles hold
// events of one line mask; k_row is specialised per mask for up to
// kMaskedLines lines (more lines keep every line).
constexpr int kLineCutBits = 40;
constexpr int kMaskedLines = 3;
constexpr float kPsfCut = 7.0f;    // collimator-response Gaussian dropped beyond 7 sigma

// scatter surrogate network (6 -> 128 -> 128 -> 128 -> 1)
constexpr int kMlpIn = 6;
constexpr int kMlpHidden = 128;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHidden;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden * kMlpHidden;
constexpr int kOffW4 = kOffB3 + kMlpHidden;
constexpr int kOffB4 = kOffW4 + kMlpHidden;
constexpr int kMlpParams = kOffB4 + 1;            // 34049
constexpr float kMlpEc = 180.f, kMlpEs = 120.f;   // energy feature: (E - kMlpEc) / kMlpEs
constexpr int kRedRows = 32;                      // rows per chunk of the bias-gradient column sums

// Per-run constants passed by value to the kernels.
struct DevSys {
    int n, ns, nb, na, nw, nwin;
    int Qm, Qp, nsc;
    float pix, R, hs, db;
    float fwhm0, fslope;            // PSF FWHM = fwhm0 + fslope * depth
    float inv_fwhm_to_sigma;        // 1 / (2 sqrt(2 ln 2))
    float T;
    float eres_k;                   // sigma_E^2 = eres_k * E
    float mu_pow;
    float rmin;                     // planar: hs / (2 sqrt(pi)); 3-D: (3 V / 4 pi)^(1/3) / sqrt(3)
    int nz, nbz;                    // 3-D: slices and axial bins (nz = 0: the planar model)
    float Zh, dbz;                  // 3-D: axial half-length and axial bin width
    // per line
    float E[LMMEW_MAX_LINES];
    float eps[LMMEW_MAX_LINES];     // E / m_e c^2
    float f[LMMEW_MAX_LINES];       // mu(E_w)/mu_ref
    float pp[LMMEW_MAX_LINES];      // alpha_w * dtheta / (2 pi); 3-D: alpha_w * dOmega / (4 pi)
    float lsc[LMMEW_MAX_LINES];     // log2(alpha_w * f_w * dtheta / Z_w); 3-D: dOmega, sphere Z_w
    float c0[LMMEW_MAX_LINES];      // log2(e) / (2 eres_k E_w)
    float sqc0[LMMEW_MAX_LINES];    // sqrt(c0)
    float nc[LMMEW_MAX_LINES];      // -0.5 log2(2 pi eres_k E_w)
    float gnorm[LMMEW_MAX_LINES];   // 1 / sqrt(2 pi eres_k E_w)
    float wlo[LMMEW_MAX_WINDOWS], whi[LMMEW_MAX_WINDOWS];
    float sqck;                     // sqrt(log2(e) / (2 eres_k)): s_w = sqck / sqrt(E')
};

// Scatter point as seen from one angle (array [na][nsc], sorted by u).
struct ScatA {
    float x, y;         // position (mm)
    float u;            // lateral detector coordinate
    float isig;         // 1 / PSF sigma at its depth
    float gsa;          // attenuation integral at mu_ref to the detector plane
    float lc;           // log2(hs^2 * mu_s / (2 pi)); 3-D: log2(V * mu_s / (4 pi))
    float D;            // probability of landing on the detector
    int sidx;           // index into the [nsc][Qp] pixel->scatter table
};

// Work tile of the per-event kernel: events [e0, e0+cnt) of one angle and
// one case; entries [k0, k1) of the plan's scatter list name the angle's
// (u-sorted) scatter points whose response reaches at least one of them.
struct Tile {
    int e0, cnt;
    int angle, ncase;
    int k0, k1;
    int lmask;          // lines whose scattered terms its events keep (bit w: line w)
    int pad;
};

// Chunk of consecutive rows of one case for the deterministic backprojection.
struct Chunk {
    int r0, r1, ncase, pad;
};

// ---- launchers (kernels.hip) ------------------------------------------------
// Attenuation tables, computed in double precision.  In 3-D, pixz and scz
// hold the z of the support voxels and of the scatter points (NULL in 2-D).
hipError_t launch_tables_d(const DevSys &S, const double *mu, const double2 *pix,
                           const double *pixz, const double2 *dirs, const double2 *sc,
                           const double *scz, float *g_qa, float *g_qs, ScatA *sa, double pixmm,
                           double R, hipStream_t st);

// Tables of one attenuation map, for plans whose cases use different maps.
struct MapTab {
    const float *g_qa;       // [na][Qp]
    const float *g_qs;       // [nsc][Qp]
    const ScatA *sa;         // [na][nsc]
    const float *ptab;       // path-parameter table (see RowArgs) or NULL
    const float *resp;       // collimator-response factors (see RowArgs)
    const float *respz;      // 3-D: axial response factors (see RowArgs)
    const float *sz;         // 3-D: scatter-point z (see RowArgs)
    int nsc, pad;
};

struct RowArgs {
    const float2 *pix_xy;
    const float2 *dirs;
    const float *g_qa;
    const float *g_qs;
    const ScatA *sa;
    const MapTab *maps;      // [ncases] tables per case, or NULL (g_qa, g_qs, sa, S.nsc)
    const float *ptab;       // scatter-path parameters [na][nsc][nw][Qp][2] (per line and
                             // pixel: log2 weight A_w, s_w; the kernel derives F_w =
                             // log2(e) / (2 k s_w)), or NULL to evaluate them in the kernel
    const float *resp;       // [na][nsc][nb] collimator-response factor of scatter point k
                             // (angle's sorted order) for bin b, 0 beyond 7 sigma
    const float *respz;      // 3-D: [na][nsc][nbz] the same for the axial bin
    const float *pix_z;      // 3-D: [Qp] z of the support voxels
    const float *sz;         // 3-D: [nsc] z of the scatter points (by g_qs row)
    const Tile *tiles;
    const int2 *slist;       // scatter list entries of the tiles: (point in the angle's
                             // sorted list, row of the point in the g_qs table)
    int ntiles;
    const int *case_tiles;   // [ncases+1]: the tiles of case c are [case_tiles[c],
                             // case_tiles[c+1]) (tiles are grouped by case): work items
                             // case-major; or NULL: block-major over all tiles
    int ncases;
    const int *ev_bin;       // sorted rows of this subset: detector bins (NULL for positions)
    const int *ev_binz;      // 3-D: sorted rows: axial bins
    const float *ev_u;       // sorted rows: continuous lateral positions (mm), or NULL (bins)
    const float *ev_E;
    float *A;                // [rows][Qp]
    int mode;                // 0: all paths, 1: scattered paths only, 2: unscattered only
    const float *pvt;        // [slist entry][event tile]: response factor of each listed
                             // point for each event of its tile (0 past the tile's events)
    const float *psft;       // planar binned events: [na][nb][Qp] bin probabilities of the
                             // unscattered paths, or NULL to form them in the kernel
};
hipError_t launch_row(const DevSys &S, const RowArgs &r, int event_tile, hipStream_t st);
// bin probability of the unscattered path of every (angle, bin, support pixel)
hipError_t launch_psf_table(const DevSys &S, const float2 *pix_xy, const float2 *dirs,
                            float *psft, hipStream_t st);
// the response-factor table of the tiles of one subset (written to pvt)
hipError_t launch_pv_table(const DevSys &S, const RowArgs &r, int event_tile, float *pvt,
                           hipStream_t st);
// collimator-response factors of every (angle, scatter point, bin); in 3-D also
// every (angle, scatter point, axial bin) into respz (sz: scatter-point z by g_qs row)
hipError_t launch_resp_table(const DevSys &S, const ScatA *sa, float *resp, const float *sz,
                             float *respz, hipStream_t st);
// scatter-path parameters of every (angle, scatter point, support pixel)
hipError_t launch_path_table(const DevSys &S, const float2 *pix_xy, const float *pix_z,
                             const float2 *dirs, const float *g_qs, const ScatA *sa,
                             const float *sz, float *ptab, hipStream_t st);

struct FwdArgs {
    const float *A;          // [rows][Qp]
    int rows;
    const int *row_case;     // [rows]
    const float *lamc;       // [ncases][Qp] image on the support pixels (0 in the padding)
    float *p;                // [rows]
    float *wt;               // [rows] 1/p (0 if p <= 0)
    double *logp;            // [rows] log p (0 if p <= 0), may be NULL
    unsigned long long *nskip;   // may be NULL
};
hipError_t launch_forward(const DevSys &S, const FwdArgs &f, hipStream_t st);
// lamc[c][i] = lambda[c][pixq[i]] on the support, 0 in the padding
hipError_t launch_compact(const DevSys &S, const float *lambda, int ncases, int Q, const int *pixq,
                          float *lamc, hipStream_t st);

struct BackArgs {
    const float *A;
    const float *wt;         // [rows]
    const Chunk *chunks;
    int nchunks;
    float *part;             // [nchunks][Qp]
    float *comp;             // [nchunks][Qp]
};
hipError_t launch_back(const DevSys &S, const BackArgs &b, hipStream_t st);

struct UpdArgs {
    const float *part, *comp;
    const int *case_chunk;   // [ncases+1] chunk ranges per case
    int ncases;
    const int *pixq;
    int Q;
    const float *sens;       // [Q] of this subset, or NULL (plain backprojection)
    long sens_stride;        // elements from one case's sensitivity to the next (0: shared)
    float *lambda;           // [ncases][Q] in/out (update) or out (backprojection)
    float *lamc;             // [ncases][Qp] support copy of the updated image, or NULL
};
hipError_t launch_update(const DevSys &S, const UpdArgs &u, hipStream_t st);

struct SensArgs {
    const float2 *pix_xy;
    const float *pix_z;      // 3-D: [Qp] voxel z
    const float *sz;         // 3-D: [nsc] scatter-point z by g_qs row
    const float2 *dirs;
    const float *g_qa;
    const float *g_qs;
    const ScatA *sa;
    const int *pixq;
    float *Sqa;              // [na][Qp]
    float *sens;             // [nsub][Q]
    int nsub, Q;
};
hipError_t launch_sens(const DevSys &S, const SensArgs &a, hipStream_t st);

struct ReduceArgs {          // deterministic sums for statistics
    const double *logp;
    int rows;
    const float *sens;       // [Q]
    long sens_stride;        // elements from one case's sensitivity to the next (0: shared)
    const float *lambda;     // [ncases][Q]
    int ncases, Q;
    double *out;             // [1]: sum logp - sum sens*lambda
};
hipError_t launch_loglik(const ReduceArgs &r, hipStream_t st);

hipError_t launch_scatter_out(const float *src, const int64_t *perm, int64_t n, float *dst,
                              hipStream_t st);
hipError_t launch_rows_out(const DevSys &S, const float *A, int rows, const int64_t *perm,
                           const int *pixq, int Q, float *out, hipStream_t st);
// out[k][pixq[i]] = A[ridx[k]][i] for k < n (rows picked from the subset scratch)
hipError_t launch_rows_pick(const DevSys &S, const float *A, const int *ridx, int n,
                            const int *pixq, int Q, float *out, hipStream_t st);
hipError_t launch_gather_w(const float *w, const int64_t *perm, int64_t n, float *dst,
                           hipStream_t st);
// out[0] = sum of x[0..n) in FP64 (fixed order: deterministic)
hipError_t launch_sum(const float *x, long n, double *out, hipStream_t st);
// out[r] = sum of row r of A [rows][Qp] in FP64, in a fixed order
hipError_t launch_row_sums(const float *A, int rows, int Qp, double *out, hipStream_t st);
hipError_t launch_roi_sums(const float *lam, int C, int Q, const uint8_t *masks, int K,
                           double *out, hipStream_t st);

// ---- scatter surrogate (mlp.hip) ------------------------------------------
struct MlpWork {             // activations of one training batch
    float *X, *Z1, *Z2, *Z3, *H3, *dZ, *dH, *y, *dy, *sq;
    float *part, *split;               // reduction partials: [M/256][8][128], [64][128][128]
    double *dsum;
    unsigned short *H1b, *H2b, *dZb;
    const unsigned short *W2b, *W3b;   // bf16 [in][out], then the transpose [out][in]
};
struct MlpRowArgs {
    const float2 *pix_xy, *dirs;
    const int *ev_bin, *ev_ang;
    const float *ev_E;
    int rows;
    float *A;
    const float *P;                    // fp32 parameters
    float c0, floor_;
    const int *ev_scale;               // rows' entries of case_scale, or NULL
    const float *case_scale;           // [cases][windows] factor on the density, or NULL (1)
    int npix;                          // positions evaluated: pix_xy[0, npix)
    int ld;                            // row stride of A (floats)
    int assign;                        // 1: A = density (coarse nodes); 0: A += density
};
// Rows' scattered densities at the support pixels by bilinear interpolation of
// the network's values at the coarse nodes (lmmew_set_scatter_grid):
// A[e][q] += sum_k w[q].k * C[e][idx[q].k] for the Qm support pixels of rows rows.
hipError_t launch_coarse_interp(const DevSys &S, const float *C, int ldc, const int4 *idx,
                                const float4 *w, int rows, float *A, hipStream_t st);
// The same rows in one pass with their unscattered part (planar, binned
// events, with the unscattered bin-probability table): A[e][i] = the
// unscattered part of row e at support pixel i, as the per-event kernel forms
// it from the table, plus the interpolated node values; 0 on padding pixels.
struct PrimInterpArgs {
    const float *psft;                 // [na][nb][Qp] unscattered bin probabilities
    const float *g_qa;                 // [na][Qp] pixel -> detector integrals (one map), or
    const MapTab *maps;                // per-case tables (then ev_case names the case), or NULL
    const int *ev_bin, *ev_ang, *ev_case;
    const float *ev_E;
    int rows;
    const float *C;                    // [rows][ldc] node values
    int ldc;
    const int4 *idx;                   // [Qp] a support pixel's four nodes
    const float4 *w;                   // [Qp] their weights
    float *A;                          // [rows][Qp] written
};
hipError_t launch_prim_interp(const DevSys &S, const PrimInterpArgs &a, hipStream_t st);
hipError_t mlp_forward_batch(const MlpWork &w, const float *P, const float *feats, const int *idx,
                             int M, const float *tgt, hipStream_t st);
hipError_t mlp_backward_batch(const MlpWork &w, const float *P, int M, float *G, hipStream_t st);
hipError_t mlp_loss(const MlpWork &w, int M, double *out, hipStream_t st);
hipError_t mlp_adam(float *P, const float *G, float *m1, float *m2, float lr, int step,
                    hipStream_t st);
hipError_t mlp_refresh(const float *P, unsigned short *W2b, unsigned short *W3b,
                       hipStream_t st);
hipError_t mlp_labels(const DevSys &S, const float2 *pix_xy, const float2 *dirs, const int *ev_bin,
                      const int *ev_ang, const float *ev_E, const float *A, int rows, float *feats,
                      float *raw, hipStream_t st);
hipError_t mlp_targets(const float *raw, long n, float floor_, float c0, float *tgt,
                       hipStream_t st);
hipError_t mlp_rows(const DevSys &S, const MlpRowArgs &a, hipStream_t st);

}  // namespace lmmew
