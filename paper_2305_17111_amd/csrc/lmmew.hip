// Host side of the lmmew C ABI: context (attenuation tables), event plans
// (validation, sorting, work tiles) and the OSEM driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace lmmew;

struct lmmew_ctx {
    lmmew_system sys{};
    DevSys S{};
    std::string err;
    int Q = 0;
    double R = 0, hs = 0, db = 0;
    std::vector<int> pixq;            // [Qp] full-grid index of support pixel i, -1 for padding
    std::vector<double> dir_c, dir_s; // [na]
    std::vector<ScatA> sa;            // [na][nsc] host copy (x, y, u, isig, lc, sidx)
    std::vector<double> sig_max;      // [na] largest PSF sigma over the scatter points
    std::vector<int> rb_lo, rb_hi;    // [na][nsc] bins reached by each scatter point's response
    std::vector<int> rbz_lo, rbz_hi;  // 3-D: [na][nsc] axial bins reached
    // device
    float2 *d_pix = nullptr;
    double2 *d_pixd = nullptr;
    int *d_pixq = nullptr;
    float2 *d_dirs = nullptr;
    double2 *d_dirsd = nullptr;
    double2 *d_scd = nullptr;
    double *d_mu = nullptr;
    float *d_gqa = nullptr, *d_gqs = nullptr;
    ScatA *d_sa = nullptr;
    float *d_Sqa = nullptr;
    hipStream_t cap_stream = nullptr; // private stream that graph captures are recorded on
    float *d_ptab = nullptr;          // scatter-path parameter table (lmmew_path_table) or NULL
    float *d_resp = nullptr;          // [na][nsc][nb] collimator-response factors
    float *d_psft = nullptr;          // planar: [na][nb][Qp] unscattered bin probabilities
    bool psft_off = false;            // the table is disabled (lmmew_psf_table) or did not fit
    float *d_respz = nullptr;         // 3-D: [na][nsc][nbz] axial response factors
    float *d_pixz = nullptr;          // 3-D: [Qp] voxel z
    double *d_pixzd = nullptr;        // 3-D: [Qp] voxel z (double, for the tables)
    float *d_scz = nullptr;           // 3-D: [nsc] scatter-point z
    double *d_sczd = nullptr;         // 3-D: [nsc] scatter-point z (double)
    lmmew_mlp *mlp = nullptr;         // scatter surrogate used by OSEM (NULL: exact model)
    // factor on the surrogate's density for this map's cases, per energy window
    float scatter_scale[LMMEW_MAX_WINDOWS] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
    std::vector<lmmew_mlp *> nets;    // networks created on this context (detached when it goes)
    int model_gen = 0;                // bumped whenever the scatter model changes
    // The exact model's scattered part evaluated at node pixels every xgrid
    // pixels and interpolated (lmmew_set_scatter_pixel_grid; 1: every pixel).
    int xgrid = 1;
    int xncn = 0, xldc = 0;           // node pixels; row stride of the node values
    float2 *d_xnode = nullptr;        // [xldc] node positions (support pixels)
    int4 *d_xidx = nullptr;           // [Qp] a support pixel's nodes (node indices)
    float4 *d_xw = nullptr;           // [Qp] their weights
    float *d_xgqa = nullptr;          // [na][xldc] pixel -> detector integrals at the nodes
    float *d_xgqs = nullptr;          // [nsc][xldc] pixel -> scatter point integrals at the nodes
};

struct lmmew_mlp {
    lmmew_ctx *ctx = nullptr;
    float *P = nullptr, *G = nullptr, *m1 = nullptr, *m2 = nullptr;   // [kMlpParams]
    unsigned short *W2b = nullptr, *W3b = nullptr;   // bf16 copies for training: [in][out],
                                                     // then the transpose [out][in]
    double c0 = 0.0, floor_ = 0.0;    // target = log(density + floor) - c0
    int step = 0;                     // Adam step count
    // Evaluation grid in OSEM (lmmew_mlp_set_grid): nodes every `grid` pixels
    // of the context's support, support pixels interpolated bilinearly
    // (grid 1: the network at every support pixel, no node tables).
    int grid = 1;
    int ncn = 0, ldc = 0;             // nodes; row stride of the node values (multiple of 64)
    float2 *d_cnode = nullptr;        // [ldc] node positions (padding repeats the last node)
    int4 *d_cidx = nullptr;           // [Qp] a support pixel's four nodes
    float4 *d_cw = nullptr;           // [Qp] their bilinear weights
    // training workspace for batches of up to cap samples
    int cap = 0;
    float *X = nullptr, *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *H3 = nullptr, *dZ = nullptr,
          *dH = nullptr, *y = nullptr, *dy = nullptr, *sq = nullptr;
    unsigned short *H1b = nullptr, *H2b = nullptr, *dZb = nullptr;
    int *idx = nullptr;
    double *dloss = nullptr;
    float *part = nullptr, *split = nullptr;
    double *dsum = nullptr;
};

struct lmmew_plan {
    lmmew_ctx *ctx = nullptr;
    std::vector<lmmew_ctx *> maps;    // [ncases] context (attenuation map) of each case, or empty
    std::vector<MapTab> maptab;       // what d_maps holds
    int nsub = 1, ncases = 1, JT = 64;
    int64_t n = 0;
    std::vector<int> bin, ang, cas;   // sorted rows
    int *d_ang = nullptr;
    std::vector<float> E;
    std::vector<int> lm;              // sorted rows: lines whose scattered terms are kept
    bool cont = false;                // events carry continuous positions (u), not bins
    std::vector<float> u;             // sorted rows: lateral position (mm) when cont
    std::vector<int> binz;            // 3-D: sorted rows: axial bins
    std::vector<int64_t> perm;        // sorted row -> input index
    struct Sub {
        int row0 = 0, rows = 0;
        int tile0 = 0, ntiles = 0;
        int chunk0 = 0, nchunks = 0;
    };
    std::vector<Sub> subs;
    std::vector<int> case_chunk;      // [nsub][ncases+1], chunk index relative to the subset
    std::vector<int> case_rows;       // [nsub][ncases+1], row index relative to the subset
    std::vector<int> case_tiles;      // [nsub][ncases+1], tile index relative to the subset
    std::vector<Tile> tiles;
    std::vector<int2> slist;          // scatter list entries of all tiles: (point, table row)
    std::vector<Chunk> chunks;
    int max_rows = 0, max_chunks = 0;
    double terms = 0, full_terms = 0;
    // device
    int *d_bin = nullptr, *d_binz = nullptr, *d_case = nullptr, *d_case_chunk = nullptr;
    int *d_case_tiles = nullptr;
    float *d_E = nullptr, *d_u = nullptr;
    int64_t *d_perm = nullptr;
    Tile *d_tiles = nullptr;
    int2 *d_slist = nullptr;
    float *d_pvt = nullptr;           // [slist entry][JT] response factors
    MapTab *d_maps = nullptr;
    MapTab *d_xmaps = nullptr;        // the cases' node tables (lmmew_set_scatter_pixel_grid)
    std::vector<MapTab> xmaptab;      // what d_xmaps holds
    Chunk *d_chunks = nullptr;
    float *d_A = nullptr, *d_p = nullptr, *d_wt = nullptr;
    float *d_C = nullptr;             // network values at the coarse nodes of a subset's rows
    size_t C_cap = 0;                 // floats in d_C
    float *d_Acache = nullptr;        // [n][Qp] rows of every subset (lmmew_plan_cache_rows) or NULL
    float *d_lamc = nullptr;          // [ncases][Qp] support copy of the current images
    float *d_cscale = nullptr;        // [ncases][nwin] surrogate density factor of each case
                                      // and energy window
    std::vector<float> cscale;        // what d_cscale holds
    int *d_sidx = nullptr;            // sorted rows: entry of d_cscale (case * nwin + window)
    int cache_gen = -1;               // scatter-model generation the cached rows were computed with
    double *d_logp = nullptr, *d_ll = nullptr;
    float *d_part = nullptr, *d_comp = nullptr;
    unsigned long long *d_nskip = nullptr;
    int stats_cap = 0;
    // captured OSEM sequence (lmmew_osem_graph) and the arguments it was captured with
    hipGraphExec_t gexec = nullptr;
    int g_iters = -1, g_jt = 0, g_gen = -1;
    const float *g_cache = nullptr, *g_tab = nullptr, *g_psft = nullptr;
    const float *g_sens = nullptr;
    float *g_lambda = nullptr;
    // optional timing of the per-event kernel launches (HIP events on the caller's stream)
    bool prof = false;
    std::vector<hipEvent_t> prof_ev;  // pairs of events around timed launches
    std::vector<int> prof_kind;       // per pair: 0 k_row, 1 k_mlp_rows
    size_t prof_used = 0;
};

namespace {

constexpr int kChunkRows = 128;
constexpr size_t kScratchBudget = size_t(2) << 30;   // per-call a_jq scratch for forward/adjoint

int fail(lmmew_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

int hipfail(lmmew_ctx *ctx, hipError_t e, const char *what)
{
    if (ctx) ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory) ? LMMEW_ENOMEM : LMMEW_EDEVICE;
}

#define HIPCHK(ctx, call)                                        \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hipfail((ctx), e_, #call);  \
    } while (0)

template <class T>
hipError_t dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

template <class T>
void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

double fwhm_per_sigma() { return 2.0 * std::sqrt(2.0 * std::log(2.0)); }

// Klein-Nishina normaliser over the sphere: the integral of P^2 (P + 1/P -
// sin^2 phi) over all directions, 2 sigma_KN / r_e^2, from the closed-form
// total Klein-Nishina cross-section (k = E / m_e c^2 >= 1e-3 here).
double kn_norm_sphere(double E, double me)
{
    const double k = E / me, l = std::log1p(2.0 * k);
    return 4.0 * kPi * ((1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k) +
                        l / (2.0 * k) - (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k)));
}

// Planar Klein-Nishina normaliser: integral over the circle of
// P^2 (P + 1/P - sin^2 phi), by the periodic trapezoid rule.
double kn_norm(double E, double me)
{
    const int N = 2048;
    const double eps = E / me;
    double s = 0.0;
    for (int k = 0; k < N; ++k) {
        const double ph = 2.0 * kPi * (k + 0.5) / N;
        const double cp = std::cos(ph);
        const double P = 1.0 / (1.0 + eps * (1.0 - cp));
        s += P * P * (P + 1.0 / P - (1.0 - cp * cp));
    }
    return s * 2.0 * kPi / N;
}

void angle_dir(int a, int na, double *c, double *s)
{
    if ((4 * a) % na == 0) {
        const int k = ((4 * a) / na) % 4;
        const double cs[4] = {1, 0, -1, 0}, sn[4] = {0, 1, 0, -1};
        *c = cs[k];
        *s = sn[k];
        return;
    }
    const double th = 2.0 * kPi * a / na;
    *c = std::cos(th);
    *s = std::sin(th);
}

int validate_sys(lmmew_ctx *ctx, const lmmew_system *s)
{
    if (s->n <= 0 || s->ns <= 0 || s->n % s->ns != 0 || ((s->n / s->ns) % 2) != 0)
        return fail(ctx, LMMEW_EINVAL, "n must be a positive multiple of ns with an even ratio");
    if (s->n_bins <= 0 || s->n_angles <= 0 || s->n_bins > 32767 || s->n_angles > 32767)
        return fail(ctx, LMMEW_EINVAL, "n_bins and n_angles must be in 1..32767");
    if (s->n_lines < 1 || s->n_lines > LMMEW_MAX_LINES)
        return fail(ctx, LMMEW_EINVAL, "n_lines must be in 1..8");
    if (s->n_windows < 1 || s->n_windows > LMMEW_MAX_WINDOWS)
        return fail(ctx, LMMEW_EINVAL, "n_windows must be in 1..8");
    if (!(s->pixel_mm > 0) || !(s->psf_fwhm0_mm > 0) || !(s->psf_fwhm_slope >= 0) ||
        !(s->coll_dtheta > 0) || !(s->eres_frac > 0) || !(s->eres_ref_keV > 0) ||
        !(s->mu_ref_keV > 0) || !std::isfinite(s->mu_power) || !(s->T > 0) ||
        !(s->electron_keV > 0))
        return fail(ctx, LMMEW_EINVAL, "non-positive or non-finite system parameter");
    for (int w = 0; w < s->n_lines; ++w)
        if (!(s->line_keV[w] > 0) || !(s->line_yield[w] >= 0) || !std::isfinite(s->line_keV[w]))
            return fail(ctx, LMMEW_EINVAL, "bad emission line");
    for (int k = 0; k < s->n_windows; ++k)
        if (!(s->win_hi_keV[k] > s->win_lo_keV[k]) || !std::isfinite(s->win_lo_keV[k]) ||
            !std::isfinite(s->win_hi_keV[k]))
            return fail(ctx, LMMEW_EINVAL, "bad energy window");
    if (s->nz < 0) return fail(ctx, LMMEW_EINVAL, "nz must be >= 0");
    if (s->nz > 0) {
        if (s->ns_z <= 0 || s->nz % s->ns_z != 0 || ((s->nz / s->ns_z) % 2) != 0)
            return fail(ctx, LMMEW_EINVAL, "nz must be a positive multiple of ns_z with an even ratio");
        if (s->n_bins_z <= 0 || s->n_bins_z > 32767)
            return fail(ctx, LMMEW_EINVAL, "n_bins_z must be in 1..32767");
        if (!(s->coll_solid_angle > 0) || !std::isfinite(s->coll_solid_angle))
            return fail(ctx, LMMEW_EINVAL, "coll_solid_angle must be positive");
        if ((int64_t)s->n * s->n * s->nz > ((int64_t)1 << 30))
            return fail(ctx, LMMEW_EINVAL, "too many voxels");
    }
    return LMMEW_OK;
}

void free_ctx(lmmew_ctx *c)
{
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    dfree(c->d_pix); dfree(c->d_pixd); dfree(c->d_pixq); dfree(c->d_dirs); dfree(c->d_dirsd);
    dfree(c->d_scd); dfree(c->d_mu); dfree(c->d_gqa); dfree(c->d_gqs); dfree(c->d_sa);
    dfree(c->d_Sqa); dfree(c->d_ptab); dfree(c->d_resp); dfree(c->d_psft);
    dfree(c->d_respz); dfree(c->d_pixz); dfree(c->d_pixzd); dfree(c->d_scz); dfree(c->d_sczd);
    dfree(c->d_xnode); dfree(c->d_xidx); dfree(c->d_xw); dfree(c->d_xgqa); dfree(c->d_xgqs);
}

void free_plan(lmmew_plan *p)
{
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
    p->prof_ev.clear();
    dfree(p->d_bin); dfree(p->d_binz); dfree(p->d_u); dfree(p->d_ang); dfree(p->d_case); dfree(p->d_case_chunk); dfree(p->d_case_tiles); dfree(p->d_E); dfree(p->d_perm);
    dfree(p->d_tiles); dfree(p->d_slist); dfree(p->d_pvt); dfree(p->d_chunks); dfree(p->d_A); dfree(p->d_p); dfree(p->d_wt);
    dfree(p->d_C);
    dfree(p->d_logp); dfree(p->d_ll); dfree(p->d_part); dfree(p->d_comp); dfree(p->d_nskip);
    dfree(p->d_maps);
    dfree(p->d_xmaps);
    dfree(p->d_Acache);
    dfree(p->d_lamc);
    dfree(p->d_cscale);
    dfree(p->d_sidx);
}

bool in_window(const lmmew_system &s, float e)
{
    if (!std::isfinite(e)) return false;
    for (int k = 0; k < s.n_windows; ++k)
        if (e >= (float)s.win_lo_keV[k] && e <= (float)s.win_hi_keV[k]) return true;
    return false;
}

// The first window that holds energy e (the same comparisons as in_window;
// 0 for an energy in none).
int window_of(const lmmew_system &s, float e)
{
    for (int k = 0; k < s.n_windows; ++k)
        if (e >= (float)s.win_lo_keV[k] && e <= (float)s.win_hi_keV[k]) return k;
    return 0;
}

// Relevant (not pruned) scatter points of one event: those whose collimator
// response reaches the event's bin within kPsfCut standard deviations.
int relevant_scatter(const lmmew_ctx *c, int a, int b, int bz = 0)
{
    const int nsc = c->S.nsc;
    const bool d3 = c->S.nz > 0;
    int cnt = 0;
    for (int k = 0; k < nsc; ++k) {
        const size_t ak = (size_t)a * nsc + k;
        cnt += (b >= c->rb_lo[ak] && b <= c->rb_hi[ak]) &&
               (!d3 || (bz >= c->rbz_lo[ak] && bz <= c->rbz_hi[ak]));
    }
    return cnt;
}

// Continuous positions: the standardised deviation of position u from scatter
// point e's projection, in the per-event kernel's float arithmetic (monotone
// in u).
inline float pos_z(const ScatA &e, float u) { return (u - e.u) * e.isig; }

// Rows [first, last) of one angle with ascending positions: the sub-range
// whose density factor for scatter point e is not cut (|z| < kPsfCut).
std::pair<int, int> reached(const ScatA &e, const float *u, int first, int last)
{
    const float *lo = std::partition_point(u + first, u + last,
                                           [&](float v) { return pos_z(e, v) <= -kPsfCut; });
    const float *hi =
        std::partition_point(lo, u + last, [&](float v) { return pos_z(e, v) < kPsfCut; });
    return {(int)(lo - u), (int)(hi - u)};
}

// Lines whose once-scattered terms an event of measured energy E keeps.  A
// line's scattered photon reaches the detector with an energy between its
// backscatter energy E_w / (1 + 2 E_w / m_e c^2) and E_w (Compton kinematics
// of the scattered energies in Eq. (5)); the energy-resolution factor of
// Eq. (3)'s event probability at E is exp(-(E - E')^2 / (2 k E')) for
// scattered energy E' (variance k E', Sec. 3.1.2).
// A line's largest factor over its reachable E' is compared with the largest
// over all lines: when it is below 2^-kLineCutBits of that, the line's
// scattered terms are dropped for the event (its unscattered term is always
// kept, and the line with the largest factor is always kept, so an energy far
// from every line's reach keeps its nearest line instead of none).  Systems
// with more than kMaskedLines lines keep every line.
int line_mask(const lmmew_system &s, float Ef)
{
    const int all = (1 << s.n_lines) - 1;
    if (s.n_lines > kMaskedLines) return all;
    const double E = Ef;
    const double fps = fwhm_per_sigma();
    const double k = s.eres_frac * s.eres_frac * s.eres_ref_keV / (fps * fps);
    const double cut = kLineCutBits * std::log(2.0);
    double x[LMMEW_MAX_LINES], xmin = INFINITY;
    for (int w = 0; w < s.n_lines; ++w) {
        const double Ew = s.line_keV[w];
        const double Emin = Ew / (1.0 + 2.0 * Ew / s.electron_keV);
        const double Ep = E < Emin ? Emin : (E > Ew ? Ew : E);   // closest reachable energy
        x[w] = (E - Ep) * (E - Ep) / (2.0 * k * Ep);             // -log of the largest factor
        xmin = std::min(xmin, x[w]);
    }
    int m = 0;
    for (int w = 0; w < s.n_lines; ++w)
        if (x[w] - xmin <= cut) m |= 1 << w;
    return m;
}

// Scatter-list entry .x: point index k and the mask of the tile's groups of 16
// events that its response reaches.
inline int slist_x(int k, unsigned gm) { return k | (int)(gm << kSlistGroupShift); }

// Mask of the groups of 16 rows that rows [first, last) of a tile touch.
inline unsigned group_span(int first, int last)
{
    unsigned gm = 0;
    for (int g = first / 16; g <= (last - 1) / 16; ++g) gm |= 1u << g;
    return gm;
}

// Builds tiles and chunks of a plan for the event tile size p->JT.
void build_tiles(lmmew_plan *p)
{
    const int na = p->ctx->S.na;
    p->tiles.clear();
    p->slist.clear();
    p->chunks.clear();
    p->case_chunk.assign((size_t)p->nsub * (p->ncases + 1), 0);
    p->case_tiles.assign((size_t)p->nsub * (p->ncases + 1), 0);
    p->max_chunks = 0;
    for (int s = 0; s < p->nsub; ++s) {
        lmmew_plan::Sub &sub = p->subs[s];
        sub.tile0 = (int)p->tiles.size();
        sub.chunk0 = (int)p->chunks.size();
        int r = sub.row0;
        const int rend = sub.row0 + sub.rows;
        int *cc = &p->case_chunk[(size_t)s * (p->ncases + 1)];
        int cur_case = 0;
        // tiles: runs of <= JT rows with the same (case, angle)
        while (r < rend) {
            int e = r;
            const int cs = p->cas[r], a = p->ang[r];
            const lmmew_ctx *c = p->maps.empty() ? p->ctx : p->maps[cs];
            const int nsc = c->S.nsc;
            while (e < rend && e - r < p->JT && p->cas[e] == cs && p->ang[e] == a &&
                   p->lm[e] == p->lm[r])
                ++e;
            const int k0 = (int)p->slist.size();
            if (c->S.nz > 0) {
                // 3-D: scatter points whose response reaches some (bin, axial bin)
                // of the tile; the tile's bounding box first, then each event
                int bmin = p->bin[r], bmax = p->bin[r], zmin = p->binz[r], zmax = p->binz[r];
                for (int k = r; k < e; ++k) {
                    bmin = std::min(bmin, p->bin[k]);
                    bmax = std::max(bmax, p->bin[k]);
                    zmin = std::min(zmin, p->binz[k]);
                    zmax = std::max(zmax, p->binz[k]);
                }
                for (int k = 0; k < nsc; ++k) {
                    const size_t ak = (size_t)a * nsc + k;
                    const int lo = c->rb_lo[ak], hi = c->rb_hi[ak];
                    const int lz = c->rbz_lo[ak], hz = c->rbz_hi[ak];
                    if (hi < bmin || lo > bmax || hz < zmin || lz > zmax) continue;
                    unsigned gm = 0;
                    for (int j = r; j < e; ++j)
                        if (p->bin[j] >= lo && p->bin[j] <= hi && p->binz[j] >= lz &&
                            p->binz[j] <= hz)
                            gm |= 1u << ((j - r) / 16);
                    if (gm) p->slist.push_back(make_int2(slist_x(k, gm), c->sa[ak].sidx));
                }
            } else if (p->cont) {
                // scatter points whose density reaches some position of the tile
                for (int k = 0; k < nsc; ++k) {
                    const ScatA &sp = c->sa[(size_t)a * nsc + k];
                    const std::pair<int, int> rr = reached(sp, p->u.data(), r, e);
                    if (rr.first < rr.second)
                        p->slist.push_back(make_int2(
                            slist_x(k, group_span(rr.first - r, rr.second - r)), sp.sidx));
                }
            } else {
                int bmin = p->bin[r], bmax = p->bin[r];
                for (int k = r; k < e; ++k) {
                    bmin = std::min(bmin, p->bin[k]);
                    bmax = std::max(bmax, p->bin[k]);
                }
                // scatter points whose response reaches some bin of the tile
                for (int k = 0; k < nsc; ++k) {
                    const size_t ak = (size_t)a * nsc + k;
                    const int lo = c->rb_lo[ak], hi = c->rb_hi[ak];
                    if (hi < bmin || lo > bmax) continue;
                    // the tile's bins are sorted: the rows inside [lo, hi] are one run
                    const int *first = p->bin.data() + r, *lastp = p->bin.data() + e;
                    const int *it = std::lower_bound(first, lastp, lo);
                    const int *ie = std::upper_bound(it, lastp, hi);
                    if (it != ie)
                        p->slist.push_back(make_int2(
                            slist_x(k, group_span((int)(it - first), (int)(ie - first))),
                            c->sa[ak].sidx));
                }
            }
            const int k1 = (int)p->slist.size();
            Tile t{};
            t.e0 = r - sub.row0;
            t.cnt = e - r;
            t.angle = a;
            t.ncase = cs;
            t.k0 = k0;
            t.k1 = k1;
            t.lmask = p->lm[r];
            p->tiles.push_back(t);
            r = e;
        }
        sub.ntiles = (int)p->tiles.size() - sub.tile0;
        // Each case's tiles together (the per-event kernel walks the work
        // items case by case, so that the tiles it runs at one time share one
        // map's tables in the L2), costliest first within a case: the launch's
        // last work items are then cheap ones, which shortens the tail in
        // which CUs run out of work.
        std::stable_sort(p->tiles.begin() + sub.tile0, p->tiles.end(),
                         [](const Tile &x, const Tile &y) {
                             if (x.ncase != y.ncase) return x.ncase < y.ncase;
                             const double cx = (double)(x.k1 - x.k0) * x.cnt *
                                               (1 + 4 * __builtin_popcount(x.lmask));
                             const double cy = (double)(y.k1 - y.k0) * y.cnt *
                                               (1 + 4 * __builtin_popcount(y.lmask));
                             return cx > cy;
                         });
        {
            int *ct = &p->case_tiles[(size_t)s * (p->ncases + 1)];
            int t = 0;
            for (int c = 0; c < p->ncases; ++c) {
                ct[c] = t;
                while (t < sub.ntiles && p->tiles[sub.tile0 + t].ncase == c) ++t;
            }
            ct[p->ncases] = t;
        }
        // chunks: runs of <= kChunkRows rows of one case
        r = sub.row0;
        for (int cs = 0; cs < p->ncases; ++cs) {
            cc[cs] = (int)p->chunks.size() - sub.chunk0;
            while (r < rend && p->cas[r] == cs) {
                int e = r;
                while (e < rend && e - r < kChunkRows && p->cas[e] == cs) ++e;
                Chunk ch{};
                ch.r0 = r - sub.row0;
                ch.r1 = e - sub.row0;
                ch.ncase = cs;
                p->chunks.push_back(ch);
                r = e;
            }
            cur_case = cs;
        }
        (void)cur_case;
        cc[p->ncases] = (int)p->chunks.size() - sub.chunk0;
        sub.nchunks = (int)p->chunks.size() - sub.chunk0;
        p->max_chunks = std::max(p->max_chunks, sub.nchunks);
    }
    (void)na;
}

RowArgs row_args(const lmmew_ctx *ctx, const lmmew_plan *p, int s);

int upload_tiles(lmmew_ctx *ctx, lmmew_plan *p, hipStream_t st)
{
    // tiles and scatter-list entries are indexed with 32-bit integers
    if (p->slist.size() > (size_t)INT32_MAX || p->tiles.size() > (size_t)INT32_MAX)
        return fail(ctx, LMMEW_ENOMEM, "plan too large: more than 2^31 scatter-list entries");
    // a captured graph refers to the arrays about to be replaced
    if (p->gexec) {
        HIPCHK(ctx, hipGraphExecDestroy(p->gexec));
        p->gexec = nullptr;
    }
    dfree(p->d_tiles);
    dfree(p->d_slist);
    dfree(p->d_pvt);
    dfree(p->d_chunks);
    dfree(p->d_case_chunk);
    dfree(p->d_case_tiles);
    dfree(p->d_part);
    dfree(p->d_comp);
    HIPCHK(ctx, dalloc(&p->d_tiles, p->tiles.size()));
    HIPCHK(ctx, dalloc(&p->d_slist, p->slist.size()));
    HIPCHK(ctx, dalloc(&p->d_chunks, p->chunks.size()));
    HIPCHK(ctx, dalloc(&p->d_case_chunk, p->case_chunk.size()));
    HIPCHK(ctx, dalloc(&p->d_case_tiles, p->case_tiles.size()));
    const size_t total_chunks = std::max<size_t>(p->chunks.size(), 1);
    HIPCHK(ctx, dalloc(&p->d_part, total_chunks * ctx->S.Qp));
    HIPCHK(ctx, dalloc(&p->d_comp, total_chunks * ctx->S.Qp));
    if (!p->tiles.empty())
        HIPCHK(ctx, hipMemcpyAsync(p->d_tiles, p->tiles.data(), p->tiles.size() * sizeof(Tile),
                                   hipMemcpyHostToDevice, st));
    if (!p->slist.empty())
        HIPCHK(ctx, hipMemcpyAsync(p->d_slist, p->slist.data(), p->slist.size() * sizeof(int2),
                                   hipMemcpyHostToDevice, st));
    if (!p->chunks.empty())
        HIPCHK(ctx, hipMemcpyAsync(p->d_chunks, p->chunks.data(),
                                   p->chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(p->d_case_chunk, p->case_chunk.data(),
                               p->case_chunk.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(p->d_case_tiles, p->case_tiles.data(),
                               p->case_tiles.size() * sizeof(int), hipMemcpyHostToDevice, st));
    // response factors of the listed (point, event) pairs: JT floats per list entry
    if (!p->slist.empty()) {
        HIPCHK(ctx, dalloc(&p->d_pvt, p->slist.size() * (size_t)p->JT));
        for (int s = 0; s < p->nsub; ++s) {
            RowArgs r = row_args(ctx, p, s);
            HIPCHK(ctx, launch_pv_table(ctx->S, r, p->JT, p->d_pvt, st));
        }
    }
    HIPCHK(ctx, hipStreamSynchronize(st));
    return LMMEW_OK;
}

// Same geometry, support and model constants: contexts that differ only in
// their attenuation map (and hence in their scatter points).
bool same_system(const lmmew_ctx *a, const lmmew_ctx *b)
{
    DevSys x = a->S, y = b->S;
    x.nsc = y.nsc = 0;
    return std::memcmp(&x, &y, sizeof(DevSys)) == 0 && a->pixq == b->pixq;
}

int sync_maps(lmmew_ctx *ctx, lmmew_plan *p, hipStream_t st);

// maps: NULL, or the context of each of the n_cases cases (maps[0] == ctx)
// The unscattered paths' bin probabilities ([na][nb][Qp], planar systems),
// read by the per-event kernel instead of two erfc per (event, pixel).  Built
// on the first plan of a context (so that the contexts of the other patients
// of a plan over several maps, whose tables the kernel does not read, never
// hold one), kept to 2 GiB; when it does not fit, or when it is disabled, the
// kernel forms the probabilities itself.
int ensure_psft(lmmew_ctx *ctx, hipStream_t st)
{
    if (ctx->d_psft || ctx->psft_off || ctx->sys.nz > 0) return LMMEW_OK;
    const size_t n = (size_t)ctx->S.na * ctx->S.nb * ctx->S.Qp;
    if (n * sizeof(float) > (size_t(2) << 30)) {
        ctx->psft_off = true;
        return LMMEW_OK;
    }
    if (dalloc(&ctx->d_psft, n) != hipSuccess) {
        (void)hipGetLastError();          // clear the allocation failure; fall back
        ctx->d_psft = nullptr;
        ctx->psft_off = true;
        return LMMEW_OK;
    }
    HIPCHK(ctx, launch_psf_table(ctx->S, ctx->d_pix, ctx->d_dirs, ctx->d_psft, st));
    return LMMEW_OK;
}

int make_plan(lmmew_ctx *ctx, const lmmew_events *ev, const int64_t *case_offsets, int n_cases,
              int n_subsets, hipStream_t st, lmmew_plan **out, lmmew_ctx *const *maps = nullptr)
{
    *out = nullptr;
    if (maps) {
        for (int c = 0; c < n_cases; ++c) {
            if (!maps[c]) return fail(ctx, LMMEW_EINVAL, "NULL context in the case list");
            if (!same_system(ctx, maps[c]))
                return fail(ctx, LMMEW_EINVAL,
                            "contexts of a plan must share the system and the support");
        }
    }
    const bool cont = ev && ev->position_mm != nullptr;
    const bool d3 = ctx->S.nz > 0;
    if (!ev || ev->n < 0 ||
        (ev->n > 0 && ((!cont && !ev->bin) || !ev->angle || !ev->energy_keV ||
                       (d3 && !ev->bin_z))))
        return fail(ctx, LMMEW_EINVAL, "events: NULL array or negative count");
    if (d3 && cont)
        return fail(ctx, LMMEW_EINVAL, "continuous positions are not supported by the 3-D model");
    if (n_subsets < 1 || n_subsets > ctx->S.na)
        return fail(ctx, LMMEW_EINVAL, "n_subsets must be in 1..n_angles");
    if (n_cases < 1) return fail(ctx, LMMEW_EINVAL, "n_cases must be >= 1");
    const int64_t n = ev->n;
    if (n > ((int64_t)1 << 31) - 1) return fail(ctx, LMMEW_EINVAL, "too many events");
    {
        const int rp = ensure_psft(ctx, st);
        if (rp != LMMEW_OK) return rp;
    }
    std::vector<int64_t> off(n_cases + 1);
    if (case_offsets) {
        for (int c = 0; c <= n_cases; ++c) off[c] = case_offsets[c];
        if (off[0] != 0 || off[n_cases] != n)
            return fail(ctx, LMMEW_EINVAL, "case_offsets must start at 0 and end at n");
        for (int c = 0; c < n_cases; ++c)
            if (off[c + 1] < off[c]) return fail(ctx, LMMEW_EINVAL, "case_offsets not sorted");
    } else {
        if (n_cases != 1) return fail(ctx, LMMEW_EINVAL, "case_offsets required for n_cases > 1");
        off[0] = 0;
        off[1] = n;
    }
    std::vector<int16_t> hb(cont ? 0 : n), ha(n), hz(d3 ? n : 0);
    std::vector<float> he(n), hu(cont ? n : 0);
    if (n > 0) {
        if (cont)
            HIPCHK(ctx, hipMemcpyAsync(hu.data(), ev->position_mm, n * sizeof(float),
                                       hipMemcpyDeviceToHost, st));
        else
            HIPCHK(ctx, hipMemcpyAsync(hb.data(), ev->bin, n * sizeof(int16_t),
                                       hipMemcpyDeviceToHost, st));
        if (d3)
            HIPCHK(ctx, hipMemcpyAsync(hz.data(), ev->bin_z, n * sizeof(int16_t),
                                       hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipMemcpyAsync(ha.data(), ev->angle, n * sizeof(int16_t), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipMemcpyAsync(he.data(), ev->energy_keV, n * sizeof(float),
                                   hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
    }
    const lmmew_system &s = ctx->sys;
    const double Rmm = 0.5 * s.n * s.pixel_mm;
    for (int64_t j = 0; j < n; ++j) {
        const bool pos_ok = (cont ? ((double)hu[j] >= -Rmm && (double)hu[j] < Rmm)
                                  : (hb[j] >= 0 && hb[j] < s.n_bins)) &&
                            (!d3 || (hz[j] >= 0 && hz[j] < s.n_bins_z));
        if (!pos_ok || ha[j] < 0 || ha[j] >= s.n_angles || !in_window(s, he[j])) {
            char buf[160];
            if (cont)
                snprintf(buf, sizeof buf,
                         "event %lld invalid (position %g mm, angle %d, energy %g keV)",
                         (long long)j, (double)hu[j], (int)ha[j], (double)he[j]);
            else if (d3)
                snprintf(buf, sizeof buf,
                         "event %lld invalid (bin %d, axial bin %d, angle %d, energy %g keV)",
                         (long long)j, (int)hb[j], (int)hz[j], (int)ha[j], (double)he[j]);
            else
                snprintf(buf, sizeof buf,
                         "event %lld invalid (bin %d, angle %d, energy %g keV)", (long long)j,
                         (int)hb[j], (int)ha[j], (double)he[j]);
            return fail(ctx, LMMEW_EINVAL, buf);
        }
    }
    lmmew_plan *p = new (std::nothrow) lmmew_plan;
    if (!p) return fail(ctx, LMMEW_ENOMEM, "host allocation");
    p->ctx = ctx;
    if (maps) p->maps.assign(maps, maps + n_cases);
    p->nsub = n_subsets;
    p->ncases = n_cases;
    p->n = n;
    p->cont = cont;
    std::vector<int> casev(n);
    for (int c = 0; c < n_cases; ++c)
        for (int64_t j = off[c]; j < off[c + 1]; ++j) casev[j] = c;
    // 3-D: an angle's events spread over the whole 2-D detector, so ordering
    // them by (bin_z, bin) makes tiles of consecutive events long strips in u
    // whose scatter lists are several times longer than one event's.  They
    // are ordered by square detector blocks first (side chosen for about 16
    // events per block at the case's mean density, so that a case orders its
    // events alike in any plan), then by (bin_z, bin).  Blocks follow a Morton
    // curve, so runs of 2 and 4 blocks (the larger event tiles) are compact too.
    auto morton = [](uint32_t x, uint32_t y) {
        int64_t r = 0;
        for (int b = 0; b < 15; ++b)
            r |= ((int64_t)((x >> b) & 1u) << (2 * b)) | ((int64_t)((y >> b) & 1u) << (2 * b + 1));
        return r;
    };
    std::vector<int64_t> blk(d3 ? n : 0);
    if (d3) {
        const double area = 2.0 * Rmm * s.nz * s.pixel_mm;
        const double dbm = 2.0 * Rmm / s.n_bins, dbzm = s.nz * s.pixel_mm / s.n_bins_z;
        for (int c = 0; c < n_cases; ++c) {
            const double per = (double)(off[c + 1] - off[c]) / s.n_angles;
            const double side = std::sqrt(16.0 * area / std::max(per, 1.0));
            const int BU = std::min(s.n_bins, std::max(1, (int)std::lround(side / dbm)));
            const int BZ = std::min(s.n_bins_z, std::max(1, (int)std::lround(side / dbzm)));
            for (int64_t j = off[c]; j < off[c + 1]; ++j)
                blk[j] = morton((uint32_t)(hb[j] / BU), (uint32_t)(hz[j] / BZ));
        }
    }
    // lines whose scattered terms each event keeps; tiles hold one mask
    std::vector<int> hm(n);
    for (int64_t j = 0; j < n; ++j) hm[j] = line_mask(ctx->sys, he[j]);
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        const int sx = ha[x] % n_subsets, sy = ha[y] % n_subsets;
        if (sx != sy) return sx < sy;
        if (casev[x] != casev[y]) return casev[x] < casev[y];
        if (ha[x] != ha[y]) return ha[x] < ha[y];
        if (hm[x] != hm[y]) return hm[x] < hm[y];
        if (d3 && blk[x] != blk[y]) return blk[x] < blk[y];
        if (d3 && hz[x] != hz[y]) return hz[x] < hz[y];
        if (cont) {
            if (hu[x] != hu[y]) return hu[x] < hu[y];
        } else if (hb[x] != hb[y]) {
            return hb[x] < hb[y];
        }
        return he[x] < he[y];
    });
    p->bin.resize(cont ? 0 : n);
    p->u.resize(cont ? n : 0);
    p->binz.resize(d3 ? n : 0);
    p->ang.resize(n);
    p->cas.resize(n);
    p->E.resize(n);
    p->lm.resize(n);
    p->perm = order;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t j = order[r];
        if (cont)
            p->u[r] = hu[j];
        else
            p->bin[r] = hb[j];
        if (d3) p->binz[r] = hz[j];
        p->ang[r] = ha[j];
        p->cas[r] = casev[j];
        p->E[r] = he[j];
        p->lm[r] = hm[j];
    }
    p->subs.assign(n_subsets, {});
    {
        int64_t r = 0;
        for (int sidx = 0; sidx < n_subsets; ++sidx) {
            p->subs[sidx].row0 = (int)r;
            while (r < n && p->ang[r] % n_subsets == sidx) ++r;
            p->subs[sidx].rows = (int)r - p->subs[sidx].row0;
            p->max_rows = std::max(p->max_rows, p->subs[sidx].rows);
        }
        // rows of each case within each subset (a subset's rows are sorted by case)
        p->case_rows.assign((size_t)n_subsets * (n_cases + 1), 0);
        for (int sidx = 0; sidx < n_subsets; ++sidx) {
            const lmmew_plan::Sub &sb = p->subs[sidx];
            int *cr = p->case_rows.data() + (size_t)sidx * (n_cases + 1);
            int rr = 0;
            for (int c = 0; c < n_cases; ++c) {
                cr[c] = rr;
                while (rr < sb.rows && p->cas[sb.row0 + rr] == c) ++rr;
            }
            cr[n_cases] = rr;
        }
    }
    // algorithmic terms per iteration
    {
        const double Qm = ctx->S.Qm, nw = ctx->S.nw, QW = Qm * nw;
        double t = 0;
        if (cont) {
            // runs of one (case, angle, line mask) have ascending positions: count each
            // scatter point's reached rows by bisection
            for (int64_t r = 0; r < n;) {
                int64_t e = r;
                while (e < n && p->cas[e] == p->cas[r] && p->ang[e] == p->ang[r] &&
                       p->lm[e] == p->lm[r])
                    ++e;
                const lmmew_ctx *c = p->maps.empty() ? ctx : p->maps[p->cas[r]];
                double rel = 0;
                for (int k = 0; k < c->S.nsc; ++k) {
                    const std::pair<int, int> rr =
                        reached(c->sa[(size_t)p->ang[r] * c->S.nsc + k], p->u.data(), (int)r, (int)e);
                    rel += rr.second - rr.first;
                }
                t += Qm * (nw * (double)(e - r) + rel * __builtin_popcount(p->lm[r]));
                r = e;
            }
        } else {
            const int nbz = d3 ? s.n_bins_z : 1;
            const size_t per = (size_t)s.n_angles * s.n_bins * nbz;
            std::vector<int> rel_cache(per * (p->maps.empty() ? 1 : n_cases), -1);
            for (int64_t r = 0; r < n; ++r) {
                const int m = p->maps.empty() ? 0 : p->cas[r];
                const int bz = d3 ? p->binz[r] : 0;
                int &rc = rel_cache[m * per + ((size_t)p->ang[r] * s.n_bins + p->bin[r]) * nbz + bz];
                if (rc < 0)
                    rc = relevant_scatter(m ? p->maps[m] : ctx, p->ang[r], p->bin[r], bz);
                t += Qm * (nw + (double)rc * __builtin_popcount(p->lm[r]));
            }
        }
        p->terms = t;
        double full = 0;
        for (int64_t r = 0; r < n; ++r)
            full += 1.0 + (p->maps.empty() ? ctx : p->maps[p->cas[r]])->S.nsc;
        p->full_terms = full * QW;
    }
    build_tiles(p);
    const int Qp = ctx->S.Qp;
    auto fin = [&](int code) {
        if (code != LMMEW_OK) {
            free_plan(p);
            delete p;
        }
        return code;
    };
#define PCHK(call)                                               \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return fin(hipfail(ctx, e_, #call)); \
    } while (0)
    if (cont)
        PCHK(dalloc(&p->d_u, n));
    else
        PCHK(dalloc(&p->d_bin, n));
    if (d3) PCHK(dalloc(&p->d_binz, n));
    PCHK(dalloc(&p->d_ang, n));
    PCHK(dalloc(&p->d_case, n));
    PCHK(dalloc(&p->d_E, n));
    PCHK(dalloc(&p->d_perm, n));
    PCHK(dalloc(&p->d_p, n));
    PCHK(dalloc(&p->d_wt, n));
    PCHK(dalloc(&p->d_logp, n));
    PCHK(dalloc(&p->d_A, (size_t)std::max(p->max_rows, 1) * Qp));
    PCHK(dalloc(&p->d_lamc, (size_t)n_cases * Qp));
    PCHK(dalloc(&p->d_cscale, (size_t)n_cases * ctx->S.nwin));
    PCHK(dalloc(&p->d_sidx, n));
    if (n > 0) {
        if (d3)
            PCHK(hipMemcpyAsync(p->d_binz, p->binz.data(), n * sizeof(int), hipMemcpyHostToDevice,
                                st));
        if (cont)
            PCHK(hipMemcpyAsync(p->d_u, p->u.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
        else
            PCHK(hipMemcpyAsync(p->d_bin, p->bin.data(), n * sizeof(int), hipMemcpyHostToDevice,
                                st));
        PCHK(hipMemcpyAsync(p->d_ang, p->ang.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
        PCHK(hipMemcpyAsync(p->d_case, p->cas.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
        PCHK(hipMemcpyAsync(p->d_E, p->E.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
        std::vector<int> sidx(n);
        for (int64_t r = 0; r < n; ++r)
            sidx[r] = p->cas[r] * ctx->S.nwin + window_of(ctx->sys, p->E[r]);
        PCHK(hipMemcpyAsync(p->d_sidx, sidx.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
        PCHK(hipStreamSynchronize(st));
        PCHK(hipMemcpyAsync(p->d_perm, p->perm.data(), n * sizeof(int64_t), hipMemcpyHostToDevice,
                            st));
    }
    if (!p->maps.empty()) PCHK(dalloc(&p->d_maps, n_cases));
    {
        const int rm = sync_maps(ctx, p, st);
        if (rm != LMMEW_OK) return fin(rm);
    }
    const int rc = upload_tiles(ctx, p, st);
    if (rc != LMMEW_OK) return fin(rc);
#undef PCHK
    *out = p;
    return LMMEW_OK;
}

// Records a timing event on the stream; two consecutive marks bracket one launch.
hipError_t prof_mark(lmmew_ctx *, lmmew_plan *p, int kind, hipStream_t st)
{
    if (p->prof_ev.size() <= p->prof_used) {
        hipEvent_t e;
        const hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        p->prof_ev.push_back(e);
    }
    if (p->prof_used % 2 == 0) p->prof_kind.resize(p->prof_used / 2 + 1);
    p->prof_kind[p->prof_used / 2] = kind;
    return hipEventRecord(p->prof_ev[p->prof_used++], st);
}

// a_jq of subset s into the plan's scratch rows.  part: 0 the context's model
// (exact, or unscattered + surrogate when a surrogate is set), 1 exact
// scattered paths only, 2 unscattered only, 3 exact (ignoring the surrogate).
// Uploads the per-case tables of a plan over several maps when they changed
// (a context's path-parameter table may be built or freed after the plan),
// and the surrogate's per-case density factors.
int sync_maps(lmmew_ctx *ctx, lmmew_plan *p, hipStream_t st)
{
    // the surrogate's density factor of every case and window
    // (lmmew_set_scatter_scale, lmmew_set_scatter_scale_windows)
    const int nwin = ctx->S.nwin;
    std::vector<float> cs((size_t)p->ncases * nwin);
    for (int c = 0; c < p->ncases; ++c)
        for (int w = 0; w < nwin; ++w)
            cs[(size_t)c * nwin + w] = (p->maps.empty() ? ctx : p->maps[c])->scatter_scale[w];
    if (cs != p->cscale) {
        HIPCHK(ctx, hipMemcpyAsync(p->d_cscale, cs.data(), cs.size() * sizeof(float),
                                   hipMemcpyHostToDevice, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        p->cscale = cs;
    }
    if (p->maps.empty()) return LMMEW_OK;
    if (ctx->xgrid > 1) {
        // the cases' node tables for the exact scattered part at the nodes
        std::vector<MapTab> xt(p->ncases);
        for (int c = 0; c < p->ncases; ++c) {
            const lmmew_ctx *m = p->maps[c];
            if (m->xgrid != ctx->xgrid)
                return fail(ctx, LMMEW_EINVAL,
                            "every context of the plan needs the plan context's scatter pixel grid");
            xt[c].g_qa = m->d_xgqa;
            xt[c].g_qs = m->d_xgqs;
            xt[c].sa = m->d_sa;
            xt[c].ptab = nullptr;
            xt[c].resp = m->d_resp;
            xt[c].respz = m->d_respz;
            xt[c].sz = m->d_scz;
            xt[c].nsc = m->S.nsc;
        }
        if (!p->d_xmaps) HIPCHK(ctx, dalloc(&p->d_xmaps, (size_t)p->ncases));
        if (xt.size() != p->xmaptab.size() ||
            std::memcmp(xt.data(), p->xmaptab.data(), xt.size() * sizeof(MapTab)) != 0) {
            HIPCHK(ctx, hipMemcpyAsync(p->d_xmaps, xt.data(), xt.size() * sizeof(MapTab),
                                       hipMemcpyHostToDevice, st));
            HIPCHK(ctx, hipStreamSynchronize(st));
            p->xmaptab = xt;
        }
    }
    std::vector<MapTab> mt(p->ncases);
    for (int c = 0; c < p->ncases; ++c) {
        const lmmew_ctx *m = p->maps[c];
        mt[c].g_qa = m->d_gqa;
        mt[c].g_qs = m->d_gqs;
        mt[c].sa = m->d_sa;
        mt[c].ptab = m->d_ptab;
        mt[c].resp = m->d_resp;
        mt[c].respz = m->d_respz;
        mt[c].sz = m->d_scz;
        mt[c].nsc = m->S.nsc;
    }
    if (mt.size() == p->maptab.size() &&
        std::memcmp(mt.data(), p->maptab.data(), mt.size() * sizeof(MapTab)) == 0)
        return LMMEW_OK;
    HIPCHK(ctx, hipMemcpyAsync(p->d_maps, mt.data(), mt.size() * sizeof(MapTab),
                               hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    p->maptab = mt;
    return LMMEW_OK;
}

// The path-parameter table the per-event kernel may use for this plan: the
// context's, or for a plan over several maps a non-NULL marker when every
// case's map has one (the kernel then reads each case's from the plan's
// table pointers); NULL to evaluate the parameters in the kernel.
const float *plan_ptab(const lmmew_ctx *ctx, const lmmew_plan *p)
{
    if (p->maps.empty()) return ctx->d_ptab;
    for (const MapTab &m : p->maptab)
        if (!m.ptab) return nullptr;
    return p->maptab.empty() ? nullptr : p->maptab[0].ptab;
}

// Rows a_jq of subset s: the cached rows, or the per-subset scratch.
float *rows_of(lmmew_plan *p, int s)
{
    return p->d_Acache ? p->d_Acache + (size_t)p->subs[s].row0 * p->ctx->S.Qp : p->d_A;
}

// Per-event kernel arguments of subset s (without output and mode).
RowArgs row_args(const lmmew_ctx *ctx, const lmmew_plan *p, int s)
{
    const lmmew_plan::Sub &sub = p->subs[s];
    RowArgs r{};
    r.pix_xy = ctx->d_pix;
    r.dirs = ctx->d_dirs;
    r.g_qa = ctx->d_gqa;
    r.g_qs = ctx->d_gqs;
    r.sa = ctx->d_sa;
    r.resp = ctx->d_resp;
    r.respz = ctx->d_respz;
    r.psft = ctx->d_psft;
    r.pix_z = ctx->d_pixz;
    r.sz = ctx->d_scz;
    r.maps = p->d_maps;
    r.ptab = plan_ptab(ctx, p);
    r.tiles = p->d_tiles + sub.tile0;
    r.slist = p->d_slist;
    r.ntiles = sub.ntiles;
    r.case_tiles = p->d_case_tiles + (size_t)s * (p->ncases + 1);
    r.ncases = p->ncases;
    r.ev_bin = p->cont ? nullptr : p->d_bin + sub.row0;
    r.ev_u = p->cont ? p->d_u + sub.row0 : nullptr;
    r.ev_binz = p->d_binz ? p->d_binz + sub.row0 : nullptr;
    r.ev_E = p->d_E + sub.row0;
    return r;
}

// Scatter network of case c: its own context's selection in a plan over
// several maps, else the plan context's.
const lmmew_mlp *case_model(const lmmew_ctx *ctx, const lmmew_plan *p, int c)
{
    if (!p->maps.empty() && p->maps[c]->mlp) return p->maps[c]->mlp;
    return ctx->mlp;
}

// Changes whenever the scatter model of any case of the plan changes.
int plan_model_gen(const lmmew_ctx *ctx, const lmmew_plan *p)
{
    int g = ctx->model_gen;
    for (size_t c = 1; c < p->maps.size(); ++c) g += p->maps[c]->model_gen;
    return g;
}

// The node-value scratch a sub-iteration's surrogate rows need: the largest
// subset's rows times the widest node row of the networks the plan's cases
// use (none when every network is evaluated at the support pixels).  Sized
// outside graph captures (lmmew_osem_graph calls it before capturing).
int coarse_scratch(lmmew_ctx *ctx, lmmew_plan *p)
{
    size_t need = 0;
    for (int c = 0; c < p->ncases; ++c) {
        const lmmew_mlp *m = case_model(ctx, p, c);
        if (m && m->grid > 1) need = std::max(need, (size_t)std::max(p->max_rows, 1) * m->ldc);
    }
    if (ctx->xgrid > 1) need = std::max(need, (size_t)std::max(p->max_rows, 1) * ctx->xldc);
    if (need <= p->C_cap) return LMMEW_OK;
    dfree(p->d_C);
    p->d_C = nullptr;
    p->C_cap = 0;
    HIPCHK(ctx, dalloc(&p->d_C, need));
    p->C_cap = need;
    return LMMEW_OK;
}

// The network's scattered densities of a.rows rows (a holds the events, the
// parameters and the density factors) added to out [rows][Qp]: evaluated at
// every support pixel, or, with a coarse grid, at the network's nodes into
// C [rows][ldc] and interpolated from there.
hipError_t net_rows(const lmmew_ctx *ctx, const lmmew_mlp *m, MlpRowArgs a, float *out, float *C,
                    hipStream_t st)
{
    if (m->grid <= 1) {
        a.pix_xy = ctx->d_pix;
        a.npix = ctx->S.Qm;
        a.ld = ctx->S.Qp;
        a.assign = 0;
        a.A = out;
        return mlp_rows(ctx->S, a, st);
    }
    if (!C) return hipErrorInvalidValue;
    a.pix_xy = m->d_cnode;
    a.npix = m->ncn;
    a.ld = m->ldc;
    a.assign = 1;
    a.A = C;
    hipError_t e = mlp_rows(ctx->S, a, st);
    if (e == hipSuccess)
        e = launch_coarse_interp(ctx->S, C, m->ldc, m->d_cidx, m->d_cw, a.rows, out, st);
    return e;
}

int run_rows(lmmew_ctx *ctx, lmmew_plan *p, int s, hipStream_t st, int part = 0,
             float *dst = nullptr)
{
    const lmmew_plan::Sub &sub = p->subs[s];
    float *const out = dst ? dst : p->d_A;
    const bool surrogate = (part == 0 && ctx->mlp != nullptr);
    if (part == 0 && !ctx->mlp)
        for (size_t c = 1; c < p->maps.size(); ++c)
            if (p->maps[c]->mlp)
                return fail(ctx, LMMEW_EINVAL,
                            "a case's context selects a scatter network but the plan's context "
                            "does not");
    if (surrogate && p->cont)
        return fail(ctx, LMMEW_EINVAL,
                    "the scatter surrogate models binned events; these carry continuous positions");
    RowArgs r = row_args(ctx, p, s);
    r.A = out;
    r.mode = surrogate ? 2 : (part == 3 ? 0 : part);
    if (!surrogate && r.mode != 2 && ctx->xgrid > 1) {
        // The exact scattered part at the node pixels, interpolated to every
        // support pixel; the unscattered part at every support pixel.
        if (!p->maps.empty() && p->xmaptab.size() != (size_t)p->ncases)
            return fail(ctx, LMMEW_EINVAL, "the plan's node tables are not set up");
        {
            const int rc = coarse_scratch(ctx, p);
            if (rc != LMMEW_OK) return rc;
        }
        r.pvt = p->d_pvt;
        const bool prof = p->prof && sub.ntiles > 0;
        // full rows of binned events with the unscattered table: the
        // unscattered part and the interpolation in one pass after the nodes
        const bool fuse = r.mode == 0 && ctx->d_psft && !p->cont;
        if (prof) HIPCHK(ctx, prof_mark(ctx, p, 0, st));
        if (r.mode == 1) {
            HIPCHK(ctx, hipMemsetAsync(out, 0, (size_t)sub.rows * ctx->S.Qp * sizeof(float), st));
        } else if (!fuse) {
            RowArgs u = r;
            u.mode = 2;
            u.case_tiles = nullptr;
            HIPCHK(ctx, launch_row(ctx->S, u, p->JT, st));
        }
        RowArgs x = r;
        x.mode = 1;
        x.pix_xy = ctx->d_xnode;
        x.g_qa = ctx->d_xgqa;
        x.g_qs = ctx->d_xgqs;
        x.psft = nullptr;
        x.ptab = nullptr;
        x.maps = p->maps.empty() ? nullptr : p->d_xmaps;
        x.A = p->d_C;
        DevSys Sx = ctx->S;
        Sx.Qm = ctx->xncn;
        Sx.Qp = ctx->xldc;
        HIPCHK(ctx, launch_row(Sx, x, p->JT, st));
        if (fuse) {
            PrimInterpArgs pa{};
            pa.psft = ctx->d_psft;
            pa.g_qa = ctx->d_gqa;
            pa.maps = p->maps.empty() ? nullptr : p->d_maps;
            pa.ev_bin = p->d_bin + sub.row0;
            pa.ev_ang = p->d_ang + sub.row0;
            pa.ev_case = p->d_case + sub.row0;
            pa.ev_E = p->d_E + sub.row0;
            pa.rows = sub.rows;
            pa.C = p->d_C;
            pa.ldc = ctx->xldc;
            pa.idx = ctx->d_xidx;
            pa.w = ctx->d_xw;
            pa.A = out;
            HIPCHK(ctx, launch_prim_interp(ctx->S, pa, st));
        } else {
            HIPCHK(ctx, launch_coarse_interp(ctx->S, p->d_C, ctx->xldc, ctx->d_xidx, ctx->d_xw,
                                             sub.rows, out, st));
        }
        if (prof) HIPCHK(ctx, prof_mark(ctx, p, 0, st));
        return LMMEW_OK;
    }
    // Without scattered paths a tile reads no map's scatter tables; its
    // pixel block's unscattered tables are shared by every case, so the
    // block-major order over all tiles keeps those in the L2 instead.
    if (r.mode == 2) r.case_tiles = nullptr;
    r.pvt = p->d_pvt;
    const bool prof = p->prof && sub.ntiles > 0;
    // Every case's network on a coarse grid, with the unscattered table: per
    // run of cases, the network at its nodes, then the unscattered part and
    // the interpolation in one pass (no separate unscattered launch).
    bool fuse = surrogate && ctx->d_psft != nullptr;
    for (int c = 0; fuse && c < p->ncases; ++c) {
        const lmmew_mlp *m = case_model(ctx, p, c);
        fuse = m && m->grid > 1;
    }
    if (!fuse) {
        if (prof) HIPCHK(ctx, prof_mark(ctx, p, 0, st));
        HIPCHK(ctx, launch_row(ctx->S, r, p->JT, st));
        if (prof) HIPCHK(ctx, prof_mark(ctx, p, 0, st));
    }
    if (surrogate) {
        // one launch per run of consecutive cases that share a network (the
        // whole subset when every case uses the plan context's)
        const bool profm = p->prof && sub.rows > 0 && !fuse;
        if (profm) HIPCHK(ctx, prof_mark(ctx, p, 1, st));
        const int *cr = p->case_rows.data() + (size_t)s * (p->ncases + 1);
        {
            const int rc = coarse_scratch(ctx, p);
            if (rc != LMMEW_OK) return rc;
        }
        for (int c0 = 0; c0 < p->ncases;) {
            const lmmew_mlp *m = case_model(ctx, p, c0);
            int c1 = c0 + 1;
            while (c1 < p->ncases && case_model(ctx, p, c1) == m) ++c1;
            const int r0 = cr[c0], r1 = cr[c1];
            if (r1 > r0) {
                MlpRowArgs a{};
                a.dirs = ctx->d_dirs;
                a.ev_bin = p->d_bin + sub.row0 + r0;
                a.ev_ang = p->d_ang + sub.row0 + r0;
                a.ev_E = p->d_E + sub.row0 + r0;
                a.rows = r1 - r0;
                a.P = m->P;
                a.c0 = (float)m->c0;
                a.floor_ = (float)m->floor_;
                a.ev_scale = p->d_sidx + sub.row0 + r0;
                a.case_scale = p->d_cscale;
                // runs follow each other on the stream: each reuses the
                // node-value scratch from its start
                if (fuse) {
                    const bool pr = p->prof;
                    a.pix_xy = m->d_cnode;
                    a.npix = m->ncn;
                    a.ld = m->ldc;
                    a.assign = 1;
                    a.A = p->d_C;
                    if (pr) HIPCHK(ctx, prof_mark(ctx, p, 1, st));
                    HIPCHK(ctx, mlp_rows(ctx->S, a, st));
                    if (pr) HIPCHK(ctx, prof_mark(ctx, p, 1, st));
                    PrimInterpArgs pa{};
                    pa.psft = ctx->d_psft;
                    pa.g_qa = ctx->d_gqa;
                    pa.maps = p->maps.empty() ? nullptr : p->d_maps;
                    pa.ev_bin = a.ev_bin;
                    pa.ev_ang = a.ev_ang;
                    pa.ev_case = p->d_case + sub.row0 + r0;
                    pa.ev_E = a.ev_E;
                    pa.rows = a.rows;
                    pa.C = p->d_C;
                    pa.ldc = m->ldc;
                    pa.idx = m->d_cidx;
                    pa.w = m->d_cw;
                    pa.A = out + (size_t)r0 * ctx->S.Qp;
                    if (pr) HIPCHK(ctx, prof_mark(ctx, p, 0, st));
                    HIPCHK(ctx, launch_prim_interp(ctx->S, pa, st));
                    if (pr) HIPCHK(ctx, prof_mark(ctx, p, 0, st));
                } else {
                    HIPCHK(ctx, net_rows(ctx, m, a, out + (size_t)r0 * ctx->S.Qp, p->d_C, st));
                }
            }
            c0 = c1;
        }
        if (profm) HIPCHK(ctx, prof_mark(ctx, p, 1, st));
    }
    return LMMEW_OK;
}

// The images on the support pixels, in the layout of the rows (read by the
// forward projection; the EM update keeps it current within an OSEM call).
int run_compact(lmmew_ctx *ctx, lmmew_plan *p, const float *lambda, hipStream_t st)
{
    HIPCHK(ctx, launch_compact(ctx->S, lambda, p->ncases, ctx->Q, ctx->d_pixq, p->d_lamc, st));
    return LMMEW_OK;
}

int run_forward(lmmew_ctx *ctx, lmmew_plan *p, int s, bool stats, int k, hipStream_t st)
{
    const lmmew_plan::Sub &sub = p->subs[s];
    FwdArgs f{};
    f.A = rows_of(p, s);
    f.rows = sub.rows;
    f.row_case = p->d_case + sub.row0;
    f.lamc = p->d_lamc;
    f.p = p->d_p + sub.row0;
    f.wt = p->d_wt + sub.row0;
    f.logp = stats ? p->d_logp + sub.row0 : nullptr;
    f.nskip = stats ? p->d_nskip + k : nullptr;
    HIPCHK(ctx, launch_forward(ctx->S, f, st));
    return LMMEW_OK;
}

int run_back(lmmew_ctx *ctx, lmmew_plan *p, int s, const float *wt_rows, float *part, float *comp,
             hipStream_t st)
{
    const lmmew_plan::Sub &sub = p->subs[s];
    BackArgs b{};
    b.A = rows_of(p, s);
    b.wt = wt_rows;
    b.chunks = p->d_chunks + sub.chunk0;
    b.nchunks = sub.nchunks;
    b.part = part;
    b.comp = comp;
    HIPCHK(ctx, launch_back(ctx->S, b, st));
    return LMMEW_OK;
}

int ensure_stats(lmmew_ctx *ctx, lmmew_plan *p, int count)
{
    if (p->stats_cap >= count) return LMMEW_OK;
    dfree(p->d_nskip);
    dfree(p->d_ll);
    HIPCHK(ctx, dalloc(&p->d_nskip, count));
    HIPCHK(ctx, dalloc(&p->d_ll, count));
    p->stats_cap = count;
    return LMMEW_OK;
}

// Static device scratch of lmmew_roi_uptake_noalloc: the region sums before
// their copy to the host.  Each device the library runs on holds its own copy
// of the array (until the process ends); host code reaches it only through the
// address hipGetSymbolAddress returns on that device, resolved once per device
// with the device current (at context creation, or on the entry point's first
// call there).
static __device__ __align__(256) double roi_scratch[LMMEW_ROI_NOALLOC_MAX];

constexpr int kMaxDevices = 64;
std::mutex g_roi_mu;
double *g_roi_ptr[kMaxDevices] = {};

hipError_t roi_scratch_ptr(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_roi_mu);
    if (!g_roi_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(roi_scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_roi_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_roi_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

const char *lmmew_status_string(int status)
{
    switch (status) {
    case LMMEW_OK: return "ok";
    case LMMEW_EINVAL: return "invalid argument";
    case LMMEW_ENOMEM: return "out of memory";
    case LMMEW_EDEVICE: return "device error";
    case LMMEW_ENUMERIC: return "non-finite result";
    default: return "unknown status";
    }
}

const char *lmmew_last_error(const lmmew_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

int lmmew_create(const lmmew_system *sys, const float *mu85, const uint8_t *support,
                 hipStream_t st, lmmew_ctx **out)
{
    if (!out) return LMMEW_EINVAL;
    *out = nullptr;
    if (!sys || !mu85) return LMMEW_EINVAL;
    lmmew_ctx *ctx = new (std::nothrow) lmmew_ctx;
    if (!ctx) return LMMEW_ENOMEM;
    auto bail = [&](int code) {
        if (code != LMMEW_OK) {
            free_ctx(ctx);
            delete ctx;
        }
        return code;
    };
    int rc = validate_sys(ctx, sys);
    if (rc != LMMEW_OK) return bail(rc);
    ctx->sys = *sys;
    const lmmew_system &s = *sys;
    // the 3-D model (nz > 0) stacks nz slices of n x n; the planar one has one
    const bool d3 = s.nz > 0;
    const int nzs = d3 ? s.nz : 1, nsz = d3 ? s.ns_z : 1;
    const int n = s.n, Q = n * n * nzs, na = s.n_angles, ns = s.ns, m = n / ns;
    const int mz = d3 ? s.nz / s.ns_z : 1;
    ctx->Q = Q;
    const double pix = s.pixel_mm, R = 0.5 * n * pix, hs = 2.0 * R / ns, db = 2.0 * R / s.n_bins;
    const double Zh = d3 ? 0.5 * s.nz * pix : 0.0;
    const double hz = d3 ? 2.0 * Zh / nsz : 0.0, dbz = d3 ? 2.0 * Zh / s.n_bins_z : 0.0;
    ctx->R = R;
    ctx->hs = hs;
    ctx->db = db;

    std::vector<float> mu_f(Q);
    std::vector<uint8_t> mask(Q, 1);
#define CCHK(call)                                                 \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return bail(hipfail(ctx, e_, #call)); \
    } while (0)
    CCHK(hipMemcpyAsync(mu_f.data(), mu85, Q * sizeof(float), hipMemcpyDeviceToHost, st));
    if (support) CCHK(hipMemcpyAsync(mask.data(), support, Q, hipMemcpyDeviceToHost, st));
    CCHK(hipStreamSynchronize(st));
    std::vector<double> mu(Q);
    for (int q = 0; q < Q; ++q) {
        if (!std::isfinite(mu_f[q]) || mu_f[q] < 0.f)
            return bail(fail(ctx, LMMEW_EINVAL, "mu85 must be finite and >= 0"));
        mu[q] = mu_f[q];
    }
    // support pixels (voxels: slice-major, q = (iz*n + iy)*n + ix)
    std::vector<double> px, py, pz;
    std::vector<int> pq;
    for (int q = 0; q < Q; ++q) {
        const int qq = q % (n * n);
        const double x = ((qq % n) + 0.5) * pix - R, y = ((qq / n) + 0.5) * pix - R;
        if (x * x + y * y <= R * R && mask[q]) {
            px.push_back(x);
            py.push_back(y);
            pz.push_back(d3 ? ((q / (n * n)) + 0.5) * pix - Zh : 0.0);
            pq.push_back(q);
        }
    }
    const int Qm = (int)pq.size();
    const int Qp = std::max(kWave, (Qm + kWave - 1) / kWave * kWave);
    std::vector<float2> pix_f(Qp);
    std::vector<double2> pix_d(Qp);
    std::vector<float> pixz_f(d3 ? Qp : 0);
    std::vector<double> pixz_d(d3 ? Qp : 0);
    ctx->pixq.assign(Qp, -1);
    for (int i = 0; i < Qp; ++i) {
        const double x = i < Qm ? px[i] : -10.0 * R, y = i < Qm ? py[i] : -10.0 * R;
        pix_f[i] = make_float2((float)x, (float)y);
        pix_d[i] = make_double2(x, y);
        if (d3) {
            pixz_d[i] = i < Qm ? pz[i] : 0.0;
            pixz_f[i] = (float)pixz_d[i];
        }
        if (i < Qm) ctx->pixq[i] = pq[i];
    }
    // scatter points: cell centres with mean attenuation of the covered pixels
    std::vector<double2> sc;
    std::vector<double> scz, smu;
    for (int kz = 0; kz < nsz; ++kz)
        for (int ky = 0; ky < ns; ++ky)
            for (int kx = 0; kx < ns; ++kx) {
                const double x = (kx + 0.5) * hs - R, y = (ky + 0.5) * hs - R;
                double acc = 0.0;
                for (int l = 0; l < mz; ++l)
                    for (int j = 0; j < m; ++j)
                        for (int i = 0; i < m; ++i)
                            acc += mu[((size_t)(kz * mz + l) * n + (ky * m + j)) * n + (kx * m + i)];
                acc /= (double)(m * m * mz);
                if (x * x + y * y <= R * R && acc > 0.0) {
                    sc.push_back(make_double2(x, y));
                    scz.push_back(d3 ? (kz + 0.5) * hz - Zh : 0.0);
                    smu.push_back(acc);
                }
            }
    if (sc.size() > (size_t)kSlistPoint)
        return bail(fail(ctx, LMMEW_EINVAL, "too many scatter points (at most 2^24 - 1)"));
    const int nsc = (int)sc.size();
    // directions and per-angle scatter lists sorted by lateral coordinate
    ctx->dir_c.resize(na);
    ctx->dir_s.resize(na);
    std::vector<float2> dirs_f(na);
    std::vector<double2> dirs_d(na);
    for (int a = 0; a < na; ++a) {
        angle_dir(a, na, &ctx->dir_c[a], &ctx->dir_s[a]);
        dirs_f[a] = make_float2((float)ctx->dir_c[a], (float)ctx->dir_s[a]);
        dirs_d[a] = make_double2(ctx->dir_c[a], ctx->dir_s[a]);
    }
    const double fps = fwhm_per_sigma();
    // planar: hs^2 mu_s / (2 pi) per unit 1/r; 3-D: V mu_s / (4 pi) per unit 1/r^2
    const double cellw = d3 ? hs * hs * hz / (4.0 * kPi) : hs * hs / (2.0 * kPi);
    ctx->sa.resize((size_t)na * nsc);
    ctx->sig_max.assign(na, 0.0);
    for (int a = 0; a < na; ++a) {
        const double c = ctx->dir_c[a], sn = ctx->dir_s[a];
        std::vector<int> idx(nsc);
        std::iota(idx.begin(), idx.end(), 0);
        std::vector<double> u(nsc);
        for (int k = 0; k < nsc; ++k) u[k] = -sc[k].x * sn + sc[k].y * c;
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return u[x] < u[y]; });
        for (int k = 0; k < nsc; ++k) {
            const int si = idx[k];
            const double depth = R - (sc[si].x * c + sc[si].y * sn);
            const double sig = (s.psf_fwhm0_mm + s.psf_fwhm_slope * depth) / fps;
            ctx->sig_max[a] = std::max(ctx->sig_max[a], sig);
            ScatA e{};
            e.x = (float)sc[si].x;
            e.y = (float)sc[si].y;
            e.u = (float)u[si];
            e.isig = (float)(1.0 / sig);
            e.gsa = 0.f;
            e.lc = (float)std::log2(cellw * smu[si]);
            e.D = 0.f;
            e.sidx = si;
            ctx->sa[(size_t)a * nsc + k] = e;
        }
    }
    // bins reached by each scatter point's response (the kernel's 7-sigma rule,
    // evaluated in the kernel's float arithmetic)
    auto reach = [](float lo0, float width, int nbins, float c, float isig, int &lo, int &hi) {
        lo = nbins;
        hi = -1;
        for (int b = 0; b < nbins; ++b) {
            const float blo = lo0 + (float)b * width;
            const float zhi = (blo + width - c) * isig, zlo = (blo - c) * isig;
            if (!(zlo >= kPsfCut || zhi <= -kPsfCut)) {
                lo = std::min(lo, b);
                hi = std::max(hi, b);
            }
        }
    };
    ctx->rb_lo.assign((size_t)na * nsc, 0);
    ctx->rb_hi.assign((size_t)na * nsc, -1);
    for (size_t ak = 0; ak < (size_t)na * nsc; ++ak) {
        const ScatA &e = ctx->sa[ak];
        reach(-(float)R, (float)db, s.n_bins, e.u, e.isig, ctx->rb_lo[ak], ctx->rb_hi[ak]);
    }
    if (d3) {
        ctx->rbz_lo.assign((size_t)na * nsc, 0);
        ctx->rbz_hi.assign((size_t)na * nsc, -1);
        for (size_t ak = 0; ak < (size_t)na * nsc; ++ak) {
            const ScatA &e = ctx->sa[ak];
            reach(-(float)Zh, (float)dbz, s.n_bins_z, (float)scz[e.sidx], e.isig,
                  ctx->rbz_lo[ak], ctx->rbz_hi[ak]);
        }
    }
    // constants
    DevSys &S = ctx->S;
    S.n = n;
    S.ns = ns;
    S.nb = s.n_bins;
    S.na = na;
    S.nw = s.n_lines;
    S.nwin = s.n_windows;
    S.Qm = Qm;
    S.Qp = Qp;
    S.nsc = nsc;
    S.pix = (float)pix;
    S.R = (float)R;
    S.hs = (float)hs;
    S.db = (float)db;
    S.nz = d3 ? s.nz : 0;
    S.nbz = d3 ? s.n_bins_z : 0;
    S.Zh = (float)Zh;
    S.dbz = (float)dbz;
    S.fwhm0 = (float)s.psf_fwhm0_mm;
    S.fslope = (float)s.psf_fwhm_slope;
    S.inv_fwhm_to_sigma = (float)(1.0 / fps);
    S.T = (float)s.T;
    const double k = s.eres_frac * s.eres_frac * s.eres_ref_keV / (fps * fps);
    S.eres_k = (float)k;
    S.sqck = (float)std::sqrt(1.0 / std::log(2.0) / (2.0 * k));
    S.mu_pow = (float)s.mu_power;
    // r is clamped below: planar at the mean of 1/r over a disk of area hs^2,
    // 3-D where 1/r^2 equals its mean over a ball of volume hs^2 hz
    S.rmin = d3 ? (float)(std::cbrt(3.0 * hs * hs * hz / (4.0 * kPi)) / std::sqrt(3.0))
                : (float)(hs / (2.0 * std::sqrt(kPi)));
    const double log2e = 1.0 / std::log(2.0);
    for (int w = 0; w < s.n_lines; ++w) {
        const double E = s.line_keV[w];
        const double f = std::pow(E / s.mu_ref_keV, -s.mu_power);
        S.E[w] = (float)E;
        S.eps[w] = (float)(E / s.electron_keV);
        S.f[w] = (float)f;
        if (d3) {
            const double Z = kn_norm_sphere(E, s.electron_keV);
            S.pp[w] = (float)(s.line_yield[w] * s.coll_solid_angle / (4.0 * kPi));
            S.lsc[w] = (float)std::log2(s.line_yield[w] * f * s.coll_solid_angle / Z);
        } else {
            const double Z = kn_norm(E, s.electron_keV);
            S.pp[w] = (float)(s.line_yield[w] * s.coll_dtheta / (2.0 * kPi));
            S.lsc[w] = (float)std::log2(s.line_yield[w] * f * s.coll_dtheta / Z);
        }
        S.c0[w] = (float)(log2e / (2.0 * k * E));
        S.sqc0[w] = (float)std::sqrt(log2e / (2.0 * k * E));
        S.nc[w] = (float)(-0.5 * std::log2(2.0 * kPi * k * E));
        S.gnorm[w] = (float)(1.0 / std::sqrt(2.0 * kPi * k * E));
    }
    for (int w = 0; w < s.n_windows; ++w) {
        S.wlo[w] = (float)s.win_lo_keV[w];
        S.whi[w] = (float)s.win_hi_keV[w];
    }
    // device tables
    CCHK(dalloc(&ctx->d_pix, Qp));
    CCHK(dalloc(&ctx->d_pixd, Qp));
    CCHK(dalloc(&ctx->d_pixq, Qp));
    CCHK(dalloc(&ctx->d_dirs, na));
    CCHK(dalloc(&ctx->d_dirsd, na));
    CCHK(dalloc(&ctx->d_scd, nsc));
    CCHK(dalloc(&ctx->d_mu, Q));
    CCHK(dalloc(&ctx->d_gqa, (size_t)na * Qp));
    CCHK(dalloc(&ctx->d_gqs, (size_t)std::max(nsc, 1) * Qp));
    CCHK(dalloc(&ctx->d_sa, (size_t)na * std::max(nsc, 1)));
    CCHK(dalloc(&ctx->d_resp, (size_t)na * std::max(nsc, 1) * s.n_bins));
    if (d3) {
        CCHK(dalloc(&ctx->d_pixz, Qp));
        CCHK(dalloc(&ctx->d_pixzd, Qp));
        CCHK(dalloc(&ctx->d_scz, std::max(nsc, 1)));
        CCHK(dalloc(&ctx->d_sczd, std::max(nsc, 1)));
        CCHK(dalloc(&ctx->d_respz, (size_t)na * std::max(nsc, 1) * s.n_bins_z));
        CCHK(hipMemcpyAsync(ctx->d_pixz, pixz_f.data(), Qp * sizeof(float), hipMemcpyHostToDevice,
                            st));
        CCHK(hipMemcpyAsync(ctx->d_pixzd, pixz_d.data(), Qp * sizeof(double),
                            hipMemcpyHostToDevice, st));
        if (nsc > 0) {
            std::vector<float> scz_f(scz.begin(), scz.end());
            CCHK(hipMemcpyAsync(ctx->d_scz, scz_f.data(), nsc * sizeof(float),
                                hipMemcpyHostToDevice, st));
            CCHK(hipMemcpyAsync(ctx->d_sczd, scz.data(), nsc * sizeof(double),
                                hipMemcpyHostToDevice, st));
            CCHK(hipStreamSynchronize(st));      // scz_f goes out of scope
        }
    }
    CCHK(hipMemcpyAsync(ctx->d_pix, pix_f.data(), Qp * sizeof(float2), hipMemcpyHostToDevice, st));
    CCHK(hipMemcpyAsync(ctx->d_pixd, pix_d.data(), Qp * sizeof(double2), hipMemcpyHostToDevice, st));
    CCHK(hipMemcpyAsync(ctx->d_pixq, ctx->pixq.data(), Qp * sizeof(int), hipMemcpyHostToDevice, st));
    CCHK(hipMemcpyAsync(ctx->d_dirs, dirs_f.data(), na * sizeof(float2), hipMemcpyHostToDevice, st));
    CCHK(hipMemcpyAsync(ctx->d_dirsd, dirs_d.data(), na * sizeof(double2), hipMemcpyHostToDevice, st));
    if (nsc > 0) {
        CCHK(hipMemcpyAsync(ctx->d_scd, sc.data(), nsc * sizeof(double2), hipMemcpyHostToDevice, st));
        CCHK(hipMemcpyAsync(ctx->d_sa, ctx->sa.data(), ctx->sa.size() * sizeof(ScatA),
                            hipMemcpyHostToDevice, st));
    }
    CCHK(hipMemcpyAsync(ctx->d_mu, mu.data(), Q * sizeof(double), hipMemcpyHostToDevice, st));
    CCHK(launch_tables_d(S, ctx->d_mu, ctx->d_pixd, ctx->d_pixzd, ctx->d_dirsd, ctx->d_scd,
                         ctx->d_sczd, ctx->d_gqa, ctx->d_gqs, ctx->d_sa, pix, R, st));
    CCHK(launch_resp_table(S, ctx->d_sa, ctx->d_resp, ctx->d_scz, ctx->d_respz, st));
    CCHK(hipStreamSynchronize(st));
    {
        double *scr = nullptr;   // resolve the no-allocation scratch on this device once
        CCHK(roi_scratch_ptr(&scr));
    }
#undef CCHK
    *out = ctx;
    return LMMEW_OK;
}

int lmmew_destroy(lmmew_ctx *ctx)
{
    if (!ctx) return LMMEW_EINVAL;
    (void)hipDeviceSynchronize();
    // networks of this context may outlive it (their destroy call must then
    // not touch it): detach them
    for (lmmew_mlp *m : ctx->nets) m->ctx = nullptr;
    ctx->nets.clear();
    ctx->mlp = nullptr;
    free_ctx(ctx);
    delete ctx;
    return LMMEW_OK;
}

int64_t lmmew_support_size(const lmmew_ctx *ctx) { return ctx ? (int64_t)ctx->S.Qm : -1; }

int lmmew_path_table(lmmew_ctx *ctx, int enable, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!enable) {
        if (ctx->d_ptab) {
            HIPCHK(ctx, hipStreamSynchronize(st));
            dfree(ctx->d_ptab);
            ctx->d_ptab = nullptr;
        }
        return LMMEW_OK;
    }
    if (ctx->d_ptab || ctx->S.nsc == 0) return LMMEW_OK;
    const size_t n = (size_t)ctx->S.na * ctx->S.nsc * 2 * ctx->S.nw * ctx->S.Qp;
    size_t fr = 0, tot = 0;
    HIPCHK(ctx, hipMemGetInfo(&fr, &tot));
    if (n * sizeof(float) + (size_t(1) << 30) > fr) {
        char buf[128];
        snprintf(buf, sizeof buf, "the path-parameter table needs %.1f GB of device memory",
                 n * sizeof(float) / 1e9);
        return fail(ctx, LMMEW_ENOMEM, buf);
    }
    float *t = nullptr;
    if (dalloc(&t, n) != hipSuccess) return fail(ctx, LMMEW_ENOMEM, "path-parameter table");
    hipError_t e = launch_path_table(ctx->S, ctx->d_pix, ctx->d_pixz, ctx->d_dirs, ctx->d_gqs,
                                     ctx->d_sa, ctx->d_scz, t, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        dfree(t);
        return hipfail(ctx, e, "path-parameter table");
    }
    ctx->d_ptab = t;
    return LMMEW_OK;
}

int lmmew_psf_table(lmmew_ctx *ctx, int enable, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!enable) {
        if (ctx->d_psft) {
            HIPCHK(ctx, hipStreamSynchronize(st));
            dfree(ctx->d_psft);
            ctx->d_psft = nullptr;
        }
        ctx->psft_off = true;
        return LMMEW_OK;
    }
    ctx->psft_off = false;
    const int rc = ensure_psft(ctx, st);
    if (rc != LMMEW_OK) return rc;
    HIPCHK(ctx, hipStreamSynchronize(st));
    return ctx->d_psft ? 1 : 0;
}

int64_t lmmew_path_table_bytes(const lmmew_ctx *ctx)
{
    if (!ctx) return -1;
    return (int64_t)ctx->S.na * ctx->S.nsc * 2 * ctx->S.nw * ctx->S.Qp * (int64_t)sizeof(float);
}

int lmmew_sensitivity(lmmew_ctx *ctx, int n_subsets, float *sens, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!sens) return fail(ctx, LMMEW_EINVAL, "sens is NULL");
    if (n_subsets < 1 || n_subsets > ctx->S.na)
        return fail(ctx, LMMEW_EINVAL, "n_subsets must be in 1..n_angles");
    if (!ctx->d_Sqa) HIPCHK(ctx, dalloc(&ctx->d_Sqa, (size_t)ctx->S.na * ctx->S.Qp));
    HIPCHK(ctx, hipMemsetAsync(sens, 0, (size_t)n_subsets * ctx->Q * sizeof(float), st));
    SensArgs g{};
    g.pix_xy = ctx->d_pix;
    g.pix_z = ctx->d_pixz;
    g.sz = ctx->d_scz;
    g.dirs = ctx->d_dirs;
    g.g_qa = ctx->d_gqa;
    g.g_qs = ctx->d_gqs;
    g.sa = ctx->d_sa;
    g.pixq = ctx->d_pixq;
    g.Sqa = ctx->d_Sqa;
    g.sens = sens;
    g.nsub = n_subsets;
    g.Q = ctx->Q;
    HIPCHK(ctx, launch_sens(ctx->S, g, st));
    return LMMEW_OK;
}

static int subsets_for_budget(const lmmew_ctx *ctx, int64_t n)
{
    const size_t row = (size_t)ctx->S.Qp * sizeof(float);
    int nsub = 1;
    while (nsub < ctx->S.na && (size_t)(n / nsub + 64) * row > kScratchBudget) nsub *= 2;
    return std::min(nsub, ctx->S.na);
}

int lmmew_forward(lmmew_ctx *ctx, const lmmew_events *ev, const float *lambda, float *p,
                  hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!ev || !lambda || (!p && ev->n > 0)) return fail(ctx, LMMEW_EINVAL, "NULL argument");
    lmmew_plan *pl = nullptr;
    int rc = make_plan(ctx, ev, nullptr, 1, subsets_for_budget(ctx, ev->n), st, &pl);
    if (rc != LMMEW_OK) return rc;
    if (rc == LMMEW_OK) rc = run_compact(ctx, pl, lambda, st);
    for (int s = 0; s < pl->nsub && rc == LMMEW_OK; ++s) {
        rc = run_rows(ctx, pl, s, st);
        if (rc == LMMEW_OK) rc = run_forward(ctx, pl, s, false, 0, st);
    }
    if (rc == LMMEW_OK) {
        hipError_t e = launch_scatter_out(pl->d_p, pl->d_perm, pl->n, p, st);
        if (e != hipSuccess) rc = hipfail(ctx, e, "scatter");
    }
    hipError_t e = hipStreamSynchronize(st);
    if (rc == LMMEW_OK && e != hipSuccess) rc = hipfail(ctx, e, "synchronize");
    lmmew_plan_destroy(pl);
    return rc;
}

int lmmew_backproject(lmmew_ctx *ctx, const lmmew_events *ev, const float *w, float *out,
                      hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!ev || !out || (!w && ev->n > 0)) return fail(ctx, LMMEW_EINVAL, "NULL argument");
    lmmew_plan *pl = nullptr;
    int rc = make_plan(ctx, ev, nullptr, 1, subsets_for_budget(ctx, ev->n), st, &pl);
    if (rc != LMMEW_OK) return rc;
    hipError_t e = hipMemsetAsync(out, 0, (size_t)ctx->Q * sizeof(float), st);
    if (e != hipSuccess) rc = hipfail(ctx, e, "memset");
    if (rc == LMMEW_OK) {
        e = launch_gather_w(w, pl->d_perm, pl->n, pl->d_wt, st);
        if (e != hipSuccess) rc = hipfail(ctx, e, "gather");
    }
    for (int s = 0; s < pl->nsub && rc == LMMEW_OK; ++s) {
        const lmmew_plan::Sub &sub = pl->subs[s];
        rc = run_rows(ctx, pl, s, st);
        if (rc == LMMEW_OK)
            rc = run_back(ctx, pl, s, pl->d_wt + sub.row0, pl->d_part + (size_t)sub.chunk0 * ctx->S.Qp,
                          pl->d_comp + (size_t)sub.chunk0 * ctx->S.Qp, st);
    }
    if (rc == LMMEW_OK) {
        const int total = (int)pl->chunks.size();
        int *d_cc = nullptr;
        const int cc[2] = {0, total};
        e = dalloc(&d_cc, 2);
        if (e == hipSuccess) e = hipMemcpyAsync(d_cc, cc, sizeof cc, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            UpdArgs u{};
            u.part = pl->d_part;
            u.comp = pl->d_comp;
            u.case_chunk = d_cc;
            u.ncases = 1;
            u.pixq = ctx->d_pixq;
            u.Q = ctx->Q;
            u.sens = nullptr;
            u.lambda = out;
            e = launch_update(ctx->S, u, st);
        }
        hipError_t e2 = hipStreamSynchronize(st);
        if (e == hipSuccess) e = e2;
        dfree(d_cc);
        if (e != hipSuccess) rc = hipfail(ctx, e, "backprojection");
    } else {
        (void)hipStreamSynchronize(st);
    }
    lmmew_plan_destroy(pl);
    return rc;
}

static int osem_run(lmmew_ctx *ctx, lmmew_plan *p, int first_subset, int count, const float *sens,
                    float *lambda, lmmew_stats *stats, hipStream_t st);

int lmmew_osem_graph(lmmew_ctx *ctx, lmmew_plan *p, int n_iters, const float *sens,
                     float *lambda, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!p || p->ctx != ctx) return fail(ctx, LMMEW_EINVAL, "plan does not belong to context");
    if (!sens || !lambda) return fail(ctx, LMMEW_EINVAL, "NULL image or sensitivity");
    if (n_iters < 0) return fail(ctx, LMMEW_EINVAL, "n_iters < 0");
    if (n_iters == 0) return LMMEW_OK;
    {
        const int rm = sync_maps(ctx, p, st);
        if (rm != LMMEW_OK) return rm;
    }
    if (!p->d_Acache && (ctx->mlp || ctx->xgrid > 1)) {
        const int rc = coarse_scratch(ctx, p);   // no allocation inside the capture
        if (rc != LMMEW_OK) return rc;
    }
    if (!p->gexec || p->g_iters != n_iters || p->g_sens != sens || p->g_lambda != lambda ||
        p->g_jt != p->JT || p->g_gen != plan_model_gen(ctx, p) || p->g_cache != p->d_Acache ||
        p->g_tab != plan_ptab(ctx, p) || p->g_psft != ctx->d_psft) {
        if (p->gexec) {
            HIPCHK(ctx, hipGraphExecDestroy(p->gexec));
            p->gexec = nullptr;
        }
        // Capture records launches without running them; it happens on a private
        // stream (the caller's may be the null stream, which cannot be captured)
        // and the graph is then launched on the caller's stream.
        if (!ctx->cap_stream)
            HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = ctx->cap_stream;
        const bool prof_was = p->prof;
        p->prof = false;                 // no event records inside the capture
        HIPCHK(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const int rc = osem_run(ctx, p, 0, n_iters * p->nsub, sens, lambda, nullptr, cs);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(cs, &g);
        p->prof = prof_was;
        if (rc != LMMEW_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (ec != hipSuccess) return hipfail(ctx, ec, "hipStreamEndCapture");
        const hipError_t ei = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            p->gexec = nullptr;
            return hipfail(ctx, ei, "hipGraphInstantiate");
        }
        p->g_iters = n_iters;
        p->g_sens = sens;
        p->g_lambda = lambda;
        p->g_jt = p->JT;
        p->g_gen = plan_model_gen(ctx, p);
        p->g_cache = p->d_Acache;
        p->g_tab = plan_ptab(ctx, p);
        p->g_psft = ctx->d_psft;
    }
    HIPCHK(ctx, hipGraphLaunch(p->gexec, st));
    return LMMEW_OK;
}

int lmmew_plan_create(lmmew_ctx *ctx, const lmmew_events *ev, const int64_t *case_offsets,
                      int n_cases, int n_subsets, hipStream_t st, lmmew_plan **out)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!out) return fail(ctx, LMMEW_EINVAL, "out is NULL");
    return make_plan(ctx, ev, case_offsets, n_cases, n_subsets, st, out);
}

int lmmew_plan_create_maps(lmmew_ctx *const *ctxs, const lmmew_events *ev,
                           const int64_t *case_offsets, int n_cases, int n_subsets, hipStream_t st,
                           lmmew_plan **out)
{
    if (!ctxs || !ctxs[0]) return LMMEW_EINVAL;
    lmmew_ctx *ctx = ctxs[0];
    if (!out) return fail(ctx, LMMEW_EINVAL, "out is NULL");
    if (n_cases < 1) return fail(ctx, LMMEW_EINVAL, "n_cases must be >= 1");
    return make_plan(ctx, ev, case_offsets, n_cases, n_subsets, st, out, ctxs);
}

int lmmew_plan_cache_rows(lmmew_ctx *ctx, lmmew_plan *p, int enable, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!p || p->ctx != ctx) return fail(ctx, LMMEW_EINVAL, "plan does not belong to context");
    if (p->gexec) {                      // a captured graph may refer to the rows
        HIPCHK(ctx, hipStreamSynchronize(st));
        HIPCHK(ctx, hipGraphExecDestroy(p->gexec));
        p->gexec = nullptr;
    }
    if (p->d_Acache) {
        HIPCHK(ctx, hipStreamSynchronize(st));
        dfree(p->d_Acache);
        p->d_Acache = nullptr;
        p->cache_gen = -1;
    }
    if (!enable || p->n == 0) return LMMEW_OK;
    {
        const int rm = sync_maps(ctx, p, st);
        if (rm != LMMEW_OK) return rm;
    }
    const size_t bytes = (size_t)p->n * ctx->S.Qp * sizeof(float);
    size_t fr = 0, tot = 0;
    HIPCHK(ctx, hipMemGetInfo(&fr, &tot));
    if (bytes + (size_t(1) << 30) > fr)
        return fail(ctx, LMMEW_ENOMEM, "not enough free device memory for the cached rows");
    float *c = nullptr;
    if (dalloc(&c, (size_t)p->n * ctx->S.Qp) != hipSuccess)
        return fail(ctx, LMMEW_ENOMEM, "cached rows");
    int rc = LMMEW_OK;
    for (int s = 0; s < p->nsub && rc == LMMEW_OK; ++s)
        rc = run_rows(ctx, p, s, st, 0, c + (size_t)p->subs[s].row0 * ctx->S.Qp);
    const hipError_t e = hipStreamSynchronize(st);
    if (rc == LMMEW_OK && e != hipSuccess) rc = hipfail(ctx, e, "caching rows");
    if (rc != LMMEW_OK) {
        dfree(c);
        return rc;
    }
    p->d_Acache = c;
    p->cache_gen = plan_model_gen(ctx, p);
    return LMMEW_OK;
}

int lmmew_plan_destroy(lmmew_plan *plan)
{
    if (!plan) return LMMEW_EINVAL;
    (void)hipDeviceSynchronize();
    free_plan(plan);
    delete plan;
    return LMMEW_OK;
}

int lmmew_plan_set_event_tile(lmmew_ctx *ctx, lmmew_plan *plan, int event_tile, hipStream_t st)
{
    if (!ctx || !plan || plan->ctx != ctx) return LMMEW_EINVAL;
    if (event_tile != 16 && event_tile != 32 && event_tile != 64)
        return fail(ctx, LMMEW_EINVAL, "event_tile must be 16, 32 or 64");
    if (event_tile == plan->JT) return LMMEW_OK;
    HIPCHK(ctx, hipStreamSynchronize(st));
    plan->JT = event_tile;
    build_tiles(plan);
    return upload_tiles(ctx, plan, st);
}

int lmmew_plan_get_event_tile(const lmmew_plan *plan) { return plan ? plan->JT : 0; }

namespace {
// Autotuner cache: problem shape -> fastest event tile.
struct TuneKey {
    int Qm, nsc, nw, na, nsub, per_angle, nz, cont;
    bool operator==(const TuneKey &o) const
    {
        return Qm == o.Qm && nsc == o.nsc && nw == o.nw && na == o.na && nsub == o.nsub &&
               per_angle == o.per_angle && nz == o.nz && cont == o.cont;
    }
};
std::vector<std::pair<TuneKey, int>> g_tune_cache;

TuneKey tune_key(const lmmew_ctx *ctx, const lmmew_plan *p)
{
    // events per (case, angle), bucketed by powers of two
    const double per = (double)p->n / std::max(1, p->ncases) / std::max(1, ctx->S.na);
    int b = 0;
    while ((1 << b) < per) ++b;
    return TuneKey{ctx->S.Qm, ctx->S.nsc, ctx->S.nw, ctx->S.na, p->nsub, b, ctx->S.nz,
                   p->cont ? 1 : 0};
}
}  // namespace

int lmmew_autotune(lmmew_ctx *ctx, lmmew_plan *p, int use_cache, hipStream_t st, int *chosen)
{
    if (!ctx || !p || p->ctx != ctx) return LMMEW_EINVAL;
    {
        const int rm = sync_maps(ctx, p, st);
        if (rm != LMMEW_OK) return rm;
    }
    const TuneKey key = tune_key(ctx, p);
    if (use_cache) {
        for (const auto &kv : g_tune_cache)
            if (kv.first == key) {
                if (chosen) *chosen = kv.second;
                return lmmew_plan_set_event_tile(ctx, p, kv.second, st);
            }
    }
    int big = 0;
    for (int s = 1; s < p->nsub; ++s)
        if (p->subs[s].rows > p->subs[big].rows) big = s;
    const bool prof_was = p->prof;
    p->prof = false;
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    int best = 16;
    float best_ms = 0.f;
    int rc = LMMEW_OK;
    for (int jt : {16, 32, 64}) {
        rc = lmmew_plan_set_event_tile(ctx, p, jt, st);
        if (rc != LMMEW_OK) break;
        // the per-event kernel alone (it writes only the plan's scratch rows) on
        // the largest subset: once to warm up, once timed
        rc = run_rows(ctx, p, big, st);
        if (rc != LMMEW_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = LMMEW_EDEVICE; break; }
        rc = run_rows(ctx, p, big, st);
        if (rc != LMMEW_OK) break;
        float ms = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(ctx, LMMEW_EDEVICE, "autotune timing failed");
            break;
        }
        if (jt == 16 || ms < best_ms) {
            best = jt;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->prof = prof_was;
    if (rc != LMMEW_OK) return rc;
    g_tune_cache.push_back({key, best});
    if (chosen) *chosen = best;
    return lmmew_plan_set_event_tile(ctx, p, best, st);
}

int lmmew_plan_profile(lmmew_ctx *ctx, lmmew_plan *plan, int enable)
{
    if (!ctx || !plan || plan->ctx != ctx) return LMMEW_EINVAL;
    plan->prof = enable != 0;
    plan->prof_used = 0;
    return LMMEW_OK;
}

int lmmew_plan_profile_read_kernels(lmmew_ctx *ctx, lmmew_plan *plan, double *ms,
                                    int64_t *launches)
{
    if (!ctx || !plan || plan->ctx != ctx) return LMMEW_EINVAL;
    double tot[2] = {0.0, 0.0};
    int64_t cnt[2] = {0, 0};
    for (size_t k = 0; k + 1 < plan->prof_used; k += 2) {
        HIPCHK(ctx, hipEventSynchronize(plan->prof_ev[k + 1]));
        float t = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&t, plan->prof_ev[k], plan->prof_ev[k + 1]));
        const int kind = plan->prof_kind[k / 2];
        tot[kind] += t;
        cnt[kind] += 1;
    }
    for (int i = 0; i < 2; ++i) {
        if (ms) ms[i] = tot[i];
        if (launches) launches[i] = cnt[i];
    }
    plan->prof_used = 0;
    return LMMEW_OK;
}

int lmmew_plan_profile_read(lmmew_ctx *ctx, lmmew_plan *plan, double *row_ms, int64_t *launches)
{
    double ms[2];
    int64_t cnt[2];
    const int rc = lmmew_plan_profile_read_kernels(ctx, plan, ms, cnt);
    if (rc != LMMEW_OK) return rc;
    if (row_ms) *row_ms = ms[0];
    if (launches) *launches = cnt[0];
    return LMMEW_OK;
}

int lmmew_plan_terms(const lmmew_plan *plan, double *out_terms, double *out_full_terms)
{
    if (!plan) return LMMEW_EINVAL;
    if (out_terms) *out_terms = plan->terms;
    if (out_full_terms) *out_full_terms = plan->full_terms;
    return LMMEW_OK;
}

static int osem_run(lmmew_ctx *ctx, lmmew_plan *p, int first_subset, int count, const float *sens,
                    float *lambda, lmmew_stats *stats, hipStream_t st)
{
    const int K = count;
    const bool want = stats != nullptr;
    if (p->d_Acache && p->cache_gen != plan_model_gen(ctx, p))
        return fail(ctx, LMMEW_EINVAL,
                    "cached rows are stale: the scatter model changed (cache them again)");
    if (K > 0) {
        const int rc = run_compact(ctx, p, lambda, st);
        if (rc != LMMEW_OK) return rc;
    }
    if (want) {
        int rc = ensure_stats(ctx, p, std::max(K, 1));
        if (rc != LMMEW_OK) return rc;
        HIPCHK(ctx, hipMemsetAsync(p->d_nskip, 0, sizeof(unsigned long long) * std::max(K, 1), st));
    }
    for (int k = 0; k < K; ++k) {
        const int s = (first_subset + k) % p->nsub;
        const lmmew_plan::Sub &sub = p->subs[s];
        int rc = p->d_Acache ? LMMEW_OK : run_rows(ctx, p, s, st);
        if (rc == LMMEW_OK) rc = run_forward(ctx, p, s, want, k, st);
        if (rc != LMMEW_OK) return rc;
        if (want) {
            ReduceArgs ra{};
            ra.logp = p->d_logp + sub.row0;
            ra.rows = sub.rows;
            ra.sens = sens + (size_t)s * ctx->Q;
            ra.sens_stride = p->maps.empty() ? 0 : (long)p->nsub * ctx->Q;
            ra.lambda = lambda;
            ra.ncases = p->ncases;
            ra.Q = ctx->Q;
            ra.out = p->d_ll + k;
            HIPCHK(ctx, launch_loglik(ra, st));
        }
        rc = run_back(ctx, p, s, p->d_wt + sub.row0, p->d_part, p->d_comp, st);
        if (rc != LMMEW_OK) return rc;
        UpdArgs u{};
        u.part = p->d_part;
        u.comp = p->d_comp;
        u.case_chunk = p->d_case_chunk + (size_t)s * (p->ncases + 1);
        u.ncases = p->ncases;
        u.pixq = ctx->d_pixq;
        u.Q = ctx->Q;
        u.sens = sens + (size_t)s * ctx->Q;
        u.sens_stride = p->maps.empty() ? 0 : (long)p->nsub * ctx->Q;
        u.lambda = lambda;
        u.lamc = p->d_lamc;
        HIPCHK(ctx, launch_update(ctx->S, u, st));
    }
    if (want) {
        std::vector<unsigned long long> sk(std::max(K, 1));
        std::vector<double> ll(std::max(K, 1));
        std::vector<float> lam((size_t)p->ncases * ctx->Q);
        HIPCHK(ctx, hipMemcpyAsync(sk.data(), p->d_nskip, sk.size() * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipMemcpyAsync(ll.data(), p->d_ll, ll.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipMemcpyAsync(lam.data(), lambda, lam.size() * sizeof(float),
                                   hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        stats->skipped_total = 0;
        for (int i = 0; i < K; ++i) {
            stats->skipped_total += (int64_t)sk[i];
            if (stats->skipped) stats->skipped[i] = (int64_t)sk[i];
            if (stats->subset_loglik) stats->subset_loglik[i] = ll[i];
        }
        for (float v : lam)
            if (!std::isfinite(v)) return fail(ctx, LMMEW_ENUMERIC, "non-finite image value");
    }
    return LMMEW_OK;
}

int lmmew_osem_iter(lmmew_ctx *ctx, lmmew_plan *p, int n_iters, const float *sens, float *lambda,
                    lmmew_stats *stats, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!p || p->ctx != ctx) return fail(ctx, LMMEW_EINVAL, "plan does not belong to context");
    if (!sens || !lambda) return fail(ctx, LMMEW_EINVAL, "NULL image or sensitivity");
    if (n_iters < 0) return fail(ctx, LMMEW_EINVAL, "n_iters < 0");
    const int rm = sync_maps(ctx, p, st);
    if (rm != LMMEW_OK) return rm;
    return osem_run(ctx, p, 0, n_iters * p->nsub, sens, lambda, stats, st);
}

int lmmew_osem_subiter(lmmew_ctx *ctx, lmmew_plan *p, int subset, const float *sens,
                       float *lambda, lmmew_stats *stats, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!p || p->ctx != ctx) return fail(ctx, LMMEW_EINVAL, "plan does not belong to context");
    if (!sens || !lambda) return fail(ctx, LMMEW_EINVAL, "NULL image or sensitivity");
    if (subset < 0 || subset >= p->nsub) return fail(ctx, LMMEW_EINVAL, "subset out of range");
    const int rm = sync_maps(ctx, p, st);
    if (rm != LMMEW_OK) return rm;
    return osem_run(ctx, p, subset, 1, sens, lambda, stats, st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// per-event rows and the scatter surrogate
// ---------------------------------------------------------------------------
namespace {

uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double unit_rand(uint64_t &x) { return (double)(splitmix64(x) >> 11) * (1.0 / 9007199254740992.0); }

void free_mlp(lmmew_mlp *m)
{
    dfree(m->P); dfree(m->G); dfree(m->m1); dfree(m->m2);
    dfree(m->W2b); dfree(m->W3b);
    dfree(m->X); dfree(m->Z1); dfree(m->Z2); dfree(m->Z3); dfree(m->H3); dfree(m->dZ); dfree(m->dH);
    dfree(m->y); dfree(m->dy); dfree(m->sq); dfree(m->H1b); dfree(m->H2b); dfree(m->dZb);
    dfree(m->idx); dfree(m->dloss); dfree(m->part); dfree(m->split); dfree(m->dsum);
    dfree(m->d_cnode); dfree(m->d_cidx); dfree(m->d_cw);
}

int mlp_workspace(lmmew_ctx *ctx, lmmew_mlp *m, int M)
{
    if (M <= m->cap) return LMMEW_OK;
    dfree(m->X); dfree(m->Z1); dfree(m->Z2); dfree(m->Z3); dfree(m->H3); dfree(m->dZ); dfree(m->dH);
    dfree(m->y); dfree(m->dy); dfree(m->sq); dfree(m->H1b); dfree(m->H2b); dfree(m->dZb);
    dfree(m->idx); dfree(m->part); dfree(m->split); dfree(m->dsum);
    const size_t n = (size_t)M * kMlpHidden;
    HIPCHK(ctx, dalloc(&m->X, (size_t)M * kMlpIn));
    HIPCHK(ctx, dalloc(&m->Z1, n));
    HIPCHK(ctx, dalloc(&m->Z2, n));
    HIPCHK(ctx, dalloc(&m->Z3, n));
    HIPCHK(ctx, dalloc(&m->H3, n));
    HIPCHK(ctx, dalloc(&m->dZ, n));
    HIPCHK(ctx, dalloc(&m->dH, n));
    HIPCHK(ctx, dalloc(&m->H1b, n));
    HIPCHK(ctx, dalloc(&m->H2b, n));
    HIPCHK(ctx, dalloc(&m->dZb, n));
    HIPCHK(ctx, dalloc(&m->y, M));
    HIPCHK(ctx, dalloc(&m->dy, M));
    HIPCHK(ctx, dalloc(&m->sq, M));
    HIPCHK(ctx, dalloc(&m->idx, M));
    HIPCHK(ctx, dalloc(&m->part, (size_t)((M + kRedRows - 1) / kRedRows) * 8 * kMlpHidden));
    HIPCHK(ctx, dalloc(&m->split, (size_t)64 * kMlpHidden * kMlpHidden));
    HIPCHK(ctx, dalloc(&m->dsum, 1));
    m->cap = M;
    return LMMEW_OK;
}

MlpWork mlp_work(const lmmew_mlp *m)
{
    MlpWork w{};
    w.X = m->X; w.Z1 = m->Z1; w.Z2 = m->Z2; w.Z3 = m->Z3; w.H3 = m->H3; w.dZ = m->dZ; w.dH = m->dH;
    w.y = m->y; w.dy = m->dy; w.sq = m->sq; w.H1b = m->H1b; w.H2b = m->H2b; w.dZb = m->dZb;
    w.W2b = m->W2b; w.W3b = m->W3b;
    w.part = m->part; w.split = m->split; w.dsum = m->dsum;
    return w;
}

}  // namespace

extern "C" {

int lmmew_rows(lmmew_ctx *ctx, const lmmew_events *ev, int part, float *rows, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!ev || (!rows && ev->n > 0)) return fail(ctx, LMMEW_EINVAL, "NULL argument");
    if (part < 0 || part > 3) return fail(ctx, LMMEW_EINVAL, "part must be 0..3");
    lmmew_plan *pl = nullptr;
    int rc = make_plan(ctx, ev, nullptr, 1, subsets_for_budget(ctx, ev->n), st, &pl);
    if (rc != LMMEW_OK) return rc;
    hipError_t e = hipMemsetAsync(rows, 0, (size_t)ev->n * ctx->Q * sizeof(float), st);
    if (e != hipSuccess) rc = hipfail(ctx, e, "memset");
    for (int s = 0; s < pl->nsub && rc == LMMEW_OK; ++s) {
        const int mode = part == 0 ? 0 : (part == 1 ? 1 : (part == 2 ? 2 : 3));
        rc = run_rows(ctx, pl, s, st, mode);
        if (rc == LMMEW_OK) {
            const lmmew_plan::Sub &sub = pl->subs[s];
            e = launch_rows_out(ctx->S, pl->d_A, sub.rows, pl->d_perm + sub.row0, ctx->d_pixq,
                                ctx->Q, rows, st);
            if (e != hipSuccess) rc = hipfail(ctx, e, "rows out");
        }
    }
    e = hipStreamSynchronize(st);
    if (rc == LMMEW_OK && e != hipSuccess) rc = hipfail(ctx, e, "synchronize");
    lmmew_plan_destroy(pl);
    return rc;
}

int lmmew_plan_rows(lmmew_ctx *ctx, lmmew_plan *p, int subset, const int64_t *events, int64_t n,
                    float *rows, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!p || p->ctx != ctx) return fail(ctx, LMMEW_EINVAL, "plan of another context");
    if (subset < 0 || subset >= p->nsub) return fail(ctx, LMMEW_EINVAL, "subset out of range");
    if (n < 0 || (n > 0 && (!events || !rows))) return fail(ctx, LMMEW_EINVAL, "NULL argument");
    if (n == 0) return LMMEW_OK;
    const lmmew_plan::Sub &sub = p->subs[subset];
    std::vector<int> inv(p->n, -1);   // input index -> row within the subset
    for (int r = 0; r < sub.rows; ++r) inv[p->perm[sub.row0 + r]] = r;
    std::vector<int> ridx(n);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t j = events[k];
        if (j < 0 || j >= p->n || inv[j] < 0)
            return fail(ctx, LMMEW_EINVAL, "event " + std::to_string((long long)j) +
                                               " is not in subset " + std::to_string(subset));
        ridx[k] = inv[j];
    }
    int rc = sync_maps(ctx, p, st);
    if (rc == LMMEW_OK) rc = run_rows(ctx, p, subset, st);
    if (rc != LMMEW_OK) return rc;
    int *d_idx = nullptr;
    hipError_t e = dalloc(&d_idx, (size_t)n);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_idx, ridx.data(), n * sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(rows, 0, (size_t)n * ctx->Q * sizeof(float), st);
    if (e == hipSuccess)
        e = launch_rows_pick(ctx->S, p->d_A, d_idx, (int)n, ctx->d_pixq, ctx->Q, rows, st);
    const hipError_t e2 = hipStreamSynchronize(st);
    if (e == hipSuccess) e = e2;
    dfree(d_idx);
    if (e != hipSuccess) return hipfail(ctx, e, "plan rows");
    return LMMEW_OK;
}

int lmmew_mlp_create(lmmew_ctx *ctx, uint64_t seed, lmmew_mlp **out)
{
    if (!ctx || !out) return LMMEW_EINVAL;
    *out = nullptr;
    if (ctx->S.nz > 0)
        return fail(ctx, LMMEW_EINVAL, "the scatter surrogate models the planar system only");
    lmmew_mlp *m = new (std::nothrow) lmmew_mlp;
    if (!m) return fail(ctx, LMMEW_ENOMEM, "host allocation");
    m->ctx = ctx;
    auto bail = [&](int code) {
        free_mlp(m);
        delete m;
        return code;
    };
#define MCHK(call)                                                 \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return bail(hipfail(ctx, e_, #call)); \
    } while (0)
    MCHK(dalloc(&m->P, kMlpParams));
    MCHK(dalloc(&m->G, kMlpParams));
    MCHK(dalloc(&m->m1, kMlpParams));
    MCHK(dalloc(&m->m2, kMlpParams));
    MCHK(dalloc(&m->W2b, 2 * kMlpHidden * kMlpHidden));
    MCHK(dalloc(&m->W3b, 2 * kMlpHidden * kMlpHidden));
    MCHK(dalloc(&m->dloss, 1));
    // Glorot-uniform weights, zero biases, from a counter-based generator
    std::vector<float> P(kMlpParams, 0.f);
    uint64_t st_ = seed;
    auto fill = [&](int off, int fin, int fout) {
        const double a = std::sqrt(6.0 / (fin + fout));
        for (int t = 0; t < fin * fout; ++t) P[off + t] = (float)((2.0 * unit_rand(st_) - 1.0) * a);
    };
    fill(kOffW1, kMlpIn, kMlpHidden);
    fill(kOffW2, kMlpHidden, kMlpHidden);
    fill(kOffW3, kMlpHidden, kMlpHidden);
    fill(kOffW4, kMlpHidden, 1);
    MCHK(hipMemcpy(m->P, P.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    MCHK(hipMemset(m->m1, 0, sizeof(float) * kMlpParams));
    MCHK(hipMemset(m->m2, 0, sizeof(float) * kMlpParams));
    MCHK(mlp_refresh(m->P, m->W2b, m->W3b, nullptr));
    MCHK(hipStreamSynchronize(nullptr));   // the copies and the refresh ran on the null stream
#undef MCHK
    ctx->nets.push_back(m);
    *out = m;
    return LMMEW_OK;
}

int lmmew_mlp_destroy(lmmew_mlp *m)
{
    if (!m) return LMMEW_EINVAL;
    (void)hipDeviceSynchronize();
    if (m->ctx) {
        std::vector<lmmew_mlp *> &v = m->ctx->nets;
        v.erase(std::remove(v.begin(), v.end(), m), v.end());
        if (m->ctx->mlp == m) {
            m->ctx->mlp = nullptr;
            m->ctx->model_gen++;
        }
    }
    free_mlp(m);
    delete m;
    return LMMEW_OK;
}

int lmmew_mlp_get_params(const lmmew_mlp *m, float *params, double *c0, double *floor_)
{
    if (!m) return LMMEW_EINVAL;
    if (params &&
        hipMemcpy(params, m->P, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost) != hipSuccess)
        return LMMEW_EDEVICE;
    if (c0) *c0 = m->c0;
    if (floor_) *floor_ = m->floor_;
    return LMMEW_OK;
}

int lmmew_mlp_set_params(lmmew_mlp *m, const float *params, double c0, double floor_)
{
    if (!m || !params || !m->ctx) return LMMEW_EINVAL;   // NULL, or detached from its context
    lmmew_ctx *ctx = m->ctx;
    HIPCHK(ctx, hipMemcpy(m->P, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemset(m->m1, 0, sizeof(float) * kMlpParams));
    HIPCHK(ctx, hipMemset(m->m2, 0, sizeof(float) * kMlpParams));
    HIPCHK(ctx, mlp_refresh(m->P, m->W2b, m->W3b, nullptr));
    HIPCHK(ctx, hipStreamSynchronize(nullptr));   // the copies and the refresh ran on the null stream
    m->step = 0;
    m->c0 = c0;
    m->floor_ = floor_;
    ctx->model_gen++;
    return LMMEW_OK;
}

int lmmew_mlp_forward(lmmew_ctx *ctx, lmmew_mlp *m, const float *feats, int64_t n, float *y,
                      hipStream_t st)
{
    if (!ctx || !m || m->ctx != ctx) return LMMEW_EINVAL;
    if (n < 0 || (n > 0 && (!feats || !y))) return fail(ctx, LMMEW_EINVAL, "bad arguments");
    const int chunk = 65536;
    int rc = mlp_workspace(ctx, m, chunk);
    if (rc != LMMEW_OK) return rc;
    std::vector<int> idx(chunk);
    const MlpWork w = mlp_work(m);
    for (int64_t b = 0; b < n; b += chunk) {
        const int cnt = (int)std::min<int64_t>(chunk, n - b);
        const int M = (cnt + 15) / 16 * 16;
        for (int t = 0; t < M; ++t) idx[t] = (int)(b + std::min(t, cnt - 1));
        HIPCHK(ctx, hipMemcpyAsync(m->idx, idx.data(), sizeof(int) * M, hipMemcpyHostToDevice, st));
        HIPCHK(ctx, mlp_forward_batch(w, m->P, feats, m->idx, M, nullptr, st));
        HIPCHK(ctx, hipMemcpyAsync(y + b, m->y, sizeof(float) * cnt, hipMemcpyDeviceToDevice, st));
        HIPCHK(ctx, hipStreamSynchronize(st));     // idx is reused for the next chunk
    }
    return LMMEW_OK;
}

int lmmew_mlp_grad(lmmew_ctx *ctx, lmmew_mlp *m, const float *feats, const float *target,
                   int64_t n, float *grad, double *loss, hipStream_t st)
{
    if (!ctx || !m || m->ctx != ctx) return LMMEW_EINVAL;
    if (!feats || !target || !grad || n <= 0 || n % 16 != 0 || n > (1 << 24))
        return fail(ctx, LMMEW_EINVAL, "n must be a positive multiple of 16 (<= 2^24)");
    int rc = mlp_workspace(ctx, m, (int)n);
    if (rc != LMMEW_OK) return rc;
    const MlpWork w = mlp_work(m);
    HIPCHK(ctx, mlp_forward_batch(w, m->P, feats, nullptr, (int)n, target, st));
    HIPCHK(ctx, mlp_backward_batch(w, m->P, (int)n, m->G, st));
    HIPCHK(ctx, hipMemcpyAsync(grad, m->G, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, st));
    HIPCHK(ctx, mlp_loss(w, (int)n, m->dloss, st));
    double l = 0.0;
    HIPCHK(ctx, hipMemcpyAsync(&l, m->dloss, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    if (loss) *loss = l / (double)n;
    return LMMEW_OK;
}

int lmmew_mlp_train(lmmew_ctx *ctx, lmmew_mlp *m, const float *feats, const float *target,
                    int64_t n, int batch, int epochs, double lr, uint64_t seed, double *epoch_loss,
                    hipStream_t st)
{
    const double lr0 = lr;
    if (!ctx || !m || m->ctx != ctx) return LMMEW_EINVAL;
    if (!feats || !target || batch <= 0 || batch % 16 != 0 || epochs < 0 || n < batch ||
        n > ((int64_t)1 << 31) - 1)
        return fail(ctx, LMMEW_EINVAL, "bad training arguments (batch a multiple of 16, n >= batch)");
    int rc = mlp_workspace(ctx, m, batch);
    if (rc != LMMEW_OK) return rc;
    const int64_t nb = n / batch;
    // Two permutation buffers on each side: a worker thread shuffles epoch
    // ep + 1's order while this thread enqueues epoch ep (before refilling a
    // host buffer it waits only for the copy made from it two epochs
    // earlier), so the device does not wait for the shuffle once the stream's
    // queue is full; the batch losses of every epoch are read back once at
    // the end.
    int *d_perm[2] = {nullptr, nullptr};
    double *d_losses = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};
    auto release = [&]() {
        dfree(d_perm[0]);
        dfree(d_perm[1]);
        dfree(d_losses);
        for (hipEvent_t &v : copied)
            if (v) (void)hipEventDestroy(v);
    };
    if (dalloc(&d_perm[0], n) != hipSuccess || dalloc(&d_perm[1], n) != hipSuccess ||
        dalloc(&d_losses, (size_t)std::max(epochs, 1) * nb) != hipSuccess ||
        hipEventCreateWithFlags(&copied[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&copied[1], hipEventDisableTiming) != hipSuccess) {
        release();
        return fail(ctx, LMMEW_ENOMEM, "training buffers");
    }
    std::vector<int> perm[2] = {std::vector<int>(n), std::vector<int>(n)};
    uint64_t rs = seed;
    // the epochs' orders, in sequence from one generator (Fisher-Yates)
    auto shuffle = [&rs, n](std::vector<int> *pv) {
        for (int64_t t = 0; t < n; ++t) (*pv)[t] = (int)t;
        for (int64_t t = n - 1; t > 0; --t) {
            const int64_t j = (int64_t)(splitmix64(rs) % (uint64_t)(t + 1));
            std::swap((*pv)[t], (*pv)[j]);
        }
    };
    std::thread worker;
    auto finish = [&worker]() {
        if (worker.joinable()) worker.join();
    };
    if (epochs > 0) shuffle(&perm[0]);
    const MlpWork w = mlp_work(m);
    hipError_t e = hipSuccess;
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        const int k = ep & 1;
        finish();                                       // epoch ep's order is ready
        e = hipMemcpyAsync(d_perm[k], perm[k].data(), sizeof(int) * n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(copied[k], st);
        if (e == hipSuccess && ep + 1 < epochs) {
            // the other host buffer was last copied at the start of epoch ep - 1
            if (ep >= 1) e = hipEventSynchronize(copied[k ^ 1]);
            if (e == hipSuccess) {
                try {
                    worker = std::thread(shuffle, &perm[k ^ 1]);
                } catch (...) {
                    shuffle(&perm[k ^ 1]);              // no thread: shuffle here
                }
            }
        }
        for (int64_t b = 0; b < nb && e == hipSuccess; ++b) {
            const int *idx = d_perm[k] + b * batch;
            e = mlp_forward_batch(w, m->P, feats, idx, batch, target, st);
            if (e == hipSuccess) e = mlp_backward_batch(w, m->P, batch, m->G, st);
            if (e == hipSuccess) e = mlp_loss(w, batch, d_losses + (size_t)ep * nb + b, st);
            // cosine decay of the step size from lr to lr/10 over the run
            const double prog = (double)(ep * nb + b) / std::max<double>(1.0, (double)epochs * nb);
            lr = lr0 * (0.1 + 0.9 * 0.5 * (1.0 + std::cos(kPi * prog)));
            if (e == hipSuccess) e = mlp_adam(m->P, m->G, m->m1, m->m2, (float)lr, ++m->step, st);
            if (e == hipSuccess) e = mlp_refresh(m->P, m->W2b, m->W3b, st);
        }
    }
    finish();
    std::vector<double> losses((size_t)epochs * nb);
    if (e == hipSuccess && epochs > 0)
        e = hipMemcpyAsync(losses.data(), d_losses, sizeof(double) * losses.size(),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && epoch_loss) {
        for (int ep = 0; ep < epochs; ++ep) {
            double sum = 0.0;
            for (int64_t b = 0; b < nb; ++b) sum += losses[(size_t)ep * nb + b];
            epoch_loss[ep] = sum / ((double)nb * batch);
        }
    }
    release();
    if (e != hipSuccess) return hipfail(ctx, e, "training");
    ctx->model_gen++;
    return LMMEW_OK;
}

int lmmew_scatter_labels(lmmew_ctx *ctx, int64_t n_events, uint64_t seed, float *feats, float *raw,
                         hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (n_events <= 0 || !feats || !raw) return fail(ctx, LMMEW_EINVAL, "bad arguments");
    if (ctx->S.nz > 0)
        return fail(ctx, LMMEW_EINVAL, "the scatter surrogate models the planar system only");
    if ((size_t)n_events * ctx->S.Qp * sizeof(float) > kScratchBudget)
        return fail(ctx, LMMEW_EINVAL, "too many label events for one pass");
    const lmmew_system &s = ctx->sys;
    // events: bin and angle uniform, energy uniform over the union of the windows
    double wsum = 0.0;
    for (int k = 0; k < s.n_windows; ++k) wsum += s.win_hi_keV[k] - s.win_lo_keV[k];
    std::vector<int16_t> hb(n_events), ha(n_events);
    std::vector<float> he(n_events);
    uint64_t rs = seed;
    for (int64_t j = 0; j < n_events; ++j) {
        hb[j] = (int16_t)(splitmix64(rs) % (uint64_t)s.n_bins);
        ha[j] = (int16_t)(splitmix64(rs) % (uint64_t)s.n_angles);
        double x = unit_rand(rs) * wsum;
        int k = 0;
        while (k + 1 < s.n_windows && x > s.win_hi_keV[k] - s.win_lo_keV[k]) {
            x -= s.win_hi_keV[k] - s.win_lo_keV[k];
            ++k;
        }
        float E = (float)(s.win_lo_keV[k] + x);
        E = std::min(std::max(E, (float)s.win_lo_keV[k]), (float)s.win_hi_keV[k]);
        he[j] = E;
    }
    int16_t *db = nullptr, *da = nullptr;
    float *de = nullptr;
    HIPCHK(ctx, dalloc(&db, n_events));
    HIPCHK(ctx, dalloc(&da, n_events));
    HIPCHK(ctx, dalloc(&de, n_events));
    int rc = LMMEW_OK;
    hipError_t e = hipMemcpyAsync(db, hb.data(), n_events * 2, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(da, ha.data(), n_events * 2, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(de, he.data(), n_events * 4, hipMemcpyHostToDevice, st);
    lmmew_plan *pl = nullptr;
    if (e != hipSuccess) rc = hipfail(ctx, e, "label events");
    if (rc == LMMEW_OK) {
        lmmew_events ev{n_events, db, da, de};
        rc = make_plan(ctx, &ev, nullptr, 1, 1, st, &pl);
    }
    if (rc == LMMEW_OK) rc = run_rows(ctx, pl, 0, st, 1);
    if (rc == LMMEW_OK) {
        e = mlp_labels(ctx->S, ctx->d_pix, ctx->d_dirs, pl->d_bin, pl->d_ang, pl->d_E, pl->d_A,
                       (int)n_events, feats, raw, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hipfail(ctx, e, "labels");
    }
    if (pl) lmmew_plan_destroy(pl);
    dfree(db);
    dfree(da);
    dfree(de);
    return rc;
}

int lmmew_mlp_fit_labels(lmmew_ctx *ctx, lmmew_mlp *m, const float *feats, const float *raw,
                         int64_t n, int epochs, int batch, double lr, double floor_frac,
                         uint64_t seed, double *epoch_loss, hipStream_t st)
{
    if (!ctx || !m || m->ctx != ctx) return LMMEW_EINVAL;
    const bool keep = floor_frac == 0.0;
    if (!(floor_frac > 0) && !keep) return fail(ctx, LMMEW_EINVAL, "floor_frac must be >= 0");
    if (keep && !(m->floor_ > 0))
        return fail(ctx, LMMEW_EINVAL, "floor_frac 0 keeps the network's floor, which is unset");
    if (n <= 0 || !feats || !raw) return fail(ctx, LMMEW_EINVAL, "bad arguments");
    float *tgt = nullptr;
    HIPCHK(ctx, dalloc(&tgt, n));
    int rc = LMMEW_OK;
    if (keep) {
        const hipError_t e = mlp_targets(raw, n, (float)m->floor_, (float)m->c0, tgt, st);
        if (e != hipSuccess) rc = hipfail(ctx, e, "targets");
        if (rc == LMMEW_OK)
            rc = lmmew_mlp_train(ctx, m, feats, tgt, n, batch, epochs, lr, seed ^ 0x5eedull,
                                 epoch_loss, st);
        dfree(tgt);
        return rc;
    }
    // floor = floor_frac x mean density, c0 = mean of log(density + floor)
    std::vector<float> h(n);
    hipError_t e = hipMemcpyAsync(h.data(), raw, sizeof(float) * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = hipfail(ctx, e, "labels to host");
    if (rc == LMMEW_OK) {
        double mean = 0.0;
        for (float v : h) mean += v;
        mean /= (double)n;
        const double fl = mean > 0 ? floor_frac * mean : 1e-30;
        double c0 = 0.0;
        for (float v : h) c0 += std::log((double)v + fl);
        c0 /= (double)n;
        m->floor_ = fl;
        m->c0 = c0;
        e = mlp_targets(raw, n, (float)fl, (float)c0, tgt, st);
        if (e != hipSuccess) rc = hipfail(ctx, e, "targets");
    }
    if (rc == LMMEW_OK)
        rc = lmmew_mlp_train(ctx, m, feats, tgt, n, batch, epochs, lr, seed ^ 0x5eedull, epoch_loss, st);
    dfree(tgt);
    return rc;
}

int lmmew_mlp_fit(lmmew_ctx *ctx, lmmew_mlp *m, int64_t n_label_events, int epochs, int batch,
                  double lr, double floor_frac, uint64_t seed, double *epoch_loss, hipStream_t st)
{
    if (!ctx || !m || m->ctx != ctx) return LMMEW_EINVAL;
    if (n_label_events <= 0) return fail(ctx, LMMEW_EINVAL, "n_label_events must be > 0");
    const int64_t n = n_label_events * ctx->S.Qm;
    float *feats = nullptr, *raw = nullptr;
    HIPCHK(ctx, dalloc(&feats, (size_t)n * kMlpIn));
    int rc = LMMEW_OK;
    if (dalloc(&raw, n) != hipSuccess) rc = fail(ctx, LMMEW_ENOMEM, "label buffers");
    if (rc == LMMEW_OK) rc = lmmew_scatter_labels(ctx, n_label_events, seed, feats, raw, st);
    if (rc == LMMEW_OK)
        rc = lmmew_mlp_fit_labels(ctx, m, feats, raw, n, epochs, batch, lr, floor_frac, seed,
                                  epoch_loss, st);
    dfree(feats);
    dfree(raw);
    return rc;
}

int lmmew_roi_uptake_noalloc(lmmew_ctx *ctx, const float *lambda, int n_cases,
                             const uint8_t *masks, int n_rois, double *out, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (n_cases < 0 || n_rois < 0) return fail(ctx, LMMEW_EINVAL, "negative count");
    if ((int64_t)n_cases * n_rois == 0) return LMMEW_OK;
    if (!lambda || !masks || !out) return fail(ctx, LMMEW_EINVAL, "NULL argument");
    if ((int64_t)n_cases * n_rois > LMMEW_ROI_NOALLOC_MAX)
        return fail(ctx, LMMEW_EINVAL,
                    "n_cases * n_rois = " + std::to_string((int64_t)n_cases * n_rois) +
                        " exceeds the static scratch of " +
                        std::to_string(LMMEW_ROI_NOALLOC_MAX) + " sums");
    double *d = nullptr;
    HIPCHK(ctx, roi_scratch_ptr(&d));
    // every entry of the scratch that this call reads back is written by the
    // kernel first (one workgroup per (case, region)), so nothing is cleared
    hipError_t e = launch_roi_sums(lambda, n_cases, ctx->Q, masks, n_rois, d, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d, sizeof(double) * n_cases * n_rois, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hipfail(ctx, e, "roi uptake (no allocation)");
    return LMMEW_OK;
}

int lmmew_roi_uptake(lmmew_ctx *ctx, const float *lambda, int n_cases, const uint8_t *masks,
                     int n_rois, double *out, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (n_cases < 0 || n_rois < 0) return fail(ctx, LMMEW_EINVAL, "negative count");
    if ((int64_t)n_cases * n_rois == 0) return LMMEW_OK;
    if (!lambda || !masks || !out) return fail(ctx, LMMEW_EINVAL, "NULL argument");
    double *d = nullptr;
    HIPCHK(ctx, dalloc(&d, (size_t)n_cases * n_rois));
    hipError_t e = launch_roi_sums(lambda, n_cases, ctx->Q, masks, n_rois, d, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d, sizeof(double) * n_cases * n_rois, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(d);
    if (e != hipSuccess) return hipfail(ctx, e, "roi uptake");
    return LMMEW_OK;
}

int lmmew_line_mask(const lmmew_system *sys, float energy_keV)
{
    if (!sys || sys->n_lines < 1 || sys->n_lines > LMMEW_MAX_LINES || !std::isfinite(energy_keV))
        return LMMEW_EINVAL;
    return line_mask(*sys, energy_keV);
}

int lmmew_roi_metrics(const double *est, const double *truth, int S, int N, int K, double *enrmse,
                      double *bias, double *std_)
{
    if (!est || !truth || S < 1 || N < 2 || K < 1) return LMMEW_EINVAL;
    for (int i = 0; i < S * K; ++i)
        if (!(truth[i] != 0.0) || !std::isfinite(truth[i])) return LMMEW_EINVAL;
    for (int k = 0; k < K; ++k) {
        double e_sum = 0.0, b_sum = 0.0, s_sum = 0.0;
        for (int s = 0; s < S; ++s) {
            const double y = truth[(size_t)s * K + k];
            double se = 0.0, dsum = 0.0, mean = 0.0;
            for (int n = 0; n < N; ++n) {
                const double v = est[((size_t)s * N + n) * K + k];
                se += (v - y) * (v - y);
                dsum += v - y;
                mean += v;
            }
            mean /= N;
            double ss = 0.0;
            for (int n = 0; n < N; ++n) {
                const double d = est[((size_t)s * N + n) * K + k] - mean;
                ss += d * d;
            }
            e_sum += std::sqrt(se / N) / y;
            b_sum += dsum / y;
            s_sum += std::sqrt(ss / (N - 1)) / y;
        }
        if (enrmse) enrmse[k] = e_sum / S;
        if (bias) bias[k] = b_sum / ((double)S * N);
        if (std_) std_[k] = s_sum / S;
    }
    return LMMEW_OK;
}

int lmmew_set_scatter_scale(lmmew_ctx *ctx, double scale)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!(scale > 0) || !std::isfinite(scale))
        return fail(ctx, LMMEW_EINVAL, "scatter scale must be positive and finite");
    bool changed = false;
    for (int w = 0; w < ctx->S.nwin; ++w) {
        changed |= (float)scale != ctx->scatter_scale[w];
        ctx->scatter_scale[w] = (float)scale;
    }
    if (changed) ctx->model_gen++;
    return LMMEW_OK;
}

int lmmew_set_scatter_scale_windows(lmmew_ctx *ctx, const double *scales, int n_windows)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!scales || n_windows != ctx->S.nwin)
        return fail(ctx, LMMEW_EINVAL, "one scale per energy window of the system");
    for (int w = 0; w < n_windows; ++w)
        if (!(scales[w] > 0) || !std::isfinite(scales[w]))
            return fail(ctx, LMMEW_EINVAL, "scatter scale must be positive and finite");
    bool changed = false;
    for (int w = 0; w < n_windows; ++w) {
        changed |= (float)scales[w] != ctx->scatter_scale[w];
        ctx->scatter_scale[w] = (float)scales[w];
    }
    if (changed) ctx->model_gen++;
    return LMMEW_OK;
}

}  // extern "C"

// The exact model's and the network's once-scattered densities summed over
// every support pixel of the given events' rows, per energy window of the
// events (FP64; a row's sum in a fixed order, rows added in plan order).
static int scale_sums(lmmew_ctx *ctx, lmmew_mlp *m, const lmmew_events *ev, double *ex,
                      double *net, hipStream_t st)
{
    if (!m || !ev) return fail(ctx, LMMEW_EINVAL, "NULL argument");
    if (!m->ctx || (m->ctx != ctx && !same_system(ctx, m->ctx)))
        return fail(ctx, LMMEW_EINVAL, "network of a context with another system or support");
    if (ev->n < 1) return fail(ctx, LMMEW_EINVAL, "no events");
    if (ev->position_mm) return fail(ctx, LMMEW_EINVAL, "the surrogate models binned events");
    lmmew_plan *pl = nullptr;
    int rc = make_plan(ctx, ev, nullptr, 1, subsets_for_budget(ctx, ev->n), st, &pl);
    if (rc != LMMEW_OK) return rc;
    const int Qp = ctx->S.Qp;
    double *d_rs = nullptr;
    float *d_C = nullptr;
    hipError_t e = dalloc(&d_rs, 2 * (size_t)std::max(pl->max_rows, 1));
    if (e == hipSuccess && m->grid > 1) e = dalloc(&d_C, (size_t)std::max(pl->max_rows, 1) * m->ldc);
    std::vector<double> h(2 * (size_t)std::max(pl->max_rows, 1));
    for (int w = 0; w < ctx->S.nwin; ++w) ex[w] = net[w] = 0.0;
    for (int s = 0; s < pl->nsub && e == hipSuccess && rc == LMMEW_OK; ++s) {
        const lmmew_plan::Sub &sub = pl->subs[s];
        if (sub.rows == 0) continue;
        rc = run_rows(ctx, pl, s, st, 1);                         // exact scattered paths
        if (rc != LMMEW_OK) break;
        e = launch_row_sums(pl->d_A, sub.rows, Qp, d_rs, st);
        if (e == hipSuccess)
            e = hipMemsetAsync(pl->d_A, 0, (size_t)sub.rows * Qp * sizeof(float), st);
        if (e == hipSuccess) {
            MlpRowArgs a{};                                        // the network alone
            a.dirs = ctx->d_dirs;
            a.ev_bin = pl->d_bin + sub.row0;
            a.ev_ang = pl->d_ang + sub.row0;
            a.ev_E = pl->d_E + sub.row0;
            a.rows = sub.rows;
            a.P = m->P;
            a.c0 = (float)m->c0;
            a.floor_ = (float)m->floor_;
            e = net_rows(ctx, m, a, pl->d_A, d_C, st);
        }
        if (e == hipSuccess) e = launch_row_sums(pl->d_A, sub.rows, Qp, d_rs + sub.rows, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h.data(), d_rs, 2 * (size_t)sub.rows * sizeof(double),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess)
            for (int r = 0; r < sub.rows; ++r) {
                const int w = window_of(ctx->sys, pl->E[sub.row0 + r]);
                ex[w] += h[r];
                net[w] += h[sub.rows + r];
            }
    }
    const hipError_t e2 = hipStreamSynchronize(st);
    if (e == hipSuccess) e = e2;
    dfree(d_rs);
    dfree(d_C);
    lmmew_plan_destroy(pl);
    if (rc != LMMEW_OK) return rc;
    if (e != hipSuccess) return hipfail(ctx, e, "scatter scale fit");
    return LMMEW_OK;
}

extern "C" {

int lmmew_scatter_scale_fit(lmmew_ctx *ctx, lmmew_mlp *m, const lmmew_events *ev, double *scale,
                            hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!scale) return fail(ctx, LMMEW_EINVAL, "NULL argument");
    double ex[LMMEW_MAX_WINDOWS], net[LMMEW_MAX_WINDOWS];
    const int rc = scale_sums(ctx, m, ev, ex, net, st);
    if (rc != LMMEW_OK) return rc;
    double x = 0.0, y = 0.0;
    for (int w = 0; w < ctx->S.nwin; ++w) {
        x += ex[w];
        y += net[w];
    }
    if (!(y > 0) || !(x > 0) || !std::isfinite(x / y))
        return fail(ctx, LMMEW_ENUMERIC, "scattered densities vanish for these events");
    *scale = x / y;
    return LMMEW_OK;
}

int lmmew_scatter_scale_fit_windows(lmmew_ctx *ctx, lmmew_mlp *m, const lmmew_events *ev,
                                    double *scales, int n_windows, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (!scales || n_windows != ctx->S.nwin)
        return fail(ctx, LMMEW_EINVAL, "one scale per energy window of the system");
    double ex[LMMEW_MAX_WINDOWS], net[LMMEW_MAX_WINDOWS];
    const int rc = scale_sums(ctx, m, ev, ex, net, st);
    if (rc != LMMEW_OK) return rc;
    double x = 0.0, y = 0.0;
    for (int w = 0; w < n_windows; ++w) {
        x += ex[w];
        y += net[w];
    }
    if (!(y > 0) || !(x > 0) || !std::isfinite(x / y))
        return fail(ctx, LMMEW_ENUMERIC, "scattered densities vanish for these events");
    for (int w = 0; w < n_windows; ++w)
        scales[w] = (ex[w] > 0 && net[w] > 0 && std::isfinite(ex[w] / net[w])) ? ex[w] / net[w]
                                                                              : x / y;
    return LMMEW_OK;
}

int lmmew_set_scatter_model(lmmew_ctx *ctx, lmmew_mlp *m)
{
    if (!ctx || (m && m->ctx != ctx)) return LMMEW_EINVAL;
    ctx->mlp = m;
    ctx->model_gen++;
    return LMMEW_OK;
}

int lmmew_mlp_set_grid(lmmew_mlp *m, int grid)
{
    if (!m || !m->ctx) return LMMEW_EINVAL;
    lmmew_ctx *ctx = m->ctx;
    if (grid < 1 || grid > 8) return fail(ctx, LMMEW_EINVAL, "grid must be 1 to 8 pixels");
    if (grid == m->grid) return LMMEW_OK;
    // kernels still reading the old tables finish before they are replaced
    HIPCHK(ctx, hipDeviceSynchronize());
    dfree(m->d_cnode); dfree(m->d_cidx); dfree(m->d_cw);
    m->d_cnode = nullptr;
    m->d_cidx = nullptr;
    m->d_cw = nullptr;
    m->ncn = m->ldc = 0;
    m->grid = 1;
    ctx->model_gen++;
    if (grid == 1) return LMMEW_OK;
    // Node (u, v) sits at the centre of pixel (grid u, grid v); support pixel
    // (ix, iy) lies in the cell of nodes (ix / grid, iy / grid) and the next
    // ones, at fractions fx = (ix mod grid) / grid, fy likewise.  Only nodes
    // with a non-zero weight are kept, numbered row by row; a zero-weight
    // corner names the cell's first node.
    const int n = ctx->sys.n, Qm = ctx->S.Qm, Qp = ctx->S.Qp;
    const double pix = ctx->sys.pixel_mm, R = ctx->R;
    std::map<std::pair<int, int>, int> id;                         // (v, u) -> node
    std::vector<std::array<std::pair<int, int>, 4>> corner(Qm);
    std::vector<float4> w(Qp, make_float4(0.f, 0.f, 0.f, 0.f));
    for (int i = 0; i < Qm; ++i) {
        const int q = ctx->pixq[i], ix = q % n, iy = q / n;
        const int u0 = ix / grid, v0 = iy / grid;
        const double fx = (double)(ix - grid * u0) / grid, fy = (double)(iy - grid * v0) / grid;
        const double wk[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
        const std::pair<int, int> ck[4] = {{v0, u0}, {v0, u0 + 1}, {v0 + 1, u0}, {v0 + 1, u0 + 1}};
        for (int k = 0; k < 4; ++k) {
            corner[i][k] = wk[k] > 0 ? ck[k] : ck[0];
            if (wk[k] > 0) id.emplace(ck[k], 0);
        }
        w[i] = make_float4((float)wk[0], (float)wk[1], (float)wk[2], (float)wk[3]);
    }
    const int ncn = (int)id.size();
    const int ldc = (ncn + kWave - 1) / kWave * kWave;
    std::vector<float2> node(ldc);
    int k = 0;
    for (auto &kv : id) {
        kv.second = k;
        node[k++] = make_float2((float)((grid * kv.first.second + 0.5) * pix - R),
                                (float)((grid * kv.first.first + 0.5) * pix - R));
    }
    for (int j = ncn; j < ldc; ++j) node[j] = node[ncn - 1];
    std::vector<int4> idx(Qp, make_int4(0, 0, 0, 0));
    for (int i = 0; i < Qm; ++i)
        idx[i] = make_int4(id[corner[i][0]], id[corner[i][1]], id[corner[i][2]], id[corner[i][3]]);
    hipError_t e = dalloc(&m->d_cnode, ldc);
    if (e == hipSuccess) e = dalloc(&m->d_cidx, Qp);
    if (e == hipSuccess) e = dalloc(&m->d_cw, Qp);
    if (e == hipSuccess) e = hipMemcpy(m->d_cnode, node.data(), ldc * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_cidx, idx.data(), Qp * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_cw, w.data(), Qp * sizeof(float4), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dfree(m->d_cnode); dfree(m->d_cidx); dfree(m->d_cw);
        m->d_cnode = nullptr;
        m->d_cidx = nullptr;
        m->d_cw = nullptr;
        return hipfail(ctx, e, "surrogate node tables");
    }
    m->grid = grid;
    m->ncn = ncn;
    m->ldc = ldc;
    return LMMEW_OK;
}

int lmmew_set_scatter_pixel_grid(lmmew_ctx *ctx, int grid, hipStream_t st)
{
    if (!ctx) return LMMEW_EINVAL;
    if (grid < 1 || grid > 8) return fail(ctx, LMMEW_EINVAL, "grid must be 1 to 8 pixels");
    if (grid > 1 && ctx->S.nz > 0)
        return fail(ctx, LMMEW_EINVAL, "the scatter pixel grid is for the planar model");
    if (grid == ctx->xgrid) return LMMEW_OK;
    // kernels still reading the old node tables finish before they go
    HIPCHK(ctx, hipDeviceSynchronize());
    dfree(ctx->d_xnode); dfree(ctx->d_xidx); dfree(ctx->d_xw); dfree(ctx->d_xgqa); dfree(ctx->d_xgqs);
    ctx->d_xnode = nullptr;
    ctx->d_xidx = nullptr;
    ctx->d_xw = nullptr;
    ctx->d_xgqa = nullptr;
    ctx->d_xgqs = nullptr;
    ctx->xncn = ctx->xldc = 0;
    ctx->xgrid = 1;
    ctx->model_gen++;
    if (grid == 1) return LMMEW_OK;
    // Support pixel (ix, iy) lies in the cell of the pixels (g u0, g v0),
    // (g u0 + g, g v0), (g u0, g v0 + g), (g u0 + g, g v0 + g), u0 = ix / g,
    // v0 = iy / g, with bilinear weights from fx = (ix mod g) / g, fy likewise.
    // Corners outside the support (or the grid) are dropped and the remaining
    // weights renormalised; a pixel with no corner in the support is its own
    // node.  The nodes are the support pixels some stencil names, in support
    // order.
    const int n = ctx->sys.n, Qm = ctx->S.Qm, Qp = ctx->S.Qp;
    const double pix = ctx->sys.pixel_mm, R = ctx->R;
    std::vector<int> sidx((size_t)n * n, -1);
    for (int i = 0; i < Qm; ++i) sidx[ctx->pixq[i]] = i;
    std::vector<std::array<int, 4>> cn(Qm);
    std::vector<std::array<double, 4>> cw(Qm);
    std::vector<char> used(Qm, 0);
    for (int i = 0; i < Qm; ++i) {
        const int q = ctx->pixq[i], ix = q % n, iy = q / n;
        const int u0 = ix / grid, v0 = iy / grid;
        const double fx = (double)(ix - grid * u0) / grid, fy = (double)(iy - grid * v0) / grid;
        const double wk[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
        double sum = 0.0;
        for (int k = 0; k < 4; ++k) {
            const int cx = grid * (u0 + (k & 1)), cy = grid * (v0 + (k >> 1));
            const int c = (cx < n && cy < n && wk[k] > 0) ? sidx[(size_t)cy * n + cx] : -1;
            cn[i][k] = c;
            cw[i][k] = c >= 0 ? wk[k] : 0.0;
            sum += cw[i][k];
        }
        if (sum > 0) {
            for (int k = 0; k < 4; ++k) cw[i][k] /= sum;
        } else {
            cn[i] = {i, -1, -1, -1};
            cw[i] = {1.0, 0.0, 0.0, 0.0};
        }
        for (int k = 0; k < 4; ++k)
            if (cn[i][k] >= 0) used[cn[i][k]] = 1;
    }
    std::vector<int> node_of(Qm, -1), nodes;
    for (int i = 0; i < Qm; ++i)
        if (used[i]) {
            node_of[i] = (int)nodes.size();
            nodes.push_back(i);
        }
    const int ncn = (int)nodes.size();
    const int ldc = (ncn + kWave - 1) / kWave * kWave;
    std::vector<double2> pos_d(ldc);
    std::vector<float2> pos_f(ldc);
    for (int k = 0; k < ldc; ++k) {
        const int q = ctx->pixq[nodes[std::min(k, ncn - 1)]];
        const double x = ((q % n) + 0.5) * pix - R, y = ((q / n) + 0.5) * pix - R;
        pos_d[k] = make_double2(x, y);
        pos_f[k] = make_float2((float)x, (float)y);
    }
    std::vector<int4> idx(Qp, make_int4(0, 0, 0, 0));
    std::vector<float4> w(Qp, make_float4(0.f, 0.f, 0.f, 0.f));
    for (int i = 0; i < Qm; ++i) {
        int k4[4];
        for (int k = 0; k < 4; ++k) k4[k] = cn[i][k] >= 0 ? node_of[cn[i][k]] : 0;
        // a dropped corner names a kept node with weight 0
        const int first = cn[i][0] >= 0 ? k4[0] : (cn[i][1] >= 0 ? k4[1] : (cn[i][2] >= 0 ? k4[2] : k4[3]));
        for (int k = 0; k < 4; ++k)
            if (cn[i][k] < 0) k4[k] = first;
        idx[i] = make_int4(k4[0], k4[1], k4[2], k4[3]);
        w[i] = make_float4((float)cw[i][0], (float)cw[i][1], (float)cw[i][2], (float)cw[i][3]);
    }
    // the node pixels' attenuation integrals, by the same kernels and inputs
    // as the context's own tables
    DevSys Sx = ctx->S;
    Sx.Qm = ncn;
    Sx.Qp = ldc;
    const int na = ctx->S.na, nsc = std::max(ctx->S.nsc, 1);
    double2 *d_pd = nullptr;
    ScatA *d_sa = nullptr;
    hipError_t e = dalloc(&ctx->d_xnode, ldc);
    if (e == hipSuccess) e = dalloc(&ctx->d_xidx, Qp);
    if (e == hipSuccess) e = dalloc(&ctx->d_xw, Qp);
    if (e == hipSuccess) e = dalloc(&ctx->d_xgqa, (size_t)na * ldc);
    if (e == hipSuccess) e = dalloc(&ctx->d_xgqs, (size_t)nsc * ldc);
    if (e == hipSuccess) e = dalloc(&d_pd, ldc);
    if (e == hipSuccess) e = dalloc(&d_sa, (size_t)na * nsc);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_xnode, pos_f.data(), ldc * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_xidx, idx.data(), Qp * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_xw, w.data(), Qp * sizeof(float4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_pd, pos_d.data(), ldc * sizeof(double2), hipMemcpyHostToDevice);
    // the scatter-point entries are updated in place by the table kernels: a copy
    if (e == hipSuccess)
        e = hipMemcpy(d_sa, ctx->d_sa, (size_t)na * nsc * sizeof(ScatA), hipMemcpyDeviceToDevice);
    if (e == hipSuccess)
        e = launch_tables_d(Sx, ctx->d_mu, d_pd, nullptr, ctx->d_dirsd, ctx->d_scd, nullptr,
                            ctx->d_xgqa, ctx->d_xgqs, d_sa, pix, R, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(d_pd);
    dfree(d_sa);
    if (e != hipSuccess) {
        dfree(ctx->d_xnode); dfree(ctx->d_xidx); dfree(ctx->d_xw); dfree(ctx->d_xgqa); dfree(ctx->d_xgqs);
        ctx->d_xnode = nullptr;
        ctx->d_xidx = nullptr;
        ctx->d_xw = nullptr;
        ctx->d_xgqa = nullptr;
        ctx->d_xgqs = nullptr;
        return hipfail(ctx, e, "scatter pixel grid tables");
    }
    ctx->xgrid = grid;
    ctx->xncn = ncn;
    ctx->xldc = ldc;
    return LMMEW_OK;
}

int lmmew_scatter_pixel_grid_nodes(const lmmew_ctx *ctx)
{
    if (!ctx) return LMMEW_EINVAL;
    return ctx->xgrid > 1 ? ctx->xncn : ctx->S.Qm;
}

int lmmew_mlp_grid_nodes(const lmmew_mlp *m)
{
    if (!m) return LMMEW_EINVAL;
    return m->grid > 1 ? m->ncn : (m->ctx ? m->ctx->S.Qm : LMMEW_EINVAL);
}

}  // extern "C"
