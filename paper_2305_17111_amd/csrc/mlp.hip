// Scatter surrogate network on gfx950: 6 -> 128 -> 128 -> 128 -> 1 with the tanh
// form of GELU.  Training: the two 128x128 layers run on BF16 MFMA
// (v_mfma_f32_16x16x16 bf16, FP32 accumulation), the first and last layers on
// FP32 VALU, Adam on the FP32 master copy.  Inference inside OSEM (k_mlp_rows):
// every layer on 16x16x32 MFMA (first layer BF16 with high/low splitting,
// hidden layers FP16), GELUs by linear interpolation in an FP16 table in LDS.
//
// Parameter vector (FP32 master copy, 34049 floats):
//   W1[6][128] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] w4[128] b4[1]
// W[i][o] maps input unit i to output unit o.
//
// MFMA 16x16x16 operand layout (lane l, r = l % 16, g = l / 16, item t = 0..3):
//   A[i][k]: i = r, k = 4g + t;  B[k][j]: k = 4g + t, j = r;  D[i][j]: i = 4g + t, j = r.
// The D layout equals the B layout with k = i, so the output of one layer
// computed as Z^T = W^T H^T is directly the B operand of the next.
// The fused inference kernel uses the 16x16x32 MFMAs (8 items per lane and
// operand, one contraction slot per (g, t) shared by A and B); it orders
// the contraction index so that two consecutive D fragments form one B
// fragment (see k_mlp_rows).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "internal.h"

namespace lmmew {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

constexpr int H = kMlpHidden;

// round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned short f2bf(float f)
{
    return __builtin_bit_cast(unsigned short, (__bf16)f);
}

__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// tanh-form GELU: 0.5 z (1 + tanh(c (z + 0.044715 z^3))) = z * sigmoid(2 c (z + 0.044715 z^3)),
// c = sqrt(2/pi).  The sigmoid is 1 / (1 + 2^s) with s = -2 c log2(e) (z + 0.044715 z^3),
// evaluated with the hardware exp2 and reciprocal (1 ulp each); both limits are
// exact (2^s = inf gives 0, 2^s = 0 gives z).
constexpr float kGeluK1 = -2.f * 0.7978845608028654f * 1.4426950408889634f;
constexpr float kGeluK2 = kGeluK1 * 0.044715f;

__device__ __forceinline__ float gelu_sigmoid(float z)
{
    const float e = __builtin_amdgcn_exp2f(z * fmaf(kGeluK2, z * z, kGeluK1));
    return __builtin_amdgcn_rcpf(1.f + e);
}

__device__ __forceinline__ float gelu(float z) { return z * gelu_sigmoid(z); }

__device__ __forceinline__ float gelu_prime(float z)
{
    const float c2 = 2.f * 0.7978845608028654f;
    const float sg = gelu_sigmoid(z);
    const float du = c2 * fmaf(3.f * 0.044715f, z * z, 1.f);
    return sg + z * sg * (1.f - sg) * du;
}

// ---------------------------------------------------------------------------
// training GEMMs on v_mfma_f32_16x16x32_bf16 (bf16 operands, FP32 results)
//
// Operand fragments: lane (g, r) of a wavefront supplies row r of A and
// column r of B at the contraction indices 32 kc + 8 g + {0..7} of chunk kc,
// 16 contiguous bytes when the contraction index is the fastest one; lane
// (g, r) receives D[4 g + t][r], t = 0..3.
// ---------------------------------------------------------------------------
constexpr int kPitch = H + 8;          // LDS row pitch in bf16 (272 B): the 16-byte
                                       // reads of a wavefront's 16 rows spread over the banks

// C[m][j] = sum_k A[m][k] Bt[j][k] for m < M, j, k < 128 (A, Bt row-major with
// rows of 128; C row stride ldc).  Workgroup: 4 wavefronts x 16 rows; Bt is
// staged in LDS once per workgroup, each wavefront keeps its rows' A
// fragments in registers and runs 8 column tiles x 4 chunks of MFMAs.
constexpr int kNtRows = 64;
__global__ __launch_bounds__(256) void k_gemm_nt(const unsigned short *A,
                                                 const unsigned short *Bt, float *C, long ldc,
                                                 int M)
{
    __shared__ uint4 sB[H * kPitch / 8];                           // 34 KB
    for (int c = threadIdx.x; c < H * (H / 8); c += 256)
        sB[(c >> 4) * (kPitch / 8) + (c & 15)] = reinterpret_cast<const uint4 *>(Bt)[c];
    __syncthreads();
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, r = l & 15, g = l >> 4;
    const long m0 = (long)blockIdx.x * kNtRows + 16 * w;
    if (m0 >= M) return;                                           // M is a multiple of 16
    const uint4 *arow = reinterpret_cast<const uint4 *>(A + (m0 + r) * H);
    v8bf a[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) a[kc] = __builtin_bit_cast(v8bf, arow[4 * kc + g]);
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            const v8bf b = __builtin_bit_cast(v8bf, sB[(16 * jt + r) * (kPitch / 8) + 4 * kc + g]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kc], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) C[(m0 + 4 * g + t) * ldc + 16 * jt + r] = acc[t];
    }
}

// Weight gradient with the batch as the contraction: part[z][i][o] = sum over
// the samples m of slice z of X[m][i] D[m][o] (X, D row-major [M][128]).
// Workgroup z runs its slice in blocks of 128 samples: each block is staged in
// LDS transposed ([unit][sample], zero past M), then wavefront w accumulates
// the 2 x 8 output tiles of rows 32 w .. 32 w + 31 in registers.
constexpr int kWgBlock = 128;
__global__ __launch_bounds__(256) void k_gemm_wgrad(const unsigned short *X,
                                                    const unsigned short *D, int M, int per,
                                                    float *part)
{
    __shared__ unsigned short sX[H * kPitch], sD[H * kPitch];     // 2 x 34 KB
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, r = l & 15, g = l >> 4;
    v4f acc[2][8];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int ot = 0; ot < 8; ++ot) acc[u][ot] = v4f{0.f, 0.f, 0.f, 0.f};
    const long z0 = (long)blockIdx.x * per;
    for (int b0 = 0; b0 < per; b0 += kWgBlock) {
        for (int c = threadIdx.x; c < kWgBlock * (H / 8); c += 256) {
            const int m = c >> 4, u0 = (c & 15) * 8;
            const long row = z0 + b0 + m;
            uint4 vx = make_uint4(0u, 0u, 0u, 0u), vd = vx;
            if (row < M) {
                vx = reinterpret_cast<const uint4 *>(X + row * H)[c & 15];
                vd = reinterpret_cast<const uint4 *>(D + row * H)[c & 15];
            }
            const unsigned px[4] = {vx.x, vx.y, vx.z, vx.w}, pd[4] = {vd.x, vd.y, vd.z, vd.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                sX[(u0 + 2 * q) * kPitch + m] = (unsigned short)(px[q] & 0xFFFFu);
                sX[(u0 + 2 * q + 1) * kPitch + m] = (unsigned short)(px[q] >> 16);
                sD[(u0 + 2 * q) * kPitch + m] = (unsigned short)(pd[q] & 0xFFFFu);
                sD[(u0 + 2 * q + 1) * kPitch + m] = (unsigned short)(pd[q] >> 16);
            }
        }
        __syncthreads();
        const uint4 *qx = reinterpret_cast<const uint4 *>(sX);
        const uint4 *qd = reinterpret_cast<const uint4 *>(sD);
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            v8bf a[2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                a[u] = __builtin_bit_cast(v8bf, qx[(16 * (2 * w + u) + r) * (kPitch / 8) + 4 * kc + g]);
#pragma unroll
            for (int ot = 0; ot < 8; ++ot) {
                const v8bf b = __builtin_bit_cast(v8bf, qd[(16 * ot + r) * (kPitch / 8) + 4 * kc + g]);
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    acc[u][ot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b, acc[u][ot], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.x * H * H;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int ot = 0; ot < 8; ++ot)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                out[(16 * (2 * w + u) + 4 * g + t) * H + 16 * ot + r] = acc[u][ot][t];
}

// ---------------------------------------------------------------------------
// training kernels (batch of M samples, rows of [M][128] activations)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_l1(const float *feats, const int *idx, int M,
                                                const float *P, float *X, float *Z1,
                                                unsigned short *H1b)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)M * H) return;
    const int m = (int)(t / H), u = (int)(t % H);
    const long src = idx ? idx[m] : m;
    float x[kMlpIn];
#pragma unroll
    for (int d = 0; d < kMlpIn; ++d) x[d] = feats[src * kMlpIn + d];
    if (u < kMlpIn) X[(long)m * kMlpIn + u] = x[u];
    float z = P[kOffB1 + u];
#pragma unroll
    for (int d = 0; d < kMlpIn; ++d) z = fmaf(x[d], P[kOffW1 + d * H + u], z);
    Z1[t] = z;
    H1b[t] = f2bf(gelu(z));
}

// Z = C + b (in place), H = GELU(Z) as bf16 and/or fp32
__global__ __launch_bounds__(256) void k_bias_gelu(float *C, const float *b, long n,
                                                   unsigned short *Hb, float *Hf)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const float z = C[t] + b[t % H];
    C[t] = z;
    const float h = gelu(z);
    if (Hb) Hb[t] = f2bf(h);
    if (Hf) Hf[t] = h;
}

// y = b4 + sum_u w4[u] h3[u]; residual r = y - target; dy = 2 r / M
__global__ __launch_bounds__(256) void k_mlp_out(const float *H3, const float *P, const float *tgt,
                                                 const int *idx, int M, float *y, float *dy,
                                                 float *sq)
{
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    float acc = P[kOffB4];
    for (int u = 0; u < H; ++u) acc = fmaf(P[kOffW4 + u], H3[(long)m * H + u], acc);
    y[m] = acc;
    if (tgt) {
        const float r = acc - tgt[idx ? idx[m] : m];
        dy[m] = 2.f * r / (float)M;
        sq[m] = r * r;
    }
}

// dZ3 = dy w4 * GELU'(Z3)
__global__ __launch_bounds__(256) void k_dz_out(const float *dy, const float *P, const float *Z,
                                                int M, float *dZ, unsigned short *dZb)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)M * H) return;
    const int m = (int)(t / H), u = (int)(t % H);
    const float v = dy[m] * P[kOffW4 + u] * gelu_prime(Z[t]);
    dZ[t] = v;
    dZb[t] = f2bf(v);
}

// dZ = dH * GELU'(Z) (dH read from the GEMM output), fp32 and optionally bf16
__global__ __launch_bounds__(256) void k_gelu_back(const float *dH, const float *Z, long n,
                                                   float *dZ, unsigned short *dZb)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const float v = dH[t] * gelu_prime(Z[t]);
    dZ[t] = v;
    if (dZb) dZb[t] = f2bf(v);
}

// Column sums over a chunk of kRedRows rows, for the 8 x 128 outputs of one
// layer's gradients: slot 0 = sum_m a[m][u] (bias), slot 1 = sum_m a[m][u] s[m]
// (s may be NULL), slots 2..7 = sum_m X[m][d] a[m][u] (d = 0..5, X may be NULL).
// part[chunk][8][128]; reduced afterwards in chunk order (deterministic).

__global__ __launch_bounds__(128) void k_colsum_part(const float *a, const float *s,
                                                     const float *X, int M, float *part)
{
    const int u = threadIdx.x;
    const int m0 = blockIdx.x * kRedRows, n = min(kRedRows, M - m0);
    // the chunk's column is read first (all loads in flight together), then
    // summed row by row in order
    float v[kRedRows];
#pragma unroll
    for (int i = 0; i < kRedRows; ++i) v[i] = i < n ? a[(long)(m0 + i) * H + u] : 0.f;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < kRedRows; ++i) {
        if (i >= n) break;
        acc[0] += v[i];
        if (s) acc[1] = fmaf(v[i], s[m0 + i], acc[1]);
        if (X) {
#pragma unroll
            for (int d = 0; d < kMlpIn; ++d)
                acc[2 + d] = fmaf(X[(long)(m0 + i) * kMlpIn + d], v[i], acc[2 + d]);
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) part[((long)blockIdx.x * 8 + k) * H + u] = acc[k];
}

// out_slot[u] = sum over chunks of part[chunk][slot][u] for the requested slots:
// one wavefront per (slot, u); lane l sums chunks l, l + 64, ... and the lanes
// are combined by a fixed butterfly (deterministic)
__global__ __launch_bounds__(256) void k_colsum_final(const float *part, int nchunks, float *bias,
                                                      float *scaled, float *xw)
{
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= 8 * H) return;
    const int k = t / H, u = t % H;
    float acc = 0.f;
    for (int c = lane; c < nchunks; c += 64) acc += part[((long)c * 8 + k) * H + u];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane != 0) return;
    if (k == 0 && bias) bias[u] = acc;
    if (k == 1 && scaled) scaled[u] = acc;
    if (k >= 2 && xw) xw[(k - 2) * H + u] = acc;      // W1 layout [d][u]
}

// sum over split-K slices of a [128][128] gradient, in slice order
__global__ __launch_bounds__(256) void k_split_sum(const float *part, int nz, float *out)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= H * H) return;
    float acc = 0.f;
    int z = 0;
    for (; z + 8 <= nz; z += 8) {                       // eight loads in flight, then in order
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = part[(long)(z + q) * H * H + t];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += v[q];
    }
    for (; z < nz; ++z) acc += part[(long)z * H * H + t];
    out[t] = acc;
}

__global__ __launch_bounds__(256) void k_sum(const float *v, int n, double *out)
{
    __shared__ double red[256];
    double acc = 0.0;
    int i = threadIdx.x;
    for (; i + 7 * 256 < n; i += 8 * 256) {              // eight loads in flight, then in order
        float x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = v[i + q * 256];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += x[q];
    }
    for (; i < n; i += 256) acc += v[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_store_sum(const double *v, float *out) { out[0] = (float)v[0]; }

__global__ __launch_bounds__(256) void k_adam(float *P, const float *G, float *m1, float *m2,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= kMlpParams) return;
    const float g = G[t];
    const float a = b1 * m1[t] + (1.f - b1) * g;
    const float v = b2 * m2[t] + (1.f - b2) * g * g;
    m1[t] = a;
    m2[t] = v;
    P[t] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// bf16 copies of W2, W3, row-major [in][out], for the training GEMMs
// bf16 copies of W2 and W3 for training: [in][out], then the transpose [out][in]
__global__ __launch_bounds__(256) void k_refresh_bf16(const float *P, unsigned short *W2b,
                                                      unsigned short *W3b)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= H * H) return;
    const int i = t / H, o = t % H;
    const unsigned short w2 = f2bf(P[kOffW2 + t]), w3 = f2bf(P[kOffW3 + t]);
    W2b[t] = w2;
    W3b[t] = w3;
    W2b[H * H + o * H + i] = w2;
    W3b[H * H + o * H + i] = w3;
}

// ---------------------------------------------------------------------------
// features of (event, pixel) pairs and training labels
// ---------------------------------------------------------------------------
// Features of an (event, pixel) pair in the detector frame of the event's
// angle: bin centre minus the pixel's lateral projection, the pixel's depth
// below the detector plane, its lateral projection (all / R), cos and sin of
// the angle, and (E - kMlpEc) / kMlpEs.  The same information as (pixel x, y,
// bin, angle, energy), arranged so that the collimator geometry is explicit.
__device__ __forceinline__ void pair_features(const DevSys &S, float2 xy, int bin, float2 dir,
                                              float E, float *f)
{
    const float iR = 1.f / S.R;
    const float uq = -xy.x * dir.y + xy.y * dir.x;
    const float dq = S.R - (xy.x * dir.x + xy.y * dir.y);
    const float ub = -S.R + ((float)bin + 0.5f) * S.db;
    f[0] = (ub - uq) * iR;
    f[1] = dq * iR;
    f[2] = uq * iR;
    f[3] = dir.x;
    f[4] = dir.y;
    f[5] = (E - kMlpEc) * (1.f / kMlpEs);
}

// sample s = e * Qm + i: features and the raw once-scattered density a_jq
__global__ __launch_bounds__(256) void k_labels(const DevSys S, const float2 *pix_xy,
                                                const float2 *dirs, const int *ev_bin,
                                                const int *ev_ang, const float *ev_E,
                                                const float *A, int rows, float *feats, float *raw)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)rows * S.Qm) return;
    const int e = (int)(t / S.Qm), i = (int)(t % S.Qm);
    float f[kMlpIn];
    pair_features(S, pix_xy[i], ev_bin[e], dirs[ev_ang[e]], ev_E[e], f);
#pragma unroll
    for (int d = 0; d < kMlpIn; ++d) feats[t * kMlpIn + d] = f[d];
    raw[t] = A[(long)e * S.Qp + i];
}

// target = log(raw + floor) - c0
__global__ __launch_bounds__(256) void k_targets(const float *raw, long n, float floor_, float c0,
                                                 float *tgt)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) tgt[t] = logf(raw[t] + floor_) - c0;
}

// ---------------------------------------------------------------------------
// fused inference: for every (row e, support pixel i) of a subset, add the
// surrogate's once-scattered density max(exp(y + c0) - floor, 0) to A[e][i].
//
// Workgroup: 8 wavefronts, each with its own task of 32 positions x kRowsPerWG
// rows (consecutive tasks of a flat list); two workgroups per CU
// (the LDS holds two copies of the network) and at most 128 VGPRs, so that four
// wavefronts share every SIMD and one's vector work fills the gaps of another's
// matrix work (9 % faster than two per SIMD with 145 VGPRs and no spill; the
// limit costs 16 bytes of scratch).  A wavefront holds two
// groups of 16 pixels (the j dimension of the MFMAs); both groups share every
// weight fragment read from LDS.  Every layer is Z^T = W^T H^T + b on
// v_mfma_f32_16x16x32_bf16 with the weights as A fragments and the bias as
// the initial accumulator.
//
// Hidden layers: the contraction index of chunk c (32 input units) is ordered
// so that lane group g holds units 32c + 4g + {0..3} (items 0..3) and
// 32c + 16 + 4g + {0..3} (items 4..7): those are exactly the units of the D
// fragments of output blocks 2c and 2c + 1, so a layer's activations are the
// next layer's B fragments without a shuffle.
//
// First layer (6 inputs, one 32-slot chunk): inputs and weights are split into
// bf16 high and low parts, x = xh + xl, W = Wh + Wl, and the chunk carries
// xh.Wh (group 0), xl.Wh (group 1) and xh.Wl (group 2); the dropped xl.Wl is
// below 2^-16 of each product, so the first layer keeps about FP32 accuracy.
// The hidden layers run on v_mfma_f32_16x16x32_f16.  The output unit is one
// FP16 MFMA per completed 32-unit chunk of the last hidden layer, with w4 in
// row 0 of the A fragment: row 0 of the result is the unit's sum, already in
// the lanes that write the pixels.
// ---------------------------------------------------------------------------
constexpr int kRowsPerWG = 32;
constexpr int kRowGroups = 2;                  // 16-pixel groups per wavefront
constexpr int kWaves = 8;                      // wavefronts per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kFrag = 8 * 4 * 4 * 16;          // A fragments per hidden layer: (ib, c, g, r)
constexpr int kFrag1 = 8 * 4 * 16;             // first layer: (ib, g, r)

__device__ __forceinline__ int frag_index(int ib, int c, int g, int r)
{
    return ((ib * 4 + c) * 4 + g) * 16 + r;
}

// A fragment (ib, c, g, r) of W^T in FP16 (round to nearest) from the FP32
// master W[in][out] at P + off: output unit 16 ib + r, input units
// 32c + 4g + {0..3} (items 0..3) and 32c + 16 + 4g + {0..3} (items 4..7)
__device__ __forceinline__ v8h load_frag_h(const float *P, int off, int f)
{
    const int r = f & 15, g = (f >> 4) & 3, c = (f >> 6) & 3, ib = f >> 8;
    const float *W = P + off + 16 * ib + r;
    v8h v;
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (_Float16)W[(32 * c + 16 * (t >> 2) + 4 * g + (t & 3)) * H];
    return v;
}

// GELU of two values by linear interpolation in an FP16 table.  Entry k of
// kGeluTab is indexed by the top 10 bits of an FP16 encoding (sign, exponent,
// top 4 mantissa bits): z_k, the value whose encoding is k << 6, starts the
// entry's interval, and the entry holds the chord from (z_k, GELU(z_k)) to the
// next entry's point as intercept and slope, an FP16 pair: a value z in the
// interval gets intercept + slope z, one FMA.  Over every finite FP16 input
// the result is within 2.1e-3 of the exact GELU (two FP16 ulps near z = 2.8,
// mostly the FP16 rounding of the stored intercept; rounding the exact value
// once costs up to 9.7e-4); beyond |z| = 16 the chords are exactly z and 0.
// It replaces the two exp2 and two reciprocals per pair on the quarter-rate
// transcendental unit by two LDS reads and a few full-rate instructions.
constexpr int kGeluTab = 1024;

// fills the table (one entry per call) from the FP32 gelu()
__device__ __forceinline__ unsigned gelu_table_entry(int k)
{
    const float z0 = (float)__builtin_bit_cast(_Float16, (unsigned short)(k << 6));
    const float z1 = (float)__builtin_bit_cast(_Float16, (unsigned short)((k + 1) << 6));
    if (!__builtin_isfinite(z0)) return 0u;                  // Inf / NaN encodings: unused
    const float g0 = gelu(z0);
    float sl = (gelu(z1) - g0) / (z1 - z0);
    if (!__builtin_isfinite(z1) || !__builtin_isfinite(sl)) sl = z0 > 0.f ? 1.f : 0.f;
    const h2 v = {(_Float16)fmaf(-sl, z0, g0), (_Float16)sl};
    return __builtin_bit_cast(unsigned, v);
}

// GELU of two FP32 accumulators in two steps, so that the table reads can be
// issued well before their results are used.  gelu_fetch: the FP16 pair
// (round toward zero) and its two table entries; tab must sit at LDS address 0
// so that an entry's byte offset is just its index times 4.
struct GeluFetch {
    h2 z;
    unsigned e0, e1;
};

__device__ __forceinline__ GeluFetch gelu_fetch(float a, float b, const unsigned *tab)
{
    GeluFetch f;
    f.z = __builtin_bit_cast(h2, __builtin_amdgcn_cvt_pkrtz(a, b));
    // With the low 6 bits of each half cleared, an entry's byte offset is bits
    // 4..15 of the low half (one bit-field extract) and bits 20..31 of the high
    // half (one shift).  The opaque copy keeps the compiler from re-deriving
    // the offsets from the pair with a shift and a mask each.
    unsigned zk = __builtin_bit_cast(unsigned, f.z) & 0xFFC0FFC0u;
    asm volatile("" : "+v"(zk));
    const unsigned o0 = __builtin_amdgcn_ubfe(zk, 4, 12), o1 = zk >> 20;
    const char *t = reinterpret_cast<const char *>(tab);
    f.e0 = *reinterpret_cast<const unsigned *>(t + o0);
    f.e1 = *reinterpret_cast<const unsigned *>(t + o1);
    return f;
}

// gelu_finish: intercept + slope z per half, as the 32-bit encoding of the
// FP16 pair of GELUs
__device__ __forceinline__ unsigned gelu_finish(const GeluFetch &f)
{
    // (intercept, slope) of the two entries -> (intercept0, intercept1), (slope0, slope1)
    const h2 I = __builtin_bit_cast(h2, __builtin_amdgcn_perm(f.e1, f.e0, 0x05040100u));
    const h2 D = __builtin_bit_cast(h2, __builtin_amdgcn_perm(f.e1, f.e0, 0x07060302u));
    return __builtin_bit_cast(unsigned, __builtin_elementwise_fma(D, f.z, I));
}

__device__ __forceinline__ unsigned gelu_pair(float a, float b, const unsigned *tab)
{
    return gelu_finish(gelu_fetch(a, b, tab));
}

// four 32-bit words (FP16 pairs) as an MFMA operand fragment
__device__ __forceinline__ v8h frag_of(const unsigned *w)
{
    return __builtin_bit_cast(v8h, make_uint4(w[0], w[1], w[2], w[3]));
}

// two FP32 values rounded to BF16 (nearest even) as one 32-bit pair, a in
// the low half
__device__ __forceinline__ unsigned bf16_pair(float a, float b)
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __bf16 b2v __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f2v){a, b}, b2v));
}

__device__ __forceinline__ unsigned pack2(unsigned short a, unsigned short b)
{
    return (unsigned)a | ((unsigned)b << 16);
}

// first-layer A fragment (ib, g, r): unit u = 16 ib + r; items d < 6 are the
// weights of input d (high part for groups 0 and 1, low part for group 2);
// group 0 items 6 and 7 are the bias high and low parts (their B items are 1)
__device__ __forceinline__ uint4 load_frag1(const float *P, int f)
{
    const int r = f & 15, g = (f >> 4) & 3, ib = f >> 6, u = 16 * ib + r;
    unsigned short v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (g < 3) {
        for (int d = 0; d < kMlpIn; ++d) {
            const float w = P[kOffW1 + d * H + u];
            const unsigned short wh = f2bf(w);
            v[d] = g < 2 ? wh : f2bf(w - bf2f(wh));
        }
    }
    if (g == 0) {
        const float b = P[kOffB1 + u];
        const unsigned short bh = f2bf(b);
        v[6] = bh;
        v[7] = f2bf(b - bf2f(bh));
    }
    return make_uint4(pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7]));
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_mlp_rows(
    const DevSys S, const MlpRowArgs a)
{
    // one LDS buffer (77 KB, two workgroups per CU): the GELU table at address
    // 0, then the weight fragments and biases (the output weights sit in
    // registers, see w4f)
    __shared__ uint4 lds[kGeluTab / 4 + kFrag1 + 2 * kFrag + 2 * H / 4];
    unsigned *const sTab = reinterpret_cast<unsigned *>(lds);            // 4 KB
    uint4 *const sW1 = lds + kGeluTab / 4;                               // 8 KB, bf16
    v8h *const sW2 = reinterpret_cast<v8h *>(sW1 + kFrag1);               // 32 KB, fp16
    v8h *const sW3 = sW2 + kFrag;                                        // 32 KB, fp16
    float4 *const sB = reinterpret_cast<float4 *>(sW3 + kFrag);          // b2, b3

    for (int f = threadIdx.x; f < kFrag; f += kThreads) {
        sW2[f] = load_frag_h(a.P, kOffW2, f);
        sW3[f] = load_frag_h(a.P, kOffW3, f);
    }
    for (int f = threadIdx.x; f < kFrag1; f += kThreads) sW1[f] = load_frag1(a.P, f);
    for (int t = threadIdx.x; t < H / 4; t += kThreads) {
        sB[t] = reinterpret_cast<const float4 *>(a.P + kOffB2)[t];
        sB[H / 4 + t] = reinterpret_cast<const float4 *>(a.P + kOffB3)[t];
    }
    const float b4 = a.P[kOffB4];
    for (int k = threadIdx.x; k < kGeluTab; k += kThreads) sTab[k] = gelu_table_entry(k);
    __syncthreads();

    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, r = l & 15, g = l >> 4;
    // first-layer input split per lane group (see the B fragments below)
    const float keep = g == 3 ? 0.f : 1.f;
    const float lo_sign = g == 1 ? -1.f : 0.f;
    const unsigned ones = g == 0 ? bf16_pair(1.f, 1.f) : 0u;
    // A wavefront's task: one block of 32 positions of one block of rows, from
    // a flat list (row block major) shared by the workgroups, so that only the
    // last position block of each row block carries padding.  The tasks past
    // the end of the list (in the last workgroup) return; no barrier follows.
    const int npb = (a.npix + 16 * kRowGroups - 1) / (16 * kRowGroups);
    const int task = (int)blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(wv);
    const int rb = task / npb, pb = task - rb * npb;
    if (rb * kRowsPerWG >= a.rows) return;
    int ip[kRowGroups];
    float2 xy[kRowGroups];
#pragma unroll
    for (int p = 0; p < kRowGroups; ++p) {
        ip[p] = pb * 16 * kRowGroups + 16 * p + r;
        xy[p] = a.pix_xy[min(ip[p], a.npix - 1)];
    }
    // Output unit as MFMA: A fragment of chunk c holds w4 in row 0 (the lanes
    // with r = 0) and zeros elsewhere, in the item order of the B fragments
    // (input units 32c + 4g + {0..3}, 32c + 16 + 4g + {0..3}); row 0 of the
    // result, in the lanes with g = 0, is then the sum over the 128 units.
    v8h w4f[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int t = 0; t < 8; ++t)
            w4f[c][t] = r == 0 ? (_Float16)a.P[kOffW4 + 32 * c + 16 * (t >> 2) + 4 * g + (t & 3)]
                               : (_Float16)0.f;
    const int e0 = rb * kRowsPerWG, e1 = min(e0 + kRowsPerWG, a.rows);
    for (int e = e0; e < e1; ++e) {
        // An opaque zero offset keeps the weight reads inside the row loop:
        // hoisted, they would take 512 registers and leave one wavefront per SIMD.
        int off = 0;
        asm volatile("" : "+v"(off));
        const float4 *bb = sB + off;
        const v8bf *w1 = reinterpret_cast<const v8bf *>(sW1) + off;
        const v8h *w2 = sW2 + off;
        const v8h *w3 = sW3 + off;

        const int bin = a.ev_bin[e];
        const float2 dir = a.dirs[a.ev_ang[e]];
        const float E = a.ev_E[e];
        const float sc = a.case_scale ? a.case_scale[a.ev_scale[e]] : 1.f;

        // first-layer B fragments: group 0 (xh, 1, 1), group 1 (xl, 0, 0),
        // group 2 (xh, 0, 0), group 3 zero.  With x scaled by keep (0 in
        // group 3), a lane rounds x + lo_sign * xh to BF16: xh in groups 0 and
        // 2, xl = x - xh (exact in FP32) in group 1; two inputs per conversion.
        v8bf x1[kRowGroups];
#pragma unroll
        for (int p = 0; p < kRowGroups; ++p) {
            float f[kMlpIn];
            pair_features(S, xy[p], bin, dir, E, f);
            unsigned wd[4];
#pragma unroll
            for (int d = 0; d < kMlpIn; d += 2) {
                const float x0 = f[d] * keep, x1v = f[d + 1] * keep;
                const unsigned hp = bf16_pair(x0, x1v);
                const float h0 = __builtin_bit_cast(float, hp << 16);
                const float h1 = __builtin_bit_cast(float, hp & 0xFFFF0000u);
                wd[d >> 1] = bf16_pair(fmaf(h0, lo_sign, x0), fmaf(h1, lo_sign, x1v));
            }
            wd[3] = ones;
            x1[p] = __builtin_bit_cast(v8bf, make_uint4(wd[0], wd[1], wd[2], wd[3]));
        }
        // Every layer is software-pipelined by one output block: the MFMAs of
        // block ib are issued before the GELUs of block ib - 1, whose
        // accumulators they no longer touch, so the matrix unit works on one
        // block while the vector unit activates the previous one.  In the
        // hidden layers the GELU table reads of block ib - 1 are issued before
        // block ib's MFMAs and used after them, and the weight fragments and
        // bias of block ib + 1 are read from LDS while block ib runs.
        //
        // layer 1 (bf16 hi/lo MFMA): output block ib = units 16 ib + 4g + t ->
        // item 4 (ib & 1) + t of chunk ib / 2, GELU from the table
        unsigned h1[kRowGroups][4][4];            // FP16 pairs: items 2t, 2t + 1 of chunk c
        v4f pend[kRowGroups];                     // accumulators awaiting their GELU
#pragma unroll
        for (int ib = 0; ib <= 8; ++ib) {
            v4f acc[kRowGroups];
            if (ib < 8) {
                const v8bf w = w1[(ib * 4 + g) * 16 + r];
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p)
                    acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        w, x1[p], v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            }
            if (ib > 0) {
                const int jb = ib - 1;
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) {
                    h1[p][jb >> 1][2 * (jb & 1) + 0] = gelu_pair(pend[p][0], pend[p][1], sTab);
                    h1[p][jb >> 1][2 * (jb & 1) + 1] = gelu_pair(pend[p][2], pend[p][3], sTab);
                }
            }
            if (ib < 8) {
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) pend[p] = acc[p];
            }
        }
        // layer 2 (fp16 MFMA, fp32 accumulation from the bias)
        unsigned h2v[kRowGroups][4][4];
        v8h wc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) wc[c] = w2[frag_index(0, c, g, r)];
        float4 bc = bb[(4 * g) >> 2];
#pragma unroll
        for (int ib = 0; ib <= 8; ++ib) {
            v4f acc[kRowGroups];
            GeluFetch gf[kRowGroups][2];
            v8h wn[4];
            float4 bn;
            if (ib + 1 < 8) {
#pragma unroll
                for (int c = 0; c < 4; ++c) wn[c] = w2[frag_index(ib + 1, c, g, r)];
                bn = bb[(16 * (ib + 1) + 4 * g) >> 2];
            }
            if (ib > 0) {
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) {
                    gf[p][0] = gelu_fetch(pend[p][0], pend[p][1], sTab);
                    gf[p][1] = gelu_fetch(pend[p][2], pend[p][3], sTab);
                }
            }
            if (ib < 8) {
                const float4 b = bc;
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) acc[p] = v4f{b.x, b.y, b.z, b.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const v8h w = wc[c];
#pragma unroll
                    for (int p = 0; p < kRowGroups; ++p)
                        acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_f16(w, frag_of(h1[p][c]),
                                                                       acc[p], 0, 0, 0);
                }
            }
            if (ib > 0) {
                const int jb = ib - 1;
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) {
                    h2v[p][jb >> 1][2 * (jb & 1) + 0] = gelu_finish(gf[p][0]);
                    h2v[p][jb >> 1][2 * (jb & 1) + 1] = gelu_finish(gf[p][1]);
                }
            }
            if (ib < 8) {
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) pend[p] = acc[p];
            }
            if (ib + 1 < 8) {
#pragma unroll
                for (int c = 0; c < 4; ++c) wc[c] = wn[c];
                bc = bn;
            }
        }
        // layer 3 and the output unit (an MFMA per completed 32-unit chunk)
        v4f yacc[kRowGroups];
        unsigned h3[kRowGroups][4];               // the chunk being completed
#pragma unroll
        for (int p = 0; p < kRowGroups; ++p) yacc[p] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) wc[c] = w3[frag_index(0, c, g, r)];
        bc = bb[H / 4 + ((4 * g) >> 2)];
#pragma unroll
        for (int ib = 0; ib <= 8; ++ib) {
            v4f acc[kRowGroups];
            GeluFetch gf[kRowGroups][2];
            v8h wn[4];
            float4 bn;
            if (ib + 1 < 8) {
#pragma unroll
                for (int c = 0; c < 4; ++c) wn[c] = w3[frag_index(ib + 1, c, g, r)];
                bn = bb[H / 4 + ((16 * (ib + 1) + 4 * g) >> 2)];
            }
            if (ib > 0) {
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) {
                    gf[p][0] = gelu_fetch(pend[p][0], pend[p][1], sTab);
                    gf[p][1] = gelu_fetch(pend[p][2], pend[p][3], sTab);
                }
            }
            if (ib < 8) {
                const float4 b = bc;
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) acc[p] = v4f{b.x, b.y, b.z, b.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const v8h w = wc[c];
#pragma unroll
                    for (int p = 0; p < kRowGroups; ++p)
                        acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_f16(w, frag_of(h2v[p][c]),
                                                                       acc[p], 0, 0, 0);
                }
            }
            if (ib > 0) {
                const int jb = ib - 1;
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) {
                    h3[p][2 * (jb & 1) + 0] = gelu_finish(gf[p][0]);
                    h3[p][2 * (jb & 1) + 1] = gelu_finish(gf[p][1]);
                }
                if (jb & 1) {
#pragma unroll
                    for (int p = 0; p < kRowGroups; ++p)
                        yacc[p] = __builtin_amdgcn_mfma_f32_16x16x32_f16(w4f[jb >> 1],
                                                                        frag_of(h3[p]), yacc[p],
                                                                        0, 0, 0);
                }
            }
            if (ib < 8) {
#pragma unroll
                for (int p = 0; p < kRowGroups; ++p) pend[p] = acc[p];
            }
            if (ib + 1 < 8) {
#pragma unroll
                for (int c = 0; c < 4; ++c) wc[c] = wn[c];
                bc = bn;
            }
        }
#pragma unroll
        for (int p = 0; p < kRowGroups; ++p) {
            const float y = yacc[p][0];
            if (g == 0 && ip[p] < a.npix) {
                const float v = fmaxf(__expf(y + b4 + a.c0) - a.floor_, 0.f);
                float *const out = a.A + (long)e * a.ld + ip[p];
                if (a.assign)
                    *out = v * sc;
                else
                    *out += v * sc;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

// C[m][j] = sum_k A[m][k] Bt[j][k], M rows (a multiple of 16)
static hipError_t mlp_gemm_nt(const unsigned short *A, const unsigned short *Bt, float *C, int M,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_gemm_nt, dim3(nblk(M, kNtRows)), dim3(256), 0, st, A, Bt, C, (long)H, M);
    return hipGetLastError();
}

// weight gradient [128][128] with the batch dimension as the contraction: at
// most 64 slices of whole 128-sample blocks, then an ordered sum of the slices
static hipError_t mlp_gemm_wgrad(const unsigned short *X, const unsigned short *D, int M, float *out,
                                 float *scratch, hipStream_t st)
{
    const int blocks = (M + kWgBlock - 1) / kWgBlock;
    const int per = ((blocks + 63) / 64) * kWgBlock;               // samples per slice
    const int nz = (M + per - 1) / per;
    hipLaunchKernelGGL(k_gemm_wgrad, dim3(nz), dim3(256), 0, st, X, D, M, per, scratch);
    hipLaunchKernelGGL(k_split_sum, dim3(H * H / 256), dim3(256), 0, st, scratch, nz, out);
    return hipGetLastError();
}

static hipError_t mlp_colsums(const float *a, const float *s, const float *X, int M, float *part,
                              float *bias, float *scaled, float *xw, hipStream_t st)
{
    const int nc = (M + kRedRows - 1) / kRedRows;
    hipLaunchKernelGGL(k_colsum_part, dim3(nc), dim3(128), 0, st, a, s, X, M, part);
    hipLaunchKernelGGL(k_colsum_final, dim3(8 * H / 4), dim3(256), 0, st, part, nc, bias,
                       scaled, xw);
    return hipGetLastError();
}

hipError_t mlp_forward_batch(const MlpWork &w, const float *P, const float *feats, const int *idx,
                             int M, const float *tgt, hipStream_t st)
{
    const long n = (long)M * H;
    hipLaunchKernelGGL(k_mlp_l1, dim3(nblk(n, 256)), dim3(256), 0, st, feats, idx, M, P, w.X,
                       w.Z1, w.H1b);
    hipError_t e = mlp_gemm_nt(w.H1b, w.W2b + H * H, w.Z2, M, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu, dim3(nblk(n, 256)), dim3(256), 0, st, w.Z2, P + kOffB2, n,
                       w.H2b, (float *)nullptr);
    e = mlp_gemm_nt(w.H2b, w.W3b + H * H, w.Z3, M, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu, dim3(nblk(n, 256)), dim3(256), 0, st, w.Z3, P + kOffB3, n,
                       (unsigned short *)nullptr, w.H3);
    hipLaunchKernelGGL(k_mlp_out, dim3(nblk(M, 256)), dim3(256), 0, st, w.H3, P, tgt, idx, M, w.y,
                       w.dy, w.sq);
    return hipGetLastError();
}

hipError_t mlp_backward_batch(const MlpWork &w, const float *P, int M, float *G, hipStream_t st)
{
    const long n = (long)M * H;
    // output layer: dw4 = sum_m dy h3, db4 = sum_m dy
    hipError_t e = mlp_colsums(w.H3, w.dy, nullptr, M, w.part, nullptr, G + kOffW4, nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, w.dy, M, w.dsum);
    hipLaunchKernelGGL(k_store_sum, dim3(1), dim3(1), 0, st, w.dsum, G + kOffB4);
    hipLaunchKernelGGL(k_dz_out, dim3(nblk(n, 256)), dim3(256), 0, st, w.dy, P, w.Z3, M, w.dZ,
                       w.dZb);
    // layer 3: dW3 = H2^T dZ3, db3, dH2 = dZ3 W3^T
    e = mlp_gemm_wgrad(w.H2b, w.dZb, M, G + kOffW3, w.split, st);
    if (e != hipSuccess) return e;
    e = mlp_colsums(w.dZ, nullptr, nullptr, M, w.part, G + kOffB3, nullptr, nullptr, st);
    if (e != hipSuccess) return e;
    e = mlp_gemm_nt(w.dZb, w.W3b, w.dH, M, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gelu_back, dim3(nblk(n, 256)), dim3(256), 0, st, w.dH, w.Z2, n, w.dZ,
                       w.dZb);
    // layer 2
    e = mlp_gemm_wgrad(w.H1b, w.dZb, M, G + kOffW2, w.split, st);
    if (e != hipSuccess) return e;
    e = mlp_colsums(w.dZ, nullptr, nullptr, M, w.part, G + kOffB2, nullptr, nullptr, st);
    if (e != hipSuccess) return e;
    e = mlp_gemm_nt(w.dZb, w.W2b, w.dH, M, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gelu_back, dim3(nblk(n, 256)), dim3(256), 0, st, w.dH, w.Z1, n, w.dZ,
                       (unsigned short *)nullptr);
    // layer 1: dW1 = X^T dZ1, db1
    return mlp_colsums(w.dZ, nullptr, w.X, M, w.part, G + kOffB1, nullptr, G + kOffW1, st);
}

hipError_t mlp_loss(const MlpWork &w, int M, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, w.sq, M, out);
    return hipGetLastError();
}

hipError_t mlp_adam(float *P, const float *G, float *m1, float *m2, float lr, int step,
                    hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(kMlpParams, 256)), dim3(256), 0, st, P, G, m1, m2, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_refresh(const float *P, unsigned short *W2b, unsigned short *W3b,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_refresh_bf16, dim3(nblk(H * H, 256)), dim3(256), 0, st, P, W2b, W3b);
    return hipGetLastError();
}

hipError_t mlp_labels(const DevSys &S, const float2 *pix_xy, const float2 *dirs, const int *ev_bin,
                      const int *ev_ang, const float *ev_E, const float *A, int rows, float *feats,
                      float *raw, hipStream_t st)
{
    const long n = (long)rows * S.Qm;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_labels, dim3(nblk(n, 256)), dim3(256), 0, st, S, pix_xy, dirs, ev_bin,
                       ev_ang, ev_E, A, rows, feats, raw);
    return hipGetLastError();
}

hipError_t mlp_targets(const float *raw, long n, float floor_, float c0, float *tgt, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_targets, dim3(nblk(n, 256)), dim3(256), 0, st, raw, n, floor_, c0, tgt);
    return hipGetLastError();
}

// Scattered densities of the surrogate at the support pixels from its values
// at the coarse nodes: A[e][q] += w.x C[e][i.x] + w.y C[e][i.y] + w.z C[e][i.z]
// + w.w C[e][i.w], with the four bilinear weights and nodes of pixel q.  A
// thread keeps its pixel's stencil for kInterpRows rows; a row's nodes sit
// close together in C, so the gathers of neighbouring pixels share cache lines.
constexpr int kInterpRows = 32;

__global__ __launch_bounds__(256) void k_coarse_interp(const DevSys S, const float *__restrict__ C,
                                                       int ldc, const int4 *__restrict__ idx,
                                                       const float4 *__restrict__ w, int rows,
                                                       float *__restrict__ A)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= S.Qm) return;
    const int4 n = idx[q];
    const float4 f = w[q];
    const int e0 = blockIdx.y * kInterpRows, e1 = min(e0 + kInterpRows, rows);
    for (int e = e0; e < e1; ++e) {
        const float *c = C + (size_t)e * ldc;
        float v = f.x * c[n.x];
        v = fmaf(f.y, c[n.y], v);
        v = fmaf(f.z, c[n.z], v);
        v = fmaf(f.w, c[n.w], v);
        A[(size_t)e * S.Qp + q] += v;
    }
}

hipError_t launch_coarse_interp(const DevSys &S, const float *C, int ldc, const int4 *idx,
                                const float4 *w, int rows, float *A, hipStream_t st)
{
    // grid.y is limited to 65535 workgroups: launch in slices of rows
    constexpr int kSlice = 32768 * kInterpRows;
    for (int r0 = 0; r0 < rows; r0 += kSlice) {
        const int n = rows - r0 < kSlice ? rows - r0 : kSlice;
        hipLaunchKernelGGL(k_coarse_interp, dim3((S.Qm + 255) / 256, (n + kInterpRows - 1) / kInterpRows),
                           dim3(256), 0, st, S, C + (size_t)r0 * ldc, ldc, idx, w, n,
                           A + (size_t)r0 * S.Qp);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Rows of the coarse evaluation grids in one pass: the unscattered part of
// every (row, support pixel), formed as the per-event kernel forms it from the
// unscattered bin-probability table (the same operations in the same order:
// the path weight of each line from the pixel's attenuation integral to the
// detector, times the energy factor of the event's energy, summed over the
// lines, times the bin probability), plus the bilinear interpolation of the
// row's node values.  Each row element is written once, with no read of the
// row.  A workgroup takes kInterpRows rows: it stages their energy factors
// (one per row and line) in LDS, and a thread keeps its pixel's stencil, and
// its path weights while consecutive rows share the angle and the case (the
// plan sorts its events that way).
__global__ __launch_bounds__(256) void k_prim_interp(const DevSys S, const PrimInterpArgs a)
{
    __shared__ float sgq[kInterpRows * LMMEW_MAX_LINES];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int e0 = blockIdx.y * kInterpRows, e1 = min(e0 + kInterpRows, a.rows);
    for (int t = threadIdx.x; t < (e1 - e0) * S.nw; t += 256) {
        const int w = t % S.nw;
        const float d = a.ev_E[e0 + t / S.nw] - S.E[w];
        sgq[t] = S.gnorm[w] * __expf(-d * d / (2.f * S.eres_k * S.E[w]));
    }
    __syncthreads();
    if (i >= S.Qp) return;
    const bool valid = i < S.Qm;
    const int4 n = valid ? a.idx[i] : make_int4(0, 0, 0, 0);
    const float4 f = valid ? a.w[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    float Pp[LMMEW_MAX_LINES];
    int key_a = -1, key_c = -1;
    for (int e = e0; e < e1; ++e) {
        float out = 0.f;
        const int an = a.ev_ang[e], cs = a.maps ? a.ev_case[e] : 0;
        if (valid) {
            if (an != key_a || cs != key_c) {
                const float *gq_a = a.maps ? a.maps[cs].g_qa : a.g_qa;
                const float gqa = gq_a[(size_t)an * S.Qp + i];
#pragma unroll
                for (int w = 0; w < LMMEW_MAX_LINES; ++w)
                    if (w < S.nw) Pp[w] = S.pp[w] * __builtin_amdgcn_exp2f(-S.f[w] * gqa * kLog2e);
                key_a = an;
                key_c = cs;
            }
            const float ps = a.psft[((size_t)an * S.nb + a.ev_bin[e]) * S.Qp + i];
            const float *gq = sgq + (e - e0) * S.nw;
            float g = 0.f;
#pragma unroll
            for (int w = 0; w < LMMEW_MAX_LINES; ++w)
                if (w < S.nw) g = fmaf(Pp[w], gq[w], g);
            const float *c = a.C + (size_t)e * a.ldc;
            float v = f.x * c[n.x];
            v = fmaf(f.y, c[n.y], v);
            v = fmaf(f.z, c[n.z], v);
            v = fmaf(f.w, c[n.w], v);
            out = __fmul_rn(ps, g) + v;
        }
        a.A[(size_t)e * S.Qp + i] = out;
    }
}

hipError_t launch_prim_interp(const DevSys &S, const PrimInterpArgs &a, hipStream_t st)
{
    if (!a.psft || (!a.g_qa && !a.maps) || (a.maps && !a.ev_case)) return hipErrorInvalidValue;
    // grid.y is limited to 65535 workgroups: launch in slices of rows
    constexpr int kSlice = 32768 * kInterpRows;
    for (int r0 = 0; r0 < a.rows; r0 += kSlice) {
        PrimInterpArgs b = a;
        b.rows = a.rows - r0 < kSlice ? a.rows - r0 : kSlice;
        b.ev_bin += r0;
        b.ev_ang += r0;
        b.ev_E += r0;
        if (b.ev_case) b.ev_case += r0;
        b.C += (size_t)r0 * a.ldc;
        b.A += (size_t)r0 * S.Qp;
        hipLaunchKernelGGL(k_prim_interp, dim3(nblk(S.Qp, 256), nblk(b.rows, kInterpRows)), dim3(256),
                           0, st, S, b);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t mlp_rows(const DevSys &S, const MlpRowArgs &a, hipStream_t st)
{
    if (a.npix < 1 || a.ld < a.npix) return hipErrorInvalidValue;
    // slices of at most 2^20 rows keep a launch's task count (position blocks
    // x row blocks) far inside the grid's range
    constexpr int kSlice = 32768 * kRowsPerWG;
    for (int r0 = 0; r0 < a.rows; r0 += kSlice) {
        MlpRowArgs b = a;
        b.rows = std::min(kSlice, a.rows - r0);
        b.ev_bin += r0;
        b.ev_ang += r0;
        b.ev_E += r0;
        b.A += (long)r0 * a.ld;
        const long tasks = (long)nblk(a.npix, 16 * kRowGroups) * nblk(b.rows, kRowsPerWG);
        if (tasks + kWaves > INT_MAX) return hipErrorInvalidValue;   // 32-bit task index
        hipLaunchKernelGGL(k_mlp_rows, dim3(nblk(tasks, kWaves)), dim3(kThreads), 0, st, S, b);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lmmew
