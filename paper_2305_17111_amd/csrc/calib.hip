// Issue-rate calibration of the instruction chains the per-event kernel is
// built from, measured on the device it runs on (lmmew_calibrate).
//
// kind 0, the algorithmic term: one energy-Gaussian factor of a (line, path)
// pair at an event's energy, accumulated with the event's response factor,
//     u = s E - F;   x = exp2(A - u^2);   acc_j += f_j x
// that is v_fma_f32, v_fma_f32, v_exp_f32, v_fma_f32 -- the per-pixel path
// parameters (s, F, A) in vector registers, the event's energy E and
// response factor f uniform (scalar registers, read with scalar loads), as in
// the per-event kernel's pair loop.  kind 1: v_fma_f32 alone; kind 2:
// v_exp_f32 alone.  Every lane runs 16 independent chains so that latency is
// hidden, and 8 waves per SIMD fill the machine.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/lmmew.h"

namespace {

constexpr int kChains = 16;
constexpr int kBlock = 256;
constexpr int kBlocks = 2048;        // 8 waves per SIMD on 256 CUs
constexpr int kEvTab = 64;           // distinct blocks of 16 (energy, factor) pairs

__global__ __launch_bounds__(kBlock) void k_cal_terms(const float *__restrict__ ev, int iters,
                                                      float *__restrict__ out)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    // path parameters of a lane: s = sqrt(log2 e / (2 k E')), F = s E',
    // A a log2 weight, for scattered energies E' spread over 90..250 keV
    const float Ep = 90.f + 160.f * (float)(t & 255) / 255.f;
    const float sw = sqrtf(1.4426950f / (2.f * 0.2525f * Ep));
    const float Fw = sw * Ep;
    const float Aw = -20.f + 0.01f * (float)(t & 31);
    float acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = 0.f;
    for (int it = 0; it < iters; ++it) {
        const float *e = ev + (it & (kEvTab - 1)) * (2 * kChains);   // uniform: scalar loads
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            const float u = fmaf(sw, e[j], -Fw);
            const float x = __builtin_amdgcn_exp2f(fmaf(-u, u, Aw));
            acc[j] = fmaf(e[kChains + j], x, acc[j]);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += acc[j];
    out[t] = s;
}

__global__ __launch_bounds__(kBlock) void k_cal_fma(int iters, float *__restrict__ out)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const float a = 0.999f - 1e-6f * (float)(t & 63), b = 1e-3f * (float)(t & 7);
    float x[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = (float)j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) x[j] = fmaf(x[j], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += x[j];
    out[t] = s;
}

__global__ __launch_bounds__(kBlock) void k_cal_exp(int iters, float *__restrict__ out)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    float x[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = 0.01f * (float)(j + (t & 15));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) x[j] = __builtin_amdgcn_exp2f(-x[j]);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += x[j];
    out[t] = s;
}

hipError_t launch(int kind, int iters, const float *ev, float *out, hipStream_t st)
{
    if (kind == 0)
        hipLaunchKernelGGL(k_cal_terms, dim3(kBlocks), dim3(kBlock), 0, st, ev, iters, out);
    else if (kind == 1)
        hipLaunchKernelGGL(k_cal_fma, dim3(kBlocks), dim3(kBlock), 0, st, iters, out);
    else
        hipLaunchKernelGGL(k_cal_exp, dim3(kBlocks), dim3(kBlock), 0, st, iters, out);
    return hipGetLastError();
}

}  // namespace

extern "C" int lmmew_calibrate(int kind, hipStream_t st, double *rate)
{
    if (!rate || kind < 0 || kind > 2) return LMMEW_EINVAL;
    *rate = 0.0;
    const int iters = kind == 0 ? 2048 : 8192;
    const int reps = 5;
    // (energy, factor) blocks for the term chain: energies over the windows,
    // factors of the order of a collimator-response probability
    float h_ev[kEvTab * 2 * kChains];
    for (int b = 0; b < kEvTab; ++b)
        for (int j = 0; j < kChains; ++j) {
            h_ev[b * 2 * kChains + j] = 70.f + 3.5f * (float)((b * kChains + j) % 64);
            h_ev[b * 2 * kChains + kChains + j] = 1e-3f * (float)(1 + (b + j) % 7);
        }
    float *d_ev = nullptr, *d_out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&d_ev, sizeof h_ev);
    if (e == hipSuccess) e = hipMalloc(&d_out, sizeof(float) * kBlocks * kBlock);
    if (e == hipSuccess) e = hipMemcpyAsync(d_ev, h_ev, sizeof h_ev, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch(kind, iters, d_ev, d_out, st);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(kind, iters, d_ev, d_out, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d_ev) (void)hipFree(d_ev);
    if (d_out) (void)hipFree(d_out);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LMMEW_ENOMEM : LMMEW_EDEVICE;
    if (!(ms > 0.f)) return LMMEW_EDEVICE;
    const double ops = (double)reps * kBlocks * kBlock * (double)iters * kChains;
    *rate = ops / (ms * 1e-3);
    return LMMEW_OK;
}
