// Per-LOS peak of |F| and the RM spread function.
//
// Peaks: one wave64 per LOS.  Each lane scans phi k = lane, lane + 64, ...
// keeping the largest Fq^2 + Fu^2 (one rounding: fma(q, q, u * u), as the
// fused peaks of the transform kernels; strict >, so its lowest k), then a
// butterfly of cross-lane shuffles merges (value, index) pairs, ties going to
// the lower index.  A LOS whose |F|^2 is not finite somewhere (a non-finite
// Fq or Fu, or |F|^2 beyond the FP32 range) is marked (idx = -1).
// HBM-bound: 8 bytes read per (LOS, phi).
//
// RMSF, eq. (12): one thread per phi, FP64 argument reduction and FP32
// sin/cos (the same generator as the transform), FP32 accumulation.
#include <float.h>

#include "common.h"

namespace {

constexpr int WAVES = 4;

__global__ __launch_bounds__(256) void peaks_kernel(
    const float* __restrict__ Fq, const float* __restrict__ Fu, int64_t nlos, int nphi,
    const double* __restrict__ phik, int32_t* __restrict__ idx, float* __restrict__ phi_pk,
    float* __restrict__ amp, float* __restrict__ q_pk, float* __restrict__ u_pk)
{
    const int lane = threadIdx.x & 63;
    const int64_t l = (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6);
    if (l >= nlos) return;  // uniform per wave
    const float* q = Fq + l * nphi;
    const float* u = Fu + l * nphi;
    float best = -1.0f;
    int bi = 0x7fffffff;
    bool bad = false;
    int k = lane;
    for (; k + 192 < nphi; k += 256) {
        float a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) { a[i] = q[k + 64 * i]; b[i] = u[k + 64 * i]; }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float m = __builtin_fmaf(a[i], a[i], b[i] * b[i]);
            bad |= !(m <= FLT_MAX);
            if (m > best) { best = m; bi = k + 64 * i; }
        }
    }
    for (; k < nphi; k += 64) {
        const float a = q[k], b = u[k];
        const float m = __builtin_fmaf(a, a, b * b);
        bad |= !(m <= FLT_MAX);
        if (m > best) { best = m; bi = k; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const bool anybad = __any(bad);
    if (lane == 0) {
        if (anybad || bi < 0 || bi >= nphi) {
            idx[l] = -1;
            const float nan = __builtin_nanf("");
            if (phi_pk) phi_pk[l] = nan;
            if (amp) amp[l] = nan;
            if (q_pk) q_pk[l] = nan;
            if (u_pk) u_pk[l] = nan;
        } else {
            idx[l] = bi;
            if (phi_pk) phi_pk[l] = (float)phik[bi];
            if (amp) amp[l] = sqrtf(best);
            if (q_pk) q_pk[l] = q[bi];
            if (u_pk) u_pk[l] = u[bi];
        }
    }
}

__global__ __launch_bounds__(256) void rmsf_kernel(const double* __restrict__ bj,
                                                   const float* __restrict__ wj, int nchan,
                                                   const double* __restrict__ phik, int nphi,
                                                   float K, float* __restrict__ re,
                                                   float* __restrict__ im)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nphi) return;
    const double ph = phik[k];
    float sr = 0.0f, si = 0.0f;
    for (int j = 0; j < nchan; ++j) {
        const float w = wj[j];
        if (w == 0.0f) continue;
        float c, s;
        phase_cos_sin(ph * bj[j], c, s);
        sr = __builtin_fmaf(w, c, sr);
        si = __builtin_fmaf(-w, s, si);
    }
    re[k] = K * sr;
    im[k] = K * si;
}

// Polarization angle of each LOS's peak referred to lambda^2 = 0 (eq. (14)):
// half the phase of F(phi_pk) de-rotated by exp(-2i phi_pk lambda0^2), taken
// in FP64 from the FP32 peak values and wrapped to [0, pi).  NaN when an
// input is not finite.
__global__ void peak_angle_kernel(const float* __restrict__ phi_pk, const float* __restrict__ q_pk,
                                  const float* __restrict__ u_pk, int64_t nlos, double lambda0_sq,
                                  float* __restrict__ chi0)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlos) return;
    const double q = q_pk[l], u = u_pk[l], ph = phi_pk[l];
    if (!(__builtin_isfinite(q) && __builtin_isfinite(u) && __builtin_isfinite(ph))) {
        chi0[l] = __builtin_nanf("");
        return;
    }
    const double pi = 3.141592653589793;
    double chi = 0.5 * atan2(u, q) - ph * lambda0_sq;
    chi -= pi * floor(chi / pi);
    // Rounding can leave chi = pi exactly; the interval is half-open.
    float c = (float)chi;
    chi0[l] = c < (float)pi ? c : 0.0f;
}

// Sub-grid peak from stored F: |F| at idx - 1, idx, idx + 1 as the square
// root (FP64) of the FP32 |F|^2 the peak search compares (the same fma), then
// the parabola's vertex.  idx = -1 gives NaN.
__global__ void peak_fit_kernel(const float* __restrict__ Fq, const float* __restrict__ Fu,
                                const int32_t* __restrict__ idx, int64_t nlos, int nphi,
                                const double* __restrict__ phik, float* __restrict__ phi_fit,
                                float* __restrict__ amp_fit)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlos) return;
    const int k = idx[l];
    if (k < 0 || k >= nphi) {
        if (phi_fit) phi_fit[l] = __builtin_nanf("");
        if (amp_fit) amp_fit[l] = __builtin_nanf("");
        return;
    }
    const float* q = Fq + l * nphi;
    const float* u = Fu + l * nphi;
    auto amp_at = [&](int kk) -> double {
        if (kk < 0 || kk >= nphi) return __builtin_nan("");
        return __builtin_sqrt((double)__builtin_fmaf(q[kk], q[kk], u[kk] * u[kk]));
    };
    const double x0 = k > 0 ? phik[k - 1] : __builtin_nan("");
    const double x2 = k + 1 < nphi ? phik[k + 1] : __builtin_nan("");
    float pf, af;
    parabola_vertex(x0, amp_at(k - 1), phik[k], amp_at(k), x2, amp_at(k + 1), &pf, &af);
    if (phi_fit) phi_fit[l] = pf;
    if (amp_fit) amp_fit[l] = af;
}

}  // namespace

hipError_t launch_peak_fit(const rmsynth_plan_s& p, const float* Fq, const float* Fu,
                           const int32_t* idx, int64_t nlos, float* phi_fit, float* amp_fit,
                           hipStream_t s)
{
    for (int64_t l0 = 0; l0 < nlos;) {
        const int64_t n = std::min<int64_t>(nlos - l0, max_items(256, 256));
        hipLaunchKernelGGL(peak_fit_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           Fq + l0 * p.nphi, Fu + l0 * p.nphi, idx + l0, n, p.nphi, p.d_phi,
                           phi_fit ? phi_fit + l0 : nullptr, amp_fit ? amp_fit + l0 : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        l0 += n;
    }
    return hipSuccess;
}

hipError_t launch_peak_angle(const rmsynth_plan_s& p, const float* phi_pk, const float* q_pk,
                             const float* u_pk, int64_t nlos, float* chi0, hipStream_t s)
{
    for (int64_t l0 = 0; l0 < nlos;) {
        const int64_t n = std::min<int64_t>(nlos - l0, max_items(256, 256));
        hipLaunchKernelGGL(peak_angle_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           phi_pk + l0, q_pk + l0, u_pk + l0, n, p.lambda0_sq, chi0 + l0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        l0 += n;
    }
    return hipSuccess;
}

hipError_t launch_peaks(const rmsynth_plan_s& p, const float* Fq, const float* Fu, int64_t nlos,
                        int32_t* idx, float* phi_pk, float* amp, float* q_pk, float* u_pk,
                        hipStream_t s)
{
    for (int64_t l0 = 0; l0 < nlos;) {
        const int64_t n = std::min<int64_t>(nlos - l0, max_items(WAVES, 64 * WAVES));
        const int64_t blocks = (n + WAVES - 1) / WAVES;
        hipLaunchKernelGGL(peaks_kernel, dim3((unsigned)blocks), dim3(64 * WAVES), 0, s,
                           Fq + l0 * p.nphi, Fu + l0 * p.nphi, n, p.nphi, p.d_phi, idx + l0,
                           phi_pk ? phi_pk + l0 : nullptr, amp ? amp + l0 : nullptr,
                           q_pk ? q_pk + l0 : nullptr, u_pk ? u_pk + l0 : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        l0 += n;
    }
    return hipSuccess;
}

hipError_t launch_rmsf(const rmsynth_plan_s& p, float* re, float* im, hipStream_t s)
{
    const int blocks = (p.nphi + 255) / 256;
    hipLaunchKernelGGL(rmsf_kernel, dim3(blocks), dim3(256), 0, s, p.d_b, p.d_w, p.nchan, p.d_phi,
                       p.nphi, (float)p.K, re, im);
    return hipGetLastError();
}
