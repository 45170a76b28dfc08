// Training-data synthesis for the gate network: Q/U spectra of Faraday-thin
// screens and Burn slabs (Section 2.1, eqs. (1), (3), (4)) plus Gaussian
// noise, drawn from a counter-based generator so that line of sight g has the
// same content whatever batch produces it; and the labels taken from the
// transform's peak.
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011), key
// (seed mod 2^32, seed div 2^32), counters
//   (0,     g_lo, g_hi, 0)  class draw          (1 + c, g_lo, g_hi, 0)  component c
//   (m,     g_lo, g_hi, 1)  noise of channels 2m, 2m + 1
// 32-bit word x -> u = (floor(x / 2^9) + 1/2) 2^-23.  All sky-model and
// Box-Muller arithmetic is FP64; Q and U are rounded to FP32 once.
#include "mlp.h"

namespace {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__device__ __forceinline__ double u24(uint32_t x) { return ((double)(x >> 9) + 0.5) * 0x1p-23; }

struct Comp {
    double P0, phi0, chi0, W;
};

__device__ __forceinline__ Comp draw_comp(const TrainSpecDev& s, uint4 x)
{
    Comp c;
    c.P0 = s.p0_lo + (s.p0_hi - s.p0_lo) * u24(x.x);
    c.phi0 = s.phi_lo + (s.phi_hi - s.phi_lo) * u24(x.y);
    c.chi0 = M_PI * u24(x.z);
    c.W = s.w_lo + (s.w_hi - s.w_lo) * u24(x.w);
    return c;
}

// P(lambda^2) of one component: thin screen, or Burn slab when `slab`.
__device__ __forceinline__ void add_comp(const Comp& c, bool slab, double lam, double& re,
                                         double& im)
{
    double sn, cs;
    sincos(2.0 * (c.chi0 + c.phi0 * lam), &sn, &cs);
    double a = c.P0;
    if (slab) {
        const double x = c.W * lam;
        a *= sin(x) / x;
    }
    re += a * cs;
    im += a * sn;
}

// One wave per line of sight.
__global__ __launch_bounds__(256) void spectra_kernel(const double* __restrict__ lambda2, int nchan,
                                                      TrainSpecDev s, uint32_t k0, uint32_t k1,
                                                      int64_t first, int64_t nlos,
                                                      float* __restrict__ Q, float* __restrict__ U,
                                                      int32_t* __restrict__ cls_out,
                                                      float* __restrict__ truth)
{
    const int lane = threadIdx.x & 63;
    const int64_t l = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (l >= nlos) return;
    const uint64_t g = (uint64_t)(first + l);
    const uint32_t glo = (uint32_t)g, ghi = (uint32_t)(g >> 32);
    const double uc = u24(philox4x32_10(make_uint4(0u, glo, ghi, 0u), k0, k1).x);
    const int cls = uc < s.f0 ? 0 : (uc < s.f1 ? 1 : (uc < s.f2 ? 2 : 3));
    const Comp a = draw_comp(s, philox4x32_10(make_uint4(1u, glo, ghi, 0u), k0, k1));
    const Comp b = draw_comp(s, philox4x32_10(make_uint4(2u, glo, ghi, 0u), k0, k1));
    float* q = Q + (int64_t)l * nchan;
    float* u = U + (int64_t)l * nchan;
    const int npair = (nchan + 1) / 2;
    for (int m = lane; m < npair; m += 64) {
        const uint4 x = philox4x32_10(make_uint4((uint32_t)m, glo, ghi, 1u), k0, k1);
        double nq[2], nu[2];
        const double ra = sqrt(-2.0 * log(u24(x.x))), rb = sqrt(-2.0 * log(u24(x.z)));
        double st, ct;
        sincos(2.0 * M_PI * u24(x.y), &st, &ct);
        nq[0] = ra * ct;
        nu[0] = ra * st;
        sincos(2.0 * M_PI * u24(x.w), &st, &ct);
        nq[1] = rb * ct;
        nu[1] = rb * st;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = 2 * m + h;
            if (j >= nchan) break;
            const double lam = lambda2[j];
            double re = 0.0, im = 0.0;
            if (cls >= 1) add_comp(a, cls == 3, lam, re, im);
            if (cls == 2) add_comp(b, false, lam, re, im);
            q[j] = (float)(re + s.sigma * nq[h]);
            u[j] = (float)(im + s.sigma * nu[h]);
        }
    }
    if (lane == 0) {
        if (cls_out) cls_out[l] = cls;
        if (truth) {
            const float nan = __builtin_nanf("");
            float* t = truth + 4 * l;
            t[0] = cls >= 1 ? (float)a.phi0 : nan;
            t[1] = cls >= 1 ? (float)a.P0 : nan;
            t[2] = cls == 2 ? (float)b.phi0 : nan;
            t[3] = cls == 2 ? (float)b.P0 : nan;
        }
    }
}

__global__ void label_kernel(const int32_t* __restrict__ idx, const float* __restrict__ phi_pk,
                             const float* __restrict__ amp, int64_t n, float thr,
                             float* __restrict__ phi_label, float* __restrict__ det_label)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool ok = idx[i] >= 0;
    if (phi_label) phi_label[i] = ok ? phi_pk[i] : 0.0f;
    if (det_label) det_label[i] = (ok && amp[i] >= thr) ? 1.0f : 0.0f;
}

}  // namespace

hipError_t train_launch_spectra(const double* lambda2, int nchan, const TrainSpecDev& s, uint64_t seed,
                                int64_t first, int64_t nlos, float* Q, float* U, int32_t* cls,
                                float* truth, hipStream_t st)
{
    const int64_t blocks = (nlos + 3) / 4;
    if (blocks > max_blocks(256)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(spectra_kernel, dim3((unsigned)blocks), dim3(256), 0, st, lambda2, nchan, s,
                       (uint32_t)seed, (uint32_t)(seed >> 32), first, nlos, Q, U, cls, truth);
    return hipGetLastError();
}

hipError_t train_launch_labels(const int32_t* idx, const float* phi_pk, const float* amp, int64_t n,
                               float thr, float* phi_label, float* det_label, hipStream_t st)
{
    if ((n + 255) / 256 > max_blocks(256)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(label_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, idx, phi_pk,
                       amp, n, thr, phi_label, det_label);
    return hipGetLastError();
}
