// RM-CLEAN: deconvolution of the Faraday spectrum by the RMSF (the use of
// R(phi), eq. (12), that Section 2.2 names and leaves unsupported; Section 4).
// Hogbom's iteration on a uniform phi grid, for every LOS independently:
//
//   r <- F;  C <- 0
//   repeat at most max_iter times:
//     p = lowest index maximising |r_k|^2;  stop when |r_p| < cutoff
//     c = gain r_p;  C_p += c;  r_k -= c R((k - p) dphi)  for every k
//   restored_k = r_k + sum_m C_m G((k - m) dphi),  G(x) = exp(-4 ln2 x^2 / fwhm^2)
//
// One wave per LOS, the residual in registers (element k = 64 e + lane, at
// most 64 per lane: nphi <= 4096), so a pick is a lane scan plus a butterfly
// of (|r|^2, k, r) with ties to the lower k, and a subtraction is one LDS read
// of R per element.  R on the doubled grid (m - (N-1)) dphi, m = 0 .. 2N-2,
// and G on the same offsets are built per call into the workspace (FP64
// argument reduction, FP32 sin/cos and accumulation, as the RMSF); R is
// staged in LDS (at most 64 KB), G is read through the caches.  The component of a pick goes to the component row by the lane that
// owns its phi (a read-modify-write of its own earlier stores); a per-lane
// bit mask remembers which of its elements hold one, and the restore visits
// only those.  A LOS whose F is not finite is flagged (niter = -1, every
// output NaN).
#include <float.h>

#include "common.h"

namespace {

// LOS (waves) per workgroup: 8, or 4 for the widest layout (64 elements per
// lane), whose one wave per SIMD may then use the full register file.
template <int E>
constexpr int waves_of() { return E >= 64 ? 4 : 8; }

// R((m - (N-1)) dphi) = K sum_j w_j exp(-2i x a_j) and G at the same offsets.
__global__ void rmclean_tables_kernel(const double* __restrict__ bj, const float* __restrict__ wj,
                                      int nchan, int N, double dphi, float K, double fwhm,
                                      float2* __restrict__ R2, float* __restrict__ G)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= 2 * N - 1) return;
    const double x = (double)(m - (N - 1)) * dphi;
    float sr = 0.0f, si = 0.0f;
    for (int j = 0; j < nchan; ++j) {
        const float w = wj[j];
        if (w == 0.0f) continue;
        float c, s;
        phase_cos_sin(x * bj[j], c, s);
        sr = __builtin_fmaf(w, c, sr);
        si = __builtin_fmaf(-w, s, si);
    }
    R2[m] = make_float2(K * sr, K * si);
    const double z = x / fwhm;
    G[m] = (float)exp(-4.0 * 0.69314718055994530942 * z * z);
}

template <int E>
__global__ __launch_bounds__(64 * waves_of<E>()) void rmclean_kernel(
    const float* Fq, const float* Fu, int64_t nlos, int N, const float2* __restrict__ R2g,
    const float* __restrict__ Gg, float gain, float cutoff, int max_iter, float* rq, float* ru,
    float* __restrict__ cq, float* __restrict__ cu, float* __restrict__ Rq, float* __restrict__ Ru,
    int32_t* __restrict__ niter)
{
    extern __shared__ float4 smem4[];
    float2* R2 = reinterpret_cast<float2*>(smem4);
    const float* G = Gg;
    const bool restore = Rq != nullptr;
    for (int i = threadIdx.x; i < 2 * N - 1; i += blockDim.x) R2[i] = R2g[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t l = (int64_t)blockIdx.x * waves_of<E>() + (threadIdx.x >> 6);
    if (l >= nlos) return;  // uniform per wave; no block barrier follows
    const int64_t row = l * N;

    // Elements past the grid (k >= N) hold 0, are never picked (|r|^2 taken
    // as -1) and never stored; their table index is clamped into the table.
    // The loops over the register arrays are written without branches (loads
    // from clamped addresses, selects), which keeps the arrays in registers.
    float xr[E], xi[E];
    bool bad = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = 64 * e + lane;
        const int kc = k < N ? k : N - 1;
        const float a = Fq[row + kc], b = Fu[row + kc];
        xr[e] = k < N ? a : 0.0f;
        xi[e] = k < N ? b : 0.0f;
        bad |= !(__builtin_fabsf(xr[e]) <= FLT_MAX && __builtin_fabsf(xi[e]) <= FLT_MAX);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = 64 * e + lane;
        if (k < N) {
            cq[row + k] = 0.0f;
            cu[row + k] = 0.0f;
        }
    }
    if (__any(bad)) {
        const float nan = __builtin_nanf("");
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = 64 * e + lane;
            if (k < N) {
                rq[row + k] = nan;
                ru[row + k] = nan;
                cq[row + k] = nan;
                cu[row + k] = nan;
                if (restore) {
                    Rq[row + k] = nan;
                    Ru[row + k] = nan;
                }
            }
        }
        if (niter && lane == 0) niter[l] = -1;
        return;
    }

    uint64_t has = 0;  // bit e: element 64 e + lane holds a component
    const int last = 2 * N - 2;
    int it = 0;
    for (; it < max_iter; ++it) {
        float best = -1.0f, br = 0.0f, bi = 0.0f;
        int bk = 0x7fffffff;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = 64 * e + lane;
            const float a2 = k < N ? __builtin_fmaf(xr[e], xr[e], xi[e] * xi[e]) : -1.0f;
            const bool gt = a2 > best;
            best = gt ? a2 : best;
            bk = gt ? k : bk;
            br = gt ? xr[e] : br;
            bi = gt ? xi[e] : bi;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off, 64);
            const int ok = __shfl_xor(bk, off, 64);
            const float orr = __shfl_xor(br, off, 64);
            const float oi = __shfl_xor(bi, off, 64);
            const bool take = ob > best || (ob == best && ok < bk);
            best = take ? ob : best;
            bk = take ? ok : bk;
            br = take ? orr : br;
            bi = take ? oi : bi;
        }
        if (sqrtf(best) < cutoff) break;
        const float cr = gain * br, ci = gain * bi;
        if (lane == (bk & 63)) {
            cq[row + bk] += cr;
            cu[row + bk] += ci;
            has |= uint64_t(1) << (bk >> 6);
        }
        const int base = N - 1 - bk;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = base + 64 * e + lane;
            const float2 R = R2[t < last ? t : last];
            xr[e] = __builtin_fmaf(-cr, R.x, __builtin_fmaf(ci, R.y, xr[e]));
            xi[e] = __builtin_fmaf(-cr, R.y, __builtin_fmaf(-ci, R.x, xi[e]));
        }
    }
    if (niter && lane == 0) niter[l] = it;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = 64 * e + lane;
        if (k < N) {
            rq[row + k] = xr[e];
            ru[row + k] = xi[e];
        }
    }
    if (!restore) return;
    // restored = residual + components convolved with G, component by
    // component in (e, lane) order (the outer loop is kept rolled: only the
    // inner one indexes the register arrays).
#pragma unroll 1
    for (int e = 0; e < E; ++e) {
        uint64_t m = __ballot((has >> e) & 1);
        float vr = 0.0f, vi = 0.0f;
        if ((has >> e) & 1) {
            vr = cq[row + 64 * e + lane];
            vi = cu[row + 64 * e + lane];
        }
        while (m) {
            const int j = __builtin_ctzll(m);
            m &= m - 1;
            const int kc = 64 * e + j;
            const float c_r = __shfl(vr, j, 64), c_i = __shfl(vi, j, 64);
            const int base = N - 1 - kc;
#pragma unroll
            for (int e2 = 0; e2 < E; ++e2) {
                const int t = base + 64 * e2 + lane;
                const float g = G[t < last ? t : last];
                xr[e2] = __builtin_fmaf(c_r, g, xr[e2]);
                xi[e2] = __builtin_fmaf(c_i, g, xi[e2]);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = 64 * e + lane;
        if (k < N) {
            Rq[row + k] = xr[e];
            Ru[row + k] = xi[e];
        }
    }
}

template <int E>
hipError_t launch_e(const float* Fq, const float* Fu, int64_t nlos, int N, const float2* R2,
                    const float* G, float gain, float cutoff, int max_iter, float* rq, float* ru,
                    float* cq, float* cu, float* Rq, float* Ru, int32_t* niter, hipStream_t s)
{
    constexpr int W = waves_of<E>();
    const size_t lds = (size_t)(2 * N - 1) * sizeof(float2);
    for (int64_t l0 = 0; l0 < nlos;) {
        const int64_t n = std::min<int64_t>(nlos - l0, max_items(W, 64 * W));
        const int64_t off = l0 * N;
        hipLaunchKernelGGL(rmclean_kernel<E>, dim3((unsigned)((n + W - 1) / W)),
                           dim3(64 * W), lds, s, Fq + off, Fu + off, n, N, R2, G, gain, cutoff,
                           max_iter, rq + off, ru + off, cq + off, cu + off, Rq ? Rq + off : nullptr,
                           Ru ? Ru + off : nullptr, niter ? niter + l0 : nullptr);
        if (hipError_t e = hipGetLastError()) return e;
        l0 += n;
    }
    return hipSuccess;
}

}  // namespace

size_t rmclean_table_bytes(const rmsynth_plan_s& p)
{
    return (size_t)round_up((int64_t)(2 * p.nphi - 1) * (int64_t)sizeof(float2), 256) +
           (size_t)round_up((int64_t)(2 * p.nphi - 1) * (int64_t)sizeof(float), 256);
}

hipError_t launch_rmclean(const rmsynth_plan_s& p, const float* Fq, const float* Fu, int64_t nlos,
                          float gain, float cutoff, int max_iter, double fwhm, float* rq, float* ru,
                          float* cq, float* cu, float* Rq, float* Ru, int32_t* niter, void* ws,
                          hipStream_t s)
{
    const int N = p.nphi;
    float2* R2 = static_cast<float2*>(ws);
    float* G = reinterpret_cast<float*>(static_cast<char*>(ws) +
                                        round_up((int64_t)(2 * N - 1) * (int64_t)sizeof(float2), 256));
    hipLaunchKernelGGL(rmclean_tables_kernel, dim3((unsigned)((2 * N - 1 + 255) / 256)), dim3(256), 0, s,
                       p.d_b, p.d_w, p.nchan, N, p.dphi, (float)p.K, fwhm, R2, G);
    if (hipError_t e = hipGetLastError()) return e;
    if (nlos == 0) return hipSuccess;
    const int E = (N + 63) / 64;
    if (E <= 4) return launch_e<4>(Fq, Fu, nlos, N, R2, G, gain, cutoff, max_iter, rq, ru, cq, cu, Rq, Ru, niter, s);
    if (E <= 8) return launch_e<8>(Fq, Fu, nlos, N, R2, G, gain, cutoff, max_iter, rq, ru, cq, cu, Rq, Ru, niter, s);
    if (E <= 16) return launch_e<16>(Fq, Fu, nlos, N, R2, G, gain, cutoff, max_iter, rq, ru, cq, cu, Rq, Ru, niter, s);
    if (E <= 32) return launch_e<32>(Fq, Fu, nlos, N, R2, G, gain, cutoff, max_iter, rq, ru, cq, cu, Rq, Ru, niter, s);
    return launch_e<64>(Fq, Fu, nlos, N, R2, G, gain, cutoff, max_iter, rq, ru, cq, cu, Rq, Ru, niter, s);
}
