// Faraday-depth transform on a uniform phi grid by a non-uniform FFT (the
// FFT evaluation the paper proposes in place of the direct sums of
// eqs. (15)-(16), Section 4).  With phi_k = phi_c + m dphi, m = k - kc,
// eq. (11) is a type-1 non-uniform DFT in m:
//
//   F_k = sum_j c_j exp(-i m x_j),  c_j = K w_j P_j exp(-2i a_j phi_c),
//                                   x_j = 2 a_j dphi (mod 2 pi),
//
// evaluated by gridding each c_j onto n >= 2N uniform points of [0, 2 pi)
// with the "exponential of semicircle" kernel psi of width W grid cells
// (Barnett, Magland & af Klinteberg 2019), an n-point FFT, and division of
// mode m by the kernel's Fourier transform psi_hat(m).  The gridding weights
// (a per-plan CSR list per grid point: the channels within the kernel's
// reach), c_j's rotation, the twiddles and 1/psi_hat are plan-time tables
// built on the host in FP64.
//
// One workgroup (256 threads) per LOS: the channels' c_j go to LDS, each
// thread gathers grid points from its CSR lists (a fixed order, no atomics),
// the FFT runs as in-place Stockham passes in LDS (radix 4, one radix-2 pass
// when log2 n is odd; each pass reads its butterflies into registers, meets
// a barrier, then writes), and the N wanted modes are scaled and stored.
#include "common.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// -i z
__device__ __forceinline__ float2 cmul_mi(float2 z) { return make_float2(z.y, -z.x); }

template <int LOGN>
__global__ __launch_bounds__(kThreads) void nufft_kernel(
    const float* __restrict__ Q, const float* __restrict__ U, int64_t nlos, int nchan,
    const float2* __restrict__ rot, const int* __restrict__ off, const int* __restrict__ ej,
    const float* __restrict__ ew, const float2* __restrict__ tw, const float* __restrict__ deconv,
    int N, int kc, float* __restrict__ Fq, float* __restrict__ Fu, float* __restrict__ Fabs)
{
    constexpr int n = 1 << LOGN;
    constexpr int NB4 = (n / 4 + kThreads - 1) / kThreads;  // radix-4 butterflies per thread
    constexpr int NB2 = (n / 2 + kThreads - 1) / kThreads;  // radix-2 butterflies per thread
    extern __shared__ float4 smem4[];
    float2* grid = reinterpret_cast<float2*>(smem4);
    float2* cb = grid + n;
    const int t = threadIdx.x;
    const int64_t l = blockIdx.x;
    if (l >= nlos) return;  // uniform per workgroup

    // c_j = rot_j (Q_j + i U_j); flagged channels are in no gridding list.
    const float* q = Q + l * nchan;
    const float* u = U + l * nchan;
    for (int j = t; j < nchan; j += kThreads) cb[j] = cmul(rot[j], make_float2(q[j], u[j]));
    __syncthreads();
    // Gridding: g_p = sum over the channels within reach of p of psi_jp c_j.
    for (int p = t; p < n; p += kThreads) {
        float2 s = make_float2(0.0f, 0.0f);
        const int e1 = off[p + 1];
        for (int e = off[p]; e < e1; ++e) {
            const float w = ew[e];
            const float2 c = cb[ej[e]];
            s.x = __builtin_fmaf(w, c.x, s.x);
            s.y = __builtin_fmaf(w, c.y, s.y);
        }
        grid[p] = s;
    }
    __syncthreads();

    // Stockham FFT, G_m = sum_p g_p exp(-2 pi i m p / n): a pass of radix R
    // on sub-transforms of length Ns reads src[j + r n/R], twiddles it by
    // exp(-2 pi i r (j mod Ns) / (Ns R)), takes an R-point DFT and writes
    // element r to (j / Ns) Ns R + (j mod Ns) + r Ns.
    int Ns = 1;
    if (LOGN & 1) {
        float2 v[NB2][2];
#pragma unroll
        for (int b = 0; b < NB2; ++b) {
            const int j = t + kThreads * b;
            if (j < n / 2) {
                v[b][0] = grid[j];
                v[b][1] = grid[j + n / 2];
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB2; ++b) {
            const int j = t + kThreads * b;
            if (j < n / 2) {
                grid[2 * j] = cadd(v[b][0], v[b][1]);
                grid[2 * j + 1] = csub(v[b][0], v[b][1]);
            }
        }
        __syncthreads();
        Ns = 2;
    }
    for (; Ns < n; Ns *= 4) {
        const int tstep = n / (4 * Ns);  // twiddle index per unit of r k
        float2 v[NB4][4];
#pragma unroll
        for (int b = 0; b < NB4; ++b) {
            const int j = t + kThreads * b;
            if (j < n / 4) {
                const int k = j & (Ns - 1);
                float2 x0 = grid[j], x1 = grid[j + n / 4], x2 = grid[j + n / 2], x3 = grid[j + 3 * n / 4];
                x1 = cmul(x1, tw[(k * tstep) & (n - 1)]);
                x2 = cmul(x2, tw[(2 * k * tstep) & (n - 1)]);
                x3 = cmul(x3, tw[(3 * k * tstep) & (n - 1)]);
                const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
                const float2 a2 = cadd(x1, x3), a3 = cmul_mi(csub(x1, x3));
                v[b][0] = cadd(a0, a2);
                v[b][1] = cadd(a1, a3);
                v[b][2] = csub(a0, a2);
                v[b][3] = csub(a1, a3);
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB4; ++b) {
            const int j = t + kThreads * b;
            if (j < n / 4) {
                const int k = j & (Ns - 1);
                const int base = (j - k) * 4 + k;
#pragma unroll
                for (int r = 0; r < 4; ++r) grid[base + r * Ns] = v[b][r];
            }
        }
        __syncthreads();
    }

    // F_k = (2 pi / n) G_{(k - kc) mod n} / psi_hat(k - kc).
    float* fq = Fq + l * N;
    float* fu = Fu + l * N;
    for (int k = t; k < N; k += kThreads) {
        const float2 g = grid[(k - kc) & (n - 1)];
        const float d = deconv[k];
        const float a = g.x * d, b = g.y * d;
        fq[k] = a;
        fu[k] = b;
        if (Fabs) Fabs[l * N + k] = sqrtf(a * a + b * b);
    }
}

}  // namespace

size_t nufft_lds_bytes(const rmsynth_plan_s& p)
{
    return (size_t)((p.nufft_n + p.nchan) * (int64_t)sizeof(float2));
}

hipError_t launch_nufft(const rmsynth_plan_s& p, const float* Q, const float* U, int64_t nlos,
                        float* Fq, float* Fu, float* Fabs, hipStream_t s)
{
    const size_t lds = nufft_lds_bytes(p);
    int logn = 0;
    while ((1 << logn) < p.nufft_n) ++logn;
    for (int64_t l0 = 0; l0 < nlos;) {
        const int64_t n = std::min<int64_t>(nlos - l0, max_blocks(kThreads));
        const float* q = Q + l0 * p.nchan;
        const float* u = U + l0 * p.nchan;
        float* fq = Fq + l0 * p.nphi;
        float* fu = Fu + l0 * p.nphi;
        float* fa = Fabs ? Fabs + l0 * p.nphi : nullptr;
#define RMS_NUFFT(L)                                                                                  \
    hipLaunchKernelGGL(nufft_kernel<L>, dim3((unsigned)n), dim3(kThreads), lds, s, q, u, n, p.nchan,    \
                       p.d_nufft_rot, p.d_nufft_off, p.d_nufft_ej, p.d_nufft_ew, p.d_nufft_tw,          \
                       p.d_nufft_deconv, p.nphi, p.nufft_kc, fq, fu, fa)
        switch (logn) {
            case 4: RMS_NUFFT(4); break;
            case 5: RMS_NUFFT(5); break;
            case 6: RMS_NUFFT(6); break;
            case 7: RMS_NUFFT(7); break;
            case 8: RMS_NUFFT(8); break;
            case 9: RMS_NUFFT(9); break;
            case 10: RMS_NUFFT(10); break;
            case 11: RMS_NUFFT(11); break;
            case 12: RMS_NUFFT(12); break;
            case 13: RMS_NUFFT(13); break;
            default: return hipErrorInvalidValue;
        }
#undef RMS_NUFFT
        if (hipError_t e = hipGetLastError()) return e;
        l0 += n;
    }
    return hipSuccess;
}
