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
// thread sums whole grid points from their lists of entries (a fixed order,
// no atomics; only the points some channel reaches),
// the FFT runs as in-place Stockham passes in LDS (radix 16, and one pass of
// radix 2, 4 or 8 for the rest of log2 n; each pass reads its butterflies
// into registers, meets a barrier, then writes), and the N wanted modes are
// scaled and stored.
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

// DFTs of 2, 4, 8 and 16 points in registers, X_q = sum_r x_r exp(-2 pi i r q / R),
// in place.  The roots of unity are the exact values cos(pi/4) = sqrt(2)/2,
// cos(pi/8), sin(pi/8).
constexpr float kC4 = 0.70710678118654752440f;   // cos(pi/4)
constexpr float kC8 = 0.92387953251128675613f;   // cos(pi/8)
constexpr float kS8 = 0.38268343236508977173f;   // sin(pi/8)

__device__ __forceinline__ void dft2(float2* x)
{
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
}
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3)
{
    const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
    const float2 a2 = cadd(x1, x3), a3 = cmul_mi(csub(x1, x3));
    x0 = cadd(a0, a2);
    x1 = cadd(a1, a3);
    x2 = csub(a0, a2);
    x3 = csub(a1, a3);
}
__device__ __forceinline__ void dft4(float2* x) { dft4(x[0], x[1], x[2], x[3]); }
// 8 points: DFT4 of the even and the odd samples, X_q = E_q + w8^q O_q.
__device__ __forceinline__ void dft8(float2* x)
{
    float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = make_float2(kC4 * (o1.x + o1.y), kC4 * (o1.y - o1.x));     // x w8^1
    o2 = cmul_mi(o2);                                               // x w8^2
    o3 = make_float2(kC4 * (o3.y - o3.x), -kC4 * (o3.x + o3.y));    // x w8^3
    x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
    x[1] = cadd(e1, o1); x[5] = csub(e1, o1);
    x[2] = cadd(e2, o2); x[6] = csub(e2, o2);
    x[3] = cadd(e3, o3); x[7] = csub(e3, o3);
}
// 16 points as 4 x 4: r = 4 r1 + r2, q = q1 + 4 q2;
// X_{q1 + 4 q2} = sum_r2 w4^{r2 q2} w16^{r2 q1} [sum_r1 x_{4 r1 + r2} w4^{r1 q1}].
__device__ __forceinline__ void dft16(float2* x)
{
    float2 y[4][4];
#pragma unroll
    for (int r2 = 0; r2 < 4; ++r2) {
        y[r2][0] = x[r2]; y[r2][1] = x[4 + r2]; y[r2][2] = x[8 + r2]; y[r2][3] = x[12 + r2];
        dft4(y[r2]);
    }
    // w16^m for m = r2 q1: 1, 2, 3 (r2 = 1); 2, 4, 6 (r2 = 2); 3, 6, 9 (r2 = 3)
    const float2 w1 = make_float2(kC8, -kS8), w2 = make_float2(kC4, -kC4), w3 = make_float2(kS8, -kC8);
    const float2 w6 = make_float2(-kC4, -kC4), w9 = make_float2(-kC8, kS8);
    y[1][1] = cmul(y[1][1], w1); y[1][2] = cmul(y[1][2], w2); y[1][3] = cmul(y[1][3], w3);
    y[2][1] = cmul(y[2][1], w2); y[2][2] = cmul_mi(y[2][2]); y[2][3] = cmul(y[2][3], w6);
    y[3][1] = cmul(y[3][1], w3); y[3][2] = cmul(y[3][2], w6); y[3][3] = cmul(y[3][3], w9);
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
        float2 z0 = y[0][q1], z1 = y[1][q1], z2 = y[2][q1], z3 = y[3][q1];
        dft4(z0, z1, z2, z3);
        x[q1] = z0; x[q1 + 4] = z1; x[q1 + 8] = z2; x[q1 + 12] = z3;
    }
}
template <int R>
__device__ __forceinline__ void dft(float2* x)
{
    if constexpr (R == 2) dft2(x);
    else if constexpr (R == 4) dft4(x);
    else if constexpr (R == 8) dft8(x);
    else dft16(x);
}

// LDS position of grid element i: the low four bits XOR-ed with the next
// four, so that the strided accesses of the passes (stride R or R Ns
// elements across a wave) fall on distinct banks; a permutation inside each
// aligned block of 16 elements.
__device__ __forceinline__ int swz(int i) { return i ^ ((i >> 4) & 15); }

// One in-place Stockham pass of radix R on sub-transforms of length Ns: the
// butterflies' inputs are read into registers, a barrier, then the outputs
// are written (every thread's reads finish before any write).
template <int R, int LOGN>
__device__ __forceinline__ void stockham_pass(float2* grid, const float2* __restrict__ tw, int Ns, int t)
{
    constexpr int n = 1 << LOGN;
    constexpr int NB = (n / R + kThreads - 1) / kThreads;
    float2 v[NB][R];
    const int tstep = n / (R * Ns);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + kThreads * b;
        if (j < n / R) {
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = grid[swz(j + r * (n / R))];
            if (Ns > 1) {
                // w^r, w = exp(-2 pi i k / (Ns R)), from the table entries of
                // w, w^2, w^4, w^8 and at most two products each.
                float2 w[R];
                w[1] = tw[(k * tstep) & (n - 1)];
                if constexpr (R > 2) w[2] = tw[(2 * k * tstep) & (n - 1)];
                if constexpr (R > 4) w[4] = tw[(4 * k * tstep) & (n - 1)];
                if constexpr (R > 8) w[8] = tw[(8 * k * tstep) & (n - 1)];
                if constexpr (R > 2) w[3] = cmul(w[1], w[2]);
                if constexpr (R > 4) {
                    w[5] = cmul(w[4], w[1]);
                    w[6] = cmul(w[4], w[2]);
                    w[7] = cmul(w[4], w[3]);
                }
                if constexpr (R > 8) {
#pragma unroll
                    for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
                }
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], w[r]);
            }
            dft<R>(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + kThreads * b;
        if (j < n / R) {
            const int k = j & (Ns - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) grid[swz(base + r * Ns)] = v[b][r];
        }
    }
    __syncthreads();
}

template <int LOGN>
__global__ __launch_bounds__(kThreads) void nufft_kernel(
    const float* __restrict__ Q, const float* __restrict__ U, int64_t nlos, int nchan,
    const float2* __restrict__ rot, int nocc, const int* __restrict__ off,
    const int2* __restrict__ ent, const float2* __restrict__ tw, const float* __restrict__ deconv,
    int N, int kc, float* __restrict__ Fq, float* __restrict__ Fu, float* __restrict__ Fabs)
{
    constexpr int n = 1 << LOGN;
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
    // Only the points some channel reaches have entries (a narrow band of
    // lambda^2 occupies a small part of the grid): the others are zeroed, the
    // occupied ones (occ[i], entries off[i] .. off[i + 1], packed
    // (j << 13) | p with the weight's bits) summed in a fixed order.
    for (int p = t; p < n; p += kThreads) grid[swz(p)] = make_float2(0.0f, 0.0f);
    __syncthreads();
    for (int i = t; i < nocc; i += kThreads) {
        float2 acc = make_float2(0.0f, 0.0f);
        const int e1 = off[i + 1];
        int pp = 0;
        for (int e = off[i]; e < e1; ++e) {
            const int2 en = ent[e];
            pp = en.x & 8191;
            const float w = __int_as_float(en.y);
            const float2 c = cb[en.x >> 13];
            acc.x = __builtin_fmaf(w, c.x, acc.x);
            acc.y = __builtin_fmaf(w, c.y, acc.y);
        }
        grid[swz(pp)] = acc;
    }
    __syncthreads();

    // Stockham FFT, G_m = sum_p g_p exp(-2 pi i m p / n): a pass of radix R
    // on sub-transforms of length Ns reads src[j + r n/R], twiddles it by
    // exp(-2 pi i r (j mod Ns) / (Ns R)), takes an R-point DFT and writes
    // element r to (j / Ns) Ns R + (j mod Ns) + r Ns.  log2 n = 4 a + b: one
    // pass of radix 2^b (if b > 0), then a passes of radix 16.
    int Ns = 1;
    constexpr int B = LOGN & 3;
    if constexpr (B == 1) stockham_pass<2, LOGN>(grid, tw, Ns, t);
    if constexpr (B == 2) stockham_pass<4, LOGN>(grid, tw, Ns, t);
    if constexpr (B == 3) stockham_pass<8, LOGN>(grid, tw, Ns, t);
    Ns = 1 << B;
#pragma unroll 1
    for (; Ns < n; Ns *= 16) stockham_pass<16, LOGN>(grid, tw, Ns, t);

    // F_k = (2 pi / n) G_{(k - kc) mod n} / psi_hat(k - kc).
    float* fq = Fq + l * N;
    float* fu = Fu + l * N;
    for (int k = t; k < N; k += kThreads) {
        const float2 g = grid[swz((k - kc) & (n - 1))];
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
                       p.d_nufft_rot, p.nufft_nocc, p.d_nufft_off, p.d_nufft_ent, p.d_nufft_tw,        \
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
