// Plain FP32 Faraday-depth transform on FP32 MFMA (v_mfma_f32_32x32x2_f32).
//
// Real form of eq. (11) as a GEMM (eqs. (15)-(16)):
//   rows  r = 2l + part of A: part 0 (Re F) holds (w Q_j, w U_j),
//                             part 1 (Im F) holds (w U_j, -w Q_j);
//   cols  k of B: (cos theta_jk, sin theta_jk), theta_jk = 2 phi_k a_j;
//   [Re F | Im F]_l,k = K sum_j row . col.
// The phase tile of B is generated into LDS for every channel step and never
// stored in HBM.  Each workgroup owns 64 LOS (128 rows) x 128 phi; its four
// waves own 64 rows x 64 cols each (2 x 2 blocks of 32 x 32).  One MFMA
// contracts one channel: lanes 0-31 carry the Q part, lanes 32-63 the U part.
#include "common.h"

namespace {

constexpr int MT = 64;            // LOS per tile
constexpr int ROWS = 2 * MT;      // A rows
constexpr int NT = 128;           // phi per tile
constexpr int KC = 8;             // channels per K-step
constexpr int RS = 2 * KC + 4;    // padded row stride (floats): [part][KC] + pad

struct Smem {
    float a[ROWS][RS];
    float b[NT][RS];
};

template <int LAYOUT>
__global__ __launch_bounds__(256, 2) void synth_fp32_kernel(
    const float* __restrict__ Q, const float* __restrict__ U, int64_t nlos, int64_t ld,
    int nchan, int vec4, const double* __restrict__ bj, const float* __restrict__ wj, int nk,
    const double* __restrict__ phik, int nphi, int tiles_n, float K,
    float* __restrict__ Fq, float* __restrict__ Fu, float* __restrict__ Fabs)
{
    __shared__ Smem sm;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t tm = tile / tiles_n;
    const int tn = (int)(tile - tm * tiles_n);
    const int64_t l0 = tm * MT;
    const int n0 = tn * NT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    // B-generation role: channel cB, phi nB + 32 i.
    const int cB = t & 7, nB = t >> 3;
    double ph[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ph[i] = phik[n0 + nB + 32 * i];

    // A-pack role: LOS la, channel quad qA, part rA.
    const int la = t >> 2, qA = (t >> 1) & 1, rA = t & 1;
    const int64_t lg = l0 + la;
    const bool lvalid = lg < nlos;

    f32x16_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    for (int ks = 0; ks < nk; ++ks) {
        const int j0 = ks * KC;
        // ---- A operand: weighted Q/U of 4 channels, one row part.
        const int ja = j0 + 4 * qA;
        float q[4], u[4];
        if (LAYOUT == RMSYNTH_LOS_MAJOR) {
            if (vec4 && lvalid && ja + 3 < nchan) {
                const float4 q4 = *reinterpret_cast<const float4*>(Q + lg * ld + ja);
                const float4 u4 = *reinterpret_cast<const float4*>(U + lg * ld + ja);
                q[0] = q4.x; q[1] = q4.y; q[2] = q4.z; q[3] = q4.w;
                u[0] = u4.x; u[1] = u4.y; u[2] = u4.z; u[3] = u4.w;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bool ok = lvalid && (ja + i) < nchan;
                    q[i] = ok ? Q[lg * ld + ja + i] : 0.0f;
                    u[i] = ok ? U[lg * ld + ja + i] : 0.0f;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool ok = lvalid && (ja + i) < nchan;
                q[i] = ok ? Q[(int64_t)(ja + i) * ld + lg] : 0.0f;
                u[i] = ok ? U[(int64_t)(ja + i) * ld + lg] : 0.0f;
            }
        }
        const float4 w4 = *reinterpret_cast<const float4*>(wj + ja);
        const float w[4] = {w4.x, w4.y, w4.z, w4.w};
        float p0[4], p1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float x = (w[i] != 0.0f) ? w[i] * q[i] : 0.0f;
            const float y = (w[i] != 0.0f) ? w[i] * u[i] : 0.0f;
            p0[i] = rA ? y : x;
            p1[i] = rA ? -x : y;
        }
        // ---- B operand: cos/sin of theta for 4 phi of one channel.
        const double b = bj[j0 + cB];
        float cs[4], sn[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) phase_cos_sin(ph[i] * b, cs[i], sn[i]);

        __syncthreads();
        {
            float* ar = &sm.a[2 * la + rA][0];
            *reinterpret_cast<float4*>(ar + 4 * qA) = make_float4(p0[0], p0[1], p0[2], p0[3]);
            *reinterpret_cast<float4*>(ar + KC + 4 * qA) = make_float4(p1[0], p1[1], p1[2], p1[3]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                sm.b[nB + 32 * i][cB] = cs[i];
                sm.b[nB + 32 * i][KC + cB] = sn[i];
            }
        }
        __syncthreads();

        // ---- MFMA: 2 x 2 blocks, 8 channels.
        const int part = lane >> 5, r = lane & 31;
#pragma unroll
        for (int cq = 0; cq < KC / 4; ++cq) {
            float4 af[2], bf[2];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
                af[rb] = *reinterpret_cast<const float4*>(&sm.a[64 * wr + 32 * rb + r][part * KC + 4 * cq]);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
                bf[cb] = *reinterpret_cast<const float4*>(&sm.b[64 * wc + 32 * cb + r][part * KC + 4 * cq]);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[rb].x, bf[cb].x, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[rb].y, bf[cb].y, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[rb].z, bf[cb].z, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[rb].w, bf[cb].w, acc[rb][cb], 0, 0, 0);
                }
        }
    }

    // ---- Epilogue: x K, planar phi-fastest store, optional |F|.
    const int half = lane >> 5, col = lane & 31;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int n = n0 + 64 * wc + 32 * cb + col;
#pragma unroll
            for (int v = 0; v < 16; v += 2) {
                const int row = 64 * wr + 32 * rb + 8 * (v >> 2) + 4 * half + (v & 3);
                const int64_t l = l0 + (row >> 1);
                if (l < nlos && n < nphi) {
                    const float fq = K * acc[rb][cb][v];
                    const float fu = K * acc[rb][cb][v + 1];
                    Fq[l * nphi + n] = fq;
                    Fu[l * nphi + n] = fu;
                    if (Fabs) Fabs[l * nphi + n] = sqrtf(fq * fq + fu * fu);
                }
            }
        }
}

}  // namespace

hipError_t launch_synth_fp32(const rmsynth_plan_s& p, const ExecArgs& a)
{
    const int tiles_n = (p.nphi + NT - 1) / NT;
    const int nk = (p.nchan + KC - 1) / KC;
    const int64_t tiles_m = (a.nlos + MT - 1) / MT;
    const int64_t blocks = tiles_m * tiles_n;
    if (blocks <= 0) return hipSuccess;
    const float K = (float)p.K;
    if (a.layout == RMSYNTH_LOS_MAJOR)
        hipLaunchKernelGGL(synth_fp32_kernel<RMSYNTH_LOS_MAJOR>, dim3((unsigned)blocks), dim3(256), 0,
                           a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, a.vec4 ? 1 : 0, p.d_b, p.d_w,
                           nk, p.d_phi, p.nphi, tiles_n, K, a.Fq, a.Fu, a.Fabs);
    else
        hipLaunchKernelGGL(synth_fp32_kernel<RMSYNTH_FREQ_MAJOR>, dim3((unsigned)blocks), dim3(256), 0,
                           a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, a.vec4 ? 1 : 0, p.d_b, p.d_w,
                           nk, p.d_phi, p.nphi, tiles_n, K, a.Fq, a.Fu, a.Fabs);
    return hipGetLastError();
}
