// Split-precision Faraday-depth transform on 16-bit MFMA with FP32 accumulation.
//
// Same real-form GEMM as the FP32 path (rows 2l + part of A, columns k of the
// generated phase tile B; see synth_fp32.hip).  Every operand value x is split
// into x = hi + lo in the 16-bit format (bfloat16 or IEEE half), and the
// product is accumulated as hi*hi + hi*lo + lo*hi, which restores close to
// FP32 accuracy; the lo*lo term (relative size 2^-18 for bfloat16) is dropped.
//
// MFMA: v_mfma_f32_32x32x16_{bf16,f16}.  One instruction contracts 16 k
// values = 8 channels x (Q part, U part).  Lane l supplies row (or column)
// l % 32 and the 8 k values of channel half l / 32, i.e. 16 bytes from LDS
// laid out as [half][row][4 channels x 2 parts].
//
// Workgroup tile: 128 LOS (256 rows) x 128 phi, 4 waves of 128 rows x 64
// cols (4 x 2 blocks of 32 x 32, 128 accumulators per lane).
#include "common.h"

namespace {

constexpr int MT = 128;
constexpr int ROWS = 2 * MT;
constexpr int NT = 128;
constexpr int KC = 8;

struct Smem {
    uint4 a_hi[2][ROWS];
    uint4 a_lo[2][ROWS];
    uint4 b_hi[2][NT];
    uint4 b_lo[2][NT];
};

template <bool FP16>
__device__ __forceinline__ void split2(float a, float b, uint32_t& hi, uint32_t& lo)
{
    if (FP16) split2_f16(a, b, hi, lo);
    else split2_bf16(a, b, hi, lo);
}

template <bool FP16>
__device__ __forceinline__ f32x16_t mfma16(uint4 a, uint4 b, f32x16_t c)
{
    if (FP16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a),
                                                      __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

template <int LAYOUT, bool FP16>
__global__ __launch_bounds__(256, 2) void synth_split_kernel(
    const float* __restrict__ Q, const float* __restrict__ U, int64_t nlos, int64_t ld,
    int nchan, int vec4, const double* __restrict__ bj, const float* __restrict__ wj, int nk,
    const double* __restrict__ phik, int nphi, int tiles_n, float K,
    float* __restrict__ Fq, float* __restrict__ Fu, float* __restrict__ Fabs,
    const float* __restrict__ los_scale)
{
    __shared__ Smem sm;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t tm = tile / tiles_n;
    const int tn = (int)(tile - tm * tiles_n);
    const int64_t l0 = tm * MT;
    const int n0 = tn * NT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    // B-generation role: channel 4 hB + cB, phi nB + 32 i.
    const int cB = t & 3, hB = (t >> 2) & 1, nB = t >> 3;
    double ph[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ph[i] = phik[n0 + nB + 32 * i];

    // A-pack role: LOS la, channel half hA (4 channels).
    const int la = t >> 1, hA = t & 1;
    const int64_t lg = l0 + la;
    const bool lvalid = lg < nlos;
    // FP16: per-LOS power-of-two scale keeping both halves of the split in
    // half precision's normal range (from the weighted data, K not applied);
    // undone exactly in the epilogue.
    const float lsc = FP16 && lvalid ? los_scale[lg] : 1.0f;

    f32x16_t acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    for (int ks = 0; ks < nk; ++ks) {
        const int j0 = ks * KC;
        // ---- A operand.
        const int ja = j0 + 4 * hA;
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
        uint32_t rh[4], rl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float x = (w[i] != 0.0f) ? w[i] * q[i] : 0.0f;
            float y = (w[i] != 0.0f) ? w[i] * u[i] : 0.0f;
            if (FP16) {
                x *= lsc;
                y *= lsc;
            }
            split2<FP16>(x, y, rh[i], rl[i]);
        }
        // ---- B operand.
        const double b = bj[j0 + 4 * hB + cB];
        uint32_t bh[4], bl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float c, s;
            phase_cos_sin(ph[i] * b, c, s);
            split2<FP16>(c, s, bh[i], bl[i]);
        }

        __syncthreads();
        sm.a_hi[hA][2 * la] = make_uint4(rh[0], rh[1], rh[2], rh[3]);
        sm.a_lo[hA][2 * la] = make_uint4(rl[0], rl[1], rl[2], rl[3]);
        sm.a_hi[hA][2 * la + 1] = make_uint4(swap_negate(rh[0]), swap_negate(rh[1]),
                                             swap_negate(rh[2]), swap_negate(rh[3]));
        sm.a_lo[hA][2 * la + 1] = make_uint4(swap_negate(rl[0]), swap_negate(rl[1]),
                                             swap_negate(rl[2]), swap_negate(rl[3]));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            reinterpret_cast<uint32_t*>(&sm.b_hi[hB][nB + 32 * i])[cB] = bh[i];
            reinterpret_cast<uint32_t*>(&sm.b_lo[hB][nB + 32 * i])[cB] = bl[i];
        }
        __syncthreads();

        // ---- MFMA.
        const int h = lane >> 5, r = lane & 31;
        uint4 ah[4], al[4], bhf[2], blf[2];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            ah[rb] = sm.a_hi[h][128 * wr + 32 * rb + r];
            al[rb] = sm.a_lo[h][128 * wr + 32 * rb + r];
        }
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            bhf[cb] = sm.b_hi[h][64 * wc + 32 * cb + r];
            blf[cb] = sm.b_lo[h][64 * wc + 32 * cb + r];
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                acc[rb][cb] = mfma16<FP16>(al[rb], bhf[cb], acc[rb][cb]);
                acc[rb][cb] = mfma16<FP16>(ah[rb], blf[cb], acc[rb][cb]);
                acc[rb][cb] = mfma16<FP16>(ah[rb], bhf[cb], acc[rb][cb]);
            }
    }

    // ---- Epilogue.
    const int half = lane >> 5, col = lane & 31;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int n = n0 + 64 * wc + 32 * cb + col;
#pragma unroll
            for (int v = 0; v < 16; v += 2) {
                const int row = 128 * wr + 32 * rb + 8 * (v >> 2) + 4 * half + (v & 3);
                const int64_t l = l0 + (row >> 1);
                if (l < nlos && n < nphi) {
                    float aq = acc[rb][cb][v], au = acc[rb][cb][v + 1];
                    if (FP16) {  // multiply by 2^-e of the scale 2^e: exact
                        const float inv = __builtin_ldexpf(1.0f, 1 - __builtin_amdgcn_frexp_expf(los_scale[l]));
                        aq *= inv;
                        au *= inv;
                    }
                    const float fq = K * aq;
                    const float fu = K * au;
                    Fq[l * nphi + n] = fq;
                    Fu[l * nphi + n] = fu;
                    if (Fabs) Fabs[l * nphi + n] = sqrtf(fq * fq + fu * fu);
                }
            }
        }
}

template <bool FP16>
hipError_t launch_t(const rmsynth_plan_s& p, const ExecArgs& a)
{
    const int tiles_n = (p.nphi + NT - 1) / NT;
    const int nk = (p.nchan + KC - 1) / KC;
    const int64_t tiles_m = (a.nlos + MT - 1) / MT;
    const int64_t blocks = tiles_m * tiles_n;
    if (blocks <= 0) return hipSuccess;
    const float K = (float)p.K;
    if (a.layout == RMSYNTH_LOS_MAJOR)
        hipLaunchKernelGGL((synth_split_kernel<RMSYNTH_LOS_MAJOR, FP16>), dim3((unsigned)blocks),
                           dim3(256), 0, a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, a.vec4 ? 1 : 0,
                           p.d_b, p.d_w, nk, p.d_phi, p.nphi, tiles_n, K, a.Fq, a.Fu, a.Fabs,
                           a.los_scale);
    else
        hipLaunchKernelGGL((synth_split_kernel<RMSYNTH_FREQ_MAJOR, FP16>), dim3((unsigned)blocks),
                           dim3(256), 0, a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, a.vec4 ? 1 : 0,
                           p.d_b, p.d_w, nk, p.d_phi, p.nphi, tiles_n, K, a.Fq, a.Fu, a.Fabs,
                           a.los_scale);
    return hipGetLastError();
}

}  // namespace

int64_t split_los_per_tile() { return MT; }

hipError_t launch_synth_split(const rmsynth_plan_s& p, const ExecArgs& a, int precision)
{
    return precision == RMSYNTH_SPLIT_FP16 ? launch_t<true>(p, a) : launch_t<false>(p, a);
}
