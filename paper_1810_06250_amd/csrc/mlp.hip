// Surrogate network that gates the fine-grid RM synthesis: input
// normalisation, FP16-MFMA GEMMs with fused epilogues (bias, ReLU, ReLU'
// masks), the two-output head with its loss and output gradient,
// deterministic reductions and Adam.
//
// Network (per line of sight, nin = 2 nchan padded to a multiple of 32):
//   x = [w Q | w U] / rms;  h1 = relu(W1 x + b1);  h2 = relu(W2 h1 + b2);
//   o = W3 h2 + b3,  o0 = phi_hat / phi_scale,  o1 = detection logit;
//   loss = mean_b [ BCE(sigmoid(o1), det) + det (o0 - phi / phi_scale)^2 ].
// x, h1, h2, the weights and the back-propagated dz are rounded to IEEE half
// for the matrix units (FP32 accumulation).  Backward works with the
// gradient of the batch SUM so that half-precision dz stays in the normal
// range; weight gradients are scaled by 1/batch in FP32.
#include "mlp.h"

#include <algorithm>

namespace {

typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));

// FP32 to half, the FP32 value rounded first: the empty asm keeps the
// compiler from fusing the multiply or add that produced x and the
// conversion into one mixed-precision FMA (a single rounding from the exact
// result), so every half below is the nearest half to an FP32 number, in the
// training kernels and in fused inference alike.
__device__ __forceinline__ _Float16 half_of(float x)
{
    asm volatile("" : "+v"(x));
    return (_Float16)x;
}

// ----------------------------------------------------------------- input
// One wave per row.  Rows b < nvalid: x = [w Q | w U] / rms (half), columns
// [2 nchan, ldx) zero.  Rows nvalid <= b < nrows: all zero (batch padding).
// A non-finite unflagged input makes the whole row non-finite.
__global__ __launch_bounds__(256) void input_kernel(const float* __restrict__ Q,
                                                    const float* __restrict__ U, int64_t nvalid,
                                                    int64_t nrows, int nchan,
                                                    const float* __restrict__ w,
                                                    _Float16* __restrict__ X, int ldx)
{
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= nrows) return;
    _Float16* x = X + b * ldx;
    if (b >= nvalid) {
        for (int j = lane; j < ldx; j += 64) x[j] = (_Float16)0.0f;
        return;
    }
    const float* q = Q + b * nchan;
    const float* u = U + b * nchan;
    float ss = 0.0f;
    for (int j = lane; j < nchan; j += 64) {
        const float a = w[j] == 0.0f ? 0.0f : w[j] * q[j];
        const float c = w[j] == 0.0f ? 0.0f : w[j] * u[j];
        ss = __builtin_fmaf(a, a, __builtin_fmaf(c, c, ss));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    const float inv = ss > 0.0f ? 1.0f / sqrtf(ss / (float)(2 * nchan))
                                : (ss == 0.0f ? 0.0f : ss);  // NaN stays NaN
    for (int j = lane; j < nchan; j += 64) {
        x[j] = half_of(w[j] == 0.0f ? 0.0f : w[j] * q[j] * inv);
        x[nchan + j] = half_of(w[j] == 0.0f ? 0.0f : w[j] * u[j] * inv);
    }
    for (int j = 2 * nchan + lane; j < ldx; j += 64) x[j] = (_Float16)0.0f;
}

// ----------------------------------------------------------------- GEMM
// C[m][n] = sum_k A(m,k) B(n,k), half inputs, FP32 accumulation.
//   A(m,k) = A[m*lda + k]  (ATR = false)   or  A[k*lda + m]  (ATR = true)
//   B(n,k) = B[n*ldb + k]  (BTR = false)   or  B[k*ldb + n]  (BTR = true)
// M, N multiples of 64, K a multiple of 32, all pointers 16-byte aligned with
// leading dimensions multiples of 8.  Workgroup tile 64 x 64 (four waves,
// one 32 x 32 block each), K-step 32 = two v_mfma_f32_32x32x16_f16.
// Epilogue:  z = alpha acc + bias[n];  if mask: z = mask[m][n] > 0 ? z : 0;
//            C32[m][n] = z;  C16[m][n] = relu ? max(z, 0) : z  (either NULL).
// Split K (weight gradients, where M x N alone gives too few workgroups):
// blockIdx.y of gridDim.y takes an even share of the K/32 steps and, with
// part given, stores its raw sums to part[blockIdx.y][m][n] (plane = M N
// floats each); reduce_split_kernel adds the planes in order.
constexpr int GT = 64, GK = 32, GRS = GK + 8;  // LDS row stride in halves
constexpr int64_t kMaxSplit = 16, kSplitCap = int64_t(1) << 22;  // split-K planes, floats

template <bool TR>
__device__ __forceinline__ void load_tile(const _Float16* __restrict__ P, int64_t ld, int64_t r0,
                                          int64_t k0, int t, uint4& v)
{
    if (!TR) v = *reinterpret_cast<const uint4*>(P + (r0 + (t >> 2)) * ld + k0 + (t & 3) * 8);
    else     v = *reinterpret_cast<const uint4*>(P + (k0 + (t >> 3)) * ld + r0 + (t & 7) * 8);
}

template <bool TR>
__device__ __forceinline__ void store_tile(_Float16 (*s)[GRS], int t, const uint4& v)
{
    if (!TR) {
        *reinterpret_cast<uint4*>(&s[t >> 2][(t & 3) * 8]) = v;
    } else {
        const f16x8_t h = __builtin_bit_cast(f16x8_t, v);
        const int k = t >> 3, r = (t & 7) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) s[r + i][k] = h[i];
    }
}

template <bool ATR, bool BTR>
__global__ __launch_bounds__(256) void gemm_kernel(
    const _Float16* __restrict__ A, int64_t lda, const _Float16* __restrict__ B, int64_t ldb,
    int64_t N, int64_t K, float alpha, const float* __restrict__ bias, int relu,
    const float* __restrict__ mask, int64_t ldm, float* __restrict__ C32, int64_t ldc,
    _Float16* __restrict__ C16, int64_t ldc16, float* __restrict__ part, int64_t plane)
{
    __shared__ _Float16 sa[GT][GRS];
    __shared__ _Float16 sb[GT][GRS];
    const int64_t tiles_n = N / GT;
    const int64_t m0 = (int64_t)(blockIdx.x / tiles_n) * GT;
    const int64_t n0 = (int64_t)(blockIdx.x % tiles_n) * GT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    f32x16_t acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    const int64_t ks = K / GK;
    const int64_t kb = (int64_t)blockIdx.y * ks / gridDim.y * GK;
    const int64_t ke = (int64_t)(blockIdx.y + 1) * ks / gridDim.y * GK;
    uint4 av, bv;
    load_tile<ATR>(A, lda, m0, kb, t, av);
    load_tile<BTR>(B, ldb, n0, kb, t, bv);
    for (int64_t k0 = kb; k0 < ke; k0 += GK) {
        __syncthreads();
        store_tile<ATR>(sa, t, av);
        store_tile<BTR>(sb, t, bv);
        __syncthreads();
        if (k0 + GK < ke) {
            load_tile<ATR>(A, lda, m0, k0 + GK, t, av);
            load_tile<BTR>(B, ldb, n0, k0 + GK, t, bv);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int kk = 16 * s + 8 * (lane >> 5);
            const uint4 a = *reinterpret_cast<const uint4*>(&sa[32 * wr + (lane & 31)][kk]);
            const uint4 b = *reinterpret_cast<const uint4*>(&sb[32 * wc + (lane & 31)][kk]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a),
                                                         __builtin_bit_cast(f16x8_t, b), acc, 0, 0, 0);
        }
    }
    // D layout of the 32x32 block: column = lane % 32, row = 8(v/4) + 4(lane/32) + v%4.
    const int64_t n = n0 + 32 * wc + (lane & 31);
    if (part) {
        float* __restrict__ P = part + (int64_t)blockIdx.y * plane;
#pragma unroll
        for (int v = 0; v < 16; ++v)
            P[(m0 + 32 * wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)) * N + n] = acc[v];
        return;
    }
    const float bn = bias ? bias[n] : 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int64_t m = m0 + 32 * wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        float z = __builtin_fmaf(alpha, acc[v], bn);
        if (mask && !(mask[m * ldm + n] > 0.0f)) z = 0.0f;
        if (C32) C32[m * ldc + n] = z;
        if (C16) C16[m * ldc16 + n] = half_of((relu && z < 0.0f) ? 0.0f : z);
    }
}

// ----------------------------------------------------------------- head
// One wave per row.  o = W3 h2 + b3 (half operands, FP32 sums in a fixed
// butterfly order).  Training (labels given), rows b < nvalid: per-row loss,
// output gradient g (of the batch sum), dz2 = (g W3) * (z2 > 0) as FP32 and
// half; rows nvalid <= b < nrows: dz2 = 0.  Inference: phi_hat = o0 phi_scale,
// score = sigmoid(o1) for rows b < nvalid.
__global__ __launch_bounds__(256) void head_kernel(
    const _Float16* __restrict__ H2, const float* __restrict__ Z2, int h2,
    const _Float16* __restrict__ W3, const float* __restrict__ b3, int64_t nvalid, int64_t nrows,
    float phi_scale, const float* __restrict__ phi_label, const float* __restrict__ det_label,
    float* __restrict__ loss_b, float* __restrict__ g_out, float* __restrict__ dz2,
    _Float16* __restrict__ dz2_16, float* __restrict__ phi_hat, float* __restrict__ score)
{
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= nrows) return;
    if (b >= nvalid) {
        if (phi_label) {
            for (int i = lane; i < h2; i += 64) {
                dz2[b * h2 + i] = 0.0f;
                dz2_16[b * h2 + i] = (_Float16)0.0f;
            }
        }
        return;
    }
    const _Float16* h = H2 + b * h2;
    float s0 = 0.0f, s1 = 0.0f;
    for (int i = lane; i < h2; i += 64) {
        const float hv = (float)h[i];
        s0 = __builtin_fmaf(hv, (float)W3[i], s0);
        s1 = __builtin_fmaf(hv, (float)W3[h2 + i], s1);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
    }
    const float o0 = s0 + b3[0], o1 = s1 + b3[1];
    if (!phi_label) {
        if (lane == 0) {
            phi_hat[b] = o0 * phi_scale;
            const float e = expf(-fabsf(o1));
            score[b] = o1 >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
        }
        return;
    }
    const float d = det_label[b];
    const float err = o0 - phi_label[b] / phi_scale;
    const float e = expf(-fabsf(o1));
    const float sig = o1 >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
    const float g0 = 2.0f * d * err, g1 = sig - d;
    if (lane == 0) {
        loss_b[b] = fmaxf(o1, 0.0f) + log1pf(e) - d * o1 + d * err * err;
        g_out[2 * b] = g0;
        g_out[2 * b + 1] = g1;
    }
    for (int i = lane; i < h2; i += 64) {
        float g = __builtin_fmaf(g0, (float)W3[i], g1 * (float)W3[h2 + i]);
        if (!(Z2[b * h2 + i] > 0.0f)) g = 0.0f;
        dz2[b * h2 + i] = g;
        dz2_16[b * h2 + i] = half_of(g);
    }
}

// Deterministic column reductions in two levels: workgroup (x, y) sums the
// rows of chunk y for 64 columns (four row phases, combined in a fixed
// order) into part[y][n]; reduce_parts then adds the chunks in order.
constexpr int RCH = 32;  // row chunks

// part[y][n] = sum over rows m of chunk y of X[m][n].
__global__ __launch_bounds__(256) void colsum_part_kernel(const float* __restrict__ X, int64_t M,
                                                          int64_t N, float* __restrict__ part)
{
    __shared__ float red[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t n = (int64_t)blockIdx.x * 64 + tx;
    const int64_t per = (M + RCH - 1) / RCH;
    const int64_t m0 = blockIdx.y * per, m1 = m0 + per < M ? m0 + per : M;
    float s = 0.0f;
    if (n < N)
        for (int64_t m = m0 + ty; m < m1; m += 4) s += X[m * N + n];
    red[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && n < N) part[blockIdx.y * N + n] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

// part[y][c h2 + i] = sum_b g[b][c] h2[b][i] and part[y][2 h2 + c] = sum_b g[b][c]
// over the rows b of chunk y.
__global__ __launch_bounds__(256) void head_wgrad_part_kernel(const float* __restrict__ g,
                                                              const _Float16* __restrict__ H2,
                                                              int h2, int64_t nb,
                                                              float* __restrict__ part)
{
    __shared__ float red[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int N = 2 * h2 + 2;
    const int n = blockIdx.x * 64 + tx;
    const int64_t per = (nb + RCH - 1) / RCH;
    const int64_t b0 = blockIdx.y * per, b1 = b0 + per < nb ? b0 + per : nb;
    float s = 0.0f;
    if (n < 2 * h2) {
        const int c = n / h2, i = n - c * h2;
        for (int64_t b = b0 + ty; b < b1; b += 4) s = __builtin_fmaf(g[2 * b + c], (float)H2[b * h2 + i], s);
    } else if (n < N) {
        const int c = n - 2 * h2;
        for (int64_t b = b0 + ty; b < b1; b += 4) s += g[2 * b + c];
    }
    red[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && n < N) part[blockIdx.y * N + n] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

// out[n] = alpha sum_y part[y][n] (chunks in order); with out2, columns
// n >= split go to out2[n - split].
__global__ void reduce_parts_kernel(const float* __restrict__ part, int64_t N, float alpha,
                                    float* __restrict__ out, int64_t split, float* __restrict__ out2)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int y = 0; y < RCH; ++y) s += part[y * N + n];
    if (out2 && n >= split) out2[n - split] = alpha * s;
    else out[n] = alpha * s;
}

// C[m][n] = alpha sum_y part[y][m][n] over the nsplit planes, in order.
__global__ void reduce_split_kernel(const float* __restrict__ part, int nsplit, int64_t N,
                                    int64_t plane, float alpha, float* __restrict__ C, int64_t ldc)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t i = (int64_t)blockIdx.y * N + n;
    float s = part[i];
    for (int y = 1; y < nsplit; ++y) s += part[y * plane + i];
    C[(int64_t)blockIdx.y * ldc + n] = alpha * s;
}

// Adam (Kingma & Ba, bias-corrected) on the FP32 master parameters.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float beta1, float beta2, float eps, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Half copies of W1, W2, W3 (the parameter block with its biases removed).
__global__ void weights16_kernel(const float* __restrict__ p, int64_t nW1, int64_t nb1,
                                 int64_t nW2, int64_t nb2, int64_t nW3, _Float16* __restrict__ w16)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nW1) w16[i] = (_Float16)p[i];
    else if (i < nW1 + nW2) w16[i] = (_Float16)p[i + nb1];
    else if (i < nW1 + nW2 + nW3) w16[i] = (_Float16)p[i + nb1 + nb2];
}

// Mean of n values in one workgroup, fixed summation order.
__global__ __launch_bounds__(256) void mean_kernel(const float* __restrict__ x, int64_t n,
                                                   float* __restrict__ out)
{
    __shared__ float part[256];
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0] / (float)n;
}

// ----------------------------------------------------------------- fused inference
// One workgroup per 64 LOS, hidden widths 256 and 256.  Thread t loads row
// t / 4, inputs (t % 4) * 8 .. + 7 of every 32-wide K-chunk.  Pass 1 over the
// row accumulates sum (w Q)^2 + (w U)^2 (the four threads of a row combine
// theirs by shuffles, a fixed order); pass 2 streams the same chunks again
// (mostly from L2/MALL) two chunks ahead of their use, normalises and rounds
// them to half on their way into LDS, and feeds layer 1; layer 2 reads the
// half h1 tile from LDS; the head reduces over lanes and waves.  Weights come
// in MFMA-fragment order (frag16_kernel), so each fragment is one contiguous
// 1 KB read per wave, two K-chunks ahead of its use.  No activation leaves
// the CU.  Three workgroups share a CU (46 KB of LDS, at most 168 VGPRs
// each), so that loads of one overlap the matrix work of the others.
// VEC: nchan % 32 == 0 (so nin_pad = 2 nchan) and 16-byte aligned rows, so
// every chunk lies in Q or in U and loads as two float4.  UNITW: every channel
// weight is 1, so none are loaded.
constexpr int FR = 64;                 // LOS per workgroup
constexpr int FH = 256;                // hidden width
constexpr int FHS = FH + 8;            // LDS row stride of h1 (halves)

// Fragment order of an N x K half matrix W (row n at W + n ldw): fragment
// (b, s) covers rows 32 b .. + 31 and columns 16 s .. + 15 and is 64 uint4,
// lane l holding row 32 b + (l & 31), columns 16 s + 8 (l >> 5) .. + 7 (the
// B operand of v_mfma_f32_32x32x16_f16), at out[(b K/16 + s) 64 + l].
__global__ void frag16_kernel(const _Float16* __restrict__ W, int64_t N, int64_t K, int64_t ldw,
                              uint4* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ks = K / 16;
    if (i >= (N / 32) * ks * 64) return;
    const int l = (int)(i & 63);
    const int64_t f = i >> 6, b = f / ks, sl = f - b * ks;
    const int64_t n = 32 * b + (l & 31), k = 16 * sl + 8 * (l >> 5);
    out[i] = *reinterpret_cast<const uint4*>(W + n * ldw + k);
}

template <bool VEC, bool UNITW>
__global__ __launch_bounds__(256, 3) void infer_fused_kernel(
    const float* __restrict__ Q, const float* __restrict__ U, int64_t nlos, int nchan,
    const float* __restrict__ w, int nin_pad, const uint4* __restrict__ W1f,
    const float* __restrict__ b1, const uint4* __restrict__ W2f, const float* __restrict__ b2,
    const _Float16* __restrict__ W3, const float* __restrict__ b3, float phi_scale,
    float* __restrict__ phi_hat, float* __restrict__ score)
{
    __shared__ _Float16 sx[2][FR][GRS];  // K-chunks of the input tile, double buffered
    __shared__ _Float16 sh[FR][FHS];     // h1
    __shared__ float part[4][FR][2];     // head partial sums per wave
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t r0 = (int64_t)blockIdx.x * FR;
    const int lrow = t >> 2, lk = (t & 3) * 8;
    // Rows past the end read the last LOS (in bounds); their outputs are never stored.
    const int64_t ll = r0 + lrow < nlos ? r0 + lrow : nlos - 1;
    const float* qrow = Q + ll * nchan;
    const float* urow = U + ll * nchan;
    const int nin = 2 * nchan;
    const int nch = nin_pad / GK;

    // The thread's 8 inputs of chunk k0 (raw data) and their channel weights.
    // VEC: nin is a multiple of 64, so nin_pad = nin and every chunk is data.
    struct In {
        float v[8], wv[8];
    };
    auto load = [&](int k0) -> In {
        In x;
        if (VEC) {
            const bool inq = k0 < nchan;
            const int j = (inq ? k0 : k0 - nchan) + lk;
            const float* src = (inq ? qrow : urow) + j;
            const float4 a = *reinterpret_cast<const float4*>(src);
            const float4 b = *reinterpret_cast<const float4*>(src + 4);
            const float4 c = UNITW ? make_float4(1.0f, 1.0f, 1.0f, 1.0f)
                                   : *reinterpret_cast<const float4*>(w + j);
            const float4 d = UNITW ? make_float4(1.0f, 1.0f, 1.0f, 1.0f)
                                   : *reinterpret_cast<const float4*>(w + j + 4);
            x.v[0] = a.x; x.v[1] = a.y; x.v[2] = a.z; x.v[3] = a.w;
            x.v[4] = b.x; x.v[5] = b.y; x.v[6] = b.z; x.v[7] = b.w;
            x.wv[0] = c.x; x.wv[1] = c.y; x.wv[2] = c.z; x.wv[3] = c.w;
            x.wv[4] = d.x; x.wv[5] = d.y; x.wv[6] = d.z; x.wv[7] = d.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + lk + e;
                const int j = k < nchan ? k : k - nchan;
                const bool ok = k < nin;
                x.v[e] = ok ? (k < nchan ? qrow[j] : urow[j]) : 0.0f;
                x.wv[e] = ok ? w[j] : 0.0f;
            }
        }
        return x;
    };

    // Pass 1: sum of squares of the weighted inputs of the row, chunks in
    // order (six in flight: the accumulators are not live yet).
    float ss = 0.0f;
    {
        int c = 0;
        for (; c + 6 <= nch; c += 6) {
            In x[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) x[i] = load((c + i) * GK);
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float a = x[i].wv[e] == 0.0f ? 0.0f : x[i].wv[e] * x[i].v[e];
                    ss = __builtin_fmaf(a, a, ss);
                }
        }
        for (; c < nch; ++c) {
            const In x0 = load(c * GK);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float a = x0.wv[e] == 0.0f ? 0.0f : x0.wv[e] * x0.v[e];
                ss = __builtin_fmaf(a, a, ss);
            }
        }
    }
    ss += __shfl_xor(ss, 1, 64);
    ss += __shfl_xor(ss, 2, 64);
    const float inv = ss > 0.0f ? 1.0f / sqrtf(ss / (float)nin) : (ss == 0.0f ? 0.0f : ss);

    const int r = lane & 31, hsel = lane >> 5;
    const int ncol = 64 * wave;              // this wave's 64 hidden units
    f32x16_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    // B fragments of K-chunk k0 (two 16-wide slices) for the wave's two
    // 32-unit blocks.
    auto wfrag = [&](const uint4* Wf, int ks, int k0, uint4 (&bv)[2][2]) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int sl = 0; sl < 2; ++sl)
                bv[cb][sl] = Wf[((int64_t)(2 * wave + cb) * ks + (k0 >> 4) + sl) * 64 + lane];
    };
    auto copy = [](uint4 (&d)[2][2], const uint4 (&s)[2][2]) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) d[cb][sl] = s[cb][sl];
    };
    auto stage = [&](int buf, const In& x) {
        f16x8_t xv;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            xv[e] = half_of(x.wv[e] == 0.0f ? 0.0f : x.wv[e] * x.v[e] * inv);
        *reinterpret_cast<f16x8_t*>(&sx[buf][lrow][lk]) = xv;
    };
    // Pass 2: layer 1.  Chunk c is contracted from sx[buf]; chunk c + 1 is
    // already in registers and staged at the end; chunk c + 2 (data and
    // weights) loads meanwhile.
    const int ks1 = nin_pad / 16;
    {
        In xn = load(0), xf;
        uint4 bv[2][2], b1n[2][2], b2n[2][2];
        stage(0, xn);
        wfrag(W1f, ks1, 0, bv);
        if (nch > 1) {
            xn = load(GK);
            wfrag(W1f, ks1, GK, b1n);
        }
        __syncthreads();
        int buf = 0;
        for (int c = 0; c < nch; ++c) {
            if (c + 2 < nch) {
                xf = load((c + 2) * GK);
                wfrag(W1f, ks1, (c + 2) * GK, b2n);
            }
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const uint4 a = *reinterpret_cast<const uint4*>(&sx[buf][32 * rb + r][16 * sl + 8 * hsel]);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, bv[cb][sl]),
                            acc[rb][cb], 0, 0, 0);
                }
            }
            if (c + 1 < nch) stage(buf ^ 1, xn);
            copy(bv, b1n);
            copy(b1n, b2n);
            xn = xf;
            __syncthreads();
            buf ^= 1;
        }
    }
    // The first two W2 chunks load while h1 is written.
    constexpr int ks2 = FH / 16, nch2 = FH / GK;
    uint4 w2a[2][2], w2b[2][2];
    wfrag(W2f, ks2, 0, w2a);
    wfrag(W2f, ks2, GK, w2b);
    // h1 = relu(z1 + b1) as half into LDS.
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int n = ncol + 32 * cb + r;
        const float bn = b1[n];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int m = 32 * rb + 8 * (v >> 2) + 4 * hsel + (v & 3);
                const float z = __builtin_fmaf(1.0f, acc[rb][cb][v], bn);
                sh[m][n] = half_of(z < 0.0f ? 0.0f : z);
                acc[rb][cb][v] = 0.0f;
            }
    }
    __syncthreads();

    // Layer 2 from the h1 tile, W2 fragments two chunks ahead.
    {
        uint4 bv[2][2], b1n[2][2], b2n[2][2];
        copy(bv, w2a);
        copy(b1n, w2b);
#pragma unroll
        for (int c = 0; c < nch2; ++c) {
            if (c + 2 < nch2) wfrag(W2f, ks2, (c + 2) * GK, b2n);
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const uint4 a = *reinterpret_cast<const uint4*>(&sh[32 * rb + r][c * GK + 16 * sl + 8 * hsel]);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, bv[cb][sl]),
                            acc[rb][cb], 0, 0, 0);
                }
            }
            copy(bv, b1n);
            copy(b1n, b2n);
        }
    }
    // Head: h2 = relu(z2 + b2) rounded to half, dotted with the two rows of W3.
    float p0[2][16], p1[2][16];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 16; ++v) p0[rb][v] = p1[rb][v] = 0.0f;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int n = ncol + 32 * cb + r;
        const float bn = b2[n], w0 = (float)W3[n], w1 = (float)W3[FH + n];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float z = __builtin_fmaf(1.0f, acc[rb][cb][v], bn);
                const float h = (float)half_of(z < 0.0f ? 0.0f : z);
                p0[rb][v] = __builtin_fmaf(h, w0, p0[rb][v]);
                p1[rb][v] = __builtin_fmaf(h, w1, p1[rb][v]);
            }
    }
    // Sum over the 32 lanes that share a row, then over the four waves.
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            float a = p0[rb][v], b = p1[rb][v];
#pragma unroll
            for (int off = 16; off > 0; off >>= 1) {
                a += __shfl_xor(a, off, 64);
                b += __shfl_xor(b, off, 64);
            }
            if (r == 0) {
                const int m = 32 * rb + 8 * (v >> 2) + 4 * hsel + (v & 3);
                part[wave][m][0] = a;
                part[wave][m][1] = b;
            }
        }
    __syncthreads();
    if (t < FR && r0 + t < nlos) {
        const float o0 = ((part[0][t][0] + part[1][t][0]) + (part[2][t][0] + part[3][t][0])) + b3[0];
        const float o1 = ((part[0][t][1] + part[1][t][1]) + (part[2][t][1] + part[3][t][1])) + b3[1];
        phi_hat[r0 + t] = o0 * phi_scale;
        const float e = expf(-fabsf(o1));
        score[r0 + t] = o1 >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
    }
}

// One-pass inference for nchan = 2 PER (PER a multiple of 16), hidden widths
// 256/256, 16-byte aligned rows.  One workgroup per 64 LOS, two per CU.  The
// block is read from HBM once, every load in flight at once: sixteen lanes
// share a row, lane k reading float4 number k + 16 p of [Q | U], so each load
// instruction covers 256 contiguous bytes of four rows (a quarter of a row
// per thread touched one cache line per lane and was 11 % slower).  The row's
// sum of squares takes four shuffles, and the normalised halves go to an LDS
// tile holding the whole 64 x 2 nchan input.  Layer 1 then runs over all
// K-chunks with no barrier and no further input loads (only the weight
// fragments, two chunks ahead); h1 reuses the tile's LDS; layer 2 and the
// head are those of infer_fused_kernel, except that the head's sums over the
// 32 lanes of a half-wave transpose as they go (below).  Rounding points and
// outputs per LOS do not depend on the LOS's position in the batch.
template <int PER, bool UNITW>
__global__ __launch_bounds__(256, 2) void infer_onepass_kernel(
    const float* __restrict__ Q, const float* __restrict__ U, int64_t nlos,
    const float* __restrict__ w, const uint4* __restrict__ W1f, const float* __restrict__ b1,
    const uint4* __restrict__ W2f, const float* __restrict__ b2, const _Float16* __restrict__ W3,
    const float* __restrict__ b3, float phi_scale, float* __restrict__ phi_hat,
    float* __restrict__ score)
{
    constexpr int nchan = 2 * PER, nin = 4 * PER;
    constexpr int XS = nin + 8;                       // row stride (halves): odd in 16-byte units
    constexpr int XB = FR * XS * 2, HB = FR * FHS * 2;
    constexpr int TB = XB > HB ? XB : HB;
    __shared__ __align__(16) unsigned char smem[TB + 4 * FR * 2 * 4];
    _Float16 (*sx)[XS] = reinterpret_cast<_Float16 (*)[XS]>(smem);
    _Float16 (*sh)[FHS] = reinterpret_cast<_Float16 (*)[FHS]>(smem);
    float (*part)[FR][2] = reinterpret_cast<float (*)[FR][2]>(smem + TB);
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t r0 = (int64_t)blockIdx.x * FR;
    {
        // Wave wv holds rows 16 wv + 4 m + g (m = 0..3, g = lane >> 4); lane
        // k = lane & 15 holds float4 number f = k + 16 p (p < NP) of the row's
        // [Q | U], whose four values are x columns 4 f .. 4 f + 3.
        constexpr int NQ = nchan / 4, NP = nin / 64;
        const int g = lane >> 4, k = lane & 15;
        float v[PER];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            // Rows past the end read the last LOS (in bounds); their outputs are never stored.
            const int64_t rr = r0 + 16 * wave + 4 * m + g;
            const int64_t ll = rr < nlos ? rr : nlos - 1;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int f = k + 16 * p;
                const float* row = (f < NQ ? Q : U) + ll * nchan;
                const float4 a = reinterpret_cast<const float4*>(row)[f < NQ ? f : f - NQ];
                float* d = &v[4 * (m * NP + p)];
                d[0] = a.x; d[1] = a.y; d[2] = a.z; d[3] = a.w;
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            float ss = 0.0f;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int f = k + 16 * p;
                const float4 wv = UNITW ? make_float4(1.0f, 1.0f, 1.0f, 1.0f)
                                        : reinterpret_cast<const float4*>(w)[f < NQ ? f : f - NQ];
                const float ww[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float& x = v[4 * (m * NP + p) + e];
                    const float a = ww[e] == 0.0f ? 0.0f : ww[e] * x;
                    x = a;
                    ss = __builtin_fmaf(a, a, ss);
                }
            }
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) ss += __shfl_xor(ss, off, 64);
            const float inv = ss > 0.0f ? 1.0f / sqrtf(ss / (float)nin) : (ss == 0.0f ? 0.0f : ss);
            const int row = 16 * wave + 4 * m + g;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                f16x4_t xv;
#pragma unroll
                for (int e = 0; e < 4; ++e) xv[e] = half_of(v[4 * (m * NP + p) + e] * inv);
                *reinterpret_cast<f16x4_t*>(&sx[row][4 * (k + 16 * p)]) = xv;
            }
        }
    }
    __syncthreads();

    const int r = lane & 31, hsel = lane >> 5;
    const int ncol = 64 * wave;
    f32x16_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    auto wfrag = [&](const uint4* Wf, int ks, int k0, uint4 (&bv)[2][2]) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int sl = 0; sl < 2; ++sl)
                bv[cb][sl] = Wf[((int64_t)(2 * wave + cb) * ks + (k0 >> 4) + sl) * 64 + lane];
    };
    // Contract K-chunk c from the tile row block of `tile` with the weight
    // fragments in `cur`, after starting the loads of chunk c + 2 into `nxt`
    // (the set chunk c - 1 used).  Three register sets rotate, so a fragment
    // load is first waited on two chunks after it was issued.
    auto chunk = [&](const _Float16* tile, int ld, const uint4* Wf, int ks, int nch, int c,
                     uint4 (&cur)[2][2], uint4 (&nxt)[2][2]) {
        if (c + 2 < nch) wfrag(Wf, ks, (c + 2) * GK, nxt);
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const uint4 a = *reinterpret_cast<const uint4*>(tile + (32 * rb + r) * ld + c * GK + 16 * sl + 8 * hsel);
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                        __builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, cur[cb][sl]),
                        acc[rb][cb], 0, 0, 0);
            }
        }
    };
    auto layer = [&](const _Float16* tile, int ld, const uint4* Wf, int ks, int nch,
                     uint4 (&B0)[2][2], uint4 (&B1)[2][2], uint4 (&B2)[2][2]) {
        int c = 0;
        for (; c + 2 < nch; c += 3) {
            chunk(tile, ld, Wf, ks, nch, c, B0, B2);
            chunk(tile, ld, Wf, ks, nch, c + 1, B1, B0);
            chunk(tile, ld, Wf, ks, nch, c + 2, B2, B1);
        }
        if (c < nch) chunk(tile, ld, Wf, ks, nch, c, B0, B2);
        if (c + 1 < nch) chunk(tile, ld, Wf, ks, nch, c + 1, B1, B0);
    };
    // Layer 1 over the whole input tile.
    {
        constexpr int nch = nin / GK, ks1 = nin / 16;
        uint4 B0[2][2], B1[2][2], B2[2][2];
        wfrag(W1f, ks1, 0, B0);
        wfrag(W1f, ks1, GK, B1);
        layer(&sx[0][0], XS, W1f, ks1, nch, B0, B1, B2);
    }
    constexpr int ks2 = FH / 16, nch2 = FH / GK;
    uint4 w2a[2][2], w2b[2][2];
    wfrag(W2f, ks2, 0, w2a);
    wfrag(W2f, ks2, GK, w2b);
    __syncthreads();  // every wave is done with the input tile: h1 takes its LDS
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int n = ncol + 32 * cb + r;
        const float bn = b1[n];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int m = 32 * rb + 8 * (v >> 2) + 4 * hsel + (v & 3);
                const float z = __builtin_fmaf(1.0f, acc[rb][cb][v], bn);
                sh[m][n] = half_of(z < 0.0f ? 0.0f : z);
                acc[rb][cb][v] = 0.0f;
            }
    }
    __syncthreads();
    {
        uint4 B2[2][2];
        layer(&sh[0][0], FHS, W2f, ks2, nch2, w2a, w2b, B2);
    }
    float p0[2][16], p1[2][16];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 16; ++v) p0[rb][v] = p1[rb][v] = 0.0f;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int n = ncol + 32 * cb + r;
        const float bn = b2[n], w0 = (float)W3[n], w1 = (float)W3[FH + n];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float z = __builtin_fmaf(1.0f, acc[rb][cb][v], bn);
                const float h = (float)half_of(z < 0.0f ? 0.0f : z);
                p0[rb][v] = __builtin_fmaf(h, w0, p0[rb][v]);
                p1[rb][v] = __builtin_fmaf(h, w1, p1[rb][v]);
            }
    }
    // Each row's sum over the 32 lanes of its half-wave adds the pairs
    // (r, r ^ o) for o = 16, 8, 4, 2, 1.  At 256 or 288 channels the lanes
    // transpose as they add: at offset o a lane keeps the half of its 32 row
    // sums that bit o of its lane number selects and adds the partner's copy
    // of that half, so the five steps take 31 shuffles per output instead of
    // 160 and leave row q = r in lane r; the tree, and so every sum, is the
    // one of the plain butterfly (which the 128-channel form keeps: there it
    // measured faster).
    if constexpr (PER >= 128) {
        float a0[32], a1[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) { a0[q] = p0[q >> 4][q & 15]; a1[q] = p1[q >> 4][q & 15]; }
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) {   // a lane holds 2 o row sums before this step
            const bool hi = (r & o) != 0;
#pragma unroll
            for (int j = 0; j < o; ++j) {
                const float k0 = hi ? a0[j + o] : a0[j], s0 = hi ? a0[j] : a0[j + o];
                const float k1 = hi ? a1[j + o] : a1[j], s1 = hi ? a1[j] : a1[j + o];
                a0[j] = k0 + __shfl_xor(s0, o, 64);
                a1[j] = k1 + __shfl_xor(s1, o, 64);
            }
        }
        const int m = 32 * (r >> 4) + 8 * ((r & 15) >> 2) + 4 * hsel + (r & 3);
        part[wave][m][0] = a0[0];
        part[wave][m][1] = a1[0];
    } else {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                float a = p0[rb][v], b = p1[rb][v];
#pragma unroll
                for (int off = 16; off > 0; off >>= 1) {
                    a += __shfl_xor(a, off, 64);
                    b += __shfl_xor(b, off, 64);
                }
                if (r == 0) {
                    const int m = 32 * rb + 8 * (v >> 2) + 4 * hsel + (v & 3);
                    part[wave][m][0] = a;
                    part[wave][m][1] = b;
                }
            }
    }
    __syncthreads();
    if (t < FR && r0 + t < nlos) {
        const float o0 = ((part[0][t][0] + part[1][t][0]) + (part[2][t][0] + part[3][t][0])) + b3[0];
        const float o1 = ((part[0][t][1] + part[1][t][1]) + (part[2][t][1] + part[3][t][1])) + b3[1];
        phi_hat[r0 + t] = o0 * phi_scale;
        const float e = expf(-fabsf(o1));
        score[r0 + t] = o1 >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
    }
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t mlp_launch_input(const float* Q, const float* U, int64_t nvalid, int64_t nrows, int nchan,
                            const float* w, _Float16* X, int ldx, hipStream_t s)
{
    hipLaunchKernelGGL(input_kernel, dim3(blocks_for(nrows, 4)), dim3(256), 0, s, Q, U, nvalid, nrows,
                       nchan, w, X, ldx);
    return hipGetLastError();
}

hipError_t mlp_launch_gemm(bool atr, bool btr, const _Float16* A, int64_t lda, const _Float16* B,
                           int64_t ldb, int64_t M, int64_t N, int64_t K, float alpha,
                           const float* bias, bool relu, const float* mask, int64_t ldm, float* C32,
                           int64_t ldc, _Float16* C16, int64_t ldc16, hipStream_t s)
{
    if (M <= 0 || N <= 0 || K <= 0 || M % GT || N % GT || K % GK || lda % 8 || ldb % 8)
        return hipErrorInvalidValue;
    const int64_t blocks = (M / GT) * (N / GT);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const int r = relu ? 1 : 0;
#define MLP_GEMM(a, b)                                                                           \
    hipLaunchKernelGGL((gemm_kernel<a, b>), dim3((unsigned)blocks), dim3(256), 0, s, A, lda, B,   \
                       ldb, N, K, alpha, bias, r, mask, ldm, C32, ldc, C16, ldc16, nullptr,      \
                       (int64_t)0)
    if (!atr && !btr) MLP_GEMM(false, false);
    else if (!atr && btr) MLP_GEMM(false, true);
    else if (atr && btr) MLP_GEMM(true, true);
    else MLP_GEMM(true, false);
#undef MLP_GEMM
    return hipGetLastError();
}

int64_t mlp_wgrad_part_floats(int64_t max_mn) { return std::min<int64_t>(kMaxSplit * max_mn, kSplitCap); }

hipError_t mlp_launch_gemm_wgrad(const _Float16* A, int64_t lda, const _Float16* B, int64_t ldb,
                                 int64_t M, int64_t N, int64_t K, float alpha, float* C, int64_t ldc,
                                 float* part, int64_t part_floats, hipStream_t s)
{
    if (M <= 0 || N <= 0 || K <= 0 || M % GT || N % GT || K % GK || lda % 8 || ldb % 8)
        return hipErrorInvalidValue;
    const int64_t blocks = (M / GT) * (N / GT), plane = M * N;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    // Enough workgroups to cover the chip twice, at least two K-steps each.
    int64_t nsplit = std::min<int64_t>({kMaxSplit, (K / GK) / 2, (2 * 256 + blocks - 1) / blocks});
    nsplit = std::min<int64_t>(nsplit, part ? part_floats / plane : 0);
    if (nsplit <= 1 || M > 65535)  // the reduction's grid has one row of workgroups per m
        return mlp_launch_gemm(true, true, A, lda, B, ldb, M, N, K, alpha, nullptr, false, nullptr, 0,
                               C, ldc, nullptr, 0, s);
    hipLaunchKernelGGL((gemm_kernel<true, true>), dim3((unsigned)blocks, (unsigned)nsplit), dim3(256),
                       0, s, A, lda, B, ldb, N, K, 1.0f, nullptr, 0, nullptr, (int64_t)0, nullptr,
                       (int64_t)0, nullptr, (int64_t)0, part, plane);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(reduce_split_kernel, dim3(blocks_for(N, 256), (unsigned)M), dim3(256), 0, s,
                       part, (int)nsplit, N, plane, alpha, C, ldc);
    return hipGetLastError();
}

hipError_t mlp_launch_head(const _Float16* H2, const float* Z2, int h2, const _Float16* W3,
                           const float* b3, int64_t nvalid, int64_t nrows, float phi_scale,
                           const float* phi_label, const float* det_label, float* loss_b,
                           float* g_out, float* dz2, _Float16* dz2_16, float* phi_hat, float* score,
                           hipStream_t s)
{
    hipLaunchKernelGGL(head_kernel, dim3(blocks_for(nrows, 4)), dim3(256), 0, s, H2, Z2, h2, W3, b3,
                       nvalid, nrows, phi_scale, phi_label, det_label, loss_b, g_out, dz2, dz2_16,
                       phi_hat, score);
    return hipGetLastError();
}

int64_t mlp_reduce_part_floats(int64_t ncols) { return (int64_t)RCH * ncols; }

hipError_t mlp_launch_head_wgrad(const float* g, const _Float16* H2, int h2, int64_t nb, float alpha,
                                 float* gW3, float* gb3, float* part, hipStream_t s)
{
    const int N = 2 * h2 + 2;
    hipLaunchKernelGGL(head_wgrad_part_kernel, dim3(blocks_for(N, 64), RCH), dim3(256), 0, s, g, H2, h2,
                       nb, part);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, part,
                       (int64_t)N, alpha, gW3, (int64_t)(2 * h2), gb3);
    return hipGetLastError();
}

hipError_t mlp_launch_colsum(const float* X, int64_t M, int64_t N, float alpha, float* out,
                             float* part, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_part_kernel, dim3(blocks_for(N, 64), RCH), dim3(256), 0, s, X, M, N, part);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, part, N, alpha,
                       out, N, nullptr);
    return hipGetLastError();
}

hipError_t mlp_launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr,
                       beta1, beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t mlp_launch_weights16(const float* p, int64_t nW1, int64_t nb1, int64_t nW2, int64_t nb2,
                                int64_t nW3, _Float16* w16, hipStream_t s)
{
    hipLaunchKernelGGL(weights16_kernel, dim3(blocks_for(nW1 + nW2 + nW3, 256)), dim3(256), 0, s, p,
                       nW1, nb1, nW2, nb2, nW3, w16);
    return hipGetLastError();
}

hipError_t mlp_launch_mean(const float* x, int64_t n, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

bool mlp_fused_supported(int h1, int h2, int nin_pad) { return h1 == FH && h2 == FH && nin_pad % GK == 0; }

int64_t mlp_fused_frag_uint4(int nin_pad) { return (int64_t)FH * nin_pad / 8 + (int64_t)FH * FH / 8; }

hipError_t mlp_launch_frag16(const _Float16* W1, const _Float16* W2, int nin_pad, uint4* frag,
                             hipStream_t s)
{
    const int64_t n1 = (int64_t)FH * nin_pad / 8, n2 = (int64_t)FH * FH / 8;
    hipLaunchKernelGGL(frag16_kernel, dim3(blocks_for(n1, 256)), dim3(256), 0, s, W1, (int64_t)FH,
                       (int64_t)nin_pad, (int64_t)nin_pad, frag);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(frag16_kernel, dim3(blocks_for(n2, 256)), dim3(256), 0, s, W2, (int64_t)FH,
                       (int64_t)FH, (int64_t)FH, frag + n1);
    return hipGetLastError();
}

hipError_t mlp_launch_infer_fused(const float* Q, const float* U, int64_t nlos, int nchan,
                                  const float* w, int nin_pad, const uint4* frag, const float* b1,
                                  const float* b2, const _Float16* W3, const float* b3,
                                  float phi_scale, float* phi_hat, float* score, bool unit_w,
                                  hipStream_t s)
{
    const uint4* W1 = frag;
    const uint4* W2 = frag + (int64_t)FH * nin_pad / 8;
    if (nlos <= 0) return hipSuccess;
    const bool vec = nchan % GK == 0 && nin_pad == 2 * nchan && (uintptr_t)Q % 16 == 0 &&
                     (uintptr_t)U % 16 == 0 && (uintptr_t)w % 16 == 0;
    // Batches of whole 64-LOS workgroups within the grid limit (row offsets
    // keep 16-byte alignment: nchan % GK == 0 on the vector path).
    const int64_t max_los = max_items(FR, 256);
    for (int64_t l0 = 0; l0 < nlos; l0 += max_los) {
        const int64_t n = nlos - l0 < max_los ? nlos - l0 : max_los;
        const int64_t blocks = (n + FR - 1) / FR;
        const float* q = Q + l0 * nchan;
        const float* u = U + l0 * nchan;
#define RMS_ONEPASS(P)                                                                                  \
    do {                                                                                                \
        if (unit_w)                                                                                     \
            hipLaunchKernelGGL((infer_onepass_kernel<P, true>), dim3((unsigned)blocks), dim3(256), 0, s, q, \
                               u, n, w, W1, b1, W2, b2, W3, b3, phi_scale, phi_hat + l0, score + l0);   \
        else                                                                                            \
            hipLaunchKernelGGL((infer_onepass_kernel<P, false>), dim3((unsigned)blocks), dim3(256), 0, s, \
                               q, u, n, w, W1, b1, W2, b2, W3, b3, phi_scale, phi_hat + l0, score + l0); \
    } while (0)
        if (vec && nchan == 288) RMS_ONEPASS(144);
        else if (vec && nchan == 256) RMS_ONEPASS(128);
        else if (vec && nchan == 128) RMS_ONEPASS(64);
        else if (vec) {
            if (unit_w)
                hipLaunchKernelGGL((infer_fused_kernel<true, true>), dim3((unsigned)blocks), dim3(256), 0, s,
                                   q, u, n, nchan, w, nin_pad, W1, b1, W2, b2, W3, b3, phi_scale,
                                   phi_hat + l0, score + l0);
            else
                hipLaunchKernelGGL((infer_fused_kernel<true, false>), dim3((unsigned)blocks), dim3(256), 0,
                                   s, q, u, n, nchan, w, nin_pad, W1, b1, W2, b2, W3, b3, phi_scale,
                                   phi_hat + l0, score + l0);
        } else {
            hipLaunchKernelGGL((infer_fused_kernel<false, false>), dim3((unsigned)blocks), dim3(256), 0, s,
                               q, u, n, nchan, w, nin_pad, W1, b1, W2, b2, W3, b3, phi_scale,
                               phi_hat + l0, score + l0);
        }
#undef RMS_ONEPASS
        if (hipError_t e = hipGetLastError()) return e;
    }
    return hipSuccess;
}
