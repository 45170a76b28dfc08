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

namespace {

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
        x[j] = (_Float16)(w[j] == 0.0f ? 0.0f : w[j] * q[j] * inv);
        x[nchan + j] = (_Float16)(w[j] == 0.0f ? 0.0f : w[j] * u[j] * inv);
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
constexpr int GT = 64, GK = 32, GRS = GK + 8;  // LDS row stride in halves

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
    _Float16* __restrict__ C16, int64_t ldc16)
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
    uint4 av, bv;
    load_tile<ATR>(A, lda, m0, 0, t, av);
    load_tile<BTR>(B, ldb, n0, 0, t, bv);
    for (int64_t k0 = 0; k0 < K; k0 += GK) {
        __syncthreads();
        store_tile<ATR>(sa, t, av);
        store_tile<BTR>(sb, t, bv);
        __syncthreads();
        if (k0 + GK < K) {
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
    const float bn = bias ? bias[n] : 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int64_t m = m0 + 32 * wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        float z = __builtin_fmaf(alpha, acc[v], bn);
        if (mask && !(mask[m * ldm + n] > 0.0f)) z = 0.0f;
        if (C32) C32[m * ldc + n] = z;
        if (C16) C16[m * ldc16 + n] = (_Float16)((relu && z < 0.0f) ? 0.0f : z);
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
        dz2_16[b * h2 + i] = (_Float16)g;
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
// t / 4, inputs (t % 4) * 8 .. + 7 of every 32-wide K-chunk, one chunk ahead
// of its use.  Pass 1 over the row accumulates sum (w Q)^2 + (w U)^2 (the
// four threads of a row combine theirs by shuffles, a fixed order); pass 2
// streams the same chunks again (mostly from L2/MALL), normalises and rounds
// them to half on their way into LDS, and feeds layer 1; layer 2 reads the
// half h1 tile from LDS; the head reduces over lanes and waves.  Weights are
// read from L2 straight into the B-operand registers.  No activation leaves
// the CU.  VEC: nchan % 32 == 0 and 16-byte aligned rows, so every chunk lies
// in Q or in U and loads as two float4.
constexpr int FR = 64;                 // LOS per workgroup
constexpr int FH = 256;                // hidden width
constexpr int FHS = FH + 8;            // LDS row stride of h1 (halves)

template <bool VEC>
__global__ __launch_bounds__(256, 2) void infer_fused_kernel(
    const float* __restrict__ Q, const float* __restrict__ U, int64_t nlos, int nchan,
    const float* __restrict__ w, int nin_pad, const _Float16* __restrict__ W1,
    const float* __restrict__ b1, const _Float16* __restrict__ W2, const float* __restrict__ b2,
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

    // The thread's 8 inputs of chunk k0 (raw data) and their channel weights.
    auto load = [&](int k0, float (&v)[8], float (&wv)[8]) {
        if (VEC) {
            const int k = k0 + lk;
            if (k0 < nin) {
                const float* src = k0 < nchan ? qrow + k : urow + (k - nchan);
                const float* ws = w + (k0 < nchan ? k : k - nchan);
                const float4 a = *reinterpret_cast<const float4*>(src);
                const float4 b = *reinterpret_cast<const float4*>(src + 4);
                const float4 c = *reinterpret_cast<const float4*>(ws);
                const float4 d = *reinterpret_cast<const float4*>(ws + 4);
                v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
                v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
                wv[0] = c.x; wv[1] = c.y; wv[2] = c.z; wv[3] = c.w;
                wv[4] = d.x; wv[5] = d.y; wv[6] = d.z; wv[7] = d.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = wv[e] = 0.0f;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + lk + e;
                const int j = k < nchan ? k : k - nchan;
                const bool ok = k < nin;
                v[e] = ok ? (k < nchan ? qrow[j] : urow[j]) : 0.0f;
                wv[e] = ok ? w[j] : 0.0f;
            }
        }
    };

    // Pass 1: sum of squares of the weighted inputs of the row.
    float ss = 0.0f;
    {
        float v[8], wv[8], vn[8], wn[8];
        load(0, v, wv);
        for (int k0 = 0; k0 < nin_pad; k0 += GK) {
            if (k0 + GK < nin_pad) load(k0 + GK, vn, wn);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float a = wv[e] == 0.0f ? 0.0f : wv[e] * v[e];
                ss = __builtin_fmaf(a, a, ss);
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                v[e] = vn[e];
                wv[e] = wn[e];
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

    // Pass 2: layer 1, chunk k0 contracted from sx[buf] while chunk k0 + 32 loads.
    auto wfrag = [&](const _Float16* W, int ld, int k0, uint4 (&bv)[2][2]) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int s = 0; s < 2; ++s)
                bv[cb][s] = *reinterpret_cast<const uint4*>(
                    W + (int64_t)(ncol + 32 * cb + r) * ld + k0 + 16 * s + 8 * hsel);
    };
    auto stage = [&](int buf, const float (&v)[8], const float (&wv)[8]) {
        f16x8_t xv;
#pragma unroll
        for (int e = 0; e < 8; ++e) xv[e] = (_Float16)(wv[e] == 0.0f ? 0.0f : wv[e] * v[e] * inv);
        *reinterpret_cast<f16x8_t*>(&sx[buf][lrow][lk]) = xv;
    };
    {
        float v[8], wv[8];
        uint4 bv[2][2], bn[2][2];
        load(0, v, wv);
        stage(0, v, wv);
        wfrag(W1, nin_pad, 0, bv);
        __syncthreads();
        int buf = 0;
        for (int k0 = 0; k0 < nin_pad; k0 += GK) {
            const bool more = k0 + GK < nin_pad;
            if (more) {
                load(k0 + GK, v, wv);
                wfrag(W1, nin_pad, k0 + GK, bn);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const uint4 a = *reinterpret_cast<const uint4*>(&sx[buf][32 * rb + r][16 * s + 8 * hsel]);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, bv[cb][s]),
                            acc[rb][cb], 0, 0, 0);
                }
            }
            if (more) {
                stage(buf ^ 1, v, wv);
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int s = 0; s < 2; ++s) bv[cb][s] = bn[cb][s];
            }
            __syncthreads();
            buf ^= 1;
        }
    }
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
                sh[m][n] = (_Float16)(z < 0.0f ? 0.0f : z);
                acc[rb][cb][v] = 0.0f;
            }
    }
    __syncthreads();

    // Layer 2 from the h1 tile, W2 fragments one chunk ahead.
    {
        uint4 bv[2][2], bn[2][2];
        wfrag(W2, FH, 0, bv);
        for (int k0 = 0; k0 < FH; k0 += GK) {
            const bool more = k0 + GK < FH;
            if (more) wfrag(W2, FH, k0 + GK, bn);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const uint4 a = *reinterpret_cast<const uint4*>(&sh[32 * rb + r][k0 + 16 * s + 8 * hsel]);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, bv[cb][s]),
                            acc[rb][cb], 0, 0, 0);
                }
            }
            if (more) {
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int s = 0; s < 2; ++s) bv[cb][s] = bn[cb][s];
            }
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
                const float h = (float)(_Float16)(z < 0.0f ? 0.0f : z);
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
                       ldb, N, K, alpha, bias, r, mask, ldm, C32, ldc, C16, ldc16)
    if (!atr && !btr) MLP_GEMM(false, false);
    else if (!atr && btr) MLP_GEMM(false, true);
    else if (atr && btr) MLP_GEMM(true, true);
    else MLP_GEMM(true, false);
#undef MLP_GEMM
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

hipError_t mlp_launch_infer_fused(const float* Q, const float* U, int64_t nlos, int nchan,
                                  const float* w, int nin_pad, const _Float16* W1, const float* b1,
                                  const _Float16* W2, const float* b2, const _Float16* W3,
                                  const float* b3, float phi_scale, float* phi_hat, float* score,
                                  hipStream_t s)
{
    const int64_t blocks = (nlos + FR - 1) / FR;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const bool vec = nchan % GK == 0 && (uintptr_t)Q % 16 == 0 && (uintptr_t)U % 16 == 0 &&
                     (uintptr_t)w % 16 == 0;
    if (vec)
        hipLaunchKernelGGL(infer_fused_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, Q, U, nlos,
                           nchan, w, nin_pad, W1, b1, W2, b2, W3, b3, phi_scale, phi_hat, score);
    else
        hipLaunchKernelGGL(infer_fused_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, Q, U,
                           nlos, nchan, w, nin_pad, W1, b1, W2, b2, W3, b3, phi_scale, phi_hat, score);
    return hipGetLastError();
}
