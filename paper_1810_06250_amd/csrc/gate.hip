// Gating kernels: per-LOS gate decision, order-preserving stream compaction
// of the gated lines of sight, gather of their spectra and scatter of their
// peaks back to the full output.
#include "mlp.h"

namespace {

constexpr int kPerThread = 4;
constexpr int kCompactBlock = 256 * kPerThread;  // elements per workgroup

__device__ __forceinline__ bool is_gated(float phi_hat, float score, float tau, float edge)
{
    if (!__builtin_isfinite(phi_hat) || !__builtin_isfinite(score)) return true;
    return score >= tau || fabsf(phi_hat) > edge;
}

// gated[l] = decision; non-gated lines of sight get idx = -1 and amp = NaN
// (phi_pk already holds phi_hat).  counts[block] = gated lines in the block.
__global__ __launch_bounds__(256) void gate_flag_kernel(const float* __restrict__ phi_hat,
                                                        const float* __restrict__ score,
                                                        int64_t nlos, float tau, float edge,
                                                        int32_t* __restrict__ gated,
                                                        int32_t* __restrict__ idx,
                                                        float* __restrict__ amp,
                                                        int32_t* __restrict__ counts)
{
    const int64_t base = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x * kPerThread;
    int c = 0;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
        const int64_t l = base + i;
        if (l < nlos) {
            const bool g = is_gated(phi_hat[l], score[l], tau, edge);
            gated[l] = g ? 1 : 0;
            if (!g) {
                idx[l] = -1;
                amp[l] = __builtin_nanf("");
            }
            c += g ? 1 : 0;
        }
    }
    __shared__ int part[256];
    part[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = part[0];
}

// Exclusive scan of counts[0..n) in place, total in counts[n]; one workgroup.
__global__ __launch_bounds__(256) void scan_counts_kernel(int32_t* __restrict__ counts, int64_t n)
{
    __shared__ int buf[256];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < n; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int v = i < n ? counts[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {  // Hillis-Steele inclusive scan
            const int add = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        const int c0 = carry;
        if (i < n) counts[i] = c0 + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255) carry = c0 + buf[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[n] = carry;
}

// list[offsets[block] + rank] = l for every gated l, in ascending order.
__global__ __launch_bounds__(256) void gate_list_kernel(const int32_t* __restrict__ gated,
                                                        int64_t nlos,
                                                        const int32_t* __restrict__ offsets,
                                                        int64_t* __restrict__ list)
{
    const int64_t base = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x * kPerThread;
    int f[kPerThread];
    int c = 0;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
        f[i] = (base + i < nlos) ? gated[base + i] : 0;
        c += f[i];
    }
    __shared__ int buf[256];
    buf[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t pos = (int64_t)offsets[blockIdx.x] + buf[threadIdx.x] - c;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i)
        if (f[i]) list[pos++] = base + i;
}

// One wave per gathered row: gQ[r][:] = Q[list[r]][:], same for U.
__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ Q,
                                                     const float* __restrict__ U,
                                                     const int64_t* __restrict__ list, int64_t n,
                                                     int nchan, float* __restrict__ gQ,
                                                     float* __restrict__ gU)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const int64_t l = list[r];
    for (int j = lane; j < nchan; j += 64) {
        gQ[r * nchan + j] = Q[l * nchan + j];
        gU[r * nchan + j] = U[l * nchan + j];
    }
}

__global__ void scatter_kernel(const int64_t* __restrict__ list, int64_t n,
                               const int32_t* __restrict__ gidx, const float* __restrict__ gphi,
                               const float* __restrict__ gamp, int32_t* __restrict__ idx,
                               float* __restrict__ phi_pk, float* __restrict__ amp)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t l = list[r];
    idx[l] = gidx[r];
    phi_pk[l] = gphi[r];
    amp[l] = gamp[r];
}

}  // namespace

int64_t gate_num_blocks(int64_t nlos) { return (nlos + kCompactBlock - 1) / kCompactBlock; }

hipError_t gate_launch_compact(const float* phi_hat, const float* score, int64_t nlos, float tau,
                               float edge, int32_t* gated, int32_t* idx, float* amp,
                               int32_t* counts, int64_t* list, hipStream_t s)
{
    const int64_t nb = gate_num_blocks(nlos);
    if (nb > max_blocks(256)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gate_flag_kernel, dim3((unsigned)nb), dim3(256), 0, s, phi_hat, score, nlos,
                       tau, edge, gated, idx, amp, counts);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(256), 0, s, counts, nb);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(gate_list_kernel, dim3((unsigned)nb), dim3(256), 0, s, gated, nlos, counts,
                       list);
    return hipGetLastError();
}

hipError_t gate_launch_gather(const float* Q, const float* U, const int64_t* list, int64_t n,
                              int nchan, float* gQ, float* gU, hipStream_t s)
{
    if ((n + 3) / 4 > max_blocks(256)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, Q, U, list, n,
                       nchan, gQ, gU);
    return hipGetLastError();
}

hipError_t gate_launch_scatter(const int64_t* list, int64_t n, const int32_t* gidx,
                               const float* gphi, const float* gamp, int32_t* idx, float* phi_pk,
                               float* amp, hipStream_t s)
{
    if ((n + 255) / 256 > max_blocks(256)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, list, n,
                       gidx, gphi, gamp, idx, phi_pk, amp);
    return hipGetLastError();
}
