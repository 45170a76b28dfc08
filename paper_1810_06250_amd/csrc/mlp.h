// Launchers of the surrogate-network and gating kernels (mlp.hip, gate.hip).
#pragma once
#include "common.h"

hipError_t mlp_launch_input(const float* Q, const float* U, int64_t nvalid, int64_t nrows, int nchan,
                            const float* w, _Float16* X, int ldx, hipStream_t s);
hipError_t mlp_launch_gemm(bool atr, bool btr, const _Float16* A, int64_t lda, const _Float16* B,
                           int64_t ldb, int64_t M, int64_t N, int64_t K, float alpha,
                           const float* bias, bool relu, const float* mask, int64_t ldm, float* C32,
                           int64_t ldc, _Float16* C16, int64_t ldc16, hipStream_t s);
// Weight gradient C[m][n] = alpha sum_k A[k][m] B[k][n] (both operands
// K-major, the GEMM's transposed loads), split over K when M x N alone gives
// too few workgroups; part holds part_floats floats of partial sums, at most
// mlp_wgrad_part_floats(M N) are used.  Deterministic for a given K.
int64_t mlp_wgrad_part_floats(int64_t max_mn);
hipError_t mlp_launch_gemm_wgrad(const _Float16* A, int64_t lda, const _Float16* B, int64_t ldb,
                                 int64_t M, int64_t N, int64_t K, float alpha, float* C, int64_t ldc,
                                 float* part, int64_t part_floats, hipStream_t s);
hipError_t mlp_launch_head(const _Float16* H2, const float* Z2, int h2, const _Float16* W3,
                           const float* b3, int64_t nvalid, int64_t nrows, float phi_scale,
                           const float* phi_label, const float* det_label, float* loss_b,
                           float* g_out, float* dz2, _Float16* dz2_16, float* phi_hat, float* score,
                           hipStream_t s);
// Deterministic column reductions use a partial buffer of
// mlp_reduce_part_floats(ncols) floats.
int64_t mlp_reduce_part_floats(int64_t ncols);
hipError_t mlp_launch_head_wgrad(const float* g, const _Float16* H2, int h2, int64_t nb, float alpha,
                                 float* gW3, float* gb3, float* part, hipStream_t s);
hipError_t mlp_launch_colsum(const float* X, int64_t M, int64_t N, float alpha, float* out,
                             float* part, hipStream_t s);
hipError_t mlp_launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t mlp_launch_weights16(const float* p, int64_t nW1, int64_t nb1, int64_t nW2, int64_t nb2,
                                int64_t nW3, _Float16* w16, hipStream_t s);
hipError_t mlp_launch_mean(const float* x, int64_t n, float* out, hipStream_t s);
// Fused inference (hidden widths 256 and 256 only): phi_hat and score per LOS.
// It reads W1 and W2 from a copy in MFMA-fragment order of
// mlp_fused_frag_uint4(nin_pad) uint4, made from the half weights by
// mlp_launch_frag16 (W1 [256][nin_pad], W2 [256][256]).  unit_w: every channel
// weight is 1 (the weights are then not read).
bool mlp_fused_supported(int h1, int h2, int nin_pad);
int64_t mlp_fused_frag_uint4(int nin_pad);
hipError_t mlp_launch_frag16(const _Float16* W1, const _Float16* W2, int nin_pad, uint4* frag,
                             hipStream_t s);
hipError_t mlp_launch_infer_fused(const float* Q, const float* U, int64_t nlos, int nchan,
                                  const float* w, int nin_pad, const uint4* frag, const float* b1,
                                  const float* b2, const _Float16* W3, const float* b3,
                                  float phi_scale, float* phi_hat, float* score, bool unit_w,
                                  hipStream_t s);

// Gate (gate.hip).  Compaction works on blocks of 1024 lines of sight:
// counts needs gate_num_blocks(nlos) + 1 entries and ends holding the
// exclusive offsets and, at [nblocks], the number of gated lines of sight.
int64_t gate_num_blocks(int64_t nlos);
hipError_t gate_launch_compact(const float* phi_hat, const float* score, int64_t nlos, float tau,
                               float edge, int32_t* gated, int32_t* idx, float* amp,
                               int32_t* counts, int64_t* list, hipStream_t s);
hipError_t gate_launch_gather(const float* Q, const float* U, const int64_t* list, int64_t n,
                              int nchan, float* gQ, float* gU, hipStream_t s);
hipError_t gate_launch_scatter(const int64_t* list, int64_t n, const int32_t* gidx,
                               const float* gphi, const float* gamp, int32_t* idx, float* phi_pk,
                               float* amp, hipStream_t s);

// Training-data synthesis (train.hip).  Uniform ranges [lo, hi]; class
// thresholds f0 < f1 < f2 are the cumulative fractions of noise-only, one-
// screen and two-screen lines of sight (the rest are slabs).
struct TrainSpecDev {
    double f0, f1, f2;
    double p0_lo, p0_hi, phi_lo, phi_hi, w_lo, w_hi;
    double sigma;
};
hipError_t train_launch_spectra(const double* lambda2, int nchan, const TrainSpecDev& s, uint64_t seed,
                                int64_t first, int64_t nlos, float* Q, float* U, int32_t* cls,
                                float* truth, hipStream_t st);
hipError_t train_launch_labels(const int32_t* idx, const float* phi_pk, const float* amp, int64_t n,
                               float thr, float* phi_label, float* det_label, hipStream_t st);
