// Shared device helpers and the host-side plan of librmsynth (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch_limits.h"
#include "rmsynth.h"

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Plan (host object).  The device tables are padded so that kernels can read
// whole channel steps and whole phi tiles without bounds checks:
//   d_b   [nchan_pad]  FP64 (lambda_j^2 - lambda0^2) / pi; 0 in the padding,
//                      so that 2 phi (lambda^2 - lambda0^2) = 2 pi phi b
//   d_w   [nchan_pad]  FP32 w_j; 0 in the padding (= flagged)
//   d_phi [nphi_pad]   FP64 phi_k; 0 in the padding
// ---------------------------------------------------------------------------
struct rmsynth_plan_s {
    int device;
    int32_t nchan, nphi, nchan_pad, nphi_pad;
    double K, lambda0_sq, fwhm_est, phimax_est;
    double phi_absmax;   // largest |phi_k| of the grid
    double* d_b;
    double* d_lambda2;   // [nchan] lambda^2 as given
    float* d_w;
    double* d_phi;
    // Factored phase tables, present when the phi grid is uniform
    // (phi_k = phi_0 + k dphi).  With tiles of kFactorTile phi,
    //   exp(-i theta_{j,k0+m}) = exp(-i theta_{j,k0}) * exp(-2i a_j m dphi):
    //   d_base [ftiles][nchan_pad] float2  K w_j (cos, sin)(theta_{j,k0}), k0 = tile start
    //   d_T{bf,hf}[hi/lo] [nchan_pad/4][kFactorTile] uint4: 4 channels x (cos, sin)
    //                   of 2 a_j m dphi, split into 16-bit hi/lo (bfloat16, half)
    bool uniform;
    double phi0, dphi;
    int32_t ftiles;
    float2* d_base;
    uint4* d_Tbf[2];
    uint4* d_Thf[2];
    bool any_flagged;    // some channel has weight 0
    // Channel-factored tables (synth_factored.hip, KF), present when the
    // contracted axis is uniform, b_j = kb0 + j kdb, and the output grid is
    // not (the adjoint plan of a uniform phi grid).  K-tiles of kKTile
    // channels, the lowest one starting kpad channels below channel 0:
    //   d_kw    [nchan_pad] float2  (w_j, 0)
    //   d_kbase [nphi_pad]  float2  K (cos, sin)(2 pi (kb0 - kpad kdb) g_k)
    //   d_krot  [nphi_pad]  float2  (cos, sin)(2 pi kKTile kdb g_k)
    //   d_K{bf,hf}[hi/lo] [kKTile/4][nphi_pad] uint4: 4 channels x (cos, sin)
    //                   of 2 pi i kdb g_k, i = 0 .. kKTile-1, split into hi/lo
    bool cuniform;
    double kb0, kdb;
    int32_t kpad;
    // Explicit split phase table (synth_factored.hip, ET), present when
    // neither axis is uniform and the table fits kEtabMaxBytes:
    //   d_ew [nchan_pad] float2  (K w_j, 0)
    //   d_E{bf,hf}[hi/lo] [nchan_pad/4][nphi_pad] uint4: 4 channels x (cos, sin)
    //                   of 2 pi b_j phi_k, split into hi/lo
    bool etab;
    float2* d_ew;
    uint4* d_Ebf[2];
    uint4* d_Ehf[2];
    float2* d_kw;
    float2* d_kbase;
    float2* d_krot;
    uint4* d_Kbf[2];
    uint4* d_Khf[2];
    // The adjoint transform's plan (axes exchanged, see build_adjoint_plan);
    // owned, NULL inside an adjoint plan itself.
    rmsynth_plan_s* adj;
    // NUFFT evaluation (uniform grids with nufft_n <= kNufftMaxGrid; nufft_n
    // = 0 otherwise): tables of nufft_plan.cpp.
    int32_t nufft_n, nufft_kc, nufft_nocc;
    float2* d_nufft_rot;    // [nchan]
    int* d_nufft_off;       // [nocc + 1] first entry of each occupied grid point
    int2* d_nufft_ent;      // [entries] ((channel << 13) | grid point, weight bits)
    float2* d_nufft_tw;     // [n]
    float* d_nufft_deconv;  // [nphi]
};

constexpr int kNufftWidth = 8;       // kernel width in grid cells
constexpr int kNufftMaxGrid = 8192;  // largest grid (LDS: 8 bytes per point)
constexpr int kNufftMaxChan = 4096;  // channels staged in LDS
int build_nufft_tables(rmsynth_plan_s* p, const double* lambda2, const double* weights);
size_t nufft_lds_bytes(const rmsynth_plan_s& p);
hipError_t launch_nufft(const rmsynth_plan_s& p, const float* Q, const float* U, int64_t nlos,
                        float* Fq, float* Fu, float* Fabs, hipStream_t s);

constexpr int kFactorTile = 128;  // phi per tile of the factored kernels
constexpr int kKTile = 96;        // channels per K-tile of the channel-factored form
constexpr size_t kEtabMaxBytes = size_t(256) << 20;  // largest explicit phase table (4 arrays)

constexpr int kChanPad = 32;    // channel padding granule (largest K-step)
constexpr int kPhiPad = 256;    // phi padding granule (largest phi tile)

// ---------------------------------------------------------------------------
// Phase generator.  theta = 2 phi a = 2 pi t with t = phi * (a / pi) in
// revolutions.  The reduction runs in FP64: q = nearest quarter turn,
// f = t - q/4 (exact, |f| <= 1/8), x = 2 pi f in [-pi/4, pi/4], rounded once
// to FP32.  sin x and cos x are the Taylor series of the functions with exact
// reciprocal-factorial coefficients, truncated after x^9 and x^10, whose
// truncation error on [-pi/4, pi/4] is below 2e-9 (under half an FP32 ulp);
// the quarter-turn index then selects sign and swap.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void phase_cos_sin(double t, float& c, float& s)
{
    const double q = __builtin_rint(4.0 * t);
    const double f = __builtin_fma(q, -0.25, t);
    const float x = (float)(f * 6.283185307179586476925286766559);
    const int n = (int)q & 3;
    const float x2 = x * x;
    float sp = 1.0f / 362880.0f;
    sp = __builtin_fmaf(sp, x2, -1.0f / 5040.0f);
    sp = __builtin_fmaf(sp, x2, 1.0f / 120.0f);
    sp = __builtin_fmaf(sp, x2, -1.0f / 6.0f);
    sp = __builtin_fmaf(sp * x2, x, x);
    float cp = -1.0f / 3628800.0f;
    cp = __builtin_fmaf(cp, x2, 1.0f / 40320.0f);
    cp = __builtin_fmaf(cp, x2, -1.0f / 720.0f);
    cp = __builtin_fmaf(cp, x2, 1.0f / 24.0f);
    cp = __builtin_fmaf(cp, x2, -0.5f);
    cp = __builtin_fmaf(cp, x2, 1.0f);
    const float cc = (n & 1) ? sp : cp;
    const float ss = (n & 1) ? cp : sp;
    c = ((n + 1) & 2) ? -cc : cc;
    s = (n & 2) ? -ss : ss;
}

// ---------------------------------------------------------------------------
// hi/lo splits.  x = hi + lo + r with hi = RNE(x), lo = RNE(x - hi) in the
// 16-bit format; x - hi is exact in FP32.  Pairs are packed into one dword,
// first element in the low half (the lower MFMA k slot).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pack2_bf16(float a, float b)
{
    bf16x2_t v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ void split2_bf16(float a, float b, uint32_t& hi, uint32_t& lo)
{
    hi = pack2_bf16(a, b);
    // Opaque to the optimiser: otherwise it re-converts a alone for hi << 16
    // (one more conversion per pair) instead of reusing hi.
    asm("" : "+v"(hi));
    const float ra = a - __uint_as_float(hi << 16);
    const float rb = b - __uint_as_float(hi & 0xffff0000u);
    lo = pack2_bf16(ra, rb);
}

__device__ __forceinline__ uint32_t pack2_f16(float a, float b)
{
    f16x2_t v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ void split2_f16(float a, float b, uint32_t& hi, uint32_t& lo)
{
    hi = pack2_f16(a, b);
    f16x2_t h = __builtin_bit_cast(f16x2_t, hi);
    lo = pack2_f16(a - (float)h[0], b - (float)h[1]);
}

// (x, y) packed -> (y, -x) packed: the imaginary-part row of the real form.
// Flipping the sign bit of a 16-bit float is exact in both formats.
__device__ __forceinline__ uint32_t swap_negate(uint32_t d)
{
    return __builtin_amdgcn_alignbit(d, d, 16) ^ 0x80000000u;
}

// Sub-grid peak (an extension; the paper reports the grid peak): the vertex
// of the parabola through (x0, y0), (x1, y1), (x2, y2), x0 < x1 < x2, y1 the
// grid maximum, in FP64.  A missing neighbour (NaN: the peak is at an end of
// the grid) or a parabola that does not open downwards leaves the grid values.
__device__ __forceinline__ void parabola_vertex(double x0, double y0, double x1, double y1,
                                                double x2, double y2, float* phi_fit,
                                                float* amp_fit)
{
    const double d0 = x0 - x1, d2 = x2 - x1;
    const double s0 = (y0 - y1) / d0, s2 = (y2 - y1) / d2;
    const double A = (s0 - s2) / (d0 - d2);
    const double B = s0 - A * d0;
    const double t = -B / (2.0 * A);
    const double top = y1 - B * B / (4.0 * A);
    const bool ok = __builtin_isfinite(y0) && __builtin_isfinite(y2) && __builtin_isfinite(t) &&
                    A < 0.0;
    *phi_fit = (float)(ok ? x1 + t : x1);
    *amp_fit = (float)(ok ? top : y1);
}

// Map a hardware workgroup id to a logical tile so that logical neighbours
// (the phi tiles of one LOS tile, which read the same Q/U rows) run on the
// same XCD: workgroups are dispatched round-robin over the 8 XCDs, each with
// its own L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t nblk)
{
    const int64_t per = nblk >> 3;
    if (bid < (per << 3)) return (bid & 7) * per + (bid >> 3);
    return bid;
}

// ---------------------------------------------------------------------------
// Kernel launchers (one per translation unit).  Each returns a hipError_t.
// ---------------------------------------------------------------------------
// Peak of |F|^2 of one LOS within 64 phi; idx = -2 marks a non-finite |F|^2.
struct PeakPart {
    float m;
    int32_t idx;
};

// The same for a transform that stores no F: the record also carries Fq, Fu
// at the peak and the |F|^2 around it that the sub-grid fit needs: at the
// neighbours inside the 64 phi (prv, nxt) and at both ends of the 64 (first,
// last), so that a neighbour across the boundary is found in the adjacent
// record.  -1 marks a value that is not there (before the first phi of the
// 64, or past the end of the grid).
struct PeakRec {
    float m;
    int32_t idx;
    float q, u;
    float prv, nxt;
    float first, last;
};

struct ExecArgs {
    const float* Q;
    const float* U;
    int64_t nlos;      // LOS in this launch
    int64_t ld;        // LOS-major: row stride (nchan); freq-major: plane stride
    int layout;
    bool vec4;         // 16-byte loads allowed
    float* Fq;
    float* Fu;
    float* Fabs;
    float* los_scale;  // FP16 split: per-LOS scale [nlos] in the workspace
    PeakPart* peak_part;  // factored kernels: per-(LOS, half phi tile) peaks, or NULL;
    int64_t peak_part_ld; // record (h, l) at peak_part[h * peak_part_ld + l]
    PeakRec* peak_rec;    // factored kernels, F not stored (Fq = Fu = NULL): full
                          // records at peak_rec[h * peak_part_ld + l], or NULL
    hipStream_t stream;
};

hipError_t launch_synth_fp32(const rmsynth_plan_s& p, const ExecArgs& a);
hipError_t launch_synth_split(const rmsynth_plan_s& p, const ExecArgs& a, int precision);
hipError_t launch_synth_factored(const rmsynth_plan_s& p, const ExecArgs& a, int precision);
hipError_t launch_los_scale(const rmsynth_plan_s& p, const ExecArgs& a);
hipError_t launch_factor_tables(const rmsynth_plan_s& p, hipStream_t s);
hipError_t launch_kfactor_tables(const rmsynth_plan_s& p, hipStream_t s);
hipError_t launch_synth_kfactored(const rmsynth_plan_s& p, const ExecArgs& a, int precision);
hipError_t launch_etable(const rmsynth_plan_s& p, hipStream_t s);
hipError_t launch_synth_etable(const rmsynth_plan_s& p, const ExecArgs& a, int precision);
hipError_t launch_peaks(const rmsynth_plan_s& p, const float* Fq, const float* Fu, int64_t nlos,
                        int32_t* idx, float* phi_pk, float* amp, float* q_pk, float* u_pk,
                        hipStream_t s);
hipError_t launch_rmsf(const rmsynth_plan_s& p, float* re, float* im, hipStream_t s);
hipError_t launch_peak_angle(const rmsynth_plan_s& p, const float* phi_pk, const float* q_pk,
                             const float* u_pk, int64_t nlos, float* chi0, hipStream_t s);
// Fused peaks of the factored kernels: records per LOS (one per half phi
// tile), and the merge of the records into the rmsynth_peaks outputs.
int factored_peak_parts(const rmsynth_plan_s& p);
hipError_t launch_peak_merge(const rmsynth_plan_s& p, const PeakPart* part, int64_t nlos,
                             const float* Fq, const float* Fu, int32_t* idx, float* phi_pk,
                             float* amp, float* q_pk, float* u_pk, hipStream_t s);
// Merge of full records (no F stored), with the sub-grid fit; records at
// rec[h * rec_ld + l] for the nlos LOS of a batch.
hipError_t launch_peak_merge_rec(const rmsynth_plan_s& p, const PeakRec* rec, int64_t rec_ld,
                                 int64_t nlos, int32_t* idx, float* phi_pk, float* amp,
                                 float* q_pk, float* u_pk, float* phi_fit, float* amp_fit,
                                 hipStream_t s);
// RM-CLEAN (rmclean.hip): workspace bytes for the doubled-grid RMSF and beam
// tables, and the launch (tables, then one wave per LOS).
constexpr int kRmcleanMaxPhi = 4096;  // residual of a LOS held in one wave's registers
size_t rmclean_table_bytes(const rmsynth_plan_s& p);
hipError_t launch_rmclean(const rmsynth_plan_s& p, const float* Fq, const float* Fu, int64_t nlos,
                          float gain, float cutoff, int max_iter, double fwhm, float* rq, float* ru,
                          float* cq, float* cu, float* Rq, float* Ru, int32_t* niter, void* ws,
                          hipStream_t s);
// Sub-grid fit from stored F around given peak indices (peaks.hip).
hipError_t launch_peak_fit(const rmsynth_plan_s& p, const float* Fq, const float* Fu,
                           const int32_t* idx, int64_t nlos, float* phi_fit, float* amp_fit,
                           hipStream_t s);

// The peaks-only search of rmsynth_search on a given workspace (any size down
// to one 128-LOS batch); `who` names the entry point in error messages.
int search_impl(const rmsynth_plan_s* p, const float* Q, const float* U, int64_t nlos,
                int32_t layout, int32_t precision, int32_t* idx, float* phi_pk, float* amp,
                float* q_pk, float* u_pk, float* phi_fit, float* amp_fit, void* workspace,
                size_t workspace_bytes, void* stream, const char* who);
// Workspace bytes rmsynth_search needs for n LOS (0 < n).
size_t search_workspace_bytes(const rmsynth_plan_s* p, int64_t n, int32_t precision);

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Error state shared by every entry point: set the thread's last-error text
// and return `code`; rms_ok clears it and returns RMSYNTH_OK.
int rms_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int rms_ok();
int rms_hip_fail(hipError_t e, const char* what);
