// C ABI of librmsynth: plan construction, validation and dispatch.
// The arithmetic of the method runs in the HIP kernels; the host forms K and
// lambda0^2 in FP64 (eq. (13)) and uploads the phase-generator tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "common.h"

thread_local std::string g_last_error;

int rms_fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int rms_ok()
{
    g_last_error.clear();
    return RMSYNTH_OK;
}

int rms_hip_fail(hipError_t e, const char* what)
{
    return rms_fail(RMSYNTH_EHIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {


void free_plan(rmsynth_plan_s* p)
{
    if (!p) return;
    void* bufs[] = {p->d_b, p->d_lambda2, p->d_w, p->d_phi, p->d_base, p->d_Tbf[0], p->d_Tbf[1],
                    p->d_Thf[0], p->d_Thf[1]};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

// The factored kernels evaluate F at phi_0 + k dphi, dphi = (phi_last -
// phi_0) / (nphi - 1), and report the caller's phi_k.  A grid is treated as
// uniform when the phase this moves, 2 |phi_k - (phi_0 + k dphi)| |a_j| of
// eq. (11), stays below kUniformPhaseTol radians for every k and every
// channel of non-zero weight (amax = max_j |a_j| over those channels).
constexpr double kUniformPhaseTol = 1e-8;

bool detect_uniform(const double* phi, int32_t nphi, double amax, double* phi0, double* dphi)
{
    *phi0 = phi[0];
    *dphi = nphi > 1 ? (phi[nphi - 1] - phi[0]) / (nphi - 1) : 0.0;
    double dev = 0.0;
    for (int32_t k = 0; k < nphi; ++k) dev = std::max(dev, std::fabs(phi[k] - (*phi0 + k * *dphi)));
    return 2.0 * dev * amax <= kUniformPhaseTol;
}

int build_factor_tables(rmsynth_plan_s* p)
{
    p->ftiles = (int32_t)((p->nphi + kFactorTile - 1) / kFactorTile);
    const size_t nT = (size_t)(p->nchan_pad / 4) * kFactorTile;
    hipError_t e;
    if ((e = hipMalloc(&p->d_base, sizeof(float2) * (size_t)p->ftiles * p->nchan_pad)) != hipSuccess ||
        (e = hipMalloc(&p->d_Tbf[0], sizeof(uint4) * nT)) != hipSuccess ||
        (e = hipMalloc(&p->d_Tbf[1], sizeof(uint4) * nT)) != hipSuccess ||
        (e = hipMalloc(&p->d_Thf[0], sizeof(uint4) * nT)) != hipSuccess ||
        (e = hipMalloc(&p->d_Thf[1], sizeof(uint4) * nT)) != hipSuccess)
        return rms_fail(RMSYNTH_ENOMEM, "rmsynth_plan: hipMalloc (phase tables): %s", hipGetErrorString(e));
    hipStream_t s = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
        return rms_hip_fail(e, "rmsynth_plan: hipStreamCreate");
    e = launch_factor_tables(*p, s);
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_plan: phase-table kernel");
    if (e2 != hipSuccess) return rms_hip_fail(e2, "rmsynth_plan: phase-table kernel");
    return RMSYNTH_OK;
}

int check_device(const rmsynth_plan_s* p)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rms_hip_fail(e, "hipGetDevice");
    if (dev != p->device)
        return rms_fail(RMSYNTH_EINVAL, "plan was created on device %d but device %d is current",
                    p->device, dev);
    return RMSYNTH_OK;
}

}  // namespace

extern "C" {

const char* rmsynth_last_error(void) { return g_last_error.c_str(); }

const char* rmsynth_version(void) { return "rmsynth-gfx950 0.1"; }

int rmsynth_plan(const double* lambda2, const double* weights, int32_t nchan, const double* phi,
                 int32_t nphi, double lambda0_sq, rmsynth_plan_t* out)
{
    if (!out) return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: out is NULL");
    *out = nullptr;
    if (!lambda2 || !weights || !phi) return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: NULL array");
    if (nchan < 1 || nchan > 65536) return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: nchan=%d", nchan);
    if (nphi < 1 || nphi > (1 << 20)) return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: nphi=%d", nphi);
    double sw = 0.0, swl = 0.0, lo = INFINITY, hi = -INFINITY;
    bool any_flagged = false;
    for (int32_t j = 0; j < nchan; ++j) {
        const double w = weights[j], l = lambda2[j];
        if (!std::isfinite(w) || w < 0.0)
            return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: weight %d is %g", j, w);
        if (!std::isfinite(l)) return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: lambda2 %d is %g", j, l);
        sw += w;
        swl += w * l;
        if (w == 0.0) any_flagged = true;
        if (w > 0.0) { lo = std::min(lo, l); hi = std::max(hi, l); }
    }
    if (!(sw > 0.0)) return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: sum of weights is %g", sw);
    for (int32_t k = 0; k < nphi; ++k)
        if (!std::isfinite(phi[k])) return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: phi %d is %g", k, phi[k]);
    if (!std::isnan(lambda0_sq) && !std::isfinite(lambda0_sq))
        return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan: lambda0_sq is %g", lambda0_sq);

    auto* p = new (std::nothrow) rmsynth_plan_s{};
    if (!p) return rms_fail(RMSYNTH_ENOMEM, "rmsynth_plan: host allocation");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { free_plan(p); return rms_hip_fail(e, "hipGetDevice"); }
    p->nchan = nchan;
    p->nphi = nphi;
    p->any_flagged = any_flagged;
    p->nchan_pad = (int32_t)round_up(nchan, kChanPad);
    p->nphi_pad = (int32_t)round_up(nphi, kPhiPad);
    p->K = 1.0 / sw;
    p->lambda0_sq = std::isnan(lambda0_sq) ? p->K * swl : lambda0_sq;
    p->fwhm_est = hi > lo ? 2.0 * std::sqrt(3.0) / (hi - lo) : INFINITY;
    std::vector<double> sorted(lambda2, lambda2 + nchan);
    std::sort(sorted.begin(), sorted.end());
    double gap = 0.0;
    for (int32_t j = 1; j < nchan; ++j) gap = std::max(gap, sorted[j] - sorted[j - 1]);
    p->phimax_est = gap > 0.0 ? std::sqrt(3.0) / gap : INFINITY;

    std::vector<double> hb(p->nchan_pad, 0.0), hphi(p->nphi_pad, 0.0);
    std::vector<float> hw(p->nchan_pad, 0.0f);
    for (int32_t j = 0; j < nchan; ++j) {
        hb[j] = (lambda2[j] - p->lambda0_sq) / M_PI;
        hw[j] = (float)weights[j];
    }
    std::copy(phi, phi + nphi, hphi.begin());
    for (int32_t k = 0; k < nphi; ++k) p->phi_absmax = std::max(p->phi_absmax, std::fabs(phi[k]));

    if ((e = hipMalloc(&p->d_b, sizeof(double) * p->nchan_pad)) != hipSuccess ||
        (e = hipMalloc(&p->d_w, sizeof(float) * p->nchan_pad)) != hipSuccess ||
        (e = hipMalloc(&p->d_phi, sizeof(double) * p->nphi_pad)) != hipSuccess ||
        (e = hipMalloc(&p->d_lambda2, sizeof(double) * nchan)) != hipSuccess) {
        free_plan(p);
        return rms_fail(RMSYNTH_ENOMEM, "rmsynth_plan: hipMalloc: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(p->d_b, hb.data(), sizeof(double) * p->nchan_pad, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_w, hw.data(), sizeof(float) * p->nchan_pad, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_phi, hphi.data(), sizeof(double) * p->nphi_pad, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_lambda2, lambda2, sizeof(double) * nchan, hipMemcpyHostToDevice)) != hipSuccess) {
        free_plan(p);
        return rms_hip_fail(e, "rmsynth_plan: hipMemcpy");
    }
    double amax = 0.0;
    for (int32_t j = 0; j < nchan; ++j)
        if (weights[j] > 0.0) amax = std::max(amax, std::fabs(lambda2[j] - p->lambda0_sq));
    p->uniform = detect_uniform(phi, nphi, amax, &p->phi0, &p->dphi);
    if (p->uniform) {
        if (int rc = build_factor_tables(p)) {
            free_plan(p);
            return rc;
        }
    }
    *out = p;
    return rms_ok();
}

int rmsynth_plan_info(rmsynth_plan_t p, double* K, double* lambda0_sq, double* fwhm_est,
                      double* phimax_est, int32_t* nchan, int32_t* nphi)
{
    if (!p) return rms_fail(RMSYNTH_EINVAL, "rmsynth_plan_info: plan is NULL");
    if (K) *K = p->K;
    if (lambda0_sq) *lambda0_sq = p->lambda0_sq;
    if (fwhm_est) *fwhm_est = p->fwhm_est;
    if (phimax_est) *phimax_est = p->phimax_est;
    if (nchan) *nchan = p->nchan;
    if (nphi) *nphi = p->nphi;
    return rms_ok();
}

int rmsynth_workspace_size(rmsynth_plan_t p, int64_t nlos, int32_t layout, int32_t precision,
                           size_t* bytes)
{
    if (!p || !bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_workspace_size: NULL argument");
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "rmsynth_workspace_size: nlos=%lld", (long long)nlos);
    if (layout != RMSYNTH_LOS_MAJOR && layout != RMSYNTH_FREQ_MAJOR)
        return rms_fail(RMSYNTH_EINVAL, "rmsynth_workspace_size: layout=%d", layout);
    if (precision < RMSYNTH_FP32 || precision > RMSYNTH_SPLIT_FP16)
        return rms_fail(RMSYNTH_EINVAL, "rmsynth_workspace_size: precision=%d", precision);
    *bytes = precision == RMSYNTH_SPLIT_FP16 ? (size_t)round_up(std::max<int64_t>(nlos, 1) * 4, 256) : 0;
    return rms_ok();
}

int rmsynth_rmsf(rmsynth_plan_t p, float* R_re, float* R_im, void* stream)
{
    if (!p || !R_re || !R_im) return rms_fail(RMSYNTH_EINVAL, "rmsynth_rmsf: NULL argument");
    if (int rc = check_device(p)) return rc;
    hipError_t e = launch_rmsf(*p, R_re, R_im, (hipStream_t)stream);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_rmsf launch");
    return rms_ok();
}

}  // extern "C"

namespace {

size_t scale_bytes(int64_t nlos) { return (size_t)round_up(std::max<int64_t>(nlos, 1) * 4, 256); }

bool fused_peaks(const rmsynth_plan_s* p, int32_t precision)
{
    return precision != RMSYNTH_FP32 && p->uniform;
}

int check_execute_args(const rmsynth_plan_s* p, int64_t nlos, int32_t layout, int32_t precision,
                       const char* who)
{
    if (!p) return rms_fail(RMSYNTH_EINVAL, "%s: plan is NULL", who);
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "%s: nlos=%lld", who, (long long)nlos);
    if (layout != RMSYNTH_LOS_MAJOR && layout != RMSYNTH_FREQ_MAJOR)
        return rms_fail(RMSYNTH_EINVAL, "%s: layout=%d", who, layout);
    if (precision < RMSYNTH_FP32 || precision > RMSYNTH_SPLIT_FP16)
        return rms_fail(RMSYNTH_EINVAL, "%s: precision=%d", who, precision);
    if (precision == RMSYNTH_SPLIT_FP16 && !p->uniform)
        return rms_fail(RMSYNTH_EUNSUPPORTED, "%s: the FP16 split needs a uniform phi grid", who);
    return RMSYNTH_OK;
}

// The transform in LOS batches (each grid within the dispatch limit, tiles of
// at least 64 LOS of 256 threads); with parts, the factored kernels also
// write their per-tile peaks.
int run_execute(const rmsynth_plan_s* p, const float* Q, const float* U, int64_t nlos, int32_t layout,
                int32_t precision, float* Fq, float* Fu, float* Fabs, float* scales, PeakPart* parts,
                hipStream_t stream, const char* who)
{
    const int64_t tiles_n = (p->nphi + 127) / 128;
    const int64_t max_los = max_los_tiled(tiles_n, 64, 256);
    for (int64_t l0 = 0; l0 < nlos;) {
        const int64_t n = std::min(nlos - l0, max_los);
        ExecArgs a{};
        if (layout == RMSYNTH_LOS_MAJOR) {
            a.Q = Q + l0 * p->nchan;
            a.U = U + l0 * p->nchan;
            a.ld = p->nchan;
            a.vec4 = (p->nchan % 4 == 0) && ((uintptr_t)Q % 16 == 0) && ((uintptr_t)U % 16 == 0);
        } else {
            a.Q = Q + l0;
            a.U = U + l0;
            a.ld = nlos;
            a.vec4 = false;
        }
        a.nlos = n;
        a.layout = layout;
        a.Fq = Fq + l0 * p->nphi;
        a.Fu = Fu + l0 * p->nphi;
        a.Fabs = Fabs ? Fabs + l0 * p->nphi : nullptr;
        a.los_scale = precision == RMSYNTH_SPLIT_FP16 ? scales + l0 : nullptr;
        a.peak_part = parts ? parts + l0 : nullptr;
        a.peak_part_ld = nlos;
        a.stream = stream;
        if (precision == RMSYNTH_SPLIT_FP16) {
            hipError_t e = launch_los_scale(*p, a);
            if (e != hipSuccess) return rms_hip_fail(e, who);
        }
        hipError_t e;
        if (precision == RMSYNTH_FP32) e = launch_synth_fp32(*p, a);
        else if (p->uniform) e = launch_synth_factored(*p, a, precision);
        else e = launch_synth_split(*p, a, precision);
        if (e != hipSuccess) return rms_hip_fail(e, who);
        l0 += n;
    }
    return RMSYNTH_OK;
}

}  // namespace

extern "C" {

int rmsynth_execute(rmsynth_plan_t p, const float* Q, const float* U, int64_t nlos, int32_t layout,
                    int32_t precision, float* Fq, float* Fu, float* Fabs, void* workspace,
                    size_t workspace_bytes, void* stream)
{
    if (int rc = check_execute_args(p, nlos, layout, precision, "rmsynth_execute")) return rc;
    if (nlos == 0) return rms_ok();
    if (!Q || !U || !Fq || !Fu) return rms_fail(RMSYNTH_EINVAL, "rmsynth_execute: NULL buffer");
    if (precision == RMSYNTH_SPLIT_FP16) {
        const size_t need = (size_t)round_up(nlos * 4, 256);
        if (!workspace || workspace_bytes < need)
            return rms_fail(RMSYNTH_EWORKSPACE, "rmsynth_execute: FP16 split needs %zu workspace bytes, got %zu",
                            need, workspace ? workspace_bytes : (size_t)0);
    }
    if (int rc = check_device(p)) return rc;
    if (int rc = run_execute(p, Q, U, nlos, layout, precision, Fq, Fu, Fabs,
                             static_cast<float*>(workspace), nullptr, (hipStream_t)stream,
                             "rmsynth_execute launch"))
        return rc;
    return rms_ok();
}

int rmsynth_execute_peaks_workspace_size(rmsynth_plan_t p, int64_t nlos, int32_t layout,
                                         int32_t precision, size_t* bytes)
{
    if (!bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_execute_peaks_workspace_size: bytes is NULL");
    if (int rc = check_execute_args(p, nlos, layout, precision, "rmsynth_execute_peaks_workspace_size"))
        return rc;
    size_t b = precision == RMSYNTH_SPLIT_FP16 ? scale_bytes(nlos) : 0;
    if (fused_peaks(p, precision))
        b += (size_t)round_up(std::max<int64_t>(nlos, 1) * factored_peak_parts(*p) * (int64_t)sizeof(PeakPart), 256);
    *bytes = b;
    return rms_ok();
}

int rmsynth_execute_peaks(rmsynth_plan_t p, const float* Q, const float* U, int64_t nlos,
                          int32_t layout, int32_t precision, float* Fq, float* Fu, float* Fabs,
                          int32_t* idx, float* phi_pk, float* amp, float* q_pk, float* u_pk,
                          void* workspace, size_t workspace_bytes, void* stream)
{
    const char* who = "rmsynth_execute_peaks";
    if (int rc = check_execute_args(p, nlos, layout, precision, who)) return rc;
    if (nlos == 0) return rms_ok();
    if (!Q || !U || !Fq || !Fu || !idx) return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    size_t need = 0;
    if (int rc = rmsynth_execute_peaks_workspace_size(p, nlos, layout, precision, &need)) return rc;
    if (need && (!workspace || workspace_bytes < need))
        return rms_fail(RMSYNTH_EWORKSPACE, "%s: needs %zu workspace bytes, got %zu", who, need,
                        workspace ? workspace_bytes : (size_t)0);
    if (int rc = check_device(p)) return rc;
    hipStream_t s = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    float* scales = reinterpret_cast<float*>(ws);
    const size_t sb = precision == RMSYNTH_SPLIT_FP16 ? scale_bytes(nlos) : 0;
    if (!fused_peaks(p, precision)) {
        if (int rc = run_execute(p, Q, U, nlos, layout, precision, Fq, Fu, Fabs, scales, nullptr, s, who))
            return rc;
        hipError_t e = launch_peaks(*p, Fq, Fu, nlos, idx, phi_pk, amp, q_pk, u_pk, s);
        if (e != hipSuccess) return rms_hip_fail(e, who);
        return rms_ok();
    }
    PeakPart* parts = reinterpret_cast<PeakPart*>(ws + sb);
    if (int rc = run_execute(p, Q, U, nlos, layout, precision, Fq, Fu, Fabs, scales, parts, s, who))
        return rc;
    hipError_t e = launch_peak_merge(*p, parts, nlos, Fq, Fu, idx, phi_pk, amp, q_pk, u_pk, s);
    if (e != hipSuccess) return rms_hip_fail(e, who);
    return rms_ok();
}

int rmsynth_peaks(rmsynth_plan_t p, const float* Fq, const float* Fu, int64_t nlos, int32_t* idx,
                  float* phi_pk, float* amp, float* q_pk, float* u_pk, void* stream)
{
    if (!p) return rms_fail(RMSYNTH_EINVAL, "rmsynth_peaks: plan is NULL");
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "rmsynth_peaks: nlos=%lld", (long long)nlos);
    if (nlos == 0) return rms_ok();
    if (!Fq || !Fu || !idx) return rms_fail(RMSYNTH_EINVAL, "rmsynth_peaks: NULL buffer");
    if (int rc = check_device(p)) return rc;
    hipError_t e = launch_peaks(*p, Fq, Fu, nlos, idx, phi_pk, amp, q_pk, u_pk, (hipStream_t)stream);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_peaks launch");
    return rms_ok();
}

int rmsynth_peak_angle(rmsynth_plan_t p, const float* phi_pk, const float* q_pk, const float* u_pk,
                       int64_t nlos, float* chi0, void* stream)
{
    if (!p) return rms_fail(RMSYNTH_EINVAL, "rmsynth_peak_angle: plan is NULL");
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "rmsynth_peak_angle: nlos=%lld", (long long)nlos);
    if (nlos == 0) return rms_ok();
    if (!phi_pk || !q_pk || !u_pk || !chi0) return rms_fail(RMSYNTH_EINVAL, "rmsynth_peak_angle: NULL buffer");
    if (int rc = check_device(p)) return rc;
    hipError_t e = launch_peak_angle(*p, phi_pk, q_pk, u_pk, nlos, chi0, (hipStream_t)stream);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_peak_angle launch");
    return rms_ok();
}

void rmsynth_destroy(rmsynth_plan_t p) { free_plan(p); }

}  // extern "C"
