// C ABI of librmsynth: plan construction, validation and dispatch.
// The arithmetic of the method runs in the HIP kernels; the host forms K and
// lambda0^2 in FP64 (eq. (13)) and uploads the phase-generator tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
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
    free_plan(p->adj);
    void* bufs[] = {p->d_b, p->d_lambda2, p->d_w, p->d_phi, p->d_base, p->d_Tbf[0], p->d_Tbf[1],
                    p->d_Thf[0], p->d_Thf[1], p->d_nufft_rot, p->d_nufft_off, p->d_nufft_ent,
                    p->d_nufft_tw, p->d_nufft_deconv, p->d_kw, p->d_kbase, p->d_krot,
                    p->d_Kbf[0], p->d_Kbf[1], p->d_Khf[0], p->d_Khf[1], p->d_ew,
                    p->d_Ebf[0], p->d_Ebf[1], p->d_Ehf[0], p->d_Ehf[1]};
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

// The explicit split phase table of a plan whose axes are not uniform (the
// factored tables do not apply), when it fits kEtabMaxBytes; larger plans keep
// the per-element phase generator.
int build_etable(rmsynth_plan_s* p)
{
    const size_t nE = (size_t)(p->nchan_pad / 4) * p->nphi_pad;
    if (nE * sizeof(uint4) * 4 > kEtabMaxBytes) return RMSYNTH_OK;
    hipError_t e;
    if ((e = hipMalloc(&p->d_ew, sizeof(float2) * p->nchan_pad)) != hipSuccess ||
        (e = hipMalloc(&p->d_Ebf[0], sizeof(uint4) * nE)) != hipSuccess ||
        (e = hipMalloc(&p->d_Ebf[1], sizeof(uint4) * nE)) != hipSuccess ||
        (e = hipMalloc(&p->d_Ehf[0], sizeof(uint4) * nE)) != hipSuccess ||
        (e = hipMalloc(&p->d_Ehf[1], sizeof(uint4) * nE)) != hipSuccess)
        return rms_fail(RMSYNTH_ENOMEM, "rmsynth_plan: hipMalloc (phase table): %s", hipGetErrorString(e));
    hipStream_t s = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
        return rms_hip_fail(e, "rmsynth_plan: hipStreamCreate");
    e = launch_etable(*p, s);
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_plan: phase-table kernel");
    if (e2 != hipSuccess) return rms_hip_fail(e2, "rmsynth_plan: phase-table kernel");
    p->etab = true;
    p->ftiles = (int32_t)((p->nphi + kFactorTile - 1) / kFactorTile);  // peak records per LOS: 2 ftiles
    return RMSYNTH_OK;
}

// The plan of the adjoint transform (spectra from Faraday-depth components,
// eq. (4) as a sum over the grid, referred to lambda0^2):
//   P_lj = sum_k C_lk exp(+2i phi_k a_j),   a_j = lambda_j^2 - lambda0^2.
// It is the forward contraction with the roles of the two axes exchanged:
// the phi_k become the contracted "channels" (b = phi_k / pi, weight 1,
// K = 1) and -a_j the output grid, so exp(-2i (-a_j) phi_k) is the wanted
// exp(+2i phi_k a_j); the forward kernels run it unchanged.
int build_adjoint_plan(rmsynth_plan_s* p, const double* lambda2, const double* phi)
{
    auto* q = new (std::nothrow) rmsynth_plan_s{};
    if (!q) return rms_fail(RMSYNTH_ENOMEM, "rmsynth_plan: host allocation");
    p->adj = q;
    q->device = p->device;
    q->nchan = p->nphi;
    q->nphi = p->nchan;
    q->nchan_pad = (int32_t)round_up(q->nchan, kChanPad);
    q->nphi_pad = (int32_t)round_up(q->nphi, kPhiPad);
    q->K = 1.0;
    q->lambda0_sq = 0.0;
    std::vector<double> hb(q->nchan_pad, 0.0), hgrid(q->nphi_pad, 0.0);
    std::vector<float> hw(q->nchan_pad, 0.0f);
    double amax = 0.0;
    for (int32_t k = 0; k < p->nphi; ++k) {
        hb[k] = phi[k] / M_PI;
        hw[k] = 1.0f;
        amax = std::max(amax, std::fabs(phi[k]));
    }
    for (int32_t j = 0; j < p->nchan; ++j) hgrid[j] = -(lambda2[j] - p->lambda0_sq);
    hipError_t e;
    if ((e = hipMalloc(&q->d_b, sizeof(double) * q->nchan_pad)) != hipSuccess ||
        (e = hipMalloc(&q->d_w, sizeof(float) * q->nchan_pad)) != hipSuccess ||
        (e = hipMalloc(&q->d_phi, sizeof(double) * q->nphi_pad)) != hipSuccess)
        return rms_fail(RMSYNTH_ENOMEM, "rmsynth_plan: hipMalloc (adjoint): %s", hipGetErrorString(e));
    if ((e = hipMemcpy(q->d_b, hb.data(), sizeof(double) * q->nchan_pad, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(q->d_w, hw.data(), sizeof(float) * q->nchan_pad, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(q->d_phi, hgrid.data(), sizeof(double) * q->nphi_pad, hipMemcpyHostToDevice)) != hipSuccess)
        return rms_hip_fail(e, "rmsynth_plan: hipMemcpy (adjoint)");
    q->uniform = detect_uniform(hgrid.data(), q->nphi, amax, &q->phi0, &q->dphi);
    if (q->uniform) return build_factor_tables(q);
    // A uniform phi grid makes the contracted axis uniform: the channel-factored
    // tables then replace per-element phase generation (same phase tolerance,
    // now over every output lambda^2).
    double gmax = 0.0, phi0 = 0.0, dphi = 0.0;
    for (int32_t j = 0; j < p->nchan; ++j) gmax = std::max(gmax, std::fabs(hgrid[j]));
    if (p->nphi < 3 * kKTile || !detect_uniform(phi, p->nphi, gmax, &phi0, &dphi)) return build_etable(q);
    q->cuniform = true;
    q->kb0 = phi0 / M_PI;
    q->kdb = dphi / M_PI;
    {
        constexpr int kc = 8, kts = kKTile / kc;  // K-step of the factored kernel
        const int nk = (q->nchan + kc - 1) / kc;
        q->kpad = ((nk + kts - 1) / kts * kts - nk) * kc;
    }
    const size_t nT = (size_t)(kKTile / 4) * q->nphi_pad;
    if ((e = hipMalloc(&q->d_kw, sizeof(float2) * q->nchan_pad)) != hipSuccess ||
        (e = hipMalloc(&q->d_kbase, sizeof(float2) * q->nphi_pad)) != hipSuccess ||
        (e = hipMalloc(&q->d_krot, sizeof(float2) * q->nphi_pad)) != hipSuccess ||
        (e = hipMalloc(&q->d_Kbf[0], sizeof(uint4) * nT)) != hipSuccess ||
        (e = hipMalloc(&q->d_Kbf[1], sizeof(uint4) * nT)) != hipSuccess ||
        (e = hipMalloc(&q->d_Khf[0], sizeof(uint4) * nT)) != hipSuccess ||
        (e = hipMalloc(&q->d_Khf[1], sizeof(uint4) * nT)) != hipSuccess)
        return rms_fail(RMSYNTH_ENOMEM, "rmsynth_plan: hipMalloc (adjoint tables): %s", hipGetErrorString(e));
    hipStream_t s = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
        return rms_hip_fail(e, "rmsynth_plan: hipStreamCreate");
    e = launch_kfactor_tables(*q, s);
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_plan: adjoint-table kernel");
    if (e2 != hipSuccess) return rms_hip_fail(e2, "rmsynth_plan: adjoint-table kernel");
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
        if (int rc = build_nufft_tables(p, lambda2, weights)) {
            free_plan(p);
            return rc;
        }
    } else if (int rc = build_etable(p)) {
        free_plan(p);
        return rc;
    }
    if (int rc = build_adjoint_plan(p, lambda2, phi)) {
        free_plan(p);
        return rc;
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

size_t region(int64_t n, int64_t bytes_each) { return (size_t)round_up(std::max<int64_t>(n, 1) * bytes_each, 256); }

size_t scale_bytes(int64_t nlos) { return region(nlos, 4); }

bool fused_peaks(const rmsynth_plan_s* p, int32_t precision)
{
    return precision != RMSYNTH_FP32 && (p->uniform || p->etab);
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
    return RMSYNTH_OK;
}

// What a call keeps in its workspace for a batch of n LOS.
enum class Mode { Execute, ExecutePeaks, Search };

struct WsLayout {
    size_t scales = 0;  // FP16 split: per-LOS scales
    size_t parts = 0;   // fused peaks with F stored: PeakPart records
    size_t recs = 0;    // fused search: PeakRec records
    size_t fq = 0, fu = 0;  // search on the unfused paths: F of the batch
    size_t total() const { return scales + parts + recs + fq + fu; }
};

WsLayout ws_layout(const rmsynth_plan_s* p, Mode mode, int32_t precision, int64_t n)
{
    WsLayout w;
    if (precision == RMSYNTH_SPLIT_FP16) w.scales = scale_bytes(n);
    if (mode == Mode::ExecutePeaks && fused_peaks(p, precision))
        w.parts = region(n, factored_peak_parts(*p) * (int64_t)sizeof(PeakPart));
    if (mode == Mode::Search) {
        if (fused_peaks(p, precision)) {
            w.recs = region(n, factored_peak_parts(*p) * (int64_t)sizeof(PeakRec));
        } else {
            w.fq = region(n, (int64_t)p->nphi * 4);
            w.fu = w.fq;
        }
    }
    return w;
}

// LOS per batch for a workspace of `bytes`: all of them when it holds the
// whole call's needs, else the largest multiple of kBatchLos it holds.
constexpr int64_t kBatchLos = 128;

int batch_size(const rmsynth_plan_s* p, Mode mode, int32_t precision, int64_t nlos, size_t bytes,
               bool have_ws, int64_t* batch, const char* who)
{
    const size_t whole = ws_layout(p, mode, precision, nlos).total();
    if (whole == 0 || (have_ws && bytes >= whole)) {
        *batch = nlos;
        return RMSYNTH_OK;
    }
    const int64_t first = std::min(nlos, kBatchLos);
    const size_t least = ws_layout(p, mode, precision, first).total();
    if (!have_ws || bytes < least)
        return rms_fail(RMSYNTH_EWORKSPACE, "%s: needs %zu workspace bytes (%zu for the whole call), got %zu",
                        who, least, whole, have_ws ? bytes : (size_t)0);
    // The layout grows linearly in n (plus at most 255 bytes of rounding per region).
    int64_t lo = first, hi = nlos;
    while (hi - lo > kBatchLos) {
        const int64_t mid = lo + (hi - lo) / 2 / kBatchLos * kBatchLos;
        if (ws_layout(p, mode, precision, mid).total() <= bytes) lo = mid;
        else hi = mid;
    }
    *batch = lo;
    return RMSYNTH_OK;
}

// The transform of one batch of n LOS starting at LOS l0 of the call, in
// launches whose grids stay within the dispatch limit (tiles of at least 64
// LOS of 256 threads).  ld is the call's row stride (LOS-major: nchan) or
// plane stride (frequency-major: the call's nlos).  With parts or recs the
// factored kernels also write their per-tile peaks, laid out [part][n].
int run_execute(const rmsynth_plan_s* p, const float* Q, const float* U, int64_t l0, int64_t n,
                int64_t ld, int32_t layout, int32_t precision, float* Fq, float* Fu, float* Fabs,
                float* scales, PeakPart* parts, PeakRec* recs, hipStream_t stream, const char* who)
{
    const int64_t tiles_n = (p->nphi + 127) / 128;
    const int64_t max_los = max_los_tiled(tiles_n, 64, 256);
    for (int64_t b0 = 0; b0 < n;) {
        const int64_t m = std::min(n - b0, max_los);
        const int64_t l = l0 + b0;
        ExecArgs a{};
        if (layout == RMSYNTH_LOS_MAJOR) {
            a.Q = Q + l * ld;
            a.U = U + l * ld;
            a.vec4 = (ld % 4 == 0) && ((uintptr_t)Q % 16 == 0) && ((uintptr_t)U % 16 == 0);
        } else {
            a.Q = Q + l;
            a.U = U + l;
            a.vec4 = false;
        }
        a.ld = ld;
        a.nlos = m;
        a.layout = layout;
        a.Fq = Fq ? Fq + b0 * p->nphi : nullptr;
        a.Fu = Fu ? Fu + b0 * p->nphi : nullptr;
        a.Fabs = Fabs ? Fabs + b0 * p->nphi : nullptr;
        a.los_scale = precision == RMSYNTH_SPLIT_FP16 ? scales + b0 : nullptr;
        a.peak_part = parts ? parts + b0 : nullptr;
        a.peak_rec = recs ? recs + b0 : nullptr;
        a.peak_part_ld = n;
        a.stream = stream;
        if (precision == RMSYNTH_SPLIT_FP16) {
            hipError_t e = launch_los_scale(*p, a);
            if (e != hipSuccess) return rms_hip_fail(e, who);
        }
        hipError_t e;
        if (precision == RMSYNTH_FP32) e = launch_synth_fp32(*p, a);
        else if (p->uniform) e = launch_synth_factored(*p, a, precision);
        else if (p->cuniform && layout == RMSYNTH_LOS_MAJOR && !parts && !recs)
            e = launch_synth_kfactored(*p, a, precision);
        else if (p->etab) e = launch_synth_etable(*p, a, precision);
        else e = launch_synth_split(*p, a, precision);
        if (e != hipSuccess) return rms_hip_fail(e, who);
        b0 += m;
    }
    return RMSYNTH_OK;
}

struct PeakOut {
    int32_t* idx;
    float *phi_pk, *amp, *q_pk, *u_pk, *phi_fit, *amp_fit;
    PeakOut at(int64_t l) const
    {
        auto o = [l](float* x) { return x ? x + l : nullptr; };
        return PeakOut{idx + l, o(phi_pk), o(amp), o(q_pk), o(u_pk), o(phi_fit), o(amp_fit)};
    }
};

// One call of execute / execute_peaks / search over all nlos, in batches that
// fit the workspace.
int run_batched(const rmsynth_plan_s* p, Mode mode, const float* Q, const float* U, int64_t nlos,
                int32_t layout, int32_t precision, float* Fq, float* Fu, float* Fabs,
                const PeakOut& out, void* workspace, size_t workspace_bytes, hipStream_t s,
                const char* who)
{
    int64_t batch = 0;
    if (int rc = batch_size(p, mode, precision, nlos, workspace_bytes, workspace != nullptr, &batch, who))
        return rc;
    const int64_t ld = layout == RMSYNTH_LOS_MAJOR ? p->nchan : nlos;
    const bool fused = fused_peaks(p, precision);
    for (int64_t l0 = 0; l0 < nlos; l0 += batch) {
        const int64_t n = std::min(batch, nlos - l0);
        const WsLayout w = ws_layout(p, mode, precision, n);
        char* ws = static_cast<char*>(workspace);
        float* scales = w.scales ? reinterpret_cast<float*>(ws) : nullptr;
        ws += w.scales;
        PeakPart* parts = w.parts ? reinterpret_cast<PeakPart*>(ws) : nullptr;
        ws += w.parts;
        PeakRec* recs = w.recs ? reinterpret_cast<PeakRec*>(ws) : nullptr;
        ws += w.recs;
        float* bq = Fq ? Fq + l0 * p->nphi : (w.fq ? reinterpret_cast<float*>(ws) : nullptr);
        ws += w.fq;
        float* bu = Fu ? Fu + l0 * p->nphi : (w.fu ? reinterpret_cast<float*>(ws) : nullptr);
        float* ba = Fabs ? Fabs + l0 * p->nphi : nullptr;
        if (int rc = run_execute(p, Q, U, l0, n, ld, layout, precision, mode == Mode::Search && fused ? nullptr : bq,
                                 mode == Mode::Search && fused ? nullptr : bu, ba, scales, parts, recs, s, who))
            return rc;
        if (mode == Mode::Execute) continue;
        const PeakOut o = out.at(l0);
        hipError_t e = hipSuccess;
        if (recs)
            e = launch_peak_merge_rec(*p, recs, n, n, o.idx, o.phi_pk, o.amp, o.q_pk, o.u_pk, o.phi_fit,
                                      o.amp_fit, s);
        else if (parts)
            e = launch_peak_merge(*p, parts, n, bq, bu, o.idx, o.phi_pk, o.amp, o.q_pk, o.u_pk, s);
        else {
            e = launch_peaks(*p, bq, bu, n, o.idx, o.phi_pk, o.amp, o.q_pk, o.u_pk, s);
            if (e == hipSuccess && (o.phi_fit || o.amp_fit))
                e = launch_peak_fit(*p, bq, bu, o.idx, n, o.phi_fit, o.amp_fit, s);
        }
        if (e != hipSuccess) return rms_hip_fail(e, who);
    }
    return RMSYNTH_OK;
}

}  // namespace

size_t search_workspace_bytes(const rmsynth_plan_s* p, int64_t n, int32_t precision)
{
    return ws_layout(p, Mode::Search, precision, n).total();
}

extern "C" {

int rmsynth_execute(rmsynth_plan_t p, const float* Q, const float* U, int64_t nlos, int32_t layout,
                    int32_t precision, float* Fq, float* Fu, float* Fabs, void* workspace,
                    size_t workspace_bytes, void* stream)
{
    const char* who = "rmsynth_execute";
    if (int rc = check_execute_args(p, nlos, layout, precision, who)) return rc;
    if (nlos == 0) return rms_ok();
    if (!Q || !U || !Fq || !Fu) return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    if (int rc = check_device(p)) return rc;
    if (int rc = run_batched(p, Mode::Execute, Q, U, nlos, layout, precision, Fq, Fu, Fabs, PeakOut{},
                             workspace, workspace_bytes, (hipStream_t)stream, who))
        return rc;
    return rms_ok();
}

int rmsynth_execute_peaks_workspace_size(rmsynth_plan_t p, int64_t nlos, int32_t layout,
                                         int32_t precision, size_t* bytes)
{
    if (!bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_execute_peaks_workspace_size: bytes is NULL");
    if (int rc = check_execute_args(p, nlos, layout, precision, "rmsynth_execute_peaks_workspace_size"))
        return rc;
    *bytes = ws_layout(p, Mode::ExecutePeaks, precision, nlos).total();
    return rms_ok();
}

int rmsynth_search_workspace_size(rmsynth_plan_t p, int64_t nlos, int32_t layout, int32_t precision,
                                  size_t* bytes)
{
    if (!bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_search_workspace_size: bytes is NULL");
    if (int rc = check_execute_args(p, nlos, layout, precision, "rmsynth_search_workspace_size"))
        return rc;
    *bytes = ws_layout(p, Mode::Search, precision, nlos).total();
    return rms_ok();
}

int rmsynth_search(rmsynth_plan_t p, const float* Q, const float* U, int64_t nlos, int32_t layout,
                   int32_t precision, int32_t* idx, float* phi_pk, float* amp, float* q_pk,
                   float* u_pk, float* phi_fit, float* amp_fit, void* workspace,
                   size_t workspace_bytes, void* stream)
{
    return search_impl(p, Q, U, nlos, layout, precision, idx, phi_pk, amp, q_pk, u_pk, phi_fit,
                       amp_fit, workspace, workspace_bytes, stream, "rmsynth_search");
}

}  // extern "C"

int search_impl(const rmsynth_plan_s* p, const float* Q, const float* U, int64_t nlos,
                int32_t layout, int32_t precision, int32_t* idx, float* phi_pk, float* amp,
                float* q_pk, float* u_pk, float* phi_fit, float* amp_fit, void* workspace,
                size_t workspace_bytes, void* stream, const char* who)
{
    if (int rc = check_execute_args(p, nlos, layout, precision, who)) return rc;
    if (nlos == 0) return rms_ok();
    if (!Q || !U || !idx) return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    if (int rc = check_device(p)) return rc;
    const PeakOut out{idx, phi_pk, amp, q_pk, u_pk, phi_fit, amp_fit};
    if (int rc = run_batched(p, Mode::Search, Q, U, nlos, layout, precision, nullptr, nullptr, nullptr, out,
                             workspace, workspace_bytes, (hipStream_t)stream, who))
        return rc;
    return rms_ok();
}

extern "C" {

int rmsynth_execute_peaks(rmsynth_plan_t p, const float* Q, const float* U, int64_t nlos,
                          int32_t layout, int32_t precision, float* Fq, float* Fu, float* Fabs,
                          int32_t* idx, float* phi_pk, float* amp, float* q_pk, float* u_pk,
                          void* workspace, size_t workspace_bytes, void* stream)
{
    const char* who = "rmsynth_execute_peaks";
    if (int rc = check_execute_args(p, nlos, layout, precision, who)) return rc;
    if (nlos == 0) return rms_ok();
    if (!Fq && !Fu && !Fabs)  // peaks only: F is never stored
        return rmsynth_search(p, Q, U, nlos, layout, precision, idx, phi_pk, amp, q_pk, u_pk, nullptr,
                              nullptr, workspace, workspace_bytes, stream);
    if (!Q || !U || !Fq || !Fu || !idx) return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    if (int rc = check_device(p)) return rc;
    const PeakOut out{idx, phi_pk, amp, q_pk, u_pk, nullptr, nullptr};
    if (int rc = run_batched(p, Mode::ExecutePeaks, Q, U, nlos, layout, precision, Fq, Fu, Fabs, out,
                             workspace, workspace_bytes, (hipStream_t)stream, who))
        return rc;
    return rms_ok();
}

int rmsynth_adjoint_workspace_size(rmsynth_plan_t p, int64_t nlos, int32_t precision, size_t* bytes)
{
    if (!bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_adjoint_workspace_size: bytes is NULL");
    if (!p) return rms_fail(RMSYNTH_EINVAL, "rmsynth_adjoint_workspace_size: plan is NULL");
    if (int rc = check_execute_args(p->adj, nlos, RMSYNTH_LOS_MAJOR, precision,
                                    "rmsynth_adjoint_workspace_size"))
        return rc;
    *bytes = ws_layout(p->adj, Mode::Execute, precision, nlos).total();
    return rms_ok();
}

int rmsynth_adjoint(rmsynth_plan_t p, const float* Cq, const float* Cu, int64_t nlos, int32_t precision,
                    float* Pq, float* Pu, void* workspace, size_t workspace_bytes, void* stream)
{
    const char* who = "rmsynth_adjoint";
    if (!p) return rms_fail(RMSYNTH_EINVAL, "%s: plan is NULL", who);
    if (int rc = check_execute_args(p->adj, nlos, RMSYNTH_LOS_MAJOR, precision, who)) return rc;
    if (nlos == 0) return rms_ok();
    if (!Cq || !Cu || !Pq || !Pu) return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    if (int rc = check_device(p)) return rc;
    if (int rc = run_batched(p->adj, Mode::Execute, Cq, Cu, nlos, RMSYNTH_LOS_MAJOR, precision, Pq, Pu,
                             nullptr, PeakOut{}, workspace, workspace_bytes, (hipStream_t)stream, who))
        return rc;
    return rms_ok();
}

int rmsynth_execute_nufft(rmsynth_plan_t p, const float* Q, const float* U, int64_t nlos,
                          float* Fq, float* Fu, float* Fabs, void* stream)
{
    const char* who = "rmsynth_execute_nufft";
    if (!p) return rms_fail(RMSYNTH_EINVAL, "%s: plan is NULL", who);
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "%s: nlos=%lld", who, (long long)nlos);
    if (!p->nufft_n)
        return rms_fail(RMSYNTH_EUNSUPPORTED, "%s: needs a uniform phi grid of at most %d values and at most "
                        "%d channels", who, kNufftMaxGrid / 2, kNufftMaxChan);
    if (nlos == 0) return rms_ok();
    if (!Q || !U || !Fq || !Fu) return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    if (int rc = check_device(p)) return rc;
    int lds_max = 0;
    hipError_t e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
    if (e != hipSuccess) return rms_hip_fail(e, "hipDeviceGetAttribute");
    if (nufft_lds_bytes(*p) > (size_t)lds_max)
        return rms_fail(RMSYNTH_EUNSUPPORTED, "%s: %zu bytes of LDS needed, the device offers %d", who,
                        nufft_lds_bytes(*p), lds_max);
    e = launch_nufft(*p, Q, U, nlos, Fq, Fu, Fabs, (hipStream_t)stream);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_execute_nufft launch");
    return rms_ok();
}

int rmsynth_rmclean_workspace_size(rmsynth_plan_t p, size_t* bytes)
{
    if (!p || !bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_rmclean_workspace_size: NULL argument");
    *bytes = rmclean_table_bytes(*p);
    return rms_ok();
}

int rmsynth_rmclean(rmsynth_plan_t p, const float* Fq, const float* Fu, int64_t nlos, float gain,
                    float cutoff, int32_t max_iter, double fwhm, float* rq, float* ru, float* cq,
                    float* cu, float* Rq, float* Ru, int32_t* niter, void* workspace,
                    size_t workspace_bytes, void* stream)
{
    const char* who = "rmsynth_rmclean";
    if (!p) return rms_fail(RMSYNTH_EINVAL, "%s: plan is NULL", who);
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "%s: nlos=%lld", who, (long long)nlos);
    if (!p->uniform) return rms_fail(RMSYNTH_EUNSUPPORTED, "%s: needs a uniform phi grid", who);
    if (p->nphi > kRmcleanMaxPhi)
        return rms_fail(RMSYNTH_EUNSUPPORTED, "%s: nphi=%d above %d", who, p->nphi, kRmcleanMaxPhi);
    if (!(gain > 0.0f && gain <= 1.0f)) return rms_fail(RMSYNTH_EINVAL, "%s: gain=%g", who, (double)gain);
    if (!(cutoff >= 0.0f && cutoff <= FLT_MAX)) return rms_fail(RMSYNTH_EINVAL, "%s: cutoff=%g", who, (double)cutoff);
    if (max_iter < 0) return rms_fail(RMSYNTH_EINVAL, "%s: max_iter=%d", who, max_iter);
    if (std::isnan(fwhm) || fwhm <= 0.0) fwhm = p->fwhm_est;
    if (!(fwhm > 0.0 && std::isfinite(fwhm))) return rms_fail(RMSYNTH_EINVAL, "%s: fwhm=%g", who, fwhm);
    if (nlos == 0) return rms_ok();
    if (!Fq || !Fu || !rq || !ru || !cq || !cu || (!Rq) != (!Ru))
        return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    const size_t need = rmclean_table_bytes(*p);
    if (!workspace || workspace_bytes < need)
        return rms_fail(RMSYNTH_EWORKSPACE, "%s: needs %zu workspace bytes, got %zu", who, need,
                        workspace ? workspace_bytes : (size_t)0);
    if (int rc = check_device(p)) return rc;
    hipError_t e = launch_rmclean(*p, Fq, Fu, nlos, gain, cutoff, max_iter, fwhm, rq, ru, cq, cu, Rq, Ru,
                                  niter, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_rmclean launch");
    return rms_ok();
}

int rmsynth_peak_fit(rmsynth_plan_t p, const float* Fq, const float* Fu, const int32_t* idx,
                     int64_t nlos, float* phi_fit, float* amp_fit, void* stream)
{
    if (!p) return rms_fail(RMSYNTH_EINVAL, "rmsynth_peak_fit: plan is NULL");
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "rmsynth_peak_fit: nlos=%lld", (long long)nlos);
    if (nlos == 0) return rms_ok();
    if (!Fq || !Fu || !idx || (!phi_fit && !amp_fit))
        return rms_fail(RMSYNTH_EINVAL, "rmsynth_peak_fit: NULL buffer");
    if (int rc = check_device(p)) return rc;
    hipError_t e = launch_peak_fit(*p, Fq, Fu, idx, nlos, phi_fit, amp_fit, (hipStream_t)stream);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_peak_fit launch");
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
