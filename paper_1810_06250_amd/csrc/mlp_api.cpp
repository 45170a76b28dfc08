// C ABI of the learned gate: network object, training step, inference and
// the gated peak search.  The arithmetic runs in the kernels of mlp.hip and
// gate.hip; the gated lines of sight go through rmsynth_execute and
// rmsynth_peaks like any other.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mlp.h"
#include "rmsynth_mlp.h"

struct rmsynth_mlp_s {
    int device;
    int32_t nchan, nin, nin_pad, h1, h2;
    float phi_scale;
    int64_t step;
    // Internal parameter block (FP32): W1 [h1][nin_pad] (pad columns zero),
    // b1 [h1], W2 [h2][h1], b2 [h2], W3 [2][h2], b3 [2].
    int64_t nW1, nW2, nW3, np;
    std::vector<float> chan_w;
    float* d_chw = nullptr;
    float* d_p = nullptr;
    float* d_g = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    _Float16* d_w16 = nullptr;   // W1 | W2 | W3 as half
    uint4* d_wfrag = nullptr;    // W1 | W2 as half in MFMA-fragment order (fused inference)
    bool frag_stale = true;      // d_wfrag not yet rebuilt from the current half weights
    float* d_part = nullptr;     // partial sums of the column reductions
    float* d_wpart = nullptr;    // split-K partial sums of the weight gradients
    int64_t wpart_floats = 0;
    // Activation buffers, rows = capacity (multiple of 64).
    int64_t cap_fwd = 0, cap_bwd = 0;
    _Float16 *X = nullptr, *H1 = nullptr, *H2 = nullptr, *D2h = nullptr, *D1h = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *D2 = nullptr, *D1 = nullptr, *lossb = nullptr, *gout = nullptr;

    int64_t off_b1() const { return nW1; }
    int64_t off_W2() const { return nW1 + h1; }
    int64_t off_b2() const { return nW1 + h1 + nW2; }
    int64_t off_W3() const { return nW1 + h1 + nW2 + h2; }
    int64_t off_b3() const { return nW1 + h1 + nW2 + h2 + nW3; }
    int64_t canonical_size() const { return (int64_t)h1 * nin + h1 + nW2 + h2 + nW3 + 2; }
};

namespace {

constexpr int64_t kInferChunk = 65536;  // lines of sight per inference pass
constexpr int64_t kGateChunk = 65536;   // gated lines of sight per synthesis pass
constexpr int kMaxHidden = 4096;

template <class T>
void free_buf(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_acts(rmsynth_mlp_s* m)
{
    free_buf(m->X); free_buf(m->H1); free_buf(m->H2); free_buf(m->D2h); free_buf(m->D1h);
    free_buf(m->Z1); free_buf(m->Z2); free_buf(m->D2); free_buf(m->D1); free_buf(m->lossb);
    free_buf(m->gout);
    m->cap_fwd = m->cap_bwd = 0;
}

void free_mlp(rmsynth_mlp_s* m)
{
    if (!m) return;
    free_acts(m);
    free_buf(m->d_chw); free_buf(m->d_p); free_buf(m->d_g); free_buf(m->d_m); free_buf(m->d_v);
    free_buf(m->d_w16);
    free_buf(m->d_wfrag);
    free_buf(m->d_part);
    free_buf(m->d_wpart);
    delete m;
}

int check_mlp_device(const rmsynth_mlp_s* m)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rms_hip_fail(e, "hipGetDevice");
    if (dev != m->device)
        return rms_fail(RMSYNTH_EINVAL, "network was created on device %d but device %d is current",
                        m->device, dev);
    return RMSYNTH_OK;
}

// Grow the activation buffers to `rows` rows (forward set, and the backward
// set when `train`).  Waits for the device before freeing smaller buffers.
int ensure_rows(rmsynth_mlp_s* m, int64_t rows, bool train)
{
    const bool fwd = rows > m->cap_fwd, bwd = train && rows > m->cap_bwd;
    if (!fwd && !bwd) return RMSYNTH_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return rms_hip_fail(e, "hipDeviceSynchronize");
    auto alloc = [&](auto*& p, int64_t n) {
        free_buf(p);
        return hipMalloc(&p, sizeof(*p) * (size_t)std::max<int64_t>(n, 1));
    };
    if (fwd) {
        m->cap_fwd = 0;
        if ((e = alloc(m->X, rows * m->nin_pad)) != hipSuccess ||
            (e = alloc(m->H1, rows * m->h1)) != hipSuccess ||
            (e = alloc(m->H2, rows * m->h2)) != hipSuccess)
            return rms_fail(RMSYNTH_ENOMEM, "network activations (%lld rows): %s", (long long)rows,
                            hipGetErrorString(e));
        m->cap_fwd = rows;
    }
    if (bwd) {
        m->cap_bwd = 0;
        if ((e = alloc(m->Z1, rows * m->h1)) != hipSuccess ||
            (e = alloc(m->Z2, rows * m->h2)) != hipSuccess ||
            (e = alloc(m->D2, rows * m->h2)) != hipSuccess ||
            (e = alloc(m->D2h, rows * m->h2)) != hipSuccess ||
            (e = alloc(m->D1, rows * m->h1)) != hipSuccess ||
            (e = alloc(m->D1h, rows * m->h1)) != hipSuccess ||
            (e = alloc(m->lossb, rows)) != hipSuccess ||
            (e = alloc(m->gout, 2 * rows)) != hipSuccess)
            return rms_fail(RMSYNTH_ENOMEM, "network gradients (%lld rows): %s", (long long)rows,
                            hipGetErrorString(e));
        m->cap_bwd = rows;
    }
    return RMSYNTH_OK;
}

const _Float16* W1h(const rmsynth_mlp_s* m) { return m->d_w16; }
const _Float16* W2h(const rmsynth_mlp_s* m) { return m->d_w16 + m->nW1; }
const _Float16* W3h(const rmsynth_mlp_s* m) { return m->d_w16 + m->nW1 + m->nW2; }

// Forward pass of `rows` rows (nvalid real ones); with `train` the FP32
// pre-activations are kept for the ReLU masks.
hipError_t forward(rmsynth_mlp_s* m, const float* Q, const float* U, int64_t nvalid, int64_t rows,
                   bool train, hipStream_t s)
{
    hipError_t e = mlp_launch_input(Q, U, nvalid, rows, m->nchan, m->d_chw, m->X, m->nin_pad, s);
    if (e != hipSuccess) return e;
    e = mlp_launch_gemm(false, false, m->X, m->nin_pad, W1h(m), m->nin_pad, rows, m->h1, m->nin_pad,
                        1.0f, m->d_p + m->off_b1(), true, nullptr, 0, train ? m->Z1 : nullptr, m->h1,
                        m->H1, m->h1, s);
    if (e != hipSuccess) return e;
    return mlp_launch_gemm(false, false, m->H1, m->h1, W2h(m), m->h1, rows, m->h2, m->h1, 1.0f,
                           m->d_p + m->off_b2(), true, nullptr, 0, train ? m->Z2 : nullptr, m->h2,
                           m->H2, m->h2, s);
}

// Gradient of the mean loss into m->d_g (internal layout); loss (device) optional.
int gradient(rmsynth_mlp_s* m, const float* Q, const float* U, int64_t B, const float* phi,
             const float* det, float* loss, hipStream_t s, const char* who)
{
    const int64_t rows = round_up(B, 64);
    if (int rc = ensure_rows(m, rows, true)) return rc;
    const float inv_b = 1.0f / (float)B;
    hipError_t e = forward(m, Q, U, B, rows, true, s);
    if (e == hipSuccess)
        e = mlp_launch_head(m->H2, m->Z2, m->h2, W3h(m), m->d_p + m->off_b3(), B, rows, m->phi_scale,
                            phi, det, m->lossb, m->gout, m->D2, m->D2h, nullptr, nullptr, s);
    if (e == hipSuccess)
        e = mlp_launch_head_wgrad(m->gout, m->H2, m->h2, B, inv_b, m->d_g + m->off_W3(),
                                  m->d_g + m->off_b3(), m->d_part, s);
    // gW2[o][i] = sum_b dz2[b][o] h1[b][i]
    if (e == hipSuccess)
        e = mlp_launch_gemm_wgrad(m->D2h, m->h2, m->H1, m->h1, m->h2, m->h1, rows, inv_b,
                                  m->d_g + m->off_W2(), m->h1, m->d_wpart, m->wpart_floats, s);
    if (e == hipSuccess) e = mlp_launch_colsum(m->D2, B, m->h2, inv_b, m->d_g + m->off_b2(), m->d_part, s);
    // dz1[b][i] = (sum_o dz2[b][o] W2[o][i]) * (z1[b][i] > 0)
    if (e == hipSuccess)
        e = mlp_launch_gemm(false, true, m->D2h, m->h2, W2h(m), m->h1, rows, m->h1, m->h2, 1.0f,
                            nullptr, false, m->Z1, m->h1, m->D1, m->h1, m->D1h, m->h1, s);
    // gW1[i][k] = sum_b dz1[b][i] x[b][k]
    if (e == hipSuccess)
        e = mlp_launch_gemm_wgrad(m->D1h, m->h1, m->X, m->nin_pad, m->h1, m->nin_pad, rows, inv_b,
                                  m->d_g, m->nin_pad, m->d_wpart, m->wpart_floats, s);
    if (e == hipSuccess) e = mlp_launch_colsum(m->D1, B, m->h1, inv_b, m->d_g + m->off_b1(), m->d_part, s);
    if (e == hipSuccess && loss) e = mlp_launch_mean(m->lossb, B, loss, s);
    if (e != hipSuccess) return rms_hip_fail(e, who);
    return RMSYNTH_OK;
}

// Half copies of the weights after every parameter change; the fragment-order
// copy for fused inference is rebuilt lazily, by the next inference call on
// its own stream (training steps do not need it).
hipError_t refresh_half(rmsynth_mlp_s* m, hipStream_t s)
{
    m->frag_stale = true;
    return mlp_launch_weights16(m->d_p, m->nW1, m->h1, m->nW2, m->h2, m->nW3, m->d_w16, s);
}

// Internal <-> canonical layout of a parameter-shaped vector (host).
void to_canonical(const rmsynth_mlp_s* m, const float* in, float* out)
{
    for (int32_t i = 0; i < m->h1; ++i)
        std::memcpy(out + (int64_t)i * m->nin, in + (int64_t)i * m->nin_pad, sizeof(float) * m->nin);
    std::memcpy(out + (int64_t)m->h1 * m->nin, in + m->nW1, sizeof(float) * (m->np - m->nW1));
}

void from_canonical(const rmsynth_mlp_s* m, const float* in, float* out)
{
    std::fill(out, out + m->nW1, 0.0f);
    for (int32_t i = 0; i < m->h1; ++i)
        std::memcpy(out + (int64_t)i * m->nin_pad, in + (int64_t)i * m->nin, sizeof(float) * m->nin);
    std::memcpy(out + m->nW1, in + (int64_t)m->h1 * m->nin, sizeof(float) * (m->np - m->nW1));
}

int read_vec(const rmsynth_mlp_s* m, const float* d, std::vector<float>& canon, const char* who)
{
    std::vector<float> tmp(m->np);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(tmp.data(), d, sizeof(float) * m->np, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return rms_hip_fail(e, who);
    canon.resize(m->canonical_size());
    to_canonical(m, tmp.data(), canon.data());
    return RMSYNTH_OK;
}

int write_vec(rmsynth_mlp_s* m, const float* canon, float* d, const char* who)
{
    std::vector<float> tmp(m->np);
    from_canonical(m, canon, tmp.data());
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(d, tmp.data(), sizeof(float) * m->np, hipMemcpyHostToDevice);
    if (e != hipSuccess) return rms_hip_fail(e, who);
    return RMSYNTH_OK;
}

// splitmix64 (Steele, Lea & Flood 2014) and Box-Muller for the initial weights.
struct InitRng {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal()
    {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    }
};

int create(int32_t nchan, int32_t h1, int32_t h2, const float* weights, float phi_scale,
           rmsynth_mlp_t* out, const char* who)
{
    if (!out) return rms_fail(RMSYNTH_EINVAL, "%s: out is NULL", who);
    *out = nullptr;
    if (nchan < 1 || nchan > 65536) return rms_fail(RMSYNTH_EINVAL, "%s: nchan=%d", who, nchan);
    if (h1 < 64 || h1 > kMaxHidden || h1 % 64 || h2 < 64 || h2 > kMaxHidden || h2 % 64)
        return rms_fail(RMSYNTH_EINVAL, "%s: hidden widths %d, %d (multiples of 64, at most %d)", who,
                        h1, h2, kMaxHidden);
    if (!(phi_scale > 0.0f) || !std::isfinite(phi_scale))
        return rms_fail(RMSYNTH_EINVAL, "%s: phi_scale=%g", who, (double)phi_scale);
    std::vector<float> w(nchan, 1.0f);
    if (weights) {
        for (int32_t j = 0; j < nchan; ++j) {
            if (!std::isfinite(weights[j]) || weights[j] < 0.0f)
                return rms_fail(RMSYNTH_EINVAL, "%s: weight %d is %g", who, j, (double)weights[j]);
            w[j] = weights[j];
        }
    }
    auto* m = new (std::nothrow) rmsynth_mlp_s{};
    if (!m) return rms_fail(RMSYNTH_ENOMEM, "%s: host allocation", who);
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) { free_mlp(m); return rms_hip_fail(e, "hipGetDevice"); }
    m->nchan = nchan;
    m->nin = 2 * nchan;
    m->nin_pad = (int32_t)round_up(m->nin, 64);
    m->h1 = h1;
    m->h2 = h2;
    m->phi_scale = phi_scale;
    m->nW1 = (int64_t)h1 * m->nin_pad;
    m->nW2 = (int64_t)h2 * h1;
    m->nW3 = 2 * (int64_t)h2;
    m->np = m->nW1 + h1 + m->nW2 + h2 + m->nW3 + 2;
    m->chan_w = w;
    const size_t pb = sizeof(float) * (size_t)m->np;
    if ((e = hipMalloc(&m->d_chw, sizeof(float) * nchan)) != hipSuccess ||
        (e = hipMalloc(&m->d_p, pb)) != hipSuccess || (e = hipMalloc(&m->d_g, pb)) != hipSuccess ||
        (e = hipMalloc(&m->d_m, pb)) != hipSuccess || (e = hipMalloc(&m->d_v, pb)) != hipSuccess ||
        (e = hipMalloc(&m->d_w16, sizeof(_Float16) * (m->nW1 + m->nW2 + m->nW3))) != hipSuccess ||
        (mlp_fused_supported(h1, h2, m->nin_pad) &&
         (e = hipMalloc(&m->d_wfrag, sizeof(uint4) * mlp_fused_frag_uint4(m->nin_pad))) != hipSuccess) ||
        (e = hipMalloc(&m->d_part, sizeof(float) * mlp_reduce_part_floats(
                                       std::max<int64_t>(std::max(h1, h2), 2 * (int64_t)h2 + 2)))) != hipSuccess ||
        (e = hipMalloc(&m->d_wpart, sizeof(float) * (m->wpart_floats = mlp_wgrad_part_floats(
                                        std::max(m->nW1, m->nW2))))) != hipSuccess) {
        free_mlp(m);
        return rms_fail(RMSYNTH_ENOMEM, "%s: hipMalloc: %s", who, hipGetErrorString(e));
    }
    if ((e = hipMemcpy(m->d_chw, w.data(), sizeof(float) * nchan, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(m->d_p, 0, pb)) != hipSuccess || (e = hipMemset(m->d_g, 0, pb)) != hipSuccess ||
        (e = hipMemset(m->d_m, 0, pb)) != hipSuccess || (e = hipMemset(m->d_v, 0, pb)) != hipSuccess) {
        free_mlp(m);
        return rms_hip_fail(e, who);
    }
    *out = m;
    return RMSYNTH_OK;
}

}  // namespace

extern "C" {

int rmsynth_mlp_create(int32_t nchan, int32_t h1, int32_t h2, const float* weights, float phi_scale,
                       uint64_t seed, rmsynth_mlp_t* out)
{
    if (int rc = create(nchan, h1, h2, weights, phi_scale, out, "rmsynth_mlp_create")) return rc;
    rmsynth_mlp_s* m = *out;
    std::vector<float> canon(m->canonical_size(), 0.0f);
    InitRng rng{seed};
    const double s1 = std::sqrt(2.0 / m->nin), s2 = std::sqrt(2.0 / h1), s3 = std::sqrt(1.0 / h2);
    int64_t o = 0;
    for (int64_t i = 0; i < (int64_t)h1 * m->nin; ++i) canon[o++] = (float)(s1 * rng.normal());
    o += h1;
    for (int64_t i = 0; i < m->nW2; ++i) canon[o++] = (float)(s2 * rng.normal());
    o += h2;
    for (int64_t i = 0; i < m->nW3; ++i) canon[o++] = (float)(s3 * rng.normal());
    int rc = write_vec(m, canon.data(), m->d_p, "rmsynth_mlp_create");
    hipError_t e = rc ? hipSuccess : refresh_half(m, nullptr);
    if (!rc && e == hipSuccess) e = hipDeviceSynchronize();
    if (!rc && e != hipSuccess) rc = rms_hip_fail(e, "rmsynth_mlp_create");
    if (rc) {
        free_mlp(m);
        *out = nullptr;
        return rc;
    }
    return rms_ok();
}

int rmsynth_mlp_num_params(rmsynth_mlp_t m, int64_t* nparams)
{
    if (!m || !nparams) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_num_params: NULL argument");
    *nparams = m->canonical_size();
    return rms_ok();
}

int rmsynth_mlp_info(rmsynth_mlp_t m, int32_t* nchan, int32_t* h1, int32_t* h2, float* phi_scale)
{
    if (!m) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_info: network is NULL");
    if (nchan) *nchan = m->nchan;
    if (h1) *h1 = m->h1;
    if (h2) *h2 = m->h2;
    if (phi_scale) *phi_scale = m->phi_scale;
    return rms_ok();
}

int rmsynth_mlp_get_params(rmsynth_mlp_t m, float* params)
{
    if (!m || !params) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_get_params: NULL argument");
    if (int rc = check_mlp_device(m)) return rc;
    std::vector<float> canon;
    if (int rc = read_vec(m, m->d_p, canon, "rmsynth_mlp_get_params")) return rc;
    std::memcpy(params, canon.data(), sizeof(float) * canon.size());
    return rms_ok();
}

int rmsynth_mlp_set_params(rmsynth_mlp_t m, const float* params)
{
    if (!m || !params) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_set_params: NULL argument");
    if (int rc = check_mlp_device(m)) return rc;
    for (int64_t i = 0; i < m->canonical_size(); ++i)
        if (!std::isfinite(params[i]))
            return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_set_params: parameter %lld is %g",
                            (long long)i, (double)params[i]);
    if (int rc = write_vec(m, params, m->d_p, "rmsynth_mlp_set_params")) return rc;
    hipError_t e = refresh_half(m, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_mlp_set_params");
    return rms_ok();
}

static int check_batch(rmsynth_mlp_t m, const float* Q, const float* U, int64_t batch,
                       const float* phi, const float* det, const char* who)
{
    if (!m) return rms_fail(RMSYNTH_EINVAL, "%s: network is NULL", who);
    if (batch < 1 || batch > (int64_t(1) << 24))
        return rms_fail(RMSYNTH_EINVAL, "%s: batch=%lld (1 .. 2^24)", who, (long long)batch);
    if (!Q || !U || !phi || !det) return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    return check_mlp_device(m);
}

int rmsynth_mlp_grad(rmsynth_mlp_t m, const float* Q, const float* U, int64_t batch,
                     const float* phi_label, const float* det_label, float* grad, float* loss,
                     void* stream)
{
    if (int rc = check_batch(m, Q, U, batch, phi_label, det_label, "rmsynth_mlp_grad")) return rc;
    if (!grad) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_grad: grad is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (int rc = gradient(m, Q, U, batch, phi_label, det_label, loss, s, "rmsynth_mlp_grad"))
        return rc;
    // Canonical layout: W1 rows without their padding, then the rest as is.
    hipError_t e = hipMemcpy2DAsync(grad, sizeof(float) * m->nin, m->d_g, sizeof(float) * m->nin_pad,
                                    sizeof(float) * m->nin, m->h1, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grad + (int64_t)m->h1 * m->nin, m->d_g + m->nW1,
                           sizeof(float) * (m->np - m->nW1), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_mlp_grad copy");
    return rms_ok();
}

int rmsynth_mlp_train_step(rmsynth_mlp_t m, const float* Q, const float* U, int64_t batch,
                           const float* phi_label, const float* det_label, float lr, float* loss,
                           void* stream)
{
    if (int rc = check_batch(m, Q, U, batch, phi_label, det_label, "rmsynth_mlp_train_step"))
        return rc;
    if (!(lr > 0.0f) || !std::isfinite(lr))
        return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_train_step: lr=%g", (double)lr);
    hipStream_t s = (hipStream_t)stream;
    if (int rc = gradient(m, Q, U, batch, phi_label, det_label, loss, s, "rmsynth_mlp_train_step"))
        return rc;
    const double b1 = 0.9, b2 = 0.999;
    const int64_t t = m->step + 1;
    const float bc1 = (float)(1.0 - std::pow(b1, (double)t));
    const float bc2 = (float)(1.0 - std::pow(b2, (double)t));
    hipError_t e = mlp_launch_adam(m->d_p, m->d_g, m->d_m, m->d_v, m->np, lr, (float)b1, (float)b2,
                                   1e-8f, bc1, bc2, s);
    if (e == hipSuccess) e = refresh_half(m, s);
    if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_mlp_train_step");
    m->step = t;
    return rms_ok();
}

int rmsynth_mlp_infer(rmsynth_mlp_t m, const float* Q, const float* U, int64_t nlos, float* phi_hat,
                      float* score, void* stream)
{
    if (!m) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_infer: network is NULL");
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_infer: nlos=%lld", (long long)nlos);
    if (nlos == 0) return rms_ok();
    if (!Q || !U || !phi_hat || !score) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_infer: NULL buffer");
    if (int rc = check_mlp_device(m)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (mlp_fused_supported(m->h1, m->h2, m->nin_pad)) {
        // One pass over the cube, no activation buffers.
        hipError_t e = hipSuccess;
        if (m->frag_stale) {
            e = mlp_launch_frag16(W1h(m), W2h(m), m->nin_pad, m->d_wfrag, s);
            if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_mlp_infer");
            m->frag_stale = false;
        }
        e = mlp_launch_infer_fused(Q, U, nlos, m->nchan, m->d_chw, m->nin_pad,
                                              m->d_wfrag, m->d_p + m->off_b1(),
                                              m->d_p + m->off_b2(), W3h(m), m->d_p + m->off_b3(),
                                              m->phi_scale, phi_hat, score,
                                              std::all_of(m->chan_w.begin(), m->chan_w.end(),
                                                          [](float v) { return v == 1.0f; }),
                                              s);
        if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_mlp_infer");
        return rms_ok();
    }
    const int64_t chunk = std::min(round_up(nlos, 64), kInferChunk);
    if (int rc = ensure_rows(m, chunk, false)) return rc;
    for (int64_t l0 = 0; l0 < nlos; l0 += chunk) {
        const int64_t n = std::min(chunk, nlos - l0);
        const int64_t rows = round_up(n, 64);
        hipError_t e = forward(m, Q + l0 * m->nchan, U + l0 * m->nchan, n, rows, false, s);
        if (e == hipSuccess)
            e = mlp_launch_head(m->H2, nullptr, m->h2, W3h(m), m->d_p + m->off_b3(), n, rows,
                                m->phi_scale, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                phi_hat + l0, score + l0, s);
        if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_mlp_infer");
    }
    return rms_ok();
}

// Workspace of the gated search (each part 256-byte aligned):
//   score [nlos] f32 | counts [nblocks + 1] i32 | list [nlos] i64 |
//   gQ, gU [G][nchan] f32 | Fq, Fu [G][nphi] f32 | gidx [G] i32 | gphi, gamp [G] f32
struct GateLayout {
    int64_t G;
    size_t score, counts, list, gQ, gU, Fq, Fu, gidx, gphi, gamp, total;
};

// With search = true the gated LOS go through the peaks-only search
// (rmsynth_search) in the given precision: its workspace takes the place of
// the F buffers.
static GateLayout gate_layout(const rmsynth_plan_s* p, int64_t nlos, bool search = false,
                              int32_t precision = RMSYNTH_FP32)
{
    GateLayout L{};
    L.G = std::max<int64_t>(1, std::min(nlos, kGateChunk));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (size_t)round_up((int64_t)bytes, 256);
        return at;
    };
    const size_t n = (size_t)std::max<int64_t>(nlos, 1);
    L.score = take(4 * n);
    L.counts = take(4 * (size_t)(gate_num_blocks(nlos) + 1));
    L.list = take(8 * n);
    L.gQ = take(4 * (size_t)L.G * p->nchan);
    L.gU = take(4 * (size_t)L.G * p->nchan);
    if (search) {
        L.Fq = take(search_workspace_bytes(p, L.G, precision));
        L.Fu = L.Fq;
    } else {
        L.Fq = take(4 * (size_t)L.G * p->nphi);
        L.Fu = take(4 * (size_t)L.G * p->nphi);
    }
    L.gidx = take(4 * (size_t)L.G);
    L.gphi = take(4 * (size_t)L.G);
    L.gamp = take(4 * (size_t)L.G);
    L.total = o;
    return L;
}

int rmsynth_gate_workspace_size(rmsynth_plan_t p, rmsynth_mlp_t m, int64_t nlos, size_t* bytes)
{
    if (!p || !m || !bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_gate_workspace_size: NULL argument");
    if (nlos < 0 || nlos > 0x7fffffffLL)
        return rms_fail(RMSYNTH_EINVAL, "rmsynth_gate_workspace_size: nlos=%lld", (long long)nlos);
    *bytes = gate_layout(p, nlos).total;
    return rms_ok();
}

static int gate_run(rmsynth_plan_t p, rmsynth_mlp_t m, const float* Q, const float* U, int64_t nlos,
                    bool search, int32_t precision, float tau, int32_t* idx, float* phi_pk, float* amp,
                    int32_t* gated, void* workspace, size_t workspace_bytes, void* stream, const char* who)
{
    if (!p || !m) return rms_fail(RMSYNTH_EINVAL, "%s: plan or network is NULL", who);
    if (p->nchan != m->nchan)
        return rms_fail(RMSYNTH_EINVAL, "%s: plan has %d channels, network %d", who, p->nchan, m->nchan);
    if (nlos < 0 || nlos > 0x7fffffffLL)
        return rms_fail(RMSYNTH_EINVAL, "%s: nlos=%lld", who, (long long)nlos);
    if (std::isnan(tau)) return rms_fail(RMSYNTH_EINVAL, "%s: tau is NaN", who);
    if (precision < RMSYNTH_FP32 || precision > RMSYNTH_SPLIT_FP16)
        return rms_fail(RMSYNTH_EINVAL, "%s: precision=%d", who, precision);
    if (nlos == 0) return rms_ok();
    if (!Q || !U || !idx || !phi_pk || !amp || !gated)
        return rms_fail(RMSYNTH_EINVAL, "%s: NULL buffer", who);
    const GateLayout L = gate_layout(p, nlos, search, precision);
    if (!workspace || workspace_bytes < L.total)
        return rms_fail(RMSYNTH_EWORKSPACE, "%s: needs %zu workspace bytes, got %zu", who, L.total,
                        workspace ? workspace_bytes : (size_t)0);
    if (int rc = check_mlp_device(m)) return rc;
    hipStream_t s = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    auto* score = reinterpret_cast<float*>(ws + L.score);
    auto* counts = reinterpret_cast<int32_t*>(ws + L.counts);
    auto* list = reinterpret_cast<int64_t*>(ws + L.list);
    auto* gQ = reinterpret_cast<float*>(ws + L.gQ);
    auto* gU = reinterpret_cast<float*>(ws + L.gU);
    auto* Fq = reinterpret_cast<float*>(ws + L.Fq);
    auto* Fu = reinterpret_cast<float*>(ws + L.Fu);
    auto* gidx = reinterpret_cast<int32_t*>(ws + L.gidx);
    auto* gphi = reinterpret_cast<float*>(ws + L.gphi);
    auto* gamp = reinterpret_cast<float*>(ws + L.gamp);

    if (int rc = rmsynth_mlp_infer(m, Q, U, nlos, phi_pk, score, stream)) return rc;
    const float edge = (float)(p->phi_absmax - p->fwhm_est);
    hipError_t e = gate_launch_compact(phi_pk, score, nlos, tau, edge, gated, idx, amp, counts, list, s);
    int32_t ngated = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&ngated, counts + gate_num_blocks(nlos), sizeof(int32_t),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return rms_hip_fail(e, who);
    for (int64_t r0 = 0; r0 < ngated; r0 += L.G) {
        const int64_t n = std::min<int64_t>(L.G, ngated - r0);
        if ((e = gate_launch_gather(Q, U, list + r0, n, p->nchan, gQ, gU, s)) != hipSuccess)
            return rms_hip_fail(e, who);
        if (search) {
            if (int rc = search_impl(p, gQ, gU, n, RMSYNTH_LOS_MAJOR, precision, gidx, gphi, gamp, nullptr,
                                     nullptr, nullptr, nullptr, Fq, search_workspace_bytes(p, L.G, precision),
                                     stream, who))
                return rc;
        } else {
            if (int rc = rmsynth_execute(p, gQ, gU, n, RMSYNTH_LOS_MAJOR, RMSYNTH_FP32, Fq, Fu, nullptr,
                                         nullptr, 0, stream))
                return rc;
            if (int rc = rmsynth_peaks(p, Fq, Fu, n, gidx, gphi, gamp, nullptr, nullptr, stream)) return rc;
        }
        if ((e = gate_launch_scatter(list + r0, n, gidx, gphi, gamp, idx, phi_pk, amp, s)) != hipSuccess)
            return rms_hip_fail(e, who);
    }
    return rms_ok();
}

int rmsynth_gate_execute(rmsynth_plan_t p, rmsynth_mlp_t m, const float* Q, const float* U,
                         int64_t nlos, float tau, int32_t* idx, float* phi_pk, float* amp,
                         int32_t* gated, void* workspace, size_t workspace_bytes, void* stream)
{
    return gate_run(p, m, Q, U, nlos, false, RMSYNTH_FP32, tau, idx, phi_pk, amp, gated, workspace,
                    workspace_bytes, stream, "rmsynth_gate_execute");
}

int rmsynth_gate_search_workspace_size(rmsynth_plan_t p, rmsynth_mlp_t m, int64_t nlos,
                                       int32_t precision, size_t* bytes)
{
    if (!p || !m || !bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_gate_search_workspace_size: NULL argument");
    if (nlos < 0 || nlos > 0x7fffffffLL)
        return rms_fail(RMSYNTH_EINVAL, "rmsynth_gate_search_workspace_size: nlos=%lld", (long long)nlos);
    if (precision < RMSYNTH_FP32 || precision > RMSYNTH_SPLIT_FP16)
        return rms_fail(RMSYNTH_EINVAL, "rmsynth_gate_search_workspace_size: precision=%d", precision);
    *bytes = gate_layout(p, nlos, true, precision).total;
    return rms_ok();
}

int rmsynth_gate_search(rmsynth_plan_t p, rmsynth_mlp_t m, const float* Q, const float* U, int64_t nlos,
                        int32_t precision, float tau, int32_t* idx, float* phi_pk, float* amp,
                        int32_t* gated, void* workspace, size_t workspace_bytes, void* stream)
{
    return gate_run(p, m, Q, U, nlos, true, precision, tau, idx, phi_pk, amp, gated, workspace,
                    workspace_bytes, stream, "rmsynth_gate_search");
}

// Labelling workspace: Fq, Fu [C][nphi] | idx, phi, amp [C], C = min(nlos, kGateChunk).
static size_t train_ws(const rmsynth_plan_s* p, int64_t nlos, int64_t* chunk)
{
    const int64_t C = std::max<int64_t>(1, std::min(nlos, kGateChunk));
    if (chunk) *chunk = C;
    return 2 * (size_t)round_up(4 * C * (int64_t)p->nphi, 256) + 3 * (size_t)round_up(4 * C, 256);
}

int rmsynth_train_workspace_size(rmsynth_plan_t p, int64_t nlos, size_t* bytes)
{
    if (!p || !bytes) return rms_fail(RMSYNTH_EINVAL, "rmsynth_train_workspace_size: NULL argument");
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "rmsynth_train_workspace_size: nlos=%lld", (long long)nlos);
    *bytes = train_ws(p, nlos, nullptr);
    return rms_ok();
}

int rmsynth_synth_training(rmsynth_plan_t p, const rmsynth_train_spec* sp, uint64_t seed,
                           int64_t first_los, int64_t nlos, float* Q, float* U, float* phi_label,
                           float* det_label, int32_t* cls, float* truth, void* workspace,
                           size_t workspace_bytes, void* stream)
{
    const char* who = "rmsynth_synth_training";
    if (!p || !sp) return rms_fail(RMSYNTH_EINVAL, "%s: plan or spec is NULL", who);
    if (nlos < 0 || first_los < 0 || first_los > INT64_MAX - nlos)
        return rms_fail(RMSYNTH_EINVAL, "%s: first_los=%lld nlos=%lld", who, (long long)first_los,
                        (long long)nlos);
    const double fr[3] = {sp->frac_noise, sp->frac_thin1, sp->frac_thin2};
    double fsum = 0.0;
    for (double f : fr) {
        if (!(f >= 0.0 && f <= 1.0)) return rms_fail(RMSYNTH_EINVAL, "%s: class fraction %g", who, f);
        fsum += f;
    }
    if (fsum > 1.0 + 1e-12) return rms_fail(RMSYNTH_EINVAL, "%s: class fractions sum to %g", who, fsum);
    auto range_ok = [](double lo, double hi) { return std::isfinite(lo) && std::isfinite(hi) && lo <= hi; };
    if (!range_ok(sp->p0_lo, sp->p0_hi) || sp->p0_lo < 0.0)
        return rms_fail(RMSYNTH_EINVAL, "%s: P0 range [%g, %g]", who, sp->p0_lo, sp->p0_hi);
    if (!range_ok(sp->phi_lo, sp->phi_hi))
        return rms_fail(RMSYNTH_EINVAL, "%s: phi range [%g, %g]", who, sp->phi_lo, sp->phi_hi);
    if (!range_ok(sp->w_lo, sp->w_hi) || !(sp->w_lo > 0.0))
        return rms_fail(RMSYNTH_EINVAL, "%s: slab width range [%g, %g]", who, sp->w_lo, sp->w_hi);
    if (!std::isfinite(sp->sigma) || sp->sigma < 0.0)
        return rms_fail(RMSYNTH_EINVAL, "%s: sigma=%g", who, sp->sigma);
    if (std::isnan(sp->det_threshold)) return rms_fail(RMSYNTH_EINVAL, "%s: det_threshold is NaN", who);
    if (nlos == 0) return rms_ok();
    if (!Q || !U) return rms_fail(RMSYNTH_EINVAL, "%s: NULL Q or U", who);
    const bool want_labels = phi_label || det_label;
    int64_t C = 0;
    const size_t need = want_labels ? train_ws(p, nlos, &C) : 0;
    if (want_labels && (!workspace || workspace_bytes < need))
        return rms_fail(RMSYNTH_EWORKSPACE, "%s: needs %zu workspace bytes, got %zu", who, need,
                        workspace ? workspace_bytes : (size_t)0);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rms_hip_fail(e, "hipGetDevice");
    if (dev != p->device)
        return rms_fail(RMSYNTH_EINVAL, "%s: plan was created on device %d but device %d is current",
                        who, p->device, dev);
    hipStream_t s = (hipStream_t)stream;
    TrainSpecDev d{};
    d.f0 = fr[0];
    d.f1 = fr[0] + fr[1];
    d.f2 = fr[0] + fr[1] + fr[2];
    d.p0_lo = sp->p0_lo; d.p0_hi = sp->p0_hi;
    d.phi_lo = sp->phi_lo; d.phi_hi = sp->phi_hi;
    d.w_lo = sp->w_lo; d.w_hi = sp->w_hi;
    d.sigma = sp->sigma;
    // Launch in batches that keep the grid within its limit (one wave per LOS).
    const int64_t max_los = max_items(4, 256);
    for (int64_t l0 = 0; l0 < nlos; l0 += max_los) {
        const int64_t n = std::min(max_los, nlos - l0);
        e = train_launch_spectra(p->d_lambda2, p->nchan, d, seed, first_los + l0, n,
                                 Q + l0 * p->nchan, U + l0 * p->nchan, cls ? cls + l0 : nullptr,
                                 truth ? truth + 4 * l0 : nullptr, s);
        if (e != hipSuccess) return rms_hip_fail(e, who);
    }
    if (!want_labels) return rms_ok();
    char* ws = static_cast<char*>(workspace);
    float* Fq = reinterpret_cast<float*>(ws);
    float* Fu = reinterpret_cast<float*>(ws + round_up(4 * C * (int64_t)p->nphi, 256));
    char* tail = ws + 2 * round_up(4 * C * (int64_t)p->nphi, 256);
    auto* idx = reinterpret_cast<int32_t*>(tail);
    auto* phk = reinterpret_cast<float*>(tail + round_up(4 * C, 256));
    auto* amp = reinterpret_cast<float*>(tail + 2 * round_up(4 * C, 256));
    for (int64_t l0 = 0; l0 < nlos; l0 += C) {
        const int64_t n = std::min(C, nlos - l0);
        if (int rc = rmsynth_execute(p, Q + l0 * p->nchan, U + l0 * p->nchan, n, RMSYNTH_LOS_MAJOR,
                                     RMSYNTH_FP32, Fq, Fu, nullptr, nullptr, 0, stream))
            return rc;
        if (int rc = rmsynth_peaks(p, Fq, Fu, n, idx, phk, amp, nullptr, nullptr, stream)) return rc;
        e = train_launch_labels(idx, phk, amp, n, (float)sp->det_threshold,
                                phi_label ? phi_label + l0 : nullptr,
                                det_label ? det_label + l0 : nullptr, s);
        if (e != hipSuccess) return rms_hip_fail(e, who);
    }
    return rms_ok();
}

// File: "RMSMLP01", int32 nchan, h1, h2, float phi_scale, int64 step,
// float channel weights [nchan], then params, Adam m, Adam v (canonical).
int rmsynth_mlp_save(rmsynth_mlp_t m, const char* path)
{
    if (!m || !path) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_save: NULL argument");
    if (int rc = check_mlp_device(m)) return rc;
    std::vector<float> P, M, V;
    if (int rc = read_vec(m, m->d_p, P, "rmsynth_mlp_save")) return rc;
    if (int rc = read_vec(m, m->d_m, M, "rmsynth_mlp_save")) return rc;
    if (int rc = read_vec(m, m->d_v, V, "rmsynth_mlp_save")) return rc;
    FILE* f = std::fopen(path, "wb");
    if (!f) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_save: cannot open %s", path);
    const int32_t dims[3] = {m->nchan, m->h1, m->h2};
    bool good = std::fwrite("RMSMLP01", 1, 8, f) == 8 && std::fwrite(dims, 4, 3, f) == 3 &&
                std::fwrite(&m->phi_scale, 4, 1, f) == 1 && std::fwrite(&m->step, 8, 1, f) == 1 &&
                std::fwrite(m->chan_w.data(), 4, m->nchan, f) == (size_t)m->nchan;
    for (const auto* vec : {&P, &M, &V})
        good = good && std::fwrite(vec->data(), 4, vec->size(), f) == vec->size();
    good = (std::fclose(f) == 0) && good;
    if (!good) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_save: write to %s failed", path);
    return rms_ok();
}

int rmsynth_mlp_load(const char* path, rmsynth_mlp_t* out)
{
    if (!path || !out) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_load: NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_load: cannot open %s", path);
    char magic[8];
    int32_t dims[3];
    float phi_scale = 0.0f;
    int64_t step = 0;
    bool good = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "RMSMLP01", 8) == 0 &&
                std::fread(dims, 4, 3, f) == 3 && std::fread(&phi_scale, 4, 1, f) == 1 &&
                std::fread(&step, 8, 1, f) == 1 && dims[0] >= 1 && dims[0] <= 65536 && step >= 0;
    std::vector<float> w;
    if (good) {
        w.resize(dims[0]);
        good = std::fread(w.data(), 4, w.size(), f) == w.size();
    }
    rmsynth_mlp_t m = nullptr;
    int rc = RMSYNTH_OK;
    if (good) rc = create(dims[0], dims[1], dims[2], w.data(), phi_scale, &m, "rmsynth_mlp_load");
    if (good && !rc) {
        std::vector<float> vec(m->canonical_size());
        float* dst[3] = {m->d_p, m->d_m, m->d_v};
        for (int i = 0; i < 3 && good && !rc; ++i) {
            good = std::fread(vec.data(), 4, vec.size(), f) == vec.size();
            if (good) rc = write_vec(m, vec.data(), dst[i], "rmsynth_mlp_load");
        }
        if (good && !rc) {
            m->step = step;
            hipError_t e = refresh_half(m, nullptr);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (e != hipSuccess) rc = rms_hip_fail(e, "rmsynth_mlp_load");
        }
    }
    std::fclose(f);
    if (!good || rc) {
        free_mlp(m);
        return rc ? rc : rms_fail(RMSYNTH_EINVAL, "rmsynth_mlp_load: %s is not a network file", path);
    }
    *out = m;
    return rms_ok();
}

void rmsynth_mlp_destroy(rmsynth_mlp_t m) { free_mlp(m); }

}  // extern "C"
