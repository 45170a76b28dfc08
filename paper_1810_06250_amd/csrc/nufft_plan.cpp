// Plan-time tables of the NUFFT evaluation (nufft.hip), built on the host in
// FP64 when the phi grid is uniform:
//   n        grid size: the smallest power of two >= max(2 nphi, 16);
//   kc       index of the grid's centre phi_c = phi_0 + kc dphi, kc = nphi / 2;
//   rot_j    K w_j exp(-2i a_j phi_c) (the factor c_j = rot_j P_j);
//   entries  for every grid point p in order, the channels j (w_j > 0) whose
//            kernel reaches it, periodic distance d = x_p - x_j wrapped to
//            [-pi, pi), |d| < alpha, with weight psi(d); x_p = 2 pi p / n,
//            x_j = 2 a_j dphi mod 2 pi; packed ((j << 13) | p, bits of
//            psi(d)); only grid points with entries are listed, off[i] the
//            first entry of the i-th of them;
//   tw_t     exp(-2 pi i t / n);
//   deconv_k (2 pi / n) / psi_hat(k - kc), psi_hat by 512-point Gauss-Legendre
//            quadrature of int psi(t) cos(m t) dt over [-alpha, alpha];
// psi(t) = exp(beta (sqrt(1 - (t / alpha)^2) - 1)), alpha = W pi / n,
// beta = 2.30 W, W = kNufftWidth grid cells (Barnett, Magland &
// af Klinteberg, SIAM J. Sci. Comput. 41, 2019).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace {

// Nodes and weights of the m-point Gauss-Legendre rule on [-1, 1]: Newton's
// method on the Legendre polynomial P_m from the usual cosine starting values.
void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < m; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

template <typename T>
int upload(T** dst, const std::vector<T>& v)
{
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), sizeof(T) * (v.size() ? v.size() : 1));
    if (e != hipSuccess) return rms_fail(RMSYNTH_ENOMEM, "rmsynth_plan: hipMalloc (NUFFT tables): %s", hipGetErrorString(e));
    if (v.size() && (e = hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return rms_hip_fail(e, "rmsynth_plan: hipMemcpy (NUFFT tables)");
    return RMSYNTH_OK;
}

}  // namespace

int build_nufft_tables(rmsynth_plan_s* p, const double* lambda2, const double* weights)
{
    int n = 16;
    while (n < 2 * p->nphi) n *= 2;
    if (n > kNufftMaxGrid || p->nchan > kNufftMaxChan) return RMSYNTH_OK;  // no NUFFT for this plan
    const int W = kNufftWidth;
    const double alpha = W * M_PI / n, beta = 2.30 * W;
    const int kc = p->nphi / 2;
    const double phic = p->phi0 + kc * p->dphi;
    auto psi = [&](double t) {
        const double z = t / alpha;
        return std::fabs(z) < 1.0 ? std::exp(beta * (std::sqrt(1.0 - z * z) - 1.0)) : 0.0;
    };

    std::vector<float2> rot(p->nchan);
    std::vector<std::vector<std::pair<int, float>>> lists(n);
    for (int32_t j = 0; j < p->nchan; ++j) {
        const double a = lambda2[j] - p->lambda0_sq;
        const double kw = p->K * weights[j];
        rot[j] = make_float2((float)(kw * std::cos(2.0 * a * phic)), (float)(-kw * std::sin(2.0 * a * phic)));
        if (!(weights[j] > 0.0)) continue;
        double x = std::fmod(2.0 * a * p->dphi, 2.0 * M_PI);
        if (x < 0.0) x += 2.0 * M_PI;
        const long centre = (long)std::floor(x * n / (2.0 * M_PI));
        for (long o = -W - 1; o <= W + 1; ++o) {
            const long pp = ((centre + o) % n + n) % n;
            double d = std::fmod(2.0 * M_PI * pp / n - x + M_PI, 2.0 * M_PI);
            if (d < 0.0) d += 2.0 * M_PI;
            d -= M_PI;
            if (std::fabs(d) < alpha) lists[pp].push_back({j, (float)psi(d)});
        }
    }
    std::vector<int> off;
    std::vector<int2> ent;
    for (int pp = 0; pp < n; ++pp) {
        if (lists[pp].empty()) continue;
        off.push_back((int)ent.size());
        for (auto& e : lists[pp]) {
            float wt = e.second;
            int bits;
            std::memcpy(&bits, &wt, sizeof bits);
            ent.push_back(make_int2((e.first << 13) | pp, bits));
        }
    }
    const int nocc = (int)off.size();
    off.push_back((int)ent.size());
    std::vector<float2> tw(n);
    for (int t = 0; t < n; ++t)
        tw[t] = make_float2((float)std::cos(2.0 * M_PI * t / n), (float)(-std::sin(2.0 * M_PI * t / n)));
    std::vector<double> gx, gw;
    gauss_legendre(512, gx, gw);
    std::vector<float> deconv(p->nphi);
    for (int32_t k = 0; k < p->nphi; ++k) {
        const double m = (double)(k - kc);
        double s = 0.0;
        for (size_t i = 0; i < gx.size(); ++i)
            s += gw[i] * std::exp(beta * (std::sqrt(1.0 - gx[i] * gx[i]) - 1.0)) * std::cos(m * alpha * gx[i]);
        deconv[k] = (float)((2.0 * M_PI / n) / (alpha * s));
    }
    if (int rc = upload(&p->d_nufft_rot, rot)) return rc;
    if (int rc = upload(&p->d_nufft_off, off)) return rc;
    if (int rc = upload(&p->d_nufft_ent, ent)) return rc;
    if (int rc = upload(&p->d_nufft_tw, tw)) return rc;
    if (int rc = upload(&p->d_nufft_deconv, deconv)) return rc;
    p->nufft_n = n;
    p->nufft_kc = kc;
    p->nufft_nocc = nocc;
    return RMSYNTH_OK;
}
