/*
 * FP64 reference implementation of RM synthesis -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously correct definition that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product library neither
 * links nor calls it, and the two share no code.
 *
 * What it computes (Sridhar, Heald & van der Hulst, "cuFFS", Section 2.2):
 *   K       = 1 / sum_j w_j                                   eq. (13)
 *   lambda0^2 = K sum_j w_j lambda_j^2  (the weighted mean of lambda^2; the
 *             paper sets lambda0^2 to the mean of lambda^2, which this equals
 *             for unit weights, and |F| does not depend on the choice)
 *   a_j     = lambda_j^2 - lambda0^2
 *   F(phi_k) = K sum_{j: w_j > 0} w_j (Q_j + i U_j) exp(-2 i phi_k a_j)
 *                                                             eq. (11)
 *   whose real and imaginary parts are eqs. (15)-(16):
 *     Qt(phi) = K sum w (Q cos 2phi a + U sin 2phi a)
 *     Ut(phi) = K sum w (U cos 2phi a - Q sin 2phi a)
 *   |F|     = sqrt(Qt^2 + Ut^2)                               eq. (17)
 *   R(phi_k) = K sum_j w_j exp(-2 i phi_k a_j)                eq. (12)
 *   for every phi_k of the grid and every line of sight   eqs. (18)-(19)
 *   phi_peak = the grid phi where |F| is largest (Section 2.2, after
 *             eq. (14)); ties go to the lowest index.
 *   resolution 2 sqrt(3) / Delta lambda^2 and largest scale sqrt(3) /
 *             delta lambda^2                                eqs. (20)-(21)
 *   work estimate 15 N_chan N_phi N_los FLOP                 Section 2.3
 *
 * Channels of weight 0 are skipped, so whatever they hold (NaN included)
 * has no effect.  Sums run over ascending channel index in FP64; cos and sin
 * are libm's, applied to theta = 2 phi_k a_j with no manual reduction.
 * "Table mode" evaluates the same cos/sin once per (channel, phi) and then
 * runs the identical loop, so its results are bitwise those of literal mode.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_LOS_MAJOR 0
#define ORACLE_FREQ_MAJOR 1

/* eq. (13) and the lambda0^2 definition.  Returns 0, or -1 on invalid input
 * (nchan < 1, a weight negative or non-finite, lambda^2 non-finite, sum w <= 0). */
int oracle_plan(const double* lambda2, const double* w, int32_t nchan,
                double lambda0_sq_in, double* K_out, double* lambda0_sq_out)
{
    if (nchan < 1 || !lambda2 || !w) return -1;
    double sw = 0.0, swl = 0.0;
    for (int32_t j = 0; j < nchan; ++j) {
        if (!isfinite(w[j]) || w[j] < 0.0 || !isfinite(lambda2[j])) return -1;
        sw += w[j];
        swl += w[j] * lambda2[j];
    }
    if (!(sw > 0.0)) return -1;
    double K = 1.0 / sw;
    *K_out = K;
    *lambda0_sq_out = isnan(lambda0_sq_in) ? K * swl : lambda0_sq_in;
    return 0;
}

/* eqs. (20)-(21).  Delta lambda^2 is the span of lambda^2 over channels of
 * non-zero weight; delta lambda^2 (the channel width) is taken as the widest
 * gap between adjacent channel centres, all channels included. */
static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

int oracle_plan_info(const double* lambda2, const double* w, int32_t nchan,
                     double* fwhm_est, double* phimax_est)
{
    if (nchan < 1) return -1;
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t j = 0; j < nchan; ++j)
        if (w[j] > 0.0) {
            if (lambda2[j] < lo) lo = lambda2[j];
            if (lambda2[j] > hi) hi = lambda2[j];
        }
    *fwhm_est = (hi > lo) ? 2.0 * sqrt(3.0) / (hi - lo) : INFINITY;
    double* s = (double*)malloc(sizeof(double) * (size_t)nchan);
    if (!s) return -1;
    memcpy(s, lambda2, sizeof(double) * (size_t)nchan);
    qsort(s, (size_t)nchan, sizeof(double), cmp_double);
    double gap = 0.0;
    for (int32_t j = 1; j < nchan; ++j)
        if (s[j] - s[j - 1] > gap) gap = s[j] - s[j - 1];
    free(s);
    *phimax_est = (gap > 0.0) ? sqrt(3.0) / gap : INFINITY;
    return 0;
}

/* Section 2.3: ~15 N_chan N_phi N_los floating-point operations. */
double oracle_cost_flop(int64_t nlos, int64_t nchan, int64_t nphi)
{
    return 15.0 * (double)nchan * (double)nphi * (double)nlos;
}

/* The Faraday-depth transform, eqs. (11), (15)-(16), for every LOS.
 * Q, U: layout 0 = [nlos][nchan], layout 1 = [nchan][nlos].
 * Fq, Fu: [nlos][nphi] (phi fastest).
 * table_mode != 0 evaluates cos/sin per (phi, channel) once up front. */
int oracle_fdf(const double* Q, const double* U, int64_t nlos, int32_t layout,
               const double* lambda2, const double* w, int32_t nchan,
               const double* phi, int32_t nphi, double K, double lambda0_sq,
               int32_t table_mode, double* Fq, double* Fu)
{
    if (nlos < 0 || nchan < 1 || nphi < 1) return -1;
    if (layout != ORACLE_LOS_MAJOR && layout != ORACLE_FREQ_MAJOR) return -1;
    double* ctab = NULL;
    double* stab = NULL;
    if (table_mode) {
        size_t n = (size_t)nphi * (size_t)nchan;
        ctab = (double*)malloc(sizeof(double) * n);
        stab = (double*)malloc(sizeof(double) * n);
        if (!ctab || !stab) { free(ctab); free(stab); return -1; }
        for (int32_t k = 0; k < nphi; ++k)
            for (int32_t j = 0; j < nchan; ++j) {
                double theta = 2.0 * phi[k] * (lambda2[j] - lambda0_sq);
                ctab[(size_t)k * nchan + j] = cos(theta);
                stab[(size_t)k * nchan + j] = sin(theta);
            }
    }
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t l = 0; l < nlos; ++l) {
        for (int32_t k = 0; k < nphi; ++k) {
            double re = 0.0, im = 0.0;
            for (int32_t j = 0; j < nchan; ++j) {
                if (!(w[j] > 0.0)) continue;          /* flagged channel */
                size_t at = (layout == ORACLE_LOS_MAJOR) ? (size_t)l * nchan + j
                                                         : (size_t)j * nlos + l;
                double x = w[j] * Q[at];
                double y = w[j] * U[at];
                double c, s;
                if (table_mode) {
                    c = ctab[(size_t)k * nchan + j];
                    s = stab[(size_t)k * nchan + j];
                } else {
                    double theta = 2.0 * phi[k] * (lambda2[j] - lambda0_sq);
                    c = cos(theta);
                    s = sin(theta);
                }
                re += x * c + y * s;
                im += y * c - x * s;
            }
            Fq[(size_t)l * nphi + k] = K * re;
            Fu[(size_t)l * nphi + k] = K * im;
        }
    }
    free(ctab);
    free(stab);
    return 0;
}

/* eq. (4) with the integral over phi replaced by the sum over the grid: the
 * spectrum of a Faraday dispersion function made of components C_k at the
 * grid depths phi_k, referred to lambda0^2 as eq. (11) refers F,
 *   P(lambda_j^2) = sum_k C_k exp(+2 i phi_k (lambda_j^2 - lambda0^2)),
 * for every channel (weights play no part) and every line of sight.
 * C: [nlos][nphi] (phi fastest); P: [nlos][nchan].  K w_j P_j is the adjoint
 * of eq. (11) applied to C. */
int oracle_adjoint(const double* Cre, const double* Cim, int64_t nlos, const double* phi,
                   int32_t nphi, const double* lambda2, int32_t nchan, double lambda0_sq,
                   double* Pre, double* Pim)
{
    if (nlos < 0 || nchan < 1 || nphi < 1) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t l = 0; l < nlos; ++l) {
        for (int32_t j = 0; j < nchan; ++j) {
            double re = 0.0, im = 0.0;
            for (int32_t k = 0; k < nphi; ++k) {
                double theta = 2.0 * phi[k] * (lambda2[j] - lambda0_sq);
                double c = cos(theta), s = sin(theta);
                double x = Cre[(size_t)l * nphi + k], y = Cim[(size_t)l * nphi + k];
                re += x * c - y * s;
                im += y * c + x * s;
            }
            Pre[(size_t)l * nchan + j] = re;
            Pim[(size_t)l * nchan + j] = im;
        }
    }
    return 0;
}

/* eq. (12): the RMSF on the phi grid. */
int oracle_rmsf(const double* lambda2, const double* w, int32_t nchan,
                const double* phi, int32_t nphi, double K, double lambda0_sq,
                double* R_re, double* R_im)
{
    if (nchan < 1 || nphi < 1) return -1;
    for (int32_t k = 0; k < nphi; ++k) {
        double re = 0.0, im = 0.0;
        for (int32_t j = 0; j < nchan; ++j) {
            if (!(w[j] > 0.0)) continue;
            double theta = 2.0 * phi[k] * (lambda2[j] - lambda0_sq);
            re += w[j] * cos(theta);
            im -= w[j] * sin(theta);
        }
        R_re[k] = K * re;
        R_im[k] = K * im;
    }
    return 0;
}

/* Peak of |F| per LOS: idx = smallest k attaining the maximum of
 * hypot(Fq, Fu); phi_pk = phi[idx]; amp = |F| there; q_pk, u_pk = Fq, Fu
 * there; margin = (largest - second largest) / largest over k != idx.
 * A LOS with any non-finite |F| gets idx = -1 and NaN outputs. */
int oracle_peaks(const double* Fq, const double* Fu, int64_t nlos, int32_t nphi,
                 const double* phi, int32_t* idx, double* phi_pk, double* amp,
                 double* q_pk, double* u_pk, double* margin)
{
    if (nlos < 0 || nphi < 1) return -1;
    #pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < nlos; ++l) {
        const double* q = Fq + (size_t)l * nphi;
        const double* u = Fu + (size_t)l * nphi;
        int32_t best = 0;
        double m1 = -1.0;
        int finite = 1;
        for (int32_t k = 0; k < nphi; ++k) {
            double a = hypot(q[k], u[k]);
            if (!isfinite(a)) { finite = 0; break; }
            if (a > m1) { m1 = a; best = k; }
        }
        if (!finite) {
            idx[l] = -1;
            phi_pk[l] = amp[l] = q_pk[l] = u_pk[l] = margin[l] = NAN;
            continue;
        }
        double m2 = 0.0;
        for (int32_t k = 0; k < nphi; ++k) {
            if (k == best) continue;
            double a = hypot(q[k], u[k]);
            if (a > m2) m2 = a;
        }
        idx[l] = best;
        phi_pk[l] = phi[best];
        amp[l] = m1;
        q_pk[l] = q[best];
        u_pk[l] = u[best];
        margin[l] = (m1 > 0.0) ? (m1 - m2) / m1 : 0.0;
    }
    return 0;
}

/* Number of OpenMP threads the parallel loops above use. */
#ifdef _OPENMP
#include <omp.h>
#endif
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
