"""Pins of the FP64 RM-CLEAN oracle (oracle/rmclean.py).

* One on-grid thin screen (eqs. (1), (3)): its F is a R(phi - phi0) (the
  shift identity of eq. (11)/(12)), so every iteration removes the fraction
  gain of what is left at phi0: after n iterations the residual is exactly
  (1 - gain)^n F, the clean component (1 - (1 - gain)^n) a at phi0, and n is
  the first count at which (1 - gain)^n |a| < cutoff.
* Gain 1 on one screen: one iteration, zero residual.
* Bookkeeping for any run: F = sum_m C_m R(phi - phi_m) + residual.
* Nothing above the cutoff: no iteration, residual = F, restored = F.
* The restoring beam has peak 1 and half maximum at +-fwhm/2.
"""
import numpy as np
import pytest

from oracle import rmclean as rc
from synthetic import WORKLOADS, thin_spectrum, band_lambda2


def _setup(oracle_mod, nphi=201, step=2.0):
    wl = WORKLOADS["c3"]
    lam, w = wl.lambda2(), wl.weights()
    phi = -step * (nphi // 2) + step * np.arange(nphi)
    R2 = rc.rmsf_doubled(oracle_mod.rmsf, lam, w, step, nphi)
    fwhm, _ = oracle_mod.plan_info(lam, w)
    return lam, w, phi, R2, fwhm


@pytest.mark.parametrize("gain", [0.1, 0.3, 1.0])
def test_single_screen_closed_form(oracle_mod, gain):
    lam, w, phi, R2, fwhm = _setup(oracle_mod)
    k0s = np.array([100, 37, 180])
    P0 = np.array([0.05, 0.08, 0.02])
    P = thin_spectrum(lam, P0, phi[k0s], np.array([0.3, 1.1, 2.0]))
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    a = Fq[np.arange(3), k0s] + 1j * Fu[np.arange(3), k0s]
    cutoff = 1e-3
    out = rc.rmclean(Fq, Fu, R2, 2.0, gain, cutoff, 10000, fwhm)
    for l in range(3):
        n = 0
        while (1 - gain) ** n * abs(a[l]) >= cutoff:
            n += 1
        assert out["niter"][l] == n
        F = Fq[l] + 1j * Fu[l]
        np.testing.assert_allclose(out["resid"][l], (1 - gain) ** n * F, rtol=0, atol=1e-13)
        expect_cc = np.zeros(phi.size, complex)
        expect_cc[k0s[l]] = (1 - (1 - gain) ** n) * a[l]
        np.testing.assert_allclose(out["cc"][l], expect_cc, rtol=0, atol=1e-13)
    if gain == 1.0:
        assert np.all(out["niter"] == 1) and np.max(np.abs(out["resid"])) < 1e-14


def test_bookkeeping_holds_for_any_run(oracle_mod):
    """Several screens (off-grid too), noise, a thick slab: whatever the loop
    picks, the dirty spectrum is the components convolved with the RMSF plus
    the residual."""
    lam, w, phi, R2, fwhm = _setup(oracle_mod, nphi=151, step=2.0)
    rng = np.random.default_rng(4)
    n = 6
    P = 1e-3 * (rng.standard_normal((n, lam.size)) + 1j * rng.standard_normal((n, lam.size)))
    P += thin_spectrum(lam, rng.uniform(0.02, 0.1, n), rng.uniform(-100, 100, n), rng.uniform(0, 3, n))
    P += thin_spectrum(lam, rng.uniform(0.02, 0.1, n), rng.uniform(-100, 100, n), rng.uniform(0, 3, n))
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    out = rc.rmclean(Fq, Fu, R2, 2.0, 0.1, 5e-3, 500, fwhm)
    assert np.all(out["niter"] > 10)
    N = phi.size
    conv = np.array([[np.sum(out["cc"][l] * R2[(N - 1) + k - np.arange(N)]) for k in range(N)]
                     for l in range(n)])
    np.testing.assert_allclose(conv + out["resid"], Fq + 1j * Fu, rtol=0, atol=1e-13)
    # stopped because the residual peak fell below the cutoff
    assert np.all(np.abs(out["resid"]).max(axis=1) < 5e-3)


def test_nothing_above_the_cutoff(oracle_mod):
    lam, w, phi, R2, fwhm = _setup(oracle_mod, nphi=101)
    rng = np.random.default_rng(1)
    P = 1e-4 * (rng.standard_normal((3, lam.size)) + 1j * rng.standard_normal((3, lam.size)))
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    out = rc.rmclean(Fq, Fu, R2, 2.0, 0.1, 1.0, 100, fwhm)
    assert np.all(out["niter"] == 0)
    np.testing.assert_array_equal(out["resid"], Fq + 1j * Fu)
    np.testing.assert_array_equal(out["restored"], Fq + 1j * Fu)
    assert np.all(out["cc"] == 0)


def test_restoring_beam_and_restored_spectrum(oracle_mod):
    """A single component restores to a x Gaussian of peak 1 whose half
    maximum lies at +-fwhm/2, on top of the residual."""
    assert rc.restoring_beam(0.0, 7.0) == 1.0
    np.testing.assert_allclose(rc.restoring_beam([3.5, -3.5], 7.0), [0.5, 0.5], rtol=1e-15)
    lam, w, phi, R2, fwhm = _setup(oracle_mod)
    P = thin_spectrum(lam, 0.05, phi[100], 0.4)
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    out = rc.rmclean(Fq, Fu, R2, 2.0, 1.0, 1e-6, 1, fwhm)
    a = Fq[0, 100] + 1j * Fu[0, 100]
    expect = a * rc.restoring_beam(phi - phi[100], fwhm) + out["resid"][0]
    np.testing.assert_allclose(out["restored"][0], expect, rtol=0, atol=1e-15)


def test_the_rmsf_table_is_centred(oracle_mod):
    """R2[N - 1] = R(0) = 1 and R2 is Hermitian about it (eq. (12))."""
    lam, w, phi, R2, fwhm = _setup(oracle_mod, nphi=51)
    N = 51
    assert abs(R2[N - 1] - 1.0) < 1e-15
    np.testing.assert_allclose(R2[::-1], np.conj(R2), rtol=0, atol=1e-15)


def test_decisions_record_their_margins(oracle_mod):
    """Two equal screens make the first pick a tie (margin 0)."""
    lam = band_lambda2(700.0, 1800.0, 300)
    w = np.ones(lam.size)
    phi = np.arange(-100.0, 100.5, 2.0)
    R2 = rc.rmsf_doubled(oracle_mod.rmsf, lam, w, 2.0, phi.size)
    fwhm, _ = oracle_mod.plan_info(lam, w)
    P = thin_spectrum(lam, [0.05, 0.05], [-60.0, 60.0], [0.0, 0.0]).sum(axis=0, keepdims=True)
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    out = rc.rmclean(Fq, Fu, R2, 2.0, 0.5, 1e-3, 3, fwhm)
    assert out["pick_margin"][0] < 1e-9


def test_a_peak_equal_to_the_cutoff_is_cleaned(oracle_mod):
    """The loop stops only when |r_p| is below the cutoff: at equality it
    takes one more component (gain 1 then leaves a zero residual)."""
    lam, w, phi, R2, fwhm = _setup(oracle_mod, nphi=101)
    P = thin_spectrum(lam, 0.05, phi[40], 0.7)
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    a2 = Fq[0] ** 2 + Fu[0] ** 2
    cutoff = float(np.sqrt(a2[np.argmax(a2)]))
    out = rc.rmclean(Fq, Fu, R2, 2.0, 1.0, cutoff, 10, fwhm)
    assert out["niter"][0] == 1
