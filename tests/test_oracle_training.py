"""Pins of the training-data oracle: Philox4x32-10 against its published
known-answer vectors, the uniform and normal variates against their exact
properties and distributions, the class mix, and the sky model against the
closed forms of a noiseless Faraday-thin screen and Burn slab (Section 2.1,
eqs. (1), (3), (4)), whose transforms peak at the injected depth."""
import json
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import training as tr
from synthetic import band_lambda2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")

SPEC = dict(frac_noise=0.25, frac_thin1=0.30, frac_thin2=0.20, p0_lo=1e-3, p0_hi=2e-2,
            phi_lo=-300.0, phi_hi=300.0, w_lo=10.0, w_hi=100.0, sigma=1e-3, det_threshold=5e-4)


def test_philox_known_answers():
    for v in json.load(open(GOLDEN))["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = tr.philox4x32_10(np.array([ctr], dtype=np.uint64), key)[0]
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_uniform24_exact_in_fp32_and_open_interval():
    x = np.array([0, 511, 512, 2 ** 31, 2 ** 32 - 1], dtype=np.uint64)
    u = tr.uniform24(x)
    assert np.all(u > 0) and np.all(u < 1)
    np.testing.assert_array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == u[1] == 2.0 ** -24 and u[2] == 1.5 * 2.0 ** -23
    assert u[3] == 0.5 + 2.0 ** -24 and u[-1] == 1.0 - 2.0 ** -24
    # Every output of a large sample is exact in FP32 too.
    w = tr.philox4x32_10(np.arange(4000, dtype=np.uint64).reshape(-1, 4), (1, 2)).ravel()
    uw = tr.uniform24(w)
    np.testing.assert_array_equal(uw.astype(np.float32).astype(np.float64), uw)


def test_noise_is_standard_normal_and_independent():
    nQ, nU = tr.noise(12345, np.arange(2000, dtype=np.uint64), 101)
    z = np.concatenate([nQ.ravel(), nU.ravel()])
    assert z.size == 2 * 2000 * 101
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # Q and U of one channel, and neighbouring channels, are uncorrelated.
    assert abs(np.corrcoef(nQ.ravel(), nU.ravel())[0, 1]) < 5 / np.sqrt(nQ.size)
    assert abs(np.corrcoef(nQ[:, :-1].ravel(), nQ[:, 1:].ravel())[0, 1]) < 5 / np.sqrt(nQ.size)
    # A different seed or line of sight gives different draws.
    a, _ = tr.noise(12346, np.arange(2000, dtype=np.uint64), 101)
    assert not np.allclose(a, nQ)


def test_class_fractions_and_components():
    g = np.arange(200_000, dtype=np.uint64)
    cls = tr.classes(SPEC, 7, g)
    want = [0.25, 0.30, 0.20, 0.25]
    for k, f in enumerate(want):
        frac = np.mean(cls == k)
        assert abs(frac - f) < 5 * np.sqrt(f * (1 - f) / g.size), (k, frac)
    P0, phi0, chi0, W = tr.components(SPEC, 7, g, 0)
    assert P0.min() >= SPEC["p0_lo"] and P0.max() <= SPEC["p0_hi"]
    assert phi0.min() >= -300 and phi0.max() <= 300 and abs(phi0.mean()) < 2.0
    assert chi0.min() > 0 and chi0.max() < np.pi
    assert W.min() >= 10 and W.max() <= 100
    assert stats.kstest((phi0 + 300) / 600, "uniform").pvalue > 1e-3


def test_noiseless_thin_screen_closed_form_and_peak():
    lam = band_lambda2(800.0, 1088.0, 288)
    spec = dict(SPEC, sigma=0.0, frac_noise=0.0, frac_thin1=1.0, frac_thin2=0.0)
    Q, U, cls, truth = tr.spectra(spec, 99, 1000, 16, lam)
    assert np.all(cls == 1) and np.all(np.isnan(truth[:, 2]))
    P = Q + 1j * U
    phi0, P0 = truth[:, 0], truth[:, 1]
    # |P| = P0 on every channel; the phase advances as 2 phi0 lambda^2 (eq. (3)).
    np.testing.assert_allclose(np.abs(P), P0[:, None] * np.ones_like(lam), rtol=2e-7)
    derot = P * np.exp(-2j * phi0[:, None] * lam[None, :])
    np.testing.assert_allclose(derot, derot[:, :1] * np.ones_like(lam), rtol=1e-6, atol=1e-9)
    # The transform of a noiseless screen peaks at phi0 within half a grid step.
    w = np.ones(lam.size)
    phi = np.arange(-300.0, 300.0 + 0.25, 0.5)
    phi_label, det, pk, _ = tr.labels(Q, U, lam, w, phi, spec["det_threshold"], oracle.fdf, oracle.peaks)
    assert np.all(np.abs(phi_label - phi0) <= 0.25 + 1e-9)
    np.testing.assert_allclose(pk["amp"], P0, rtol=1e-3)
    assert np.all(det == (P0 >= spec["det_threshold"]))


def test_noiseless_slab_closed_form():
    lam = band_lambda2(800.0, 1088.0, 288)
    spec = dict(SPEC, sigma=0.0, frac_noise=0.0, frac_thin1=0.0, frac_thin2=0.0)
    Q, U, cls, truth = tr.spectra(spec, 5, 0, 8, lam)
    assert np.all(cls == 3)
    _, _, _, W = tr.components(spec, 5, np.arange(8, dtype=np.uint64), 0)
    x = W[:, None] * lam[None, :]
    np.testing.assert_allclose(np.hypot(Q, U), truth[:, 1:2] * np.abs(np.sin(x) / x), rtol=2e-6,
                               atol=1e-12)


def test_two_screens_are_the_sum_of_their_parts():
    lam = band_lambda2(800.0, 1088.0, 64)
    spec2 = dict(SPEC, sigma=0.0, frac_noise=0.0, frac_thin1=0.0, frac_thin2=1.0)
    Q, U, cls, truth = tr.spectra(spec2, 3, 0, 10, lam)
    assert np.all(cls == 2) and np.all(np.isfinite(truth))
    g = np.arange(10, dtype=np.uint64)
    P = np.zeros((10, lam.size), complex)
    for c in (0, 1):
        P0, phi0, chi0, _ = tr.components(spec2, 3, g, c)
        P += P0[:, None] * np.exp(2j * (chi0[:, None] + phi0[:, None] * lam[None, :]))
    np.testing.assert_allclose(Q, P.real, atol=1e-9)
    np.testing.assert_allclose(U, P.imag, atol=1e-9)


def test_counter_addressing_is_position_free():
    """Line of sight g gets the same content whatever batch it is made in."""
    lam = band_lambda2(800.0, 1088.0, 40)
    a = tr.spectra(SPEC, 11, 100, 50, lam)
    b = tr.spectra(SPEC, 11, 130, 5, lam)
    np.testing.assert_array_equal(a[0][30:35], b[0])
    np.testing.assert_array_equal(a[2][30:35], b[2])
