"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each checks it against an
independent fact -- a library FFT, a closed form, a symmetry, an invariance,
or a value the paper prints -- so that a dropped term, a wrong sign or index,
or a transposed operand fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

from synthetic import band_lambda2, thin_spectrum, make_small_cube, WORKLOADS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _uniform_lambda2(n, start=0.05, delta=0.001):
    return start + delta * np.arange(n)


# ---------------------------------------------------------------- eq. (11)
def test_fft_special_case(oracle_mod):
    """Uniform lambda^2 spacing d, unit weights and phi_k = pi k / (N d):
    eq. (11) becomes a length-N DFT, F_k = K exp(i pi k (N-1)/N) FFT(P)_k."""
    rng = np.random.default_rng(1)
    for n in (7, 16, 33):
        d = 0.0013
        lam = _uniform_lambda2(n, 0.07, d)
        w = np.ones(n)
        phi = np.pi * np.arange(n) / (n * d)
        P = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
        Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
        k = np.arange(n)
        expect = (1.0 / n) * np.exp(1j * np.pi * k * (n - 1) / n) * np.fft.fft(P, axis=1)
        np.testing.assert_allclose(Fq + 1j * Fu, expect, rtol=0, atol=1e-12)


def test_thin_source_on_grid(oracle_mod):
    """A noise-free Faraday-thin screen (eqs. (1), (3)) at a grid depth phi0
    gives |F(phi0)| = P0, its peak at phi0 and arg F(phi0) = 2(chi0 + phi0 l0^2)."""
    lam = band_lambda2(120.0, 168.0, 128)
    w = np.ones(lam.size)
    phi = np.arange(-100.0, 100.5, 1.0)
    P0, phi0, chi0 = 0.0731, 37.0, 0.4
    P = thin_spectrum(lam, P0, phi0, chi0)
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    K, l0 = oracle_mod.plan(lam, w)
    k0 = int(np.flatnonzero(phi == phi0)[0])
    assert abs(np.hypot(Fq[0, k0], Fu[0, k0]) - P0) < 1e-13
    pk = oracle_mod.peaks(Fq, Fu, phi)
    assert pk["idx"][0] == k0 and pk["phi_pk"][0] == phi0
    ang = np.angle(Fq[0, k0] + 1j * Fu[0, k0])
    d = np.angle(np.exp(1j * (ang - 2 * (chi0 + phi0 * l0))))
    assert abs(d) < 1e-12


def test_thin_source_shift_identity(oracle_mod):
    """F(phi) = P0 exp(2i(chi0 + phi0 l0^2)) R(phi - phi0): the transform of a
    thin screen is the RMSF (eq. (12)) moved to phi0."""
    lam = band_lambda2(700.0, 1800.0, 400)
    rng = np.random.default_rng(3)
    w = (rng.uniform(size=lam.size) > 0.1).astype(float) * rng.uniform(0.5, 2.0, lam.size)
    phi = np.linspace(-300, 300, 241)
    P0, phi0, chi0 = 0.05, 12.345, 2.1
    P = thin_spectrum(lam, P0, phi0, chi0)
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    K, l0 = oracle_mod.plan(lam, w)
    Rr, Ri = oracle_mod.rmsf(lam, w, phi - phi0)
    expect = P0 * np.exp(2j * (chi0 + phi0 * l0)) * (Rr + 1j * Ri)
    np.testing.assert_allclose(Fq[0] + 1j * Fu[0], expect, rtol=0, atol=1e-13)


def test_peak_angle_recovers_the_screen_angle(oracle_mod):
    """Eq. (14): for thin screens (eqs. (1), (3)) the angle at the peak,
    referred to lambda^2 = 0, is the screen's intrinsic angle chi0 (mod pi),
    whatever lambda0^2 the transform used, although the phase of F(phi_pk)
    itself moves with lambda0^2."""
    lam = band_lambda2(120.0, 168.0, 128)
    w = np.ones(lam.size)
    phi = np.arange(-100.0, 100.5, 1.0)
    rng = np.random.default_rng(17)
    n = 40
    phi0 = phi[rng.integers(10, phi.size - 10, n)]
    chi0 = rng.uniform(-2 * np.pi, 2 * np.pi, n)
    P = thin_spectrum(lam, rng.uniform(0.01, 0.1, n), phi0, chi0)
    phases = []
    for l0 in (float("nan"), 0.0, 3.7):
        Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi, lambda0_sq=l0)
        pk = oracle_mod.peaks(Fq, Fu, phi)
        np.testing.assert_array_equal(pk["phi_pk"], phi0)
        used = oracle_mod.plan(lam, w)[1] if np.isnan(l0) else l0
        chi = oracle_mod.peak_angle(pk["q_pk"], pk["u_pk"], pk["phi_pk"], used)
        assert np.all((chi >= 0) & (chi < np.pi))
        d = np.angle(np.exp(2j * (chi - chi0))) / 2
        assert np.max(np.abs(d)) < 1e-12
        phases.append(np.angle(pk["q_pk"] + 1j * pk["u_pk"]))
    assert np.max(np.abs(np.angle(np.exp(1j * (phases[1] - phases[2]))))) > 0.1
    nan = oracle_mod.peak_angle([np.nan, 1.0], [0.0, np.inf], [0.0, 1.0], 0.5)
    assert np.all(np.isnan(nan))


def test_off_grid_source_peaks_at_nearest_node(oracle_mod):
    """|R| is symmetric and falls monotonically on its main lobe, so a
    noise-free screen between grid nodes peaks at the nearest node."""
    wl = WORKLOADS["c1"]
    lam, w, phi = wl.lambda2(), wl.weights(), wl.phi()
    rng = np.random.default_rng(5)
    phi0 = rng.uniform(-80, 80, 50)
    P = thin_spectrum(lam, rng.uniform(0.01, 0.1, 50), phi0, rng.uniform(0, np.pi, 50))
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    pk = oracle_mod.peaks(Fq, Fu, phi)
    np.testing.assert_array_equal(pk["idx"], np.rint(phi0 - phi[0]).astype(int))


def test_linearity_complex_scalars(oracle_mod):
    """F is linear over complex scalars in P = Q + iU."""
    c = make_small_cube(4, 50, 21, seed=7, nsrc=2)
    d = make_small_cube(4, 50, 21, seed=8, nsrc=1)
    a, b = 0.3 - 1.7j, -2.2 + 0.4j
    P1, P2 = c["Q"] + 1j * c["U"], d["Q"] + 1j * d["U"]
    args = (c["lambda2"], c["weights"], c["phi"])
    F1 = np.add(*[x * y for x, y in zip(oracle_mod.fdf(P1.real, P1.imag, *args), (1, 1j))])
    F2 = np.add(*[x * y for x, y in zip(oracle_mod.fdf(P2.real, P2.imag, *args), (1, 1j))])
    Pm = a * P1 + b * P2
    Fq, Fu = oracle_mod.fdf(Pm.real, Pm.imag, *args)
    np.testing.assert_allclose(Fq + 1j * Fu, a * F1 + b * F2, rtol=0, atol=1e-14)


def test_flagged_channels_have_no_effect(oracle_mod):
    """Channels of weight 0 contribute nothing, whatever they hold, and the
    result equals the transform of the unflagged channels alone."""
    c = make_small_cube(6, 80, 31, seed=11, nflag=9, nsrc=3)
    lam, w, phi = c["lambda2"], c["weights"], c["phi"]
    Q, U = c["Q"].copy(), c["U"].copy()
    ref = oracle_mod.fdf(Q, U, lam, w, phi)
    flagged = w == 0
    Q[:, flagged] = np.nan
    U[:, flagged] = 1e30
    got = oracle_mod.fdf(Q, U, lam, w, phi)
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1], ref[1])
    keep = ~flagged
    K, l0 = oracle_mod.plan(lam, w)
    alone = oracle_mod.fdf(c["Q"][:, keep], c["U"][:, keep], lam[keep], w[keep], phi,
                           lambda0_sq=l0)
    np.testing.assert_allclose(alone[0], ref[0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(alone[1], ref[1], rtol=0, atol=1e-15)


def test_amplitude_independent_of_lambda0(oracle_mod):
    """Changing lambda0^2 multiplies F(phi) by exp(2i phi (l0'^2 - l0^2)): the
    Q/U phases move and |F| does not."""
    c = make_small_cube(5, 64, 41, seed=13, nsrc=2)
    lam, w, phi = c["lambda2"], c["weights"], c["phi"]
    K, l0 = oracle_mod.plan(lam, w)
    F0 = np.add(*[x * y for x, y in zip(oracle_mod.fdf(c["Q"], c["U"], lam, w, phi), (1, 1j))])
    for l0b in (0.0, 1.7, l0 * 0.5):
        q, u = oracle_mod.fdf(c["Q"], c["U"], lam, w, phi, lambda0_sq=l0b)
        F1 = q + 1j * u
        np.testing.assert_allclose(np.abs(F1), np.abs(F0), rtol=0, atol=1e-14)
        np.testing.assert_allclose(F1, F0 * np.exp(2j * phi * (l0b - l0)), rtol=0, atol=1e-14)


def test_weights_normalised_by_K(oracle_mod):
    """Scaling every weight by the same factor leaves F unchanged (eq. (13))."""
    c = make_small_cube(3, 40, 17, seed=17, nflag=4, nsrc=1)
    lam, w, phi = c["lambda2"], c["weights"], c["phi"]
    a = oracle_mod.fdf(c["Q"], c["U"], lam, w, phi)
    b = oracle_mod.fdf(c["Q"], c["U"], lam, 3.7 * w, phi)
    np.testing.assert_allclose(a[0], b[0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(a[1], b[1], rtol=0, atol=1e-13)


def test_layouts_agree(oracle_mod):
    """A frequency-major cube gives the same F as its LOS-major transpose."""
    c = make_small_cube(7, 30, 13, seed=19, nsrc=2)
    args = (c["lambda2"], c["weights"], c["phi"])
    a = oracle_mod.fdf(c["Q"], c["U"], *args, layout=0)
    b = oracle_mod.fdf(c["Q"].T.copy(), c["U"].T.copy(), *args, layout=1)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_table_mode_bitwise_equals_literal(oracle_mod):
    c = make_small_cube(4, 60, 25, seed=23, nflag=5, nsrc=2)
    args = (c["Q"], c["U"], c["lambda2"], c["weights"], c["phi"])
    a = oracle_mod.fdf(*args, table_mode=True)
    b = oracle_mod.fdf(*args, table_mode=False)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_triple_loop_matches_matrix_product(oracle_mod):
    """Second, independent evaluation: one complex128 matrix product."""
    for seed, nflag in ((29, 0), (31, 6)):
        c = make_small_cube(9, 48, 19, seed=seed, nflag=nflag, nsrc=3)
        args = (c["Q"], c["U"], c["lambda2"], c["weights"], c["phi"])
        a = oracle_mod.fdf(*args)
        b = oracle_mod.fdf_bruteforce(*args)
        np.testing.assert_allclose(a[0], b[0], rtol=0, atol=1e-13)
        np.testing.assert_allclose(a[1], b[1], rtol=0, atol=1e-13)


# ---------------------------------------------------------------- eq. (12)
def test_rmsf_dirichlet_closed_form(oracle_mod):
    """Unit weights on a uniform lambda^2 grid of spacing d, centred by
    lambda0^2 = mean: R(phi) = sin(N phi d) / (N sin(phi d)), real."""
    for n in (8, 25, 100):
        d = 0.0007
        lam = _uniform_lambda2(n, 0.2, d)
        phi = np.linspace(-400.3, 400.1, 301)
        Rr, Ri = oracle_mod.rmsf(lam, np.ones(n), phi)
        expect = np.sin(n * phi * d) / (n * np.sin(phi * d))
        np.testing.assert_allclose(Rr, expect, rtol=0, atol=2e-14)
        np.testing.assert_allclose(Ri, 0.0, rtol=0, atol=2e-14)


def test_rmsf_properties(oracle_mod):
    """R(0) = 1, |R| <= 1, R(-phi) = conj R(phi)."""
    lam = band_lambda2(110.0, 190.0, 300)
    rng = np.random.default_rng(37)
    w = rng.uniform(0, 2, lam.size) * (rng.uniform(size=lam.size) > 0.2)
    phi = np.linspace(-50, 50, 201)  # symmetric, contains 0
    Rr, Ri = oracle_mod.rmsf(lam, w, phi)
    assert abs(Rr[100] - 1.0) < 1e-15 and abs(Ri[100]) < 1e-15
    assert np.all(np.hypot(Rr, Ri) <= 1.0 + 1e-15)
    np.testing.assert_allclose(Rr[::-1], Rr, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Ri[::-1], -Ri, rtol=0, atol=1e-15)


def test_unit_spectrum_gives_rmsf(oracle_mod):
    """Q = 1, U = 0 in every channel: eq. (11) reduces to eq. (12)."""
    lam = band_lambda2(800.0, 1088.0, 288)
    rng = np.random.default_rng(41)
    w = (rng.uniform(size=lam.size) > 0.05).astype(float)
    phi = np.arange(-300, 300.25, 0.5)
    q, u = oracle_mod.fdf(np.ones((1, lam.size)), np.zeros((1, lam.size)), lam, w, phi)
    Rr, Ri = oracle_mod.rmsf(lam, w, phi)
    np.testing.assert_allclose(q[0], Rr, rtol=0, atol=1e-15)
    np.testing.assert_allclose(u[0], Ri, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_rmsf_fwhm_near_eq20(oracle_mod, name):
    """eq. (20) is an estimate: the measured FWHM of |R| on a fine grid must
    sit within [1.0, 1.45] times 2 sqrt(3) / Delta lambda^2 for the bands of
    the synthetic workloads."""
    wl = WORKLOADS[name]
    lam, w = wl.lambda2(), wl.weights()
    est, _ = oracle_mod.plan_info(lam, w)
    phi = np.linspace(0, 2.0 * est, 4001)
    Rr, Ri = oracle_mod.rmsf(lam, w, phi)
    a = np.hypot(Rr, Ri)
    k = int(np.argmax(a < 0.5))
    x = phi[k - 1] + (0.5 - a[k - 1]) * (phi[k] - phi[k - 1]) / (a[k] - a[k - 1])
    ratio = 2 * x / est
    assert 1.0 <= ratio <= 1.45, ratio


# ---------------------------------------------------------------- peaks
def test_peak_rules(oracle_mod):
    phi = np.array([-2.0, -1.0, 0.0, 1.0, 2.0])
    Fq = np.array([[0.1, 0.5, 0.2, 0.5, 0.0],       # tie -> lowest index
                   [0.0, 0.0, 0.0, 0.0, 0.3],
                   [0.1, np.nan, 0.0, 0.0, 0.0],    # non-finite -> idx -1
                   [0.0, 0.0, 0.0, 0.0, 0.0]])      # all zero -> idx 0, margin 0
    Fu = np.array([[0.0, 0.0, 0.0, 0.0, 0.0],
                   [0.0, -0.4, 0.0, 0.0, 0.0],
                   [0.0, 0.0, 0.0, 0.0, 0.0],
                   [0.0, 0.0, 0.0, 0.0, 0.0]])
    p = oracle_mod.peaks(Fq, Fu, phi)
    assert list(p["idx"]) == [1, 1, -1, 0]
    assert p["margin"][0] == 0.0
    assert abs(p["margin"][1] - 0.25) < 1e-15 and p["phi_pk"][1] == -1.0
    assert p["u_pk"][1] == -0.4 and p["amp"][1] == 0.4
    assert np.isnan(p["amp"][2])


# ---------------------------------------------------------------- printed values
def test_paper_cost_example(oracle_mod):
    g = json.load(open(GOLDEN))["wsrt_sings_cost"]
    tflop = oracle_mod.cost_flop(g["nlos"], g["nchan"], g["nphi"]) / 1e12
    assert round(tflop, g["digits"]) == g["tflop_printed"]


def test_paper_lofar_resolution_example(oracle_mod):
    """LOFAR_LR: 48.8 kHz channels over 120.238-166.087 MHz (RFI-free subset)
    give a resolution of 1.17 rad/m^2 and a largest scale of about 350."""
    g = json.load(open(GOLDEN))["lofar_lr_resolution"]
    nu = np.arange(g["f_lo_mhz"], g["f_hi_mhz"] + 1e-9, g["chan_width_mhz"])
    lam = (299.792458 / nu) ** 2
    rng = np.random.default_rng(43)
    w = np.zeros(lam.size)
    w[0] = w[-1] = 1.0
    inner = rng.choice(np.arange(1, lam.size - 1), size=g["nchan_rfi_free"] - 2, replace=False)
    w[inner] = 1.0
    fwhm, phimax = oracle_mod.plan_info(lam, w)
    assert round(fwhm, g["delta_phi_digits"]) == g["delta_phi_printed"]
    assert abs(phimax - g["phimax_printed_about"]) / g["phimax_printed_about"] < g["phimax_rel_tol"]


def test_plan_rejects_invalid(oracle_mod):
    lam = band_lambda2(120, 168, 10)
    with pytest.raises(ValueError):
        oracle_mod.plan(lam, np.zeros(10))
    with pytest.raises(ValueError):
        oracle_mod.plan(lam, -np.ones(10))
    w = np.ones(10)
    w[3] = np.nan
    with pytest.raises(ValueError):
        oracle_mod.plan(lam, w)
