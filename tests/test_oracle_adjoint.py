"""Pins of the oracle's spectrum synthesis (oracle.adjoint): eq. (4) with the
integral over phi replaced by the sum over grid components C_k, referred to
lambda0^2 as eq. (11) refers F.

Pinned by the closed form of a Faraday-thin screen (eqs. (1), (3)), by the
adjoint identity with the oracle's own forward transform (an independent
loop: <F(P), C> = <P, K w A(C)>), by the inverse-FFT special case, and by the
shift identity of a transform of a synthesised thin screen."""
import numpy as np

from synthetic import band_lambda2, thin_spectrum, WORKLOADS


def test_one_component_is_a_thin_screen(oracle_mod):
    """C = P0 exp(2i(chi0 + phi0 lambda0^2)) at phi0 alone gives the thin
    screen P0 exp(2i(chi0 + phi0 lambda^2)) in every channel."""
    lam = band_lambda2(120.0, 168.0, 64)
    rng = np.random.default_rng(2)
    w = rng.uniform(0.5, 1.5, lam.size)
    phi = np.linspace(-50, 50, 101)
    _, l0 = oracle_mod.plan(lam, w)
    n = 6
    ks = rng.integers(0, phi.size, n)
    P0, chi0 = rng.uniform(0.1, 1.0, n), rng.uniform(0, np.pi, n)
    C = np.zeros((n, phi.size), complex)
    C[np.arange(n), ks] = P0 * np.exp(2j * (chi0 + phi[ks] * l0))
    Pq, Pu = oracle_mod.adjoint(C.real, C.imag, lam, w, phi)
    np.testing.assert_allclose(Pq + 1j * Pu, thin_spectrum(lam, P0, phi[ks], chi0), rtol=0, atol=1e-12)


def test_adjoint_identity_with_the_forward_transform(oracle_mod):
    """<F(P), C> = <P, K w A(C)> for random P, C: the synthesis is the adjoint
    of eq. (11) up to the weights K w_j."""
    wl = WORKLOADS["c2"]
    lam, w = wl.lambda2()[:120], wl.weights()[:120]
    w[5] = 0.0
    phi = np.linspace(-300, 300, 77)
    rng = np.random.default_rng(5)
    P = rng.standard_normal((4, lam.size)) + 1j * rng.standard_normal((4, lam.size))
    C = rng.standard_normal((4, phi.size)) + 1j * rng.standard_normal((4, phi.size))
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    Aq, Au = oracle_mod.adjoint(C.real, C.imag, lam, w, phi)
    K, _ = oracle_mod.plan(lam, w)
    lhs = np.sum(np.conj(Fq + 1j * Fu) * C, axis=1)
    rhs = np.sum(np.conj(P) * (K * w) * (Aq + 1j * Au), axis=1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_inverse_fft_special_case(oracle_mod):
    """lambda^2 spaced d from lambda0^2 = lambda_0^2 of the first channel and
    phi_k = pi k / (N d): P_j = sum_k C_k exp(2 pi i k j / N) = N ifft(C)_j."""
    rng = np.random.default_rng(9)
    for n in (5, 16, 31):
        d = 0.0017
        lam = 0.09 + d * np.arange(n)
        phi = np.pi * np.arange(n) / (n * d)
        C = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
        Pq, Pu = oracle_mod.adjoint(C.real, C.imag, lam, np.ones(n), phi, lambda0_sq=lam[0])
        np.testing.assert_allclose(Pq + 1j * Pu, n * np.fft.ifft(C, axis=1), rtol=0, atol=1e-11)


def test_round_trip_of_a_component_is_the_shifted_rmsf(oracle_mod):
    """Transforming the spectrum of one component C_k0 gives C_k0 R(phi - phi_k0)
    (eq. (12)), so F(phi_k0) = C_k0 exactly."""
    lam = band_lambda2(700.0, 1800.0, 200)
    w = np.ones(lam.size)
    phi = np.linspace(-200, 200, 201)
    C = np.zeros((1, phi.size), complex)
    C[0, 120] = 0.3 - 0.4j
    Pq, Pu = oracle_mod.adjoint(C.real, C.imag, lam, w, phi)
    Fq, Fu = oracle_mod.fdf(Pq, Pu, lam, w, phi)
    Rr, Ri = oracle_mod.rmsf(lam, w, phi - phi[120])
    np.testing.assert_allclose(Fq[0] + 1j * Fu[0], C[0, 120] * (Rr + 1j * Ri), rtol=0, atol=1e-13)
    assert abs(Fq[0, 120] + 1j * Fu[0, 120] - C[0, 120]) < 1e-13
