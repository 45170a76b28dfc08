"""Pins of the FP64 NUFFT evaluation of eq. (11) (oracle/nufft.py) against
the direct sum of the C oracle: at kernel width 8 on the 2x oversampled grid
it agrees to 1e-6 of max|F| per LOS on every synthetic band, the error falls
steeply with the width, and the kernel's Fourier transform is checked
against a direct quadrature at a few modes."""
import numpy as np
import pytest

from oracle import nufft
from synthetic import WORKLOADS, make_cube


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_nufft_matches_the_direct_sum(oracle_mod, name):
    wl = WORKLOADS[name]
    cube = make_cube(wl, nlos=24, device="cpu", layout=0)
    Q, U = cube["Q"].double().numpy(), cube["U"].double().numpy()
    lam, w, phi = cube["lambda2"], cube["weights"], cube["phi"]
    rq, ru = oracle_mod.fdf(Q, U, lam, w, phi)
    e = {}
    for width in (6, 8, 10):
        nq, nu = nufft.fdf_nufft(Q, U, lam, w, phi, width=width)
        e[width] = oracle_mod.per_los_error(nq, nu, rq, ru).max()
    assert e[8] < 1e-6
    assert e[10] < e[8] / 20 and e[8] < e[6] / 20


def test_psi_hat_by_direct_quadrature():
    alpha, beta = nufft.kernel_params(8, 256)
    t = np.linspace(-alpha, alpha, 200001)
    for m in (0, 5, 60, 127):
        f = nufft.psi(t, alpha, beta) * np.cos(m * t)
        direct = np.sum((f[1:] + f[:-1]) / 2) * (t[1] - t[0])
        assert abs(nufft.psi_hat([m], alpha, beta)[0] - direct) < 1e-9 * abs(direct) + 1e-14


def test_flagged_channels_are_ignored(oracle_mod):
    wl = WORKLOADS["c2"]
    cube = make_cube(wl, nlos=4, device="cpu", layout=0)
    Q, U = cube["Q"].double().numpy(), cube["U"].double().numpy()
    lam, w, phi = cube["lambda2"], cube["weights"], cube["phi"][:301]
    a = nufft.fdf_nufft(Q, U, lam, w, phi)
    Q2 = Q.copy()
    Q2[:, w == 0] = 1e30
    b = nufft.fdf_nufft(Q2, U, lam, w, phi)
    np.testing.assert_array_equal(a[0], b[0])


def test_off_centre_grid(oracle_mod):
    """A grid not centred on phi = 0 (the phase referred to its centre phi_c
    is part of every coefficient)."""
    wl = WORKLOADS["c3"]
    cube = make_cube(wl, nlos=8, device="cpu", layout=0)
    Q, U = cube["Q"].double().numpy(), cube["U"].double().numpy()
    lam, w = cube["lambda2"], cube["weights"]
    phi = 137.0 + 2.0 * np.arange(300)
    rq, ru = oracle_mod.fdf(Q, U, lam, w, phi)
    nq, nu = nufft.fdf_nufft(Q, U, lam, w, phi)
    assert oracle_mod.per_los_error(nq, nu, rq, ru).max() < 1e-6
