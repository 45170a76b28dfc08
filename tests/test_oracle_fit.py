"""Pins of the oracle's sub-grid peak (peak_fit, peak_fit_from_spectra).

The paper reports phi_peak on the grid (Section 2.2, after eq. (14)); the
three-point parabola through |F| at the grid peak and its neighbours is an
extension.  It is pinned here by exact parabolas (whose vertex it must return
exactly, on uniform and irregular grids), by off-grid Faraday-thin screens
(eqs. (1), (3)) whose true depth it must recover far closer than the grid
does, and by its edge rules.
"""
import numpy as np
import pytest

from synthetic import WORKLOADS, thin_spectrum


@pytest.mark.parametrize("grid", ["uniform", "irregular"])
def test_exact_parabola_vertex(oracle_mod, grid):
    rng = np.random.default_rng(3)
    n = 50
    x1 = rng.uniform(-100, 100, n)
    if grid == "uniform":
        h = rng.uniform(0.1, 3.0, n)
        x0, x2 = x1 - h, x1 + h
    else:
        x0, x2 = x1 - rng.uniform(0.1, 3.0, n), x1 + rng.uniform(0.1, 3.0, n)
    # vertex within half a spacing of x1, on the side of the larger neighbour
    xv = x1 + rng.uniform(-0.45, 0.45, n) * np.minimum(x1 - x0, x2 - x1)
    a, b = rng.uniform(0.5, 2.0, n), rng.uniform(0.01, 1.0, n)
    y = lambda x: a - b * (x - xv) ** 2
    pf, af = oracle_mod.peak_fit(y(x0), y(x1), y(x2), x0, x1, x2)
    np.testing.assert_allclose(pf, xv, rtol=0, atol=1e-10)
    np.testing.assert_allclose(af, a, rtol=1e-12)


def test_offgrid_thin_screens_are_recovered(oracle_mod):
    """Thin screens at random off-grid depths: the grid peak is up to half a
    step (1 rad m^-2) away, the fitted peak within 0.005 of a step, because the
    main lobe of |R| is close to a parabola over +-1 step when the step is a
    tenth of the RMSF width (700-1800 MHz band, step 2 rad m^-2)."""
    wl = WORKLOADS["c3"]
    lam, w = wl.lambda2(), wl.weights()
    phi = np.arange(-100.0, 100.0 + 1e-9, 2.0)
    rng = np.random.default_rng(11)
    phi0 = rng.uniform(-60, 60, 300)
    P0 = rng.uniform(0.01, 0.1, 300)
    P = thin_spectrum(lam, P0, phi0, rng.uniform(0, np.pi, 300))
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    pk = oracle_mod.peaks(Fq, Fu, phi)
    assert np.max(np.abs(pk["phi_pk"] - phi0)) > 0.9      # the grid alone is off by ~1
    pf, af = oracle_mod.peak_fit_from_spectra(Fq, Fu, phi, pk["idx"])
    assert np.max(np.abs(pf - phi0)) < 0.01
    # and the fitted amplitude is closer to P0 than the grid amplitude
    assert np.max(np.abs(af - P0) / P0) < 0.5 * np.max(np.abs(pk["amp"] - P0) / P0)
    assert np.all(af >= pk["amp"])


def test_symmetric_neighbours_leave_the_grid_peak(oracle_mod):
    pf, af = oracle_mod.peak_fit(np.array([0.5]), np.array([1.0]), np.array([0.5]),
                                 np.array([1.0]), np.array([2.0]), np.array([3.0]))
    assert pf[0] == 2.0 and af[0] == 1.0


def test_edges_and_missing_peaks(oracle_mod):
    """A peak at either end of the grid keeps its grid values; idx -1 gives NaN."""
    # (rows 0 and 1 would give a downward parabola if the grid were wrapped around)
    Fq = np.array([[5.0, 4.0, 1.0, 0.5], [0.5, 1.0, 4.0, 5.0], [1.0, 3.0, 2.0, 0.5],
                   [1.0, 1.0, 1.0, 1.0]])
    Fu = np.zeros_like(Fq)
    phi = np.array([-1.0, 0.0, 1.0, 2.0])
    pf, af = oracle_mod.peak_fit_from_spectra(Fq, Fu, phi, np.array([0, 3, 1, -1]))
    assert pf[0] == -1.0 and af[0] == 5.0
    assert pf[1] == 2.0 and af[1] == 5.0
    # interior: y = 1, 3, 2 around phi = 0 -> vertex (1 - 2) / (2 (1 - 6 + 2)) = 1/6
    assert abs(pf[2] - 1.0 / 6.0) < 1e-15
    assert abs(af[2] - (3.0 - (1.0 - 2.0) ** 2 / (8.0 * (1.0 - 6.0 + 2.0)))) < 1e-15
    assert np.isnan(pf[3]) and np.isnan(af[3])


def test_the_fit_uses_the_amplitude_of_the_complex_F(oracle_mod):
    """|F| = hypot(Fq, Fu): putting the same amplitudes into Fu instead of Fq,
    or splitting them between the two, changes nothing."""
    amps = np.array([[1.0, 3.0, 2.0]])
    phi = np.array([0.0, 1.0, 2.0])
    a = oracle_mod.peak_fit_from_spectra(amps, 0 * amps, phi, np.array([1]))
    b = oracle_mod.peak_fit_from_spectra(0 * amps, amps, phi, np.array([1]))
    c = oracle_mod.peak_fit_from_spectra(0.6 * amps, 0.8 * amps, phi, np.array([1]))
    for r in (b, c):
        np.testing.assert_allclose(r[0], a[0], rtol=1e-15)
        np.testing.assert_allclose(r[1], a[1], rtol=1e-15)
