"""RM-CLEAN (rmsynth_rmclean) against the FP64 oracle (oracle.rmclean), through
the C ABI.

The GPU iterates in FP32 with an FP32 table of the RMSF on the doubled grid;
the oracle in FP64.  Where every decision of the oracle's loop is clear
(relative margin of each pick over the runner-up and of each comparison with
the cutoff above 1e-4), the GPU must take the same decisions: the same
number of iterations, and components, residual and restored spectrum within

    bar_l = 2 (niter_l + 1) (eps_R + 2^-21) max_k |F_lk|,

eps_R the largest difference of the GPU's RMSF table from the oracle's (per
unit R(0) = 1), 2^-21 covering the FP32 roundings of one subtraction (of
|c R| and |r|, both at most max |F|); each iteration adds at most that much
error to every residual element, and the restored spectrum sums the
components (|G| <= 1).  Elsewhere the GPU's outputs must be a valid run:
F = C * R + r within the same bar, and the residual peak below the cutoff
unless the iteration limit was reached.
"""
import numpy as np
import pytest

import oracle
from oracle import rmclean as orc
import paper_1810_06250_amd as rs
from synthetic import (WORKLOADS, band_lambda2, flag_channels, make_cube, noise_sigma_F,
                       slab_spectrum, stratified_subsample, thin_spectrum, LOS_MAJOR)
from gpu_util import dev32, host, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs.load_library()
    oracle.build(force=False)


def _cube(lam, w, phi, n, sigma, seed):
    """n LOS: a quarter noise only, the rest one or two thin screens or a slab."""
    rng = np.random.default_rng(seed)
    P = sigma * (rng.standard_normal((n, lam.size)) + 1j * rng.standard_normal((n, lam.size)))
    span = 0.7 * np.max(np.abs(phi))
    kind = rng.integers(0, 4, n)
    for l in range(n):
        if kind[l] >= 1:
            P[l] += thin_spectrum(lam, rng.uniform(0.01, 0.1), rng.uniform(-span, span),
                                  rng.uniform(0, np.pi))[0]
        if kind[l] == 2:
            P[l] += thin_spectrum(lam, rng.uniform(0.01, 0.1), rng.uniform(-span, span),
                                  rng.uniform(0, np.pi))[0]
        if kind[l] == 3:
            P[l] += slab_spectrum(lam, rng.uniform(0.01, 0.1), rng.uniform(-span, span),
                                  rng.uniform(1, 5), rng.uniform(0, np.pi))[0]
    Fq, Fu = oracle.fdf(P.real, P.imag, lam, w, phi)
    return Fq.astype(np.float32), Fu.astype(np.float32)


def _table_error(lam, w, phi):
    """eps_R: the GPU's RMSF on the doubled grid against the oracle's."""
    N = phi.size
    dphi = (phi[-1] - phi[0]) / (N - 1)
    grid = (np.arange(2 * N - 1) - (N - 1)) * dphi
    p2 = rs.Plan(lam, w, grid)
    re, im = (host(t) for t in p2.rmsf())
    p2.close()
    R2 = orc.rmsf_doubled(oracle.rmsf, lam, w, dphi, N)
    return float(np.max(np.abs(re + 1j * im - R2))), R2, dphi


def _run(lam, w, phi, Fq, Fu, gain, cutoff, max_iter, fwhm=float("nan")):
    plan = rs.Plan(lam, w, phi)
    o = plan.rmclean(dev32(Fq), dev32(Fu), gain, cutoff, max_iter, fwhm)
    out = {k: host(v) for k, v in o.items()}
    plan.close()
    return out


def _compare(lam, w, phi, Fq, Fu, gain, cutoff, max_iter):
    g = _run(lam, w, phi, Fq, Fu, gain, cutoff, max_iter)
    return _verify(lam, w, phi, Fq, Fu, g, gain, cutoff, max_iter)


def _verify(lam, w, phi, Fq, Fu, g, gain, cutoff, max_iter):
    """The checks of the module docstring on GPU outputs g (host arrays) of the
    LOS whose input spectra are Fq, Fu."""
    eps_R, R2, dphi = _table_error(lam, w, phi)
    fwhm, _ = oracle.plan_info(lam, w)
    ref = orc.rmclean(Fq.astype(np.float64), Fu.astype(np.float64), R2, dphi, gain, cutoff,
                      max_iter, fwhm)
    N = phi.size
    F = Fq.astype(np.float64) + 1j * Fu
    scale = np.abs(F).max(axis=1)
    clear = (ref["pick_margin"] > 1e-4) & (ref["stop_margin"] > 1e-4)
    niter = g["niter"]
    bar = 2 * (np.maximum(niter, ref["niter"]) + 1) * (eps_R + 2.0 ** -21) * scale
    resid = g["rq"] + 1j * g["ru"]
    cc = g["cq"] + 1j * g["cu"]
    rest = g["Rq"] + 1j * g["Ru"]
    note(f"  eps_R {eps_R:.2e}; {clear.sum()} of {len(clear)} LOS with clear decisions; "
         f"niter {niter.min()}..{niter.max()}")
    np.testing.assert_array_equal(niter[clear], ref["niter"][clear])
    worst = 0.0
    for name, a, b in (("resid", resid, ref["resid"]), ("cc", cc, ref["cc"]),
                       ("restored", rest, ref["restored"])):
        d = np.abs(a - b).max(axis=1)
        assert np.all(d[clear] <= bar[clear]), (name, np.max(d[clear] / bar[clear]))
        worst = max(worst, float(np.max(d[clear] / scale[clear])))
    note(f"  max error / max|F| on clear LOS: {worst:.2e}")
    # every LOS: a valid run of the iteration
    conv = np.stack([np.array([np.sum(cc[l] * R2[(N - 1) + k - np.arange(N)]) for k in range(N)])
                     for l in range(len(F))])
    assert np.all(np.abs(conv + resid - F).max(axis=1) <= bar)
    done = niter < max_iter
    assert np.all(np.sqrt((resid[done] * np.conj(resid[done])).real.max(axis=1)) < cutoff * (1 + 1e-4))
    beam = orc.restoring_beam(dphi * (np.arange(N)[:, None] - np.arange(N)[None, :]), fwhm)
    assert np.all(np.abs(rest - (resid + cc @ beam.T)).max(axis=1) <= bar)
    return g, ref


@pytest.mark.parametrize("band,nphi,step", [((120.0, 168.0, 128), 201, 1.0),
                                            ((700.0, 1800.0, 400), 301, 2.0)])
def test_rmclean_matches_oracle(band, nphi, step):
    note(f"rmclean band {band} nphi {nphi}")
    lam = band_lambda2(*band)
    w = flag_channels(lam.size, lam.size // 20, np.random.default_rng(1))
    phi = (np.arange(nphi) - nphi // 2) * step
    sigma = 1e-3
    Fq, Fu = _cube(lam, w, phi, 160, sigma, seed=nphi)
    cutoff = 5 * noise_sigma_F(sigma, w)
    g, ref = _compare(lam, w, phi, Fq, Fu, 0.1, cutoff, 300)
    assert np.sum(g["niter"] > 10) > 50


def test_rmclean_large_grid():
    """4001 phi: the widest register layout (64 elements per lane)."""
    note("rmclean 4001 phi")
    lam = band_lambda2(110.0, 190.0, 256)
    w = np.ones(lam.size)
    phi = np.linspace(-1000, 1000, 4001)
    Fq, Fu = _cube(lam, w, phi, 24, 1e-4, seed=4)
    _compare(lam, w, phi, Fq, Fu, 0.2, 5 * noise_sigma_F(1e-4, w), 100)


def test_rmclean_single_screen_closed_form():
    """An on-grid screen alone: each iteration takes gain of what is left at
    its depth, so after n iterations the residual there is (1 - gain)^n P0
    and the component holds the rest."""
    lam = band_lambda2(700.0, 1800.0, 200)
    w = np.ones(lam.size)
    phi = np.arange(-100.0, 100.5, 2.0)
    P = thin_spectrum(lam, 0.05, phi[60], 0.3)
    Fq, Fu = (a.astype(np.float32) for a in oracle.fdf(P.real, P.imag, lam, w, phi))
    g = _run(lam, w, phi, Fq, Fu, 0.25, 0.0, 7)
    assert g["niter"][0] == 7
    amp = np.hypot(g["rq"][0, 60], g["ru"][0, 60])
    assert abs(amp - 0.75 ** 7 * 0.05) <= 1e-6 * 0.05
    assert abs(np.hypot(g["cq"][0, 60], g["cu"][0, 60]) - (1 - 0.75 ** 7) * 0.05) <= 1e-6 * 0.05
    nz = np.flatnonzero(g["cq"][0] != 0)
    assert list(nz) == [60]


def test_rmclean_noop_below_cutoff_and_nonfinite():
    lam = band_lambda2(120.0, 168.0, 64)
    w = np.ones(lam.size)
    phi = np.linspace(-50, 50, 101)
    rng = np.random.default_rng(3)
    Fq = (1e-4 * rng.standard_normal((6, 101))).astype(np.float32)
    Fu = (1e-4 * rng.standard_normal((6, 101))).astype(np.float32)
    Fq[4, 9] = np.inf
    g = _run(lam, w, phi, Fq, Fu, 0.1, 1.0, 50)
    keep = np.arange(6) != 4
    assert np.all(g["niter"][keep] == 0) and g["niter"][4] == -1
    np.testing.assert_array_equal(g["rq"][keep], Fq[keep])
    np.testing.assert_array_equal(g["Rq"][keep], Fq[keep])
    assert np.all(g["cq"][keep] == 0) and np.all(g["cu"][keep] == 0)
    assert np.all(np.isnan(g["rq"][4])) and np.all(np.isnan(g["Rq"][4]))


def test_rmclean_in_place_and_argument_errors():
    import torch
    lam = band_lambda2(700.0, 1800.0, 100)
    w = np.ones(lam.size)
    phi = np.linspace(-200, 200, 201)
    Fq, Fu = _cube(lam, w, phi, 40, 1e-3, seed=9)
    ref = _run(lam, w, phi, Fq, Fu, 0.1, 0.01, 100)
    plan = rs.Plan(lam, w, phi)
    q, u = dev32(Fq), dev32(Fu)
    cq, cu = torch.empty_like(q), torch.empty_like(q)
    nb = rs.rmsynth_rmclean_workspace_size(plan.handle)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    rs.rmsynth_rmclean(plan.handle, q, u, 40, 0.1, 0.01, 100, float("nan"), q, u, cq, cu,
                       workspace=ws, workspace_bytes=nb)
    np.testing.assert_array_equal(host(q), ref["rq"])
    np.testing.assert_array_equal(host(cu), ref["cu"])
    for gain in (0.0, 1.5, float("nan")):
        with pytest.raises(rs.RmsynthError) as ei:
            rs.rmsynth_rmclean(plan.handle, q, u, 40, gain, 0.01, 10, 0.0, q, u, cq, cu,
                               workspace=ws, workspace_bytes=nb)
        assert ei.value.code == rs.RMSYNTH_EINVAL
    with pytest.raises(rs.RmsynthError) as ei:
        rs.rmsynth_rmclean(plan.handle, q, u, 40, 0.1, 0.01, 10, 0.0, q, u, cq, cu,
                           workspace=ws, workspace_bytes=nb - 1)
    assert ei.value.code == rs.RMSYNTH_EWORKSPACE
    irregular = rs.Plan(lam, w, np.sort(np.random.default_rng(1).uniform(-200, 200, 201)))
    with pytest.raises(rs.RmsynthError) as ei:
        rs.rmsynth_rmclean(irregular.handle, q, u, 40, 0.1, 0.01, 10, 0.0, q, u, cq, cu,
                           workspace=ws, workspace_bytes=nb)
    assert ei.value.code == rs.RMSYNTH_EUNSUPPORTED
    wide = rs.Plan(lam, w, np.linspace(-2000, 2000, 4097))
    F = torch.zeros((2, 4097), dtype=torch.float32, device="cuda")
    with pytest.raises(rs.RmsynthError) as ei:
        rs.rmsynth_rmclean(wide.handle, F, F, 2, 0.1, 0.01, 10, 0.0, F, F, F.clone(), F.clone(),
                           workspace=ws, workspace_bytes=nb)
    assert ei.value.code == rs.RMSYNTH_EUNSUPPORTED


def test_rmclean_c3_full_size_sampled():
    """The benchmark's RM-CLEAN launch: the c3 cube's F (1 048 576 LOS x 2001
    phi, from the split transform) in one call with the benchmark's settings
    (gain 0.1, cutoff 5 sigma_F, at most 1000 iterations); 96 sampled LOS (half
    with sources) checked against the oracle as above."""
    import torch
    wl = WORKLOADS["c3"]
    note("rmclean c3 full size")
    cube = make_cube(wl, device="cuda")
    lam, w, phi = cube["lambda2"], cube["weights"], cube["phi"]
    plan = rs.Plan(lam, w, phi)
    Fq, Fu, _ = plan.execute(cube["Q"], cube["U"], LOS_MAJOR, rs.RMSYNTH_SPLIT_BF16)
    src = cube["src_los"]
    del cube
    torch.cuda.empty_cache()
    cutoff = 5 * noise_sigma_F(wl.sigma, w)
    o = plan.rmclean(Fq, Fu, 0.1, cutoff, 1000, float("nan"))
    torch.cuda.synchronize()
    sub = stratified_subsample(wl.nlos, src, 96, seed=wl.seed + 9)
    subt = torch.as_tensor(sub, device="cuda")
    g = {k: host(v[subt]) for k, v in o.items()}
    fq, fu = host(Fq[subt]), host(Fu[subt])
    del o
    plan.close()
    g2, ref = _verify(lam, w, phi, fq, fu, g, 0.1, cutoff, 1000)
    assert np.sum(ref["niter"] > 0) >= 40      # the source LOS are cleaned
