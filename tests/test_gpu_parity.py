"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Bar: per-LOS error max_k |F_gpu - F_oracle| / max_k |F_oracle| <= 1e-5 for
the FP32 and the split-bfloat16 paths; peak indices equal wherever the
oracle's peak margin exceeds 2e-5 (elsewhere the GPU index must point at a
value within that margin of the maximum).
"""
import numpy as np
import pytest

import oracle
import paper_1810_06250_amd as rs
from synthetic import (WORKLOADS, band_lambda2, thin_spectrum, make_small_cube, make_cube,
                       stratified_subsample, FREQ_MAJOR, LOS_MAJOR)
from gpu_util import PREC_TOL, SCALE_TOL, dev32, fit_bar, host, note

pytestmark = pytest.mark.gpu

PRECS = {"fp32": rs.RMSYNTH_FP32, "bf16x3": rs.RMSYNTH_SPLIT_BF16, "fp16x3": rs.RMSYNTH_SPLIT_FP16}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs.load_library()
    oracle.build(force=False)


def _run(plan, Q, U, layout, prec, want_abs=True):
    Fq, Fu, Fa = plan.execute(Q, U, layout, prec, want_abs=want_abs)
    pk = plan.peaks(Fq, Fu)
    out = dict(Fq=host(Fq), Fu=host(Fu), Fa=host(Fa) if Fa is not None else None)
    out.update({k: host(v) for k, v in pk.items()})
    return out


def _check(out, Q64, U64, lam, w, phi, layout, tol, margin=2e-5, floor=False):
    rq, ru = oracle.fdf(Q64, U64, lam, w, phi, layout=layout)
    fl = oracle.incoherent_scale(Q64, U64, w, layout=layout) if floor else None
    err = oracle.per_los_error(out["Fq"], out["Fu"], rq, ru, floor=fl)
    note(f"  max per-LOS error {err.max():.3e}")
    assert np.all(np.isfinite(err)), "non-finite GPU output"
    assert err.max() <= tol, f"max per-LOS error {err.max():.3e} > {tol:.1e}"
    ref = oracle.peaks(rq, ru, phi)
    nun, mism, bad = oracle.peak_agreement(out["idx"], rq, ru, ref, margin)
    assert mism == 0 and bad == 0, f"peak mismatches: {mism} of {nun} unambiguous, {bad} ambiguous"
    if out["Fa"] is not None:
        np.testing.assert_allclose(out["Fa"], np.hypot(out["Fq"], out["Fu"]), rtol=1e-6, atol=1e-30)
    ok = out["idx"] >= 0
    np.testing.assert_array_equal(out["phi_pk"][ok], phi[out["idx"][ok]].astype(np.float32))
    rows = np.arange(out["Fq"].shape[0])[ok]
    np.testing.assert_array_equal(out["q_pk"][ok], out["Fq"][rows, out["idx"][ok]])
    amp = np.sqrt(out["Fq"][rows, out["idx"][ok]].astype(np.float64) ** 2 +
                  out["Fu"][rows, out["idx"][ok]].astype(np.float64) ** 2)
    np.testing.assert_allclose(out["amp"][ok], amp, rtol=1e-6, atol=1e-30)
    return err, rq, ru


@pytest.mark.parametrize("prec", list(PRECS))
def test_c1_full_cube(prec):
    """64x64 LOS, 128 channels, 201 phi, 20 injected thin sources."""
    wl = WORKLOADS["c1"]
    note(f"c1 full cube, {prec}")
    cube = make_cube(wl, device="cpu")
    plan = rs.Plan(cube["lambda2"], cube["weights"], cube["phi"])
    out = _run(plan, dev32(cube["Q"]), dev32(cube["U"]), LOS_MAJOR, PRECS[prec])
    _check(out, cube["Q"].double().numpy(), cube["U"].double().numpy(), cube["lambda2"],
           cube["weights"], cube["phi"], LOS_MAJOR, PREC_TOL[prec])


@pytest.mark.parametrize("prec", list(PRECS))
def test_frequency_major_equals_los_major(prec):
    """Both input layouts feed the same arithmetic: outputs are bitwise equal."""
    note(f"layouts bitwise, {prec}")
    c = make_small_cube(333, 77, 150, seed=3, nflag=6, nsrc=5)
    plan = rs.Plan(c["lambda2"], c["weights"], c["phi"])
    a = _run(plan, dev32(c["Q"]), dev32(c["U"]), LOS_MAJOR, PRECS[prec])
    b = _run(plan, dev32(c["Q"].T), dev32(c["U"].T), FREQ_MAJOR, PRECS[prec])
    for k in ("Fq", "Fu", "Fa", "idx"):
        np.testing.assert_array_equal(a[k], b[k])


SHAPES = [(1, 1, 1), (1, 3, 5), (37, 5, 7), (64, 8, 128), (130, 13, 129), (129, 64, 257),
          (300, 33, 300), (257, 100, 1), (2, 200, 513)]
# Grids of a few phi only: there max_k |F| can be one small sample, far below
# the size of the products that make it, so the error is taken relative to
# the LOS's incoherent scale K sqrt(sum w^2 |P|^2) as well, with the split's
# per-product bound (SCALE_TOL).  Every other shape meets 1e-5 of max_k |F|.
SHORT_GRID = 7


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("layout", [LOS_MAJOR, FREQ_MAJOR], ids=["los", "freq"])
def test_ragged_shapes(prec, shape, layout):
    """Sizes that fill several tiles and leave ragged LOS, channel and phi tails."""
    nlos, nchan, nphi = shape
    note(f"ragged {shape} layout={layout} {prec}")
    c = make_small_cube(nlos, nchan, nphi, seed=nlos * 7 + nchan, nflag=nchan // 10,
                        nsrc=max(1, nlos // 20))
    plan = rs.Plan(c["lambda2"], c["weights"], c["phi"])
    Q, U = (c["Q"], c["U"]) if layout == LOS_MAJOR else (c["Q"].T, c["U"].T)
    Q32, U32 = np.float32(Q), np.float32(U)
    out = _run(plan, dev32(Q32), dev32(U32), layout, PRECS[prec])
    short = nphi <= SHORT_GRID
    _check(out, Q32.astype(np.float64), U32.astype(np.float64), c["lambda2"], c["weights"],
           c["phi"], layout, SCALE_TOL[prec] if short else PREC_TOL[prec], floor=short)


@pytest.mark.parametrize("prec", list(PRECS))
def test_flagged_and_nonfinite_channels(prec):
    """NaN/Inf in flagged channels has no effect; a NaN in an unflagged channel
    poisons only its own LOS (idx = -1)."""
    note(f"flags and NaN, {prec}")
    c = make_small_cube(200, 96, 101, seed=5, nflag=12, nsrc=4)
    plan = rs.Plan(c["lambda2"], c["weights"], c["phi"])
    Q32, U32 = np.float32(c["Q"]), np.float32(c["U"])
    base = _run(plan, dev32(Q32), dev32(U32), LOS_MAJOR, PRECS[prec])
    fl = c["weights"] == 0
    Qb, Ub = Q32.copy(), U32.copy()
    Qb[:, fl] = np.nan
    Ub[:, fl] = np.inf
    out = _run(plan, dev32(Qb), dev32(Ub), LOS_MAJOR, PRECS[prec])
    for k in ("Fq", "Fu", "idx"):
        np.testing.assert_array_equal(out[k], base[k])
    Qc = Q32.copy()
    unfl = np.flatnonzero(~fl)[3]
    Qc[17, unfl] = np.nan
    out = _run(plan, dev32(Qc), dev32(U32), LOS_MAJOR, PRECS[prec])
    assert out["idx"][17] == -1 and np.isnan(out["amp"][17])
    keep = np.arange(200) != 17
    np.testing.assert_array_equal(out["Fq"][keep], base["Fq"][keep])
    np.testing.assert_array_equal(out["idx"][keep], base["idx"][keep])


def test_plan_info_matches_oracle():
    """K and lambda0^2 (eq. (13) and the weighted mean), the resolution and the
    largest recoverable depth estimates (eqs. (20)-(21)) reported by the plan
    equal the oracle's for the five synthetic bands and the LOFAR_LR band of
    Section 3.3 (whose printed 1.17 and ~350 rad m^-2 pin the oracle)."""
    import json
    import os
    bands = {n: (WORKLOADS[n].lambda2(), WORKLOADS[n].weights()) for n in WORKLOADS}
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "paper_values.json")))["lofar_lr_resolution"]
    nu = np.arange(g["f_lo_mhz"], g["f_hi_mhz"] + 1e-9, g["chan_width_mhz"])
    lam_lf = (299.792458 / nu) ** 2
    w_lf = np.zeros(lam_lf.size)
    w_lf[0] = w_lf[-1] = 1.0
    inner = np.random.default_rng(43).choice(np.arange(1, lam_lf.size - 1),
                                             size=g["nchan_rfi_free"] - 2, replace=False)
    w_lf[inner] = 1.0
    bands["lofar_lr"] = (lam_lf, w_lf)
    phi = np.linspace(-10.0, 10.0, 21)
    for name, (lam, w) in bands.items():
        note(f"plan_info {name}")
        plan = rs.Plan(lam, w, phi)
        info = plan.info
        K, l0 = oracle.plan(lam, w)
        fwhm, phimax = oracle.plan_info(lam, w)
        assert info["K"] == pytest.approx(K, rel=1e-15), name
        assert info["lambda0_sq"] == pytest.approx(l0, rel=1e-14), name
        assert info["fwhm_est"] == pytest.approx(fwhm, rel=1e-12), name
        assert info["phimax_est"] == pytest.approx(phimax, rel=1e-12), name
        assert (info["nchan"], info["nphi"]) == (len(lam), len(phi))
        if name == "lofar_lr":
            assert round(info["fwhm_est"], g["delta_phi_digits"]) == g["delta_phi_printed"]
            assert abs(info["phimax_est"] / g["phimax_printed_about"] - 1) < g["phimax_rel_tol"]
        plan.close()
        # a caller's lambda0^2 is kept as given
        plan = rs.Plan(lam, w, phi, lambda0_sq=0.25)
        assert plan.info["lambda0_sq"] == 0.25
        plan.close()


def test_rmsf_matches_oracle_and_unit_spectrum():
    note("rmsf")
    import torch
    for name in ("c1", "c3", "c4"):
        wl = WORKLOADS[name]
        lam, w, phi = wl.lambda2(), wl.weights(), wl.phi()
        plan = rs.Plan(lam, w, phi)
        re, im = (host(x) for x in plan.rmsf())
        rr, ri = oracle.rmsf(lam, w, phi)
        assert np.max(np.hypot(re - rr, im - ri)) < 2e-6
        k0 = np.flatnonzero(phi == 0.0)
        assert abs(re[k0[0]] - 1.0) < 1e-6 and abs(im[k0[0]]) < 1e-6
        ones = torch.ones((1, lam.size), dtype=torch.float32, device="cuda")
        zeros = torch.zeros_like(ones)
        Fq, Fu, _ = plan.execute(ones, zeros, LOS_MAJOR, rs.RMSYNTH_FP32)
        np.testing.assert_allclose(host(Fq)[0], re, rtol=0, atol=2e-6)
        np.testing.assert_allclose(host(Fu)[0], im, rtol=0, atol=2e-6)


def test_phase_generator_accuracy():
    """One channel, lambda0^2 = 0: R(phi) = exp(-2 i phi lambda^2) exactly, so
    the RMSF exposes the generator's cos/sin over arguments up to ~1.5e4 rad."""
    note("phase generator accuracy")
    phi = np.linspace(-1000.0, 1000.0, 40001)
    worst = 0.0
    for lam2 in (0.0277, 0.9, 3.1, 7.43):
        plan = rs.Plan(np.array([lam2]), np.array([1.0]), phi, lambda0_sq=0.0)
        re, im = (host(x) for x in plan.rmsf())
        th = 2.0 * phi * lam2
        worst = max(worst, np.max(np.abs(re - np.cos(th))), np.max(np.abs(im + np.sin(th))))
    assert worst < 3e-7, worst


@pytest.mark.parametrize("prec", list(PRECS))
def test_thin_source_peak(prec):
    note(f"thin source peak, {prec}")
    wl = WORKLOADS["c3"]
    lam, w, phi = wl.lambda2(), wl.weights(), wl.phi()
    rng = np.random.default_rng(9)
    n = 64
    phi0 = phi[rng.integers(100, phi.size - 100, n)]
    P0 = rng.uniform(0.01, 0.1, n)
    P = thin_spectrum(lam, P0, phi0, rng.uniform(0, np.pi, n))
    plan = rs.Plan(lam, w, phi)
    out = _run(plan, dev32(P.real), dev32(P.imag), LOS_MAJOR, PRECS[prec])
    np.testing.assert_array_equal(out["phi_pk"], phi0.astype(np.float32))
    np.testing.assert_allclose(out["amp"], P0, rtol=1.5e-5)


@pytest.mark.parametrize("prec", list(PRECS))
def test_peak_angle(prec):
    """rmsynth_peak_angle (eq. (14)) against the oracle's on the same FP32 peak
    values, thin screens' intrinsic angles recovered, NaN for LOS without a
    peak, and nlos = 0 a no-op."""
    import torch
    note(f"peak angle, {prec}")
    wl = WORKLOADS["c3"]
    lam, w, phi = wl.lambda2(), wl.weights(), wl.phi()
    rng = np.random.default_rng(19)
    n = 96
    phi0 = phi[rng.integers(100, phi.size - 100, n)]
    chi0 = rng.uniform(0, np.pi, n)
    P = thin_spectrum(lam, rng.uniform(0.01, 0.1, n), phi0, chi0)
    P[-1, 7] = np.nan                       # one LOS without a peak
    plan = rs.Plan(lam, w, phi)
    Fq, Fu, _ = plan.execute(dev32(P.real), dev32(P.imag), LOS_MAJOR, PRECS[prec])
    pk = plan.peaks(Fq, Fu)
    chi = host(plan.peak_angle(pk))
    ref = oracle.peak_angle(host(pk["q_pk"]), host(pk["u_pk"]), host(pk["phi_pk"]),
                            plan.info["lambda0_sq"])
    assert np.isnan(chi[-1]) and np.isnan(ref[-1])
    ok = slice(0, n - 1)
    assert np.all((chi[ok] >= 0) & (chi[ok] < np.pi))
    d = np.angle(np.exp(2j * (chi[ok].astype(np.float64) - ref[ok]))) / 2
    assert np.max(np.abs(d)) < 1e-6, np.max(np.abs(d))
    d0 = np.angle(np.exp(2j * (chi[ok].astype(np.float64) - chi0[ok]))) / 2
    assert np.max(np.abs(d0)) < 2e-4, np.max(np.abs(d0))
    empty = torch.full((4,), 7.0, device="cuda")
    rs.rmsynth_peak_angle(plan.handle, empty, empty, empty, 0, empty)
    torch.cuda.synchronize()
    assert torch.all(empty == 7.0)


@pytest.mark.parametrize("prec", list(PRECS))
def test_linearity_and_determinism(prec):
    note(f"linearity/determinism, {prec}")
    c = make_small_cube(256, 128, 201, seed=21, nsrc=8)
    d = make_small_cube(256, 128, 201, seed=22, nsrc=8)
    plan = rs.Plan(c["lambda2"], c["weights"], c["phi"])
    a, b = 0.5 - 1.25j, -0.75 + 0.5j
    P1, P2 = c["Q"] + 1j * c["U"], d["Q"] + 1j * d["U"]
    Pm = a * P1 + b * P2
    r1 = _run(plan, dev32(P1.real), dev32(P1.imag), LOS_MAJOR, PRECS[prec])
    r2 = _run(plan, dev32(P2.real), dev32(P2.imag), LOS_MAJOR, PRECS[prec])
    rm = _run(plan, dev32(Pm.real), dev32(Pm.imag), LOS_MAJOR, PRECS[prec])
    F1, F2 = r1["Fq"] + 1j * r1["Fu"], r2["Fq"] + 1j * r2["Fu"]
    Fm = rm["Fq"] + 1j * rm["Fu"]
    scale = np.abs(Fm).max(axis=1, keepdims=True)
    assert np.max(np.abs(Fm - (a * F1 + b * F2)) / scale) < 3e-5
    again = _run(plan, dev32(P1.real), dev32(P1.imag), LOS_MAJOR, PRECS[prec])
    for k in ("Fq", "Fu", "idx"):
        np.testing.assert_array_equal(again[k], r1[k])


def test_execute_argument_errors():
    import torch
    c = make_small_cube(4, 16, 9, seed=1)
    plan = rs.Plan(c["lambda2"], c["weights"], c["phi"])
    Q = dev32(c["Q"])
    F = torch.empty((4, 9), dtype=torch.float32, device="cuda")
    with pytest.raises(rs.RmsynthError):
        rs.rmsynth_execute(plan.handle, Q, Q, 4, 7, rs.RMSYNTH_FP32, F, F)
    with pytest.raises(rs.RmsynthError):
        rs.rmsynth_execute(plan.handle, Q, Q, 4, LOS_MAJOR, 9, F, F)
    with pytest.raises(rs.RmsynthError):
        rs.rmsynth_execute(plan.handle, Q, None, 4, LOS_MAJOR, rs.RMSYNTH_FP32, F, F)
    F.fill_(7.0)
    rs.rmsynth_execute(plan.handle, Q, Q, 0, LOS_MAJOR, rs.RMSYNTH_FP32, F, F)
    torch.cuda.synchronize()
    assert torch.all(F == 7.0)
    assert rs.rmsynth_workspace_size(plan.handle, 4, LOS_MAJOR, rs.RMSYNTH_FP32) == 0


# ------------------------------------------------------------------ full-size workloads
def _full_size(name, prec_list, nsub):
    import torch
    wl = WORKLOADS[name]
    note(f"{name} full size: generating {wl.nlos} LOS x {wl.nchan} channels")
    cube = make_cube(wl, device="cuda")
    plan = rs.Plan(cube["lambda2"], cube["weights"], cube["phi"])
    sub = stratified_subsample(wl.nlos, cube["src_los"], nsub, seed=wl.seed + 11)
    subt = torch.as_tensor(sub, device="cuda")
    if cube["layout"] == LOS_MAJOR:
        Qs, Us = cube["Q"][subt], cube["U"][subt]
    else:
        Qs, Us = cube["Q"][:, subt].t(), cube["U"][:, subt].t()
    Q64, U64 = host(Qs).astype(np.float64), host(Us).astype(np.float64)
    note(f"{name}: oracle on {sub.size} LOS")
    rq, ru = oracle.fdf(Q64, U64, cube["lambda2"], cube["weights"], cube["phi"], layout=0)
    ref = oracle.peaks(rq, ru, cube["phi"])
    Fq = torch.empty((wl.nlos, len(cube["phi"])), dtype=torch.float32, device="cuda")
    Fu = torch.empty_like(Fq)
    results = {}
    for prec in prec_list:
        note(f"{name}: execute {prec}")
        plan.execute(cube["Q"], cube["U"], cube["layout"], PRECS[prec], out=(Fq, Fu, None))
        torch.cuda.synchronize()
        pk = plan.peaks(Fq, Fu)
        gq, gu = host(Fq[subt]), host(Fu[subt])
        err = oracle.per_los_error(gq, gu, rq, ru)
        idx = host(pk["idx"])[sub]
        nun, mism, bad = oracle.peak_agreement(idx, rq, ru, ref)
        note(f"{name} {prec}: max per-LOS err {err.max():.3e}, peaks {mism}/{nun} mismatched, {bad} bad ambiguous")
        results[prec] = (err.max(), mism, bad)
        assert err.max() <= PREC_TOL[prec]
        assert mism == 0 and bad == 0
        # The one-call transform + peaks gives the same peaks on the whole cube
        # (written over the same Fq, Fu: no second output cube).
        pk2 = {k: torch.empty_like(v) for k, v in pk.items()}
        nb = rs.rmsynth_execute_peaks_workspace_size(plan.handle, wl.nlos, cube["layout"], PRECS[prec])
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        rs.rmsynth_execute_peaks(plan.handle, cube["Q"], cube["U"], wl.nlos, cube["layout"],
                                 PRECS[prec], Fq, Fu, None, pk2["idx"], pk2["phi_pk"], pk2["amp"],
                                 pk2["q_pk"], pk2["u_pk"], ws, nb)
        for key in ("idx", "amp", "q_pk", "u_pk"):
            assert torch.equal(pk2[key], pk[key]), (name, prec, key)
        del pk2, ws
        # Sub-grid peak from the stored F, then the peaks-only search (F not
        # stored): the same peaks bit for bit.
        pf, af = plan.peak_fit(Fq, Fu, pk["idx"])
        torch.cuda.synchronize()
        ph = cube["phi"]
        rfit = oracle.peak_fit_from_spectra(rq, ru, ph, ref["idx"])
        same = (ref["idx"] == idx) & (ref["margin"] > 2e-5)
        bp, _ = fit_bar(rq, ru, ph, ref["idx"], err * np.hypot(rq, ru).max(axis=1))
        d = np.abs(host(pf)[sub] - rfit[0])[same]
        note(f"{name} {prec}: sub-grid peak max |dphi| {d.max():.2e} rad/m^2 (bar {bp[same].max():.2e})")
        assert np.all(d <= bp[same] + 2.0 ** -23 * np.abs(rfit[0][same]))
        note(f"{name}: search {prec}")
        # The unfused (FP32) search holds F of a batch in its workspace: cap it
        # at 16 GiB (LOS batches, same results), which keeps c4 (134 GB of F
        # already resident) within the card.
        least = rs.rmsynth_search_workspace_size(plan.handle, 128, cube["layout"], PRECS[prec])
        whole = rs.rmsynth_search_workspace_size(plan.handle, wl.nlos, cube["layout"], PRECS[prec])
        torch.cuda.empty_cache()
        s = plan.search(cube["Q"], cube["U"], cube["layout"], PRECS[prec],
                        workspace_bytes=min(whole, max(least, 16 << 30)))
        for key in ("idx", "amp", "q_pk", "u_pk"):
            assert torch.equal(s[key], pk[key]), (name, prec, "search", key)
        assert torch.equal(s["phi_fit"], pf) and torch.equal(s["amp_fit"], af)
        del s, pf, af
        torch.cuda.empty_cache()
    del Fq, Fu, cube
    torch.cuda.empty_cache()
    return results


def test_c2_full_size_sampled():
    """512^2 LOS, 800 channels (40 flagged), 1001 phi, frequency-major."""
    _full_size("c2", ["fp32", "bf16x3", "fp16x3"], 2048)


def test_c3_full_size_sampled():
    """1024^2 LOS, 400 channels, 2001 phi, LOS-major: the benchmark workload."""
    _full_size("c3", ["bf16x3", "fp32", "fp16x3"], 4096)


def test_c4_full_size_sampled():
    """2048^2 LOS, 1024 channels 110-190 MHz (phase arguments up to ~1e4 rad),
    4001 phi, frequency-major: the FP16 split against FP32 (168 GB resident)."""
    _full_size("c4", ["fp16x3", "fp32", "bf16x3"], 2048)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("layout", [LOS_MAJOR, FREQ_MAJOR], ids=["los", "freq"])
def test_nonuniform_phi_grid(prec, layout):
    """An irregular phi grid takes the per-element phase generator instead of
    the factored tables; both must agree with the oracle."""
    note(f"non-uniform phi grid, layout={layout} {prec}")
    rng = np.random.default_rng(77)
    c = make_small_cube(300, 120, 10, seed=78, nflag=7, nsrc=6)
    phi = np.sort(rng.uniform(-150, 150, 333))
    plan = rs.Plan(c["lambda2"], c["weights"], phi)
    Q, U = (c["Q"], c["U"]) if layout == LOS_MAJOR else (c["Q"].T, c["U"].T)
    Q32, U32 = np.float32(Q), np.float32(U)
    out = _run(plan, dev32(Q32), dev32(U32), layout, PRECS[prec])
    _check(out, Q32.astype(np.float64), U32.astype(np.float64), c["lambda2"], c["weights"],
           phi, layout, PREC_TOL[prec])


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_irregular_grid_above_the_table_cap(prec):
    """An irregular grid whose plan-time phase table would pass its size cap
    (4096 channels x 4200 phi) keeps the per-element phase generator; both
    forms agree with the oracle."""
    note(f"irregular grid above the table cap, {prec}")
    rng = np.random.default_rng(91)
    lam = band_lambda2(110.0, 190.0, 4096)
    w = np.ones(lam.size)
    phi = np.sort(rng.uniform(-400, 400, 4200))
    plan = rs.Plan(lam, w, phi)
    nlos = 48
    Q = np.float32(rng.standard_normal((nlos, lam.size)) * 1e-2)
    U = np.float32(rng.standard_normal((nlos, lam.size)) * 1e-2)
    out = _run(plan, dev32(Q), dev32(U), LOS_MAJOR, PRECS[prec])
    _check(out, Q.astype(np.float64), U.astype(np.float64), lam, w, phi, LOS_MAJOR, PREC_TOL[prec])


def test_fp16_split_needs_its_workspace():
    """The FP16 split keeps a per-LOS scale in the caller's workspace, on
    uniform and irregular phi grids alike."""
    import torch
    c = make_small_cube(8, 32, 9, seed=2)
    Q = dev32(c["Q"])
    F = torch.empty((8, 40), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(3)
    for phi in (np.sort(rng.uniform(-50, 50, 40)), np.linspace(-50, 50, 40)):
        plan = rs.Plan(c["lambda2"], c["weights"], phi)
        need = rs.rmsynth_workspace_size(plan.handle, 8, LOS_MAJOR, rs.RMSYNTH_SPLIT_FP16)
        assert need >= 8 * 4
        with pytest.raises(rs.RmsynthError) as ei:
            rs.rmsynth_execute(plan.handle, Q, Q, 8, LOS_MAJOR, rs.RMSYNTH_SPLIT_FP16, F, F)
        assert ei.value.code == rs.rmsynth.RMSYNTH_EWORKSPACE
        small = torch.empty(4, dtype=torch.uint8, device="cuda")
        with pytest.raises(rs.RmsynthError) as ei:
            rs.rmsynth_execute(plan.handle, Q, Q, 8, LOS_MAJOR, rs.RMSYNTH_SPLIT_FP16, F, F,
                               workspace=small, workspace_bytes=4)
        assert ei.value.code == rs.rmsynth.RMSYNTH_EWORKSPACE


@pytest.mark.parametrize("irregular", [False, True], ids=["uniform", "irregular"])
def test_fp16_split_wide_dynamic_range_any_grid(irregular):
    """Per-LOS scaling on either kernel family: LOS whose values differ by 1e8
    in size are all transformed to FP32-like accuracy."""
    note(f"fp16x3 dynamic range, irregular={irregular}")
    c = make_small_cube(96, 160, 257, seed=31, nsrc=10)
    phi = np.sort(np.random.default_rng(4).uniform(-100, 100, 257)) if irregular else c["phi"]
    scales = 10.0 ** np.linspace(-6, 2, 96)
    Q = np.float32(c["Q"] * scales[:, None])
    U = np.float32(c["U"] * scales[:, None])
    plan = rs.Plan(c["lambda2"], c["weights"], phi)
    out = _run(plan, dev32(Q), dev32(U), LOS_MAJOR, rs.RMSYNTH_SPLIT_FP16)
    _check(out, Q.astype(np.float64), U.astype(np.float64), c["lambda2"], c["weights"], phi,
           LOS_MAJOR, PREC_TOL["fp16x3"])


def _compare_fused(plan, Q, U, layout, prec):
    import torch
    Fq, Fu, _ = plan.execute(Q, U, layout, PRECS[prec])
    pk = plan.peaks(Fq, Fu)
    Fq2, Fu2, _, pk2 = plan.execute_peaks(Q, U, layout, PRECS[prec])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(Fq2), host(Fq))
    np.testing.assert_array_equal(host(Fu2), host(Fu))
    for key in ("idx", "phi_pk", "amp", "q_pk", "u_pk"):
        np.testing.assert_array_equal(host(pk2[key]), host(pk[key]), err_msg=f"{prec} {key}")
    return host(pk2["idx"])


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3", "fp32"])
@pytest.mark.parametrize("layout", [LOS_MAJOR, FREQ_MAJOR], ids=["los", "freq"])
@pytest.mark.parametrize("nlos,nchan,nphi", [(1000, 96, 300), (257, 33, 129), (128, 64, 2001)])
def test_execute_peaks_equals_execute_then_peaks(prec, layout, nlos, nchan, nphi):
    """rmsynth_execute_peaks (peaks reduced in the transform kernels' epilogue
    and merged over phi tiles) gives bit for bit the outputs of rmsynth_execute
    followed by rmsynth_peaks: ragged LOS and phi tiles, flagged channels, a
    non-finite LOS."""
    note(f"execute_peaks {prec} layout={layout} {nlos}x{nchan}x{nphi}")
    c = make_small_cube(nlos, nchan, nphi, seed=nlos + nphi, nflag=5, nsrc=12)
    Q, U = np.float32(c["Q"]), np.float32(c["U"])
    unflagged = int(np.flatnonzero(c["weights"] > 0)[0])
    flagged = int(np.flatnonzero(c["weights"] == 0)[0])
    Q[3, unflagged] = np.nan        # poisons LOS 3
    U[5, flagged] = np.inf          # ignored (weight 0)
    plan = rs.Plan(c["lambda2"], c["weights"], np.linspace(-200, 200, nphi))
    if layout == FREQ_MAJOR:
        Q, U = np.ascontiguousarray(Q.T), np.ascontiguousarray(U.T)
    idx = _compare_fused(plan, dev32(Q), dev32(U), layout, prec)
    assert idx[3] == -1 and idx[5] >= 0


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("layout", [LOS_MAJOR, FREQ_MAJOR], ids=["los", "freq"])
def test_execute_peaks_on_an_irregular_grid(prec, layout):
    """The fused peaks on the plan-time phase table (irregular grid): bit for
    bit execute + peaks, ragged tiles, flagged channels, a non-finite LOS."""
    note(f"execute_peaks irregular {prec} layout={layout}")
    c = make_small_cube(300, 72, 10, seed=44, nflag=5, nsrc=12)
    Q, U = np.float32(c["Q"]), np.float32(c["U"])
    Q[3, int(np.flatnonzero(c["weights"] > 0)[0])] = np.nan
    phi = np.sort(np.random.default_rng(45).uniform(-200, 200, 333))
    plan = rs.Plan(c["lambda2"], c["weights"], phi)
    if layout == FREQ_MAJOR:
        Q, U = np.ascontiguousarray(Q.T), np.ascontiguousarray(U.T)
    idx = _compare_fused(plan, dev32(Q), dev32(U), layout, prec)
    assert idx[3] == -1


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_execute_peaks_all_ties_take_the_first_phi(prec):
    """A zero cube: every |F| is 0, so every phi ties and the peak is phi_0."""
    c = make_small_cube(300, 40, 700, seed=9)
    plan = rs.Plan(c["lambda2"], c["weights"], np.linspace(-300, 300, 700))
    Z = dev32(np.zeros((300, 40)))
    idx = _compare_fused(plan, Z, Z, LOS_MAJOR, prec)
    assert np.all(idx == 0)


def test_execute_peaks_workspace_errors():
    import torch
    c = make_small_cube(8, 32, 300, seed=4)
    plan = rs.Plan(c["lambda2"], c["weights"], np.linspace(-100, 100, 300))
    need = rs.rmsynth_execute_peaks_workspace_size(plan.handle, 8, LOS_MAJOR, rs.RMSYNTH_SPLIT_BF16)
    assert need >= 8 * 3 * 8   # one 8-byte record per LOS and phi tile
    assert rs.rmsynth_execute_peaks_workspace_size(plan.handle, 8, LOS_MAJOR, rs.RMSYNTH_FP32) == 0
    Q = dev32(c["Q"])
    F = torch.empty((8, 300), dtype=torch.float32, device="cuda")
    idx = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(rs.RmsynthError) as ei:
        rs.rmsynth_execute_peaks(plan.handle, Q, Q, 8, LOS_MAJOR, rs.RMSYNTH_SPLIT_BF16, F, F, None, idx)
    assert ei.value.code == rs.rmsynth.RMSYNTH_EWORKSPACE
