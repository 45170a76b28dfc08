"""The peaks-only search (F never stored) and the sub-grid peak, through the C ABI.

* rmsynth_search returns bit for bit what rmsynth_execute + rmsynth_peaks
  return, and rmsynth_peak_fit on that stored F, for every precision, both
  layouts, ragged shapes, flagged and non-finite channels, with its workspace
  whole or cut down to one 128-LOS batch.
* The sub-grid peak against the oracle's three-point parabola
  (oracle.peak_fit_from_spectra): on the same F within what one FP32 rounding
  of |F|^2 can move it, and on the oracle's own F within what the per-LOS
  error of F can move it.  Both bars are the parabola's worst-case response
  to amplitude errors of that size (its value at the corners of the error
  box), times two, plus one FP32 ulp of the stored result.
"""
import numpy as np
import pytest

import oracle
import paper_1810_06250_amd as rs
from synthetic import WORKLOADS, make_small_cube, thin_spectrum, LOS_MAJOR, FREQ_MAJOR
from gpu_util import dev32, fit_bar, host, note

pytestmark = pytest.mark.gpu

PRECS = {"fp32": rs.RMSYNTH_FP32, "bf16x3": rs.RMSYNTH_SPLIT_BF16, "fp16x3": rs.RMSYNTH_SPLIT_FP16}
KEYS = ("idx", "phi_pk", "amp", "q_pk", "u_pk")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs.load_library()
    oracle.build(force=False)


def _search_vs_execute(plan, Q, U, layout, prec, nlos, workspace_bytes=None):
    import torch
    Fq, Fu, _ = plan.execute(Q, U, layout, PRECS[prec])
    pk = plan.peaks(Fq, Fu)
    pf, af = plan.peak_fit(Fq, Fu, pk["idx"])
    out = plan.search(Q, U, layout, PRECS[prec], workspace_bytes=workspace_bytes)
    torch.cuda.synchronize()
    for k in KEYS:
        np.testing.assert_array_equal(host(out[k]), host(pk[k]), err_msg=f"{prec} {k}")
    np.testing.assert_array_equal(host(out["phi_fit"]), host(pf), err_msg=f"{prec} phi_fit")
    np.testing.assert_array_equal(host(out["amp_fit"]), host(af), err_msg=f"{prec} amp_fit")
    return {k: host(v) for k, v in out.items()}, host(Fq), host(Fu)


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("layout", [LOS_MAJOR, FREQ_MAJOR], ids=["los", "freq"])
@pytest.mark.parametrize("nlos,nchan,nphi", [(1000, 96, 300), (257, 33, 129), (130, 64, 2001),
                                             (70, 17, 64), (5, 8, 1), (3, 8, 2)])
def test_search_equals_execute_peaks_fit(prec, layout, nlos, nchan, nphi):
    note(f"search {prec} layout={layout} {nlos}x{nchan}x{nphi}")
    c = make_small_cube(nlos, nchan, nphi, seed=nlos + 3 * nphi, nflag=max(1, nchan // 10),
                        nsrc=max(1, nlos // 20))
    Q, U = np.float32(c["Q"]), np.float32(c["U"])
    unflagged = int(np.flatnonzero(c["weights"] > 0)[0])
    flagged = int(np.flatnonzero(c["weights"] == 0)[0])
    Q[1, unflagged] = np.nan       # poisons LOS 1
    U[2, flagged] = np.inf         # ignored (weight 0)
    plan = rs.Plan(c["lambda2"], c["weights"], np.linspace(-150, 150, nphi))
    if layout == FREQ_MAJOR:
        Q, U = np.ascontiguousarray(Q.T), np.ascontiguousarray(U.T)
    out, _, _ = _search_vs_execute(plan, dev32(Q), dev32(U), layout, prec, nlos)
    assert out["idx"][1] == -1 and np.isnan(out["phi_fit"][1]) and np.isnan(out["amp_fit"][1])
    assert out["idx"][2] >= 0


@pytest.mark.parametrize("prec", list(PRECS))
def test_search_on_a_nonuniform_grid(prec):
    """Unfused paths hold F of a batch in the workspace; same results."""
    note(f"search non-uniform grid {prec}")
    c = make_small_cube(400, 80, 10, seed=12, nflag=4, nsrc=20)
    phi = np.sort(np.random.default_rng(5).uniform(-120, 120, 257))
    plan = rs.Plan(c["lambda2"], c["weights"], phi)
    _search_vs_execute(plan, dev32(c["Q"]), dev32(c["U"]), LOS_MAJOR, prec, 400)
    least = rs.rmsynth_search_workspace_size(plan.handle, 128, LOS_MAJOR, PRECS[prec])
    _search_vs_execute(plan, dev32(c["Q"]), dev32(c["U"]), LOS_MAJOR, prec, 400,
                       workspace_bytes=least)


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("layout", [LOS_MAJOR, FREQ_MAJOR], ids=["los", "freq"])
def test_search_in_los_batches(prec, layout):
    """A workspace that holds one 128-LOS batch (or a little more) gives the
    same outputs as the whole one; less than that is refused."""
    import torch
    note(f"search batches {prec} layout={layout}")
    nlos, nchan, nphi = 1000, 48, 400
    c = make_small_cube(nlos, nchan, nphi, seed=8, nflag=3, nsrc=30)
    plan = rs.Plan(c["lambda2"], c["weights"], np.linspace(-100, 100, nphi))
    Q, U = np.float32(c["Q"]), np.float32(c["U"])
    if layout == FREQ_MAJOR:
        Q, U = np.ascontiguousarray(Q.T), np.ascontiguousarray(U.T)
    Qd, Ud = dev32(Q), dev32(U)
    whole = plan.search(Qd, Ud, layout, PRECS[prec])
    least = rs.rmsynth_search_workspace_size(plan.handle, 128, layout, PRECS[prec])
    for nb in (least, least + 5000, 3 * least - 1):
        part = plan.search(Qd, Ud, layout, PRECS[prec], workspace_bytes=nb)
        torch.cuda.synchronize()
        for k, v in whole.items():
            np.testing.assert_array_equal(host(part[k]), host(v), err_msg=f"{nb} {k}")
    with pytest.raises(rs.RmsynthError) as ei:
        plan.search(Qd, Ud, layout, PRECS[prec], workspace_bytes=least - 256)
    assert ei.value.code == rs.RMSYNTH_EWORKSPACE
    # execute and execute_peaks batch the same way
    if prec != "fp32":
        nb = rs.rmsynth_execute_peaks_workspace_size(plan.handle, 128, layout, PRECS[prec])
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        Fq = torch.empty((nlos, nphi), dtype=torch.float32, device="cuda")
        Fu = torch.empty_like(Fq)
        pk = {k: torch.empty(nlos, dtype=torch.int32 if k == "idx" else torch.float32, device="cuda")
              for k in KEYS}
        rs.rmsynth_execute_peaks(plan.handle, Qd, Ud, nlos, layout, PRECS[prec], Fq, Fu, None,
                                 pk["idx"], pk["phi_pk"], pk["amp"], pk["q_pk"], pk["u_pk"], ws, nb)
        for k in KEYS:
            np.testing.assert_array_equal(host(pk[k]), host(whole[k]), err_msg=f"execute_peaks {k}")


def test_peak_fit_matches_oracle():
    """Sub-grid peak on a c1-band cube with sources: against the oracle's fit
    on the same F (FP32 |F|^2 rounding only), and against the oracle's fit on
    the oracle's F (the F error moves it)."""
    note("peak_fit vs oracle")
    c = make_small_cube(600, 128, 201, seed=21, nflag=6, nsrc=120)
    phi = np.linspace(-100, 100, 201)
    plan = rs.Plan(c["lambda2"], c["weights"], phi)
    for prec in ("fp32", "bf16x3"):
        out, Fq, Fu = _search_vs_execute(plan, dev32(c["Q"]), dev32(c["U"]), LOS_MAJOR, prec, 600)
        idx = out["idx"]
        ok = idx >= 0
        assert ok.all()
        # same F: one FP32 rounding of |F|^2 in each amplitude
        pf_o, af_o = oracle.peak_fit_from_spectra(Fq, Fu, phi, idx)
        amp = np.hypot(Fq, Fu).max(axis=1)
        bp, ba = fit_bar(Fq, Fu, phi, idx, 2.0 ** -23 * amp)
        assert np.all(np.abs(out["phi_fit"] - pf_o) <= bp + 2.0 ** -23 * np.abs(pf_o)), prec
        assert np.all(np.abs(out["amp_fit"] - af_o) <= ba + 2.0 ** -23 * af_o), prec
        # oracle F
        Q32, U32 = np.float32(c["Q"]).astype(np.float64), np.float32(c["U"]).astype(np.float64)
        rq, ru = oracle.fdf(Q32, U32, c["lambda2"], c["weights"], phi)
        ref = oracle.peaks(rq, ru, phi)
        err = oracle.per_los_error(Fq, Fu, rq, ru)
        same = (ref["idx"] == idx) & (ref["margin"] > 2e-5)
        assert same.sum() > 550
        pf_r, af_r = oracle.peak_fit_from_spectra(rq, ru, phi, ref["idx"])
        dy = err * np.hypot(rq, ru).max(axis=1)
        bp, ba = fit_bar(rq, ru, phi, ref["idx"], dy)
        d_p = np.abs(out["phi_fit"] - pf_r)[same]
        d_a = np.abs(out["amp_fit"] - af_r)[same]
        note(f"  {prec}: max |dphi_fit| {d_p.max():.2e} (bar {bp[same].max():.2e})")
        assert np.all(d_p <= bp[same] + 2.0 ** -23 * np.abs(pf_r[same])), prec
        assert np.all(d_a <= ba[same] + 2.0 ** -23 * af_r[same]), prec


@pytest.mark.parametrize("prec", list(PRECS))
def test_offgrid_thin_screens(prec):
    """Noise-free thin screens at random off-grid depths (700-1800 MHz band,
    step 2 rad m^-2): the grid peak is up to a step away, the fitted peak
    within 0.01 rad m^-2, as the oracle's fit is on these screens."""
    note(f"off-grid screens {prec}")
    wl = WORKLOADS["c3"]
    lam, w = wl.lambda2(), wl.weights()
    phi = np.arange(-100.0, 100.0 + 1e-9, 2.0)
    rng = np.random.default_rng(11)
    n = 300
    phi0 = rng.uniform(-60, 60, n)
    P0 = rng.uniform(0.01, 0.1, n)
    P = thin_spectrum(lam, P0, phi0, rng.uniform(0, np.pi, n))
    plan = rs.Plan(lam, w, phi)
    out = {k: host(v) for k, v in plan.search(dev32(P.real), dev32(P.imag), LOS_MAJOR,
                                               PRECS[prec]).items()}
    assert np.max(np.abs(out["phi_pk"] - phi0)) > 0.9
    assert np.max(np.abs(out["phi_fit"] - phi0)) < 0.01
    assert np.all(out["amp_fit"] >= out["amp"])


def test_peak_fit_edges():
    """Peaks at the grid ends keep their grid values, a flat spectrum too (the
    parabola does not open downwards), and idx -1 gives NaN."""
    import torch
    phi = np.array([-1.0, 0.0, 1.0, 2.0])
    c = make_small_cube(4, 8, 4, seed=1)
    plan = rs.Plan(c["lambda2"], c["weights"], phi)
    Fq = np.array([[5.0, 4.0, 1.0, 0.5], [0.5, 1.0, 4.0, 5.0], [1.0, 3.0, 2.0, 0.5],
                   [1.0, 1.0, 1.0, 1.0]], np.float32)
    Fu = np.zeros_like(Fq)
    idx = torch.as_tensor(np.array([0, 3, 1, -1], np.int32)).cuda()
    pf, af = (host(t) for t in plan.peak_fit(dev32(Fq), dev32(Fu), idx))
    assert pf[0] == -1.0 and af[0] == 5.0
    assert pf[1] == 2.0 and af[1] == 5.0
    po, ao = oracle.peak_fit_from_spectra(Fq, Fu, phi, np.array([0, 3, 1, -1]))
    assert abs(pf[2] - po[2]) < 1e-6 and abs(af[2] - ao[2]) < 1e-6
    assert np.isnan(pf[3]) and np.isnan(af[3])
    flat = dev32(np.ones((4, 4)))
    pf, af = (host(t) for t in plan.peak_fit(flat, flat * 0, torch.full((4,), 1, dtype=torch.int32,
                                                                          device="cuda")))
    assert np.all(pf == 0.0) and np.all(af == 1.0)
