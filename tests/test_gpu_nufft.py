"""The NUFFT evaluation of eq. (11) (rmsynth_execute_nufft) against the FP64
oracles, through the C ABI.

Bars, per LOS as for the direct paths: max_k |F_gpu - F_ref| / max_k |F_ref|
<= 1e-5 against the direct sum (oracle.fdf: the definition) and against the
oracle's own NUFFT of the same steps (oracle.nufft.fdf_nufft, FP64; the two
differ by the kernel truncation, below 1e-6 at width 8).  Peaks agree with
the direct sum's under the usual rule.
"""
import numpy as np
import pytest

import oracle
from oracle import nufft as onufft
import paper_1810_06250_amd as rs
from synthetic import WORKLOADS, make_cube, make_small_cube, stratified_subsample
from gpu_util import dev32, host, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs.load_library()
    oracle.build(force=False)


def _check(lam, w, phi, Q, U, tol=1e-5):
    plan = rs.Plan(lam, w, phi)
    Fq, Fu, Fa = plan.execute_nufft(dev32(Q), dev32(U), want_abs=True)
    gq, gu, ga = host(Fq), host(Fu), host(Fa)
    Q64, U64 = np.float32(Q).astype(np.float64), np.float32(U).astype(np.float64)
    rq, ru = oracle.fdf(Q64, U64, lam, w, phi)
    e_direct = oracle.per_los_error(gq, gu, rq, ru)
    nq, nu = onufft.fdf_nufft(Q64, U64, lam, w, phi)
    e_nufft = oracle.per_los_error(gq, gu, nq, nu)
    note(f"  nufft: max per-LOS error {e_direct.max():.3e} (direct sum), {e_nufft.max():.3e} (oracle NUFFT)")
    assert np.all(np.isfinite(e_direct))
    assert e_direct.max() <= tol and e_nufft.max() <= tol
    np.testing.assert_allclose(ga, np.hypot(gq, gu), rtol=1e-6, atol=1e-30)
    pk = plan.peaks(Fq, Fu)
    nun, mism, bad = oracle.peak_agreement(host(pk["idx"]), rq, ru, oracle.peaks(rq, ru, phi))
    assert mism == 0 and bad == 0, (mism, nun, bad)
    plan.close()
    return gq, gu


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_nufft_on_every_band(name):
    """Each workload's band, grid and source mix (LOS-major), a few hundred LOS:
    grids of 512 to 8192 points, odd and even log2 n."""
    note(f"nufft {name}")
    wl = WORKLOADS[name]
    cube = make_cube(wl, nlos=300, device="cpu", layout=0)
    _check(cube["lambda2"], cube["weights"], cube["phi"], cube["Q"].numpy(), cube["U"].numpy())


@pytest.mark.parametrize("nphi", [1, 2, 7, 64, 300, 1025])
def test_nufft_ragged_grids(nphi):
    note(f"nufft nphi={nphi}")
    c = make_small_cube(130, 77, nphi, seed=nphi, nflag=7, nsrc=10)
    _check(c["lambda2"], c["weights"], c["phi"], c["Q"], c["U"])


def test_nufft_off_centre_grid_and_flags():
    """A grid not centred on 0 (the phase of phi_c in every coefficient); NaN
    in flagged channels has no effect, NaN in an unflagged one poisons its LOS."""
    wl = WORKLOADS["c3"]
    cube = make_cube(wl, nlos=200, device="cpu", layout=0)
    lam, w = cube["lambda2"], cube["weights"].copy()
    w[[3, 50, 399]] = 0.0
    phi = 137.0 + 2.0 * np.arange(300)
    Q, U = cube["Q"].numpy().copy(), cube["U"].numpy().copy()
    gq, _ = _check(lam, w, phi, Q, U)
    Q[:, 50] = np.nan
    Q[7, 10] = np.nan
    plan = rs.Plan(lam, w, phi)
    Fq, Fu, _ = plan.execute_nufft(dev32(Q), dev32(U))
    hq = host(Fq)
    keep = np.arange(200) != 7
    np.testing.assert_array_equal(hq[keep], gq[keep])
    assert np.all(np.isnan(hq[7]))


def test_nufft_unsupported():
    import torch
    c = make_small_cube(4, 16, 5, seed=1)
    irregular = rs.Plan(c["lambda2"], c["weights"], np.array([0.0, 1.0, 3.0, 4.0, 9.0]))
    wide = rs.Plan(c["lambda2"], c["weights"], np.linspace(-10, 10, 4097))
    Q = dev32(c["Q"])
    for plan in (irregular, wide):
        F = torch.empty((4, plan.nphi), dtype=torch.float32, device="cuda")
        with pytest.raises(rs.RmsynthError) as ei:
            rs.rmsynth_execute_nufft(plan.handle, Q, Q, 4, F, F)
        assert ei.value.code == rs.RMSYNTH_EUNSUPPORTED


def test_nufft_c3_full_size_sampled():
    """The benchmark's NUFFT launch: the whole c3 cube (1 048 576 LOS) in one
    call; 512 sampled LOS (half with sources) against the direct-sum and the
    NUFFT oracles, and their peaks."""
    import torch
    wl = WORKLOADS["c3"]
    note("nufft c3 full size")
    cube = make_cube(wl, device="cuda")
    lam, w, phi = cube["lambda2"], cube["weights"], cube["phi"]
    plan = rs.Plan(lam, w, phi)
    Fq, Fu, _ = plan.execute_nufft(cube["Q"], cube["U"])
    torch.cuda.synchronize()
    sub = stratified_subsample(wl.nlos, cube["src_los"], 512, seed=wl.seed + 7)
    subt = torch.as_tensor(sub, device="cuda")
    Q64 = host(cube["Q"][subt]).astype(np.float64)
    U64 = host(cube["U"][subt]).astype(np.float64)
    gq, gu = host(Fq[subt]), host(Fu[subt])
    rq, ru = oracle.fdf(Q64, U64, lam, w, phi)
    nq, nu = onufft.fdf_nufft(Q64, U64, lam, w, phi)
    e_direct = oracle.per_los_error(gq, gu, rq, ru)
    e_nufft = oracle.per_los_error(gq, gu, nq, nu)
    note(f"  nufft c3: max per-LOS error {e_direct.max():.3e} (direct), {e_nufft.max():.3e} (oracle NUFFT)")
    assert e_direct.max() <= 1e-5 and e_nufft.max() <= 1e-5
    pk = plan.peaks(Fq, Fu)
    nun, mism, bad = oracle.peak_agreement(host(pk["idx"])[sub], rq, ru, oracle.peaks(rq, ru, phi))
    assert mism == 0 and bad == 0, (mism, nun, bad)
    plan.close()
