"""rmsynth_search_noalloc (the search with its workspace in the library's own
fixed device array) against rmsynth_search with a caller's workspace, through
the C ABI: two calls in a row on one device, the second with a smaller input,
for the fused split path (records in the array, several batches) on a
uniform and on an irregular phi grid, and the FP32 path (F of a batch in the
array)."""
import numpy as np
import pytest

import paper_1810_06250_amd as rs
from synthetic import make_small_cube, LOS_MAJOR, FREQ_MAJOR
from gpu_util import dev32, host, note

pytestmark = pytest.mark.gpu

KEYS = ("idx", "phi_pk", "amp", "q_pk", "u_pk", "phi_fit", "amp_fit")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs.load_library()


def _outputs(n):
    import torch
    return {k: torch.full((n,), -7, dtype=torch.int32 if k == "idx" else torch.float32,
                          device="cuda") for k in KEYS}


def _noalloc(plan, Q, U, n, layout, prec):
    out = _outputs(n)
    rs.rmsynth_search_noalloc(plan.handle, Q, U, n, layout, prec, out["idx"], out["phi_pk"],
                              out["amp"], out["q_pk"], out["u_pk"], out["phi_fit"], out["amp_fit"])
    return out


@pytest.mark.parametrize("prec,layout,nlos,nchan,nphi,irregular", [
    (rs.RMSYNTH_SPLIT_BF16, LOS_MAJOR, 150_000, 64, 2001, False),
    (rs.RMSYNTH_SPLIT_FP16, FREQ_MAJOR, 70_000, 40, 4001, False),
    (rs.RMSYNTH_SPLIT_BF16, LOS_MAJOR, 120_000, 56, 1601, True),
    (rs.RMSYNTH_FP32, LOS_MAJOR, 20_000, 48, 1501, False),
])
def test_noalloc_search_equals_search(prec, layout, nlos, nchan, nphi, irregular):
    import torch
    scratch = rs.rmsynth_search_noalloc_scratch_bytes()
    assert scratch == 64 << 20
    for call, n in enumerate((nlos, nlos // 7 + 3)):
        note(f"noalloc prec={prec} layout={layout} call {call}: {n} LOS x {nchan} x {nphi}")
        c = make_small_cube(n, nchan, nphi, seed=100 * call + prec, nflag=3, nsrc=n // 50)
        phi = c["phi"]
        if irregular:       # each phi moved by up to a fifth of the step: still sorted
            step = phi[1] - phi[0]
            phi = phi + np.random.default_rng(call).uniform(-0.2, 0.2, phi.size) * step
        plan = rs.Plan(c["lambda2"], c["weights"], phi)
        Q, U = np.float32(c["Q"]), np.float32(c["U"])
        Q[5, int(np.flatnonzero(c["weights"] > 0)[0])] = np.nan
        if layout == FREQ_MAJOR:
            Q, U = np.ascontiguousarray(Q.T), np.ascontiguousarray(U.T)
        Qd, Ud = dev32(Q), dev32(U)
        ref = plan.search(Qd, Ud, layout, prec)
        whole = rs.rmsynth_search_workspace_size(plan.handle, n, layout, prec)
        if call == 0:
            assert whole > scratch      # the array holds only part: several batches
        got = _noalloc(plan, Qd, Ud, n, layout, prec)
        torch.cuda.synchronize()
        for k in KEYS:
            np.testing.assert_array_equal(host(got[k]), host(ref[k]), err_msg=f"call {call} {k}")
        assert host(got["idx"])[5] == -1
        plan.close()


def test_noalloc_rejects_what_does_not_fit():
    """An unfused path whose 128-LOS batch of F exceeds the array is refused
    before anything runs."""
    import torch
    nphi = 70_000
    c = make_small_cube(4, 16, 3, seed=1)
    phi = np.sort(np.random.default_rng(2).uniform(-500, 500, nphi))   # non-uniform: unfused
    plan = rs.Plan(c["lambda2"], c["weights"], phi)
    Q = dev32(c["Q"])
    out = _outputs(4)
    with pytest.raises(rs.RmsynthError) as ei:
        rs.rmsynth_search_noalloc(plan.handle, Q, Q, 4, LOS_MAJOR, rs.RMSYNTH_FP32, out["idx"])
    assert ei.value.code == rs.RMSYNTH_EINVAL and "too large" in str(ei.value)
    torch.cuda.synchronize()
