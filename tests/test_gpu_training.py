"""Parity of the training-data synthesis kernel with the FP64 training oracle,
through the C ABI.

Both sides draw the same Philox4x32-10 words and evaluate the sky model and
Box-Muller in FP64; the GPU rounds to FP32 once.  Bars: classes bit-exact;
Q, U within one FP32 ulp of the oracle's FP32-rounded value (FP64 library
functions may differ in the last bit, which moves a rounding decision only
rarely) and at least 99 % bit-identical; labels equal to the oracle's wherever
the oracle's peak is unambiguous (margin > 2e-5) and its peak |F| is not
within 1e-5 (relative) of the detection threshold.
"""
import numpy as np
import pytest

import oracle
from oracle import training as otr
import paper_1810_06250_amd as rs
from synthetic import band_lambda2, phi_grid, noise_sigma_F
from gpu_util import host, note

pytestmark = pytest.mark.gpu

NCHAN = 288
LAM = band_lambda2(800.0, 1088.0, NCHAN)
W = np.ones(NCHAN)
W[[5, 77, 200]] = 0.0
PHI = phi_grid(-300.0, 300.0, 0.5)
SIGF = noise_sigma_F(1e-3, W)


def _spec(**kw):
    d = dict(frac_noise=0.25, frac_thin1=0.30, frac_thin2=0.20, p0_lo=3 * SIGF, p0_hi=50 * SIGF,
             phi_lo=-300.0, phi_hi=300.0, w_lo=10.0, w_hi=100.0, sigma=1e-3,
             det_threshold=6 * SIGF)
    d.update(kw)
    return rs.TrainSpec(**d)


@pytest.fixture(scope="module")
def plan():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs.load_library()
    oracle.build(force=False)
    return rs.Plan(LAM, W, PHI)


def _ulp32(x):
    x = np.abs(np.asarray(x, np.float32))
    return np.spacing(x).astype(np.float64)


@pytest.mark.parametrize("seed,first,n", [(1, 0, 3000), (2 ** 40 + 3, 2 ** 32 - 1500, 3000)])
def test_spectra_match_oracle(plan, seed, first, n):
    note(f"training spectra seed={seed} first={first} n={n}")
    spec = _spec()
    out = rs.make_training_data(plan, spec, seed, first, n, labels=False, extras=True)
    Q, U, cls, truth = (host(out[k]) for k in ("Q", "U", "cls", "truth"))
    Qo, Uo, clso, trutho = otr.spectra(spec.as_dict(), seed, first, n, LAM)
    np.testing.assert_array_equal(cls, clso)
    for a, b in ((Q, Qo), (U, Uo)):
        d = np.abs(a.astype(np.float64) - b)
        assert np.all(d <= _ulp32(b) * 1.0001), np.max(d / _ulp32(b))
        assert np.mean(d == 0) >= 0.99
    np.testing.assert_array_equal(np.isnan(truth), np.isnan(trutho))
    ok = ~np.isnan(trutho)
    np.testing.assert_allclose(truth[ok], trutho[ok].astype(np.float32), rtol=0, atol=0)


def test_batches_are_position_free(plan):
    spec = _spec()
    a = rs.make_training_data(plan, spec, 9, 1000, 500, labels=False)
    b = rs.make_training_data(plan, spec, 9, 1200, 100, labels=False)
    np.testing.assert_array_equal(host(a["Q"])[200:300], host(b["Q"]))
    np.testing.assert_array_equal(host(a["U"])[200:300], host(b["U"]))


def test_labels_match_oracle(plan):
    n = 2000
    note(f"training labels n={n}")
    spec = _spec()
    out = rs.make_training_data(plan, spec, 77, 5000, n, labels=True)
    Q, U = host(out["Q"]).astype(np.float64), host(out["U"]).astype(np.float64)
    phl, det = host(out["phi_label"]), host(out["det_label"])
    phl_o, det_o, pk, _ = otr.labels(Q, U, LAM, W, PHI, spec.det_threshold, oracle.fdf, oracle.peaks)
    clear = pk["margin"] > 2e-5
    # Noise-only and slab lines of sight often have flat tops; most peaks are clear.
    assert clear.mean() > 0.5
    np.testing.assert_array_equal(phl[clear], phl_o[clear].astype(np.float32))
    far = np.abs(pk["amp"] - spec.det_threshold) > 1e-5 * spec.det_threshold
    np.testing.assert_array_equal(det[far], det_o[far])
    # The class mix shows in the labels: most source-free lines are not detections.
    assert 0.3 < det.mean() < 0.8


def test_noise_only_and_zero_sigma_edge_cases(plan):
    spec = _spec(frac_noise=1.0, frac_thin1=0.0, frac_thin2=0.0)
    out = rs.make_training_data(plan, spec, 3, 0, 4000, labels=True, extras=True)
    assert np.all(host(out["cls"]) == 0)
    assert np.all(np.isnan(host(out["truth"])))
    # 6 sigma_F on ~20 independent resolution elements: false detections are rare.
    assert host(out["det_label"]).mean() < 0.01
    spec0 = _spec(sigma=0.0, frac_noise=0.0, frac_thin1=1.0, frac_thin2=0.0)
    out0 = rs.make_training_data(plan, spec0, 4, 0, 256, labels=True, extras=True)
    tr0 = host(out0["truth"])
    # A noiseless screen peaks within half a grid step of its depth, at |F| = P0
    # up to the sampling loss of half a step on an RMSF ~54 rad/m^2 wide.
    assert np.all(np.abs(host(out0["phi_label"]) - tr0[:, 0]) <= 0.25 + 1e-4)
    det0, P0 = host(out0["det_label"]), tr0[:, 1]
    thr = spec0.det_threshold
    assert np.all(det0[P0 > 1.001 * thr] == 1.0) and np.all(det0[P0 < 0.999 * thr] == 0.0)


def test_training_argument_errors(plan):
    import torch
    Q = torch.empty((4, NCHAN), dtype=torch.float32, device="cuda")
    bad = [dict(frac_noise=0.7, frac_thin1=0.5), dict(w_lo=0.0), dict(p0_lo=-1.0),
           dict(sigma=-1.0), dict(phi_lo=5.0, phi_hi=1.0)]
    for kw in bad:
        with pytest.raises(rs.RmsynthError) as e:
            rs.rmsynth_synth_training(plan.handle, _spec(**kw), 0, 0, 4, Q, Q)
        assert e.value.code == rs.RMSYNTH_EINVAL, kw
    lab = torch.empty(4, dtype=torch.float32, device="cuda")
    with pytest.raises(rs.RmsynthError) as e:
        rs.rmsynth_synth_training(plan.handle, _spec(), 0, 0, 4, Q, Q, lab, lab)
    assert e.value.code == rs.RMSYNTH_EWORKSPACE
