"""Parity of the gate network's HIP kernels with the FP64 network oracle, and of
the gated peak search with the ungated path, through the C ABI.

The reference is the FP64 network with its 16-bit inputs rounded to half (the
normalised spectrum x and the weight matrices); nothing the kernels round
inside (h1, h2, the back-propagated dz) is mirrored.  The bar is elementwise:
|gpu - oracle| <= oracle.mlp.error_bound, the probabilistic rounding-error
analysis of half rounding at those points plus FP32 accumulation (6 standard
deviations, pinned on the CPU against the same arithmetic in numpy).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
import paper_1810_06250_amd as rs
from gpu_util import dev32, host, note

pytestmark = pytest.mark.gpu

PHI_SCALE = 300.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs.load_library()
    oracle.build(force=False)


def _blocks(vec, nin, h1, h2):
    sizes = [h1 * nin, h1, h2 * h1, h2, 2 * h2, 2]
    shapes = [(h1, nin), (h1,), (h2, h1), (h2,), (2, h2), (2,)]
    out, o = [], 0
    for n, sh in zip(sizes, shapes):
        out.append(np.asarray(vec[o:o + n], np.float64).reshape(sh))
        o += n
    assert o == len(vec)
    return out


def _flat(blocks):
    return np.concatenate([np.asarray(b, np.float64).ravel() for b in blocks])


def _case(seed, B, nchan, h1, h2, flagged=0.1):
    rng = np.random.default_rng(seed)
    w = np.ones(nchan)
    w[rng.uniform(size=nchan) < flagged] = 0.0
    w[rng.uniform(size=nchan) < 0.2] = 0.5
    Q = rng.standard_normal((B, nchan)).astype(np.float32)
    U = rng.standard_normal((B, nchan)).astype(np.float32)
    phi = rng.uniform(-300, 300, B).astype(np.float32)
    det = (rng.uniform(size=B) < 0.5).astype(np.float32)
    params = omlp.init_params(2 * nchan, h1, h2, rng)
    params[1] = rng.standard_normal(h1) * 0.1
    params[3] = rng.standard_normal(h2) * 0.1
    params[5] = rng.standard_normal(2) * 0.1
    p32 = _flat(params).astype(np.float32)
    return w, Q, U, phi, det, p32


def _oracle_grad(p32, w, Q, U, phi, det, nchan, h1, h2, round16=True):
    """Loss, gradients, outputs and the elementwise error bars of the FP64
    network (round16: x and the weights rounded to half)."""
    params = _blocks(p32.astype(np.float64), 2 * nchan, h1, h2)
    x = omlp.normalise(Q.astype(np.float64), U.astype(np.float64), w)
    o, cache = omlp.forward(params, x, round16=round16)
    loss, g = omlp.loss_and_grad_out(o, phi.astype(np.float64), det.astype(np.float64), PHI_SCALE)
    grads = omlp.backward(params, cache, g, round16=round16)
    e_o, bars = omlp.error_bound(params, x, phi.astype(np.float64), det.astype(np.float64),
                                 PHI_SCALE)
    # loss bar: first order in the output error (g is d loss / d o), the
    # squared term of the phi loss, and the FP32 evaluation of the loss terms
    loss_bar = float(np.sum(np.abs(g) * e_o) + np.mean(det * e_o[:, 0] ** 2) + 1e-5 * abs(loss))
    return (loss, loss_bar), grads, o, bars


def _check_blocks(g_gpu, grads, bars, nchan, h1, h2, what):
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    for name, a, b, e in zip(names, _blocks(g_gpu, 2 * nchan, h1, h2), grads, bars):
        assert np.all(np.isfinite(a)), (what, name)
        worst = np.max(np.abs(a - b) / np.maximum(e, 1e-300))
        note(f"  {what} {name}: max |gpu - oracle| / bar = {worst:.3f}")
        assert np.all(np.abs(a - b) <= e), (what, name, worst)


def _check_outputs(ph, sc, params, x):
    """phi_hat / phi_scale and sigmoid(logit) within the error bar of o
    (the sigmoid's slope is at most 1/4; its FP32 evaluation adds < 1e-6)."""
    o, _ = omlp.forward(params, x, round16=True)
    e_o, _ = omlp.error_bound(params, x, np.zeros(len(x)), np.zeros(len(x)), PHI_SCALE)
    sig = 1.0 / (1.0 + np.exp(-o[:, 1]))
    assert np.all(np.abs(ph / PHI_SCALE - o[:, 0]) <= e_o[:, 0] + 1e-7 * np.abs(o[:, 0])), \
        np.max(np.abs(ph / PHI_SCALE - o[:, 0]) / e_o[:, 0])
    assert np.all(np.abs(sc - sig) <= 0.25 * e_o[:, 1] + 1e-6), \
        np.max(np.abs(sc - sig) / (0.25 * e_o[:, 1] + 1e-6))


# (1024, 288, 256, 256) is the gate's training step: the weight-gradient GEMMs
# split the batch into 15 uneven shares (gW1) and 16 (gW2).
@pytest.mark.parametrize("B,nchan,h1,h2", [(200, 40, 64, 128), (64, 288, 256, 256), (1000, 33, 128, 64),
                                          (1024, 288, 256, 256)])
def test_gradient_matches_oracle(B, nchan, h1, h2):
    note(f"mlp grad B={B} nchan={nchan} h1={h1} h2={h2}")
    import torch
    w, Q, U, phi, det, p32 = _case(B + nchan, B, nchan, h1, h2)
    net = rs.Mlp(nchan, h1, h2, weights=w, phi_scale=PHI_SCALE, seed=1)
    net.set_params(p32)
    g, loss = net.grad(dev32(Q), dev32(U), dev32(phi), dev32(det))
    g = host(g).astype(np.float64)
    loss = float(host(loss)[0])
    (l_or, l_bar), grads, _, bars = _oracle_grad(p32, w, Q, U, phi, det, nchan, h1, h2)
    assert abs(loss - l_or) <= l_bar, (loss, l_or, l_bar)
    _check_blocks(g, grads, bars, nchan, h1, h2, "grad")
    # Flagged channels feed nothing: their W1 columns get exactly zero gradient.
    gW1 = _blocks(g, 2 * nchan, h1, h2)[0]
    off = np.concatenate([w == 0, w == 0])
    assert np.all(gW1[:, off] == 0.0)
    # Reductions (split-K weight gradients included) run in a fixed order:
    # a second call gives the same bits.
    g2, _ = net.grad(dev32(Q), dev32(U), dev32(phi), dev32(det))
    np.testing.assert_array_equal(host(g2).astype(np.float64), g)
    net.close()
    torch.cuda.synchronize()


def test_gradient_of_unmirrored_oracle_is_close_too():
    """The FP64 network without half rounding is within the half-precision
    error of the GPU gradient (a check that the mirror hides no real bug)."""
    B, nchan, h1, h2 = 256, 64, 128, 128
    w, Q, U, phi, det, p32 = _case(7, B, nchan, h1, h2)
    net = rs.Mlp(nchan, h1, h2, weights=w, phi_scale=PHI_SCALE)
    net.set_params(p32)
    g, _ = net.grad(dev32(Q), dev32(U), dev32(phi), dev32(det))
    g = host(g).astype(np.float64)
    _, grads, _, _ = _oracle_grad(p32, w, Q, U, phi, det, nchan, h1, h2, round16=False)
    for a, b in zip(_blocks(g, 2 * nchan, h1, h2), grads):
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-12


def test_adam_steps_match_oracle():
    B, nchan, h1, h2 = 128, 48, 64, 64
    lr = 1e-3
    w, Q, U, phi, det, p32 = _case(11, B, nchan, h1, h2)
    net = rs.Mlp(nchan, h1, h2, weights=w, phi_scale=PHI_SCALE)
    net.set_params(p32)
    params = _blocks(p32.astype(np.float64), 2 * nchan, h1, h2)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    x = omlp.normalise(Q.astype(np.float64), U.astype(np.float64), w)
    Qd, Ud, phid, detd = dev32(Q), dev32(U), dev32(phi), dev32(det)
    for step in range(1, 4):
        note(f"adam step {step}")
        o, cache = omlp.forward(params, x, round16=True)
        _, g = omlp.loss_and_grad_out(o, phi.astype(np.float64), det.astype(np.float64), PHI_SCALE)
        grads = omlp.backward(params, cache, g, round16=True)
        _, bars = omlp.error_bound(params, x, phi.astype(np.float64), det.astype(np.float64),
                                   PHI_SCALE)
        omlp.adam_update(params, grads, m, v, step, lr)
        net.train_step(Qd, Ud, phid, detd, lr)
        p_gpu = net.get_params().astype(np.float64)
        for a, b, gr, e in zip(_blocks(p_gpu, 2 * nchan, h1, h2), params, grads, bars):
            # gradient sign certain (outside four error bars) and not tiny
            sure = (np.abs(gr) > 4 * e) & (np.abs(gr) > 1e-2 * np.max(np.abs(gr)))
            assert np.max(np.abs(a - b)[sure], initial=0.0) <= 0.02 * lr * step
            assert np.max(np.abs(a - b)) <= 2.0 * lr * step + 1e-7
    # Flagged-channel weights never move.
    W1 = _blocks(net.get_params(), 2 * nchan, h1, h2)[0]
    off = np.concatenate([w == 0, w == 0])
    np.testing.assert_array_equal(W1[:, off], _blocks(p32, 2 * nchan, h1, h2)[0][:, off])


@pytest.mark.parametrize("nchan,h1,h2", [(96, 128, 64), (288, 256, 256), (256, 256, 256),
                                         (128, 256, 256), (33, 256, 256)])
def test_infer_matches_oracle_and_is_chunk_invariant(nchan, h1, h2):
    """(96, 128, 64) runs the layer-by-layer path in 65 536-row chunks; the
    256 x 256 shapes run the fused kernels: the one-pass kernel for 288, 256
    and 128 channels (the head's transposing sums at 288 and 256, the plain
    butterfly at 128), the two-pass one for 33 channels (ragged K)."""
    n = 70_000                      # crosses the 65 536-row inference chunk
    note(f"mlp infer n={n} nchan={nchan} h1={h1} h2={h2}")
    w, Q, U, phi, det, p32 = _case(5, n, nchan, h1, h2)
    net = rs.Mlp(nchan, h1, h2, weights=w, phi_scale=PHI_SCALE)
    net.set_params(p32)
    Qd, Ud = dev32(Q), dev32(U)
    ph, sc = net.infer(Qd, Ud)
    ph, sc = host(ph), host(sc)
    sel = np.r_[0:300, 65_400:65_700, n - 300:n]
    params = _blocks(p32.astype(np.float64), 2 * nchan, h1, h2)
    x = omlp.normalise(Q[sel].astype(np.float64), U[sel].astype(np.float64), w)
    _check_outputs(ph[sel], sc[sel], params, x)
    # The same rows inferred alone give bit-identical outputs.
    ph2, sc2 = net.infer(Qd[65_400:65_700].contiguous(), Ud[65_400:65_700].contiguous())
    np.testing.assert_array_equal(host(ph2), ph[65_400:65_700])
    np.testing.assert_array_equal(host(sc2), sc[65_400:65_700])


@pytest.mark.parametrize("nchan", [288, 256, 128])
def test_onepass_small_batches_and_nonfinite_rows(nchan):
    """The one-pass kernel on batches of 1, 63 and 65 rows (rows past the end
    of a batch read its last LOS and are never stored) reproduces those rows
    of a larger batch bit for bit.  A non-finite value in an unflagged channel
    makes its row NaN; one in a flagged channel is ignored (the row equals
    the row with that value zeroed); an all-zero row stays finite."""
    h1 = h2 = 256
    n = 200
    w, Q, U, _, _, p32 = _case(41 + nchan, n, nchan, h1, h2)
    flagged, kept = np.flatnonzero(w == 0), np.flatnonzero(w > 0)
    assert flagged.size and kept.size
    Q[7, flagged[0]] = np.nan
    U[9, kept[0]] = np.inf
    Q[11] = 0.0
    U[11] = 0.0
    net = rs.Mlp(nchan, h1, h2, weights=w, phi_scale=PHI_SCALE)
    net.set_params(p32)
    Qd, Ud = dev32(Q), dev32(U)
    ph, sc = (host(t) for t in net.infer(Qd, Ud))
    assert np.isnan(ph[9]) and np.isnan(sc[9])
    finite = np.ones(n, bool)
    finite[9] = False
    assert np.all(np.isfinite(ph[finite])) and np.all(np.isfinite(sc[finite]))
    Q7 = Q[7:8].copy()
    Q7[0, flagged[0]] = 0.0
    p7, s7 = (host(t) for t in net.infer(dev32(Q7), Ud[7:8].contiguous()))
    np.testing.assert_array_equal(p7, ph[7:8])
    np.testing.assert_array_equal(s7, sc[7:8])
    ok = finite.copy()
    ok[7] = False
    params = _blocks(p32.astype(np.float64), 2 * nchan, h1, h2)
    x = omlp.normalise(Q[ok].astype(np.float64), U[ok].astype(np.float64), w)
    _check_outputs(ph[ok], sc[ok], params, x)
    for a, m in ((0, 1), (7, 63), (120, 65), (n - 1, 1)):
        note(f"one-pass nchan={nchan} rows {a}..{a + m}")
        p2, s2 = (host(t) for t in net.infer(Qd[a:a + m].contiguous(), Ud[a:a + m].contiguous()))
        np.testing.assert_array_equal(p2, ph[a:a + m])
        np.testing.assert_array_equal(s2, sc[a:a + m])


def test_infer_with_unit_weights_matches_oracle():
    """All channel weights 1 (the fused kernel then reads none): against the
    oracle, and equal to the network given the weights explicitly."""
    nchan, h1, h2, n = 288, 256, 256, 3000
    _, Q, U, _, _, p32 = _case(31, n, nchan, h1, h2)
    w = np.ones(nchan)
    a = rs.Mlp(nchan, h1, h2, phi_scale=PHI_SCALE)
    b = rs.Mlp(nchan, h1, h2, weights=w, phi_scale=PHI_SCALE)
    a.set_params(p32)
    b.set_params(p32)
    Qd, Ud = dev32(Q), dev32(U)
    pa, sa = (host(t) for t in a.infer(Qd, Ud))
    pb, sb = (host(t) for t in b.infer(Qd, Ud))
    np.testing.assert_array_equal(pa, pb)
    np.testing.assert_array_equal(sa, sb)
    x = omlp.normalise(Q.astype(np.float64), U.astype(np.float64), w)
    _check_outputs(pa, sa, _blocks(p32.astype(np.float64), 2 * nchan, h1, h2), x)


def test_infer_follows_parameter_changes():
    """The fused kernel reads a fragment-order copy of W1 and W2 that the first
    inference after a parameter change rebuilds: inference after set_params
    and after an Adam step must use the new parameters."""
    nchan, h1, h2, n = 288, 256, 256, 2048
    w, Q, U, phi, det, p_a = _case(21, n, nchan, h1, h2)
    _, _, _, _, _, p_b = _case(22, n, nchan, h1, h2)
    net = rs.Mlp(nchan, h1, h2, weights=w, phi_scale=PHI_SCALE)
    Qd, Ud = dev32(Q), dev32(U)
    x = omlp.normalise(Q.astype(np.float64), U.astype(np.float64), w)

    def check(p32):
        ph, sc = (host(t) for t in net.infer(Qd, Ud))
        _check_outputs(ph, sc, _blocks(np.asarray(p32, np.float64), 2 * nchan, h1, h2), x)
        return ph

    net.set_params(p_a)
    ph_a = check(p_a)
    net.set_params(p_b)
    ph_b = check(p_b)
    assert not np.array_equal(ph_a, ph_b)
    net.train_step(Qd, Ud, dev32(phi), dev32(det), lr=1e-2)
    check(net.get_params())


def test_nonfinite_inputs():
    nchan, h1, h2 = 32, 64, 64
    w = np.ones(nchan)
    w[3] = 0.0
    rng = np.random.default_rng(2)
    Q = rng.standard_normal((4, nchan)).astype(np.float32)
    U = rng.standard_normal((4, nchan)).astype(np.float32)
    Q[1, 3] = np.nan      # flagged channel: ignored
    U[2, 5] = np.inf      # unflagged: outputs NaN
    Q[3] = 0.0
    U[3] = 0.0            # all-zero spectrum: finite
    net = rs.Mlp(nchan, h1, h2, weights=w, seed=3)
    ph, sc = (host(t) for t in net.infer(dev32(Q), dev32(U)))
    assert np.isfinite(ph[[0, 1, 3]]).all() and np.isfinite(sc[[0, 1, 3]]).all()
    assert np.isnan(ph[2]) and np.isnan(sc[2])


def test_save_load_roundtrip(tmp_path):
    nchan, h1, h2 = 20, 64, 64
    w, Q, U, phi, det, p32 = _case(9, 64, nchan, h1, h2)
    net = rs.Mlp(nchan, h1, h2, weights=w, phi_scale=123.0, seed=4)
    net.train_step(dev32(Q), dev32(U), dev32(phi), dev32(det), 1e-3)
    path = str(tmp_path / "net.bin")
    net.save(path)
    net2 = rs.Mlp.load(path)
    np.testing.assert_array_equal(net.get_params(), net2.get_params())
    a = [host(t) for t in net.infer(dev32(Q), dev32(U))]
    b = [host(t) for t in net2.infer(dev32(Q), dev32(U))]
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    # Training continues identically (same Adam moments and step).
    for n in (net, net2):
        n.train_step(dev32(Q), dev32(U), dev32(phi), dev32(det), 1e-3)
    np.testing.assert_array_equal(net.get_params(), net2.get_params())


def test_create_seed_is_deterministic_and_he_scaled():
    a = rs.Mlp(100, 128, 64, seed=42).get_params()
    b = rs.Mlp(100, 128, 64, seed=42).get_params()
    c = rs.Mlp(100, 128, 64, seed=43).get_params()
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)
    W1 = a[:128 * 200]
    assert abs(W1.std() - np.sqrt(2.0 / 200)) < 0.05 * np.sqrt(2.0 / 200)


# ------------------------------------------------------------------ gate
def _gate_setup(n, nchan=64, nphi=301, seed=21):
    rng = np.random.default_rng(seed)
    nu = np.linspace(800e6, 1088e6, nchan)
    lam = (299792458.0 / nu) ** 2
    w = np.ones(nchan)
    w[rng.uniform(size=nchan) < 0.05] = 0.0
    phi = np.linspace(-300, 300, nphi)
    plan = rs.Plan(lam, w, phi)
    Q = rng.standard_normal((n, nchan)).astype(np.float32)
    U = rng.standard_normal((n, nchan)).astype(np.float32)
    net = rs.Mlp(nchan, 64, 64, weights=w, seed=seed)
    return plan, net, Q, U, lam, w, phi


@pytest.mark.parametrize("n,tau", [(5000, 0.5), (300_000, 0.55), (1000, 0.0), (777, 2.0)])
def test_gate_matches_ungated_on_gated_lines(n, tau):
    note(f"gate n={n} tau={tau}")
    plan, net, Q, U, lam, w, phi = _gate_setup(n)
    Q[n // 3, 7] = np.nan if w[7] > 0 else Q[n // 3, 7]
    Qd, Ud = dev32(Q), dev32(U)
    out = {k: host(v) for k, v in net.gate(plan, Qd, Ud, tau).items()}
    ph, sc = (host(t) for t in net.infer(Qd, Ud))
    edge = np.float32(np.max(np.abs(phi)) - plan.info["fwhm_est"])
    want = ~(np.isfinite(ph) & np.isfinite(sc)) | (sc >= np.float32(tau)) | (np.abs(ph) > edge)
    np.testing.assert_array_equal(out["gated"], want.astype(np.int32))
    Fq, Fu, _ = plan.execute(Qd, Ud)
    full = {k: host(v) for k, v in plan.peaks(Fq, Fu).items()}
    g = want
    np.testing.assert_array_equal(out["idx"][g], full["idx"][g])
    np.testing.assert_array_equal(out["phi_pk"][g], full["phi_pk"][g])
    np.testing.assert_array_equal(out["amp"][g], full["amp"][g])
    assert np.all(out["idx"][~g] == -1) and np.all(np.isnan(out["amp"][~g]))
    np.testing.assert_array_equal(out["phi_pk"][~g], ph[~g])
    if tau == 0.0:
        assert g.all()
    # Spot-check the gated peaks against the FP64 oracle.
    sel = np.flatnonzero(g & np.isfinite(out["amp"]))[:64]
    if sel.size:
        rq, ru = oracle.fdf(Q[sel].astype(np.float64), U[sel].astype(np.float64), lam, w, phi)
        n_u, mism, bad = oracle.peak_agreement(out["idx"][sel], rq, ru, oracle.peaks(rq, ru, phi))
        assert mism == 0 and bad == 0, (mism, bad)


@pytest.mark.parametrize("prec", [rs.RMSYNTH_SPLIT_BF16, rs.RMSYNTH_FP32])
def test_gate_search_matches_the_search_on_gated_lines(prec):
    """rmsynth_gate_search: the gated LOS get bit for bit what rmsynth_search
    gives over the whole cube in the same precision; the rest as the FP32 gate."""
    n = 20_000
    note(f"gate search n={n} prec={prec}")
    plan, net, Q, U, lam, w, phi = _gate_setup(n)
    Qd, Ud = dev32(Q), dev32(U)
    out = {k: host(v) for k, v in net.gate(plan, Qd, Ud, 0.5, precision=prec).items()}
    ref = {k: host(v) for k, v in net.gate(plan, Qd, Ud, 0.5).items()}
    full = {k: host(v) for k, v in plan.search(Qd, Ud, rs.RMSYNTH_LOS_MAJOR, prec).items()}
    g = out["gated"].astype(bool)
    np.testing.assert_array_equal(out["gated"], ref["gated"])
    for k in ("idx", "phi_pk", "amp"):
        np.testing.assert_array_equal(out[k][g], full[k][g])
        np.testing.assert_array_equal(out[k][~g], ref[k][~g])
    assert g.any() and (~g).any()


def test_gate_argument_errors():
    plan, net, Q, U, lam, w, phi = _gate_setup(10)
    other = rs.Plan(lam[:-1], w[:-1], phi)
    import torch
    i32 = torch.empty(10, dtype=torch.int32, device="cuda")
    f32 = torch.empty(10, dtype=torch.float32, device="cuda")
    nb = rs.rmsynth_gate_workspace_size(plan.handle, net.handle, 10)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    # The binding refuses a cube that does not fit the plan before any call...
    with pytest.raises(ValueError):
        rs.rmsynth_gate_execute(other.handle, net.handle, dev32(Q), dev32(U), 10, 0.5, i32, f32,
                                f32, i32, ws, nb)
    # ...and the library a plan whose channel count is not the network's.
    with pytest.raises(rs.RmsynthError) as e:
        rs.rmsynth_gate_execute(other.handle, net.handle, dev32(Q[:, :-1]), dev32(U[:, :-1]), 10,
                                0.5, i32, f32, f32, i32, ws, nb)
    assert e.value.code == -1
    with pytest.raises(rs.RmsynthError) as e:
        rs.rmsynth_gate_execute(plan.handle, net.handle, dev32(Q), dev32(U), 10, 0.5, i32, f32,
                                f32, i32, ws, nb - 1)
    assert e.value.code == -5
