"""Pins of the FP64 surrogate-network oracle: finite differences, closed-form
special cases of the loss, the first Adam step, and the input normalisation."""
import numpy as np

from oracle import mlp


def _setup(seed=0, B=7, nin=12, h1=9, h2=8):
    rng = np.random.default_rng(seed)
    params = mlp.init_params(nin, h1, h2, rng)
    params[1] = rng.standard_normal(h1) * 0.1
    params[3] = rng.standard_normal(h2) * 0.1
    params[5] = rng.standard_normal(2) * 0.1
    x = rng.standard_normal((B, nin))
    phi = rng.uniform(-300, 300, B)
    det = (rng.uniform(size=B) > 0.5).astype(float)
    return params, x, phi, det


def _loss(params, x, phi, det):
    o, _ = mlp.forward(params, x)
    return mlp.loss_and_grad_out(o, phi, det, 300.0)[0]


def test_backward_matches_central_differences():
    params, x, phi, det = _setup()
    o, cache = mlp.forward(params, x)
    _, g = mlp.loss_and_grad_out(o, phi, det, 300.0)
    grads = mlp.backward(params, cache, g)
    rng = np.random.default_rng(1)
    h = 1e-6
    for pi, (p, gp) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        gflat = gp.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            keep = flat[idx]
            flat[idx] = keep + h
            lp = _loss(params, x, phi, det)
            flat[idx] = keep - h
            lm = _loss(params, x, phi, det)
            flat[idx] = keep
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[idx]) <= 1e-6 * max(1.0, abs(fd)), (pi, idx, fd, gflat[idx])


def test_loss_special_cases():
    o = np.array([[0.5, 0.0], [0.2, 0.0]])
    loss, g = mlp.loss_and_grad_out(o, np.array([0.0, 60.0]), np.array([0.0, 1.0]), 300.0)
    # BCE at logit 0 is log 2 for either label; the phi term counts only where det = 1.
    assert abs(loss - (np.log(2.0) + 0.5 * (0.2 - 0.2) ** 2)) < 1e-15
    assert g[0, 0] == 0.0 and abs(g[0, 1] - 0.25) < 1e-15 and abs(g[1, 1] + 0.25) < 1e-15
    big = np.array([[0.0, 800.0], [0.0, -800.0]])
    loss2, _ = mlp.loss_and_grad_out(big, np.zeros(2), np.array([1.0, 0.0]), 300.0)
    assert loss2 == 0.0  # confident and right, no overflow


def test_first_adam_step_is_sign_step():
    """With m = v = 0, the first bias-corrected step is lr * g / (|g| + eps)."""
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    mlp.adam_update(p, g, m, v, 1, 0.01)
    expect = np.array([1.0, -2.0, 3.0]) - 0.01 * g[0] / (np.abs(g[0]) + 1e-8)
    np.testing.assert_allclose(p[0], expect, rtol=0, atol=1e-15)


def test_normalise_unit_rms_and_weights():
    rng = np.random.default_rng(4)
    Q = rng.standard_normal((5, 10))
    U = rng.standard_normal((5, 10))
    x = mlp.normalise(Q, U)
    np.testing.assert_allclose(np.sqrt(np.mean(x * x, axis=1)), 1.0, rtol=1e-14)
    w = np.ones(10)
    w[3] = 0
    xw = mlp.normalise(Q, U, w)
    assert np.all(xw[:, 3] == 0) and np.all(xw[:, 13] == 0)
    assert np.all(mlp.normalise(np.zeros((1, 4)), np.zeros((1, 4))) == 0)


def test_relu_network_forward_by_hand():
    """A 1-unit network evaluated by hand."""
    params = [np.array([[2.0, -1.0]]), np.array([0.5]), np.array([[3.0]]), np.array([-1.0]),
              np.array([[1.0], [-2.0]]), np.array([0.25, 0.0])]
    o, _ = mlp.forward(params, np.array([[1.0, 1.0], [-1.0, 1.0]]))
    # row 0: z1 = 1.5, h2 = relu(3*1.5 - 1) = 3.5 -> o = (3.75, -7); row 1: z1 = -2.5 -> 0 -> h2 = 0
    np.testing.assert_allclose(o, [[3.75, -7.0], [0.25, 0.0]], rtol=0, atol=1e-15)


def _kernel_arithmetic(params, x, phi, det, phi_scale):
    """The network evaluated the way the GPU kernels evaluate it, written
    independently of the bound: x, h1, h2 and the weights rounded to half,
    products summed in FP32, the back-propagated dz rounded to half at the
    batch-sum scale, bias gradients from the unrounded dz."""
    f32, f16 = np.float32, np.float16

    def h(a):
        return np.asarray(a, f32).astype(f16).astype(f32)

    W1, b1, W2, b2, W3, b3 = params
    W1h, W2h, W3h = h(W1), h(W2), h(W3)
    b1, b2, b3 = (np.asarray(b, f32) for b in (b1, b2, b3))
    B = len(x)
    xh = h(x)
    z1 = xh @ W1h.T + b1
    h1 = h(np.maximum(z1, 0))
    z2 = h1 @ W2h.T + b2
    h2 = h(np.maximum(z2, 0))
    o = h2 @ W3h.T + b3
    d = np.asarray(det, f32)
    t = np.asarray(phi, f32) / f32(phi_scale)
    s = o[:, 1]
    e = np.exp(-np.abs(s))
    sig = np.where(s >= 0, 1 / (1 + e), e / (1 + e)).astype(f32)
    g = np.stack([2 * d * (o[:, 0] - t), sig - d], axis=1).astype(f32)     # batch-sum gradient
    gW3, gb3 = (g.T @ h2) / f32(B), g.sum(axis=0) / f32(B)
    dz2 = (g @ W3h) * (z2 > 0)
    gW2, gb2 = (h(dz2).T @ h1) / f32(B), dz2.sum(axis=0) / f32(B)
    dz1 = (h(dz2) @ W2h) * (z1 > 0)
    gW1, gb1 = (h(dz1).T @ xh) / f32(B), dz1.sum(axis=0) / f32(B)
    return o, [gW1, gb1, gW2, gb2, gW3, gb3]


def _bound_case(seed, B=96, nin=40, nh1=48, nh2=32):
    params, x, phi, det = _setup(seed=seed, B=B, nin=nin, h1=nh1, h2=nh2)
    x = x * np.exp(np.random.default_rng(seed + 100).uniform(-3, 3, x.shape))   # wide range
    ref_o, cache = mlp.forward(params, x, round16=True)
    _, g = mlp.loss_and_grad_out(ref_o, phi, det, 300.0)
    ref_g = mlp.backward(params, cache, g, round16=True)
    sim_o, sim_g = _kernel_arithmetic(params, x, phi, det, 300.0)
    return params, x, phi, det, ref_o, ref_g, sim_o, sim_g


def test_error_bound_covers_the_kernel_arithmetic():
    """error_bound's bar holds the half/FP32 evaluation of the network element
    by element (the largest error is about a third of the bar here), and is
    tight enough to matter: a few per cent of the typical gradient (W1's bar
    is wider, from ReLU masks that may flip on these wide-range inputs)."""
    for seed in range(6):
        params, x, phi, det, ref_o, ref_g, sim_o, sim_g = _bound_case(seed)
        e_o, e_g = mlp.error_bound(params, x, phi, det, 300.0)
        assert np.all(np.abs(sim_o - ref_o) <= e_o)
        for name, a, b, e in zip("W1 b1 W2 b2 W3 b3".split(), sim_g, ref_g, e_g):
            assert np.all(np.abs(a - b) <= e), (seed, name, np.max(np.abs(a - b) / e))
        for i, tight in ((0, 0.25), (2, 0.02), (4, 0.02)):
            big = np.abs(ref_g[i]) > 0.1 * np.abs(ref_g[i]).max()
            assert np.median(e_g[i][big] / np.abs(ref_g[i][big])) < tight, (seed, i)


def test_error_bound_needs_its_half_rounding_terms():
    """With the half unit roundoff understated 16-fold the bound no longer
    holds the kernel arithmetic: the half-rounding terms carry it."""
    failed = False
    for seed in range(6):
        params, x, phi, det, ref_o, ref_g, sim_o, sim_g = _bound_case(seed)
        e_o, e_g = mlp.error_bound(params, x, phi, det, 300.0, u=2.0 ** -15)
        failed |= bool(np.any(np.abs(sim_o - ref_o) > e_o))
        for a, b, e in zip(sim_g, ref_g, e_g):
            failed |= bool(np.any(np.abs(a - b) > e))
    assert failed


def test_error_bound_is_zero_for_exact_arithmetic():
    params, x, phi, det = _setup(seed=2, B=5)
    e_o, e_g = mlp.error_bound(params, x, phi, det, 300.0, u=0.0, ua=0.0, acc=0.0)
    assert np.all(e_o == 0) and all(np.all(e == 0) for e in e_g)
