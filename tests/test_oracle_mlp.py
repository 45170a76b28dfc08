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


def test_dz_scale_only_moves_the_half_rounding_point():
    """Without half rounding dz_scale has no effect; with it, a power-of-two
    scale leaves every rounding decision unchanged (half rounding commutes with
    exact scaling by 2^k in the normal range), so the gradients agree exactly."""
    params, x, phi, det = _setup(seed=3, B=8)
    o, cache = mlp.forward(params, x, round16=False)
    _, g = mlp.loss_and_grad_out(o, phi, det, 300.0)
    a = mlp.backward(params, cache, g, round16=False, dz_scale=1.0)
    b = mlp.backward(params, cache, g, round16=False, dz_scale=8.0)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    o, cache = mlp.forward(params, x, round16=True)
    _, g = mlp.loss_and_grad_out(o, phi, det, 300.0)
    c = mlp.backward(params, cache, g, round16=True, dz_scale=8.0)
    d = mlp.backward(params, cache, g, round16=True, dz_scale=16.0)
    for u, v in zip(c, d):
        np.testing.assert_array_equal(u, v)
    # ...and the rounded gradient stays within half precision of the exact one.
    for u, v in zip(c, a):
        assert np.linalg.norm(u - v) <= 5e-3 * np.linalg.norm(v) + 1e-12
