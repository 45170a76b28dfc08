"""Pins of the oracle's comparison rules (per_los_error, incoherent_scale,
peak_agreement) against hand-built arrays of known answer.

Every GPU parity verdict passes through these three functions, so each is
checked here against values worked out by hand or fixed by the mathematics
(Parseval's theorem for incoherent_scale), with cases chosen so that a wrong
reduction axis, a dropped or inverted floor, a missing component, an inverted
ambiguity mask, a swapped result order or a lax acceptance band fails one of
them (tests/test_oracle_mutants.py plants each of these mistakes).
"""
import numpy as np
import pytest


# ---------------------------------------------------------------- per_los_error
def test_per_los_error_known_answer(oracle_mod):
    """e_l = max_k |F_gpu - F_ref| / max_k |F_ref|, one value per LOS (rows),
    with the complex modulus of the difference."""
    Fq_ref = np.array([[3.0, 0.0, 0.0],
                       [0.0, 1.0, 0.0],
                       [0.0, 0.0, 10.0]])
    Fu_ref = np.array([[4.0, 0.0, 0.0],     # max |F| = 5
                       [0.0, 0.0, 0.0],     # max |F| = 1
                       [0.0, 0.0, 0.0]])    # max |F| = 10
    dq = np.array([[0.0, 0.3, 0.0],
                   [0.0, 0.0, 0.0],
                   [0.5, 0.0, 0.0]])
    du = np.array([[0.0, 0.4, 0.0],         # |diff| 0.5 -> 0.5 / 5
                   [0.0, 0.0, 0.25],        # only Im differs: 0.25 / 1
                   [0.0, 0.0, 0.0]])        # 0.5 / 10
    e = oracle_mod.per_los_error(Fq_ref + dq, Fu_ref + du, Fq_ref, Fu_ref)
    assert e.shape == (3,)
    np.testing.assert_allclose(e, [0.1, 0.25, 0.05], rtol=1e-15)


def test_per_los_error_reduces_over_phi_not_los(oracle_mod):
    """A square case where the transposed reduction would give other values."""
    Fq_ref = np.diag([1.0, 2.0, 4.0])
    Fu_ref = np.zeros((3, 3))
    diff = np.zeros((3, 3))
    diff[0, 2] = 0.5          # LOS 0: 0.5 / 1; a column-wise reduction would see 0.5 / 4
    e = oracle_mod.per_los_error(Fq_ref + diff, Fu_ref, Fq_ref, Fu_ref)
    np.testing.assert_allclose(e, [0.5, 0.0, 0.0], rtol=1e-15)


def test_per_los_error_floor(oracle_mod):
    """The floor replaces max_k |F_ref| only where it is larger."""
    Fq_ref = np.array([[2.0, 0.0], [2.0, 0.0]])
    Fu_ref = np.zeros((2, 2))
    Fq = Fq_ref + np.array([[0.0, 0.2], [0.0, 0.2]])
    floor = np.array([4.0, 1.0])
    e = oracle_mod.per_los_error(Fq, Fu_ref, Fq_ref, Fu_ref, floor=floor)
    np.testing.assert_allclose(e, [0.2 / 4.0, 0.2 / 2.0], rtol=1e-15)
    e0 = oracle_mod.per_los_error(Fq, Fu_ref, Fq_ref, Fu_ref)
    np.testing.assert_allclose(e0, [0.1, 0.1], rtol=1e-15)


def test_per_los_error_zero_reference_row(oracle_mod):
    """A LOS whose oracle F is identically 0 reports the absolute difference."""
    z = np.zeros((2, 3))
    Fq = z.copy()
    Fq[1, 1] = 3e-7
    e = oracle_mod.per_los_error(Fq, z, z, z)
    np.testing.assert_allclose(e, [0.0, 3e-7], rtol=1e-15)


def test_per_los_error_nonfinite_gpu_value_is_not_hidden(oracle_mod):
    Fq_ref = np.ones((2, 3))
    Fu_ref = np.zeros((2, 3))
    Fq = Fq_ref.copy()
    Fq[1, 2] = np.nan
    e = oracle_mod.per_los_error(Fq, Fu_ref, Fq_ref, Fu_ref)
    assert e[0] == 0.0 and not np.isfinite(e[1])


# ------------------------------------------------------------- incoherent_scale
def test_incoherent_scale_known_answer(oracle_mod):
    """K sqrt(sum_j w_j^2 |P_j|^2), K = 1 / sum w, flagged channels out."""
    w = np.array([1.0, 2.0, 0.0, 1.0])
    Q = np.array([[1.0, 0.0, 7.0, 0.0],
                  [0.0, 0.0, np.nan, 0.0]])
    U = np.array([[0.0, 1.0, 7.0, 2.0],
                  [3.0, 0.0, np.inf, 0.0]])
    # LOS 0: w^2|P|^2 = 1*1 + 4*1 + 1*4 = 9 -> 3 / 4; LOS 1: 1*9 = 9 -> 3 / 4.
    s = oracle_mod.incoherent_scale(Q, U, w)
    np.testing.assert_allclose(s, [0.75, 0.75], rtol=1e-15)
    s1 = oracle_mod.incoherent_scale(Q.T.copy(), U.T.copy(), w, layout=1)
    np.testing.assert_allclose(s1, s, rtol=0)


def test_incoherent_scale_is_the_rms_of_F_over_a_full_period(oracle_mod):
    """Parseval: on the FFT grid phi_k = pi k / (N d) of a uniform lambda^2
    spacing d with unit weights, the mean over k of |F_k|^2 equals
    K^2 sum_j |P_j|^2 exactly, i.e. the square of the incoherent scale."""
    rng = np.random.default_rng(8)
    n, d = 24, 0.0011
    lam = 0.05 + d * np.arange(n)
    w = np.ones(n)
    phi = np.pi * np.arange(n) / (n * d)
    P = rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n))
    Fq, Fu = oracle_mod.fdf(P.real, P.imag, lam, w, phi)
    rms = np.sqrt(np.mean(Fq ** 2 + Fu ** 2, axis=1))
    np.testing.assert_allclose(oracle_mod.incoherent_scale(P.real, P.imag, w), rms, rtol=1e-12)


# --------------------------------------------------------------- peak_agreement
def _ref(oracle_mod, amps):
    amps = np.asarray(amps, np.float64)
    Fq, Fu = amps * 0.6, amps * 0.8     # |F| = amps
    return Fq, Fu, oracle_mod.peaks(Fq, Fu, np.arange(amps.shape[1], dtype=np.float64))


def test_peak_agreement_counts(oracle_mod):
    """Five unambiguous LOS with two wrong indices, three ambiguous LOS with
    one unacceptable index: (5, 2, 1) in that order."""
    amps = [[1.0, 5.0, 2.0],        # unambiguous, peak 1
            [3.0, 1.0, 2.0],        # unambiguous, peak 0
            [1.0, 2.0, 9.0],        # unambiguous, peak 2
            [4.0, 1.0, 1.0],        # unambiguous, peak 0
            [1.0, 1.0, 1.5],        # unambiguous, peak 2
            [2.0, 2.0, 1.0],        # tie: 0 or 1 acceptable
            [1.0, 7.0, 7.0],        # tie: 1 or 2 acceptable
            [3.0, 3.0, 0.5]]        # tie: 0 or 1 acceptable
    Fq, Fu, ref = _ref(oracle_mod, amps)
    gpu = np.array([1, 2, 2, 1, 2, 1, 2, 2])
    assert oracle_mod.peak_agreement(gpu, Fq, Fu, ref) == (5, 2, 1)
    assert oracle_mod.peak_agreement(ref["idx"], Fq, Fu, ref) == (5, 0, 0)


def test_peak_agreement_ambiguity_band(oracle_mod):
    """With margin_thr = 2e-5: a runner-up within 1e-5 makes the LOS
    ambiguous and is accepted; one 1e-4 below the top (which a band ten times
    wider would still accept) makes it unambiguous, and the second index is
    then a mismatch.  A margin of exactly the threshold counts as ambiguous
    (the third LOS's margin is set to it)."""
    amps = [[1.0, 1.0 - 1e-5, 0.1],
            [1.0, 1.0 - 1e-4, 0.1],
            [1.0, 1.0 - 1.5e-5, 0.1]]
    Fq, Fu, ref = _ref(oracle_mod, amps)
    ref["margin"][2] = 2e-5
    assert oracle_mod.peak_agreement(np.array([1, 1, 1]), Fq, Fu, ref) == (1, 1, 0)
    # The ambiguous rule itself: an index 3e-5 below the top is not acceptable.
    amps2 = [[1.0, 1.0 - 3e-5, 1.0 - 1e-6]]
    Fq2, Fu2, ref2 = _ref(oracle_mod, amps2)
    assert ref2["margin"][0] < 2e-5
    assert oracle_mod.peak_agreement(np.array([2]), Fq2, Fu2, ref2) == (0, 0, 0)
    assert oracle_mod.peak_agreement(np.array([1]), Fq2, Fu2, ref2) == (0, 0, 1)


def test_peak_agreement_out_of_range_index(oracle_mod):
    amps = [[1.0, 1.0, 0.5], [1.0, 1.0, 0.5]]
    Fq, Fu, ref = _ref(oracle_mod, amps)
    assert oracle_mod.peak_agreement(np.array([3, -1]), Fq, Fu, ref) == (0, 0, 2)


def test_peak_agreement_nonfinite_rows(oracle_mod):
    """The oracle flags a LOS with a non-finite |F| (idx -1): the GPU must flag
    it too, and must not flag a finite one."""
    Fq = np.array([[1.0, 2.0, 0.0], [1.0, np.nan, 0.0], [0.5, 3.0, 0.0]])
    Fu = np.zeros_like(Fq)
    ref = oracle_mod.peaks(Fq, Fu, np.arange(3.0))
    assert list(ref["idx"]) == [1, -1, 1]
    assert oracle_mod.peak_agreement(np.array([1, -1, 1]), Fq, Fu, ref) == (2, 0, 0)
    assert oracle_mod.peak_agreement(np.array([1, 0, 1]), Fq, Fu, ref) == (2, 0, 1)
    assert oracle_mod.peak_agreement(np.array([-1, -1, 1]), Fq, Fu, ref) == (2, 1, 0)


@pytest.mark.parametrize("thr", [1e-3, 2e-5])
def test_peak_agreement_threshold_argument_is_used(oracle_mod, thr):
    """The margin threshold is the caller's: a runner-up 1e-4 below the top is
    ambiguous at 1e-3 (second index accepted) and unambiguous at 2e-5."""
    Fq, Fu, ref = _ref(oracle_mod, [[1.0, 1.0 - 1e-4]])
    got = oracle_mod.peak_agreement(np.array([1]), Fq, Fu, ref, margin_thr=thr)
    assert got == ((0, 0, 0) if thr == 1e-3 else (1, 1, 0))
