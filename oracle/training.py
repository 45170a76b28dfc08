"""FP64 reference of the training-data synthesis for the gate network -- test
infrastructure only (nothing in the product path may import it).

Every line of sight g draws its content from Philox4x32-10 (Salmon, Moraes,
Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) with
key (seed mod 2^32, seed div 2^32) and counters

    (0,     g mod 2^32, g div 2^32, 0)   class draw
    (1 + c, g mod 2^32, g div 2^32, 0)   component c in {0, 1}: P0, phi0, chi0, W
    (m,     g mod 2^32, g div 2^32, 1)   noise of channels 2m and 2m + 1

A 32-bit output x becomes the uniform u = (floor(x / 2^9) + 1/2) 2^-23, exact
in FP32 (24 significant bits).  Classes: 0 noise only, 1 one Faraday-thin screen, 2 two screens,
3 one Burn slab, chosen by comparing u with the cumulative class fractions.
The sky model is that of Section 2.1 (eqs. (1), (3) and (4)):

    thin screen: P(lambda^2) = P0 exp(2i(chi0 + phi0 lambda^2))
    Burn slab:   P(lambda^2) = P0 exp(2i(chi0 + phic lambda^2)) sin(W lambda^2)/(W lambda^2)

with P0, phi0 (or phic), chi0 and W uniform over [p0_lo, p0_hi],
[phi_lo, phi_hi], [0, pi) and [w_lo, w_hi].  Noise: Box-Muller pairs
(r cos t, r sin t), r = sqrt(-2 ln u_a), t = 2 pi u_b, scaled by sigma, the
first pair for (Q, U) of channel 2m, the second for channel 2m + 1.  Q and U
are rounded to FP32 once at the end.

Labels come from the transform itself: the oracle's eq. (15) on the plan's
grid, its peak (smallest index on ties), phi_label = phi at the peak and
det_label = 1 iff the peak |F| >= det_threshold.
"""
from __future__ import annotations

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: [..., 4] integers < 2^32; key: two
    integers < 2^32.  Returns [..., 4] uint64 holding 32-bit words."""
    c = [np.asarray(ctr, dtype=np.uint64)[..., i] & MASK for i in range(4)]
    k0, k1 = np.uint64(key[0]) & MASK, np.uint64(key[1]) & MASK
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def uniform24(x):
    """32-bit word -> uniform in (0, 1) with 24 significant bits (exact in FP32)."""
    return ((np.asarray(x, dtype=np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def _key(seed):
    seed = int(seed) & (2 ** 64 - 1)
    return seed & 0xFFFFFFFF, seed >> 32


def _ctr(n, g, tag):
    g = np.asarray(g, dtype=np.uint64)
    n = np.broadcast_to(np.asarray(n, dtype=np.uint64), g.shape)
    return np.stack([n, g & MASK, g >> np.uint64(32), np.full(g.shape, tag, np.uint64)], axis=-1)


def classes(spec, seed, g):
    """Class of each line of sight g (array of global indices)."""
    u = uniform24(philox4x32_10(_ctr(0, g, 0), _key(seed))[..., 0])
    f0 = spec["frac_noise"]
    f1 = f0 + spec["frac_thin1"]
    f2 = f1 + spec["frac_thin2"]
    return np.where(u < f0, 0, np.where(u < f1, 1, np.where(u < f2, 2, 3))).astype(np.int32)


def components(spec, seed, g, c):
    """(P0, phi0, chi0, W) of component c for each line of sight g."""
    x = philox4x32_10(_ctr(1 + c, g, 0), _key(seed))
    u = uniform24(x)
    P0 = spec["p0_lo"] + (spec["p0_hi"] - spec["p0_lo"]) * u[..., 0]
    phi0 = spec["phi_lo"] + (spec["phi_hi"] - spec["phi_lo"]) * u[..., 1]
    chi0 = np.pi * u[..., 2]
    W = spec["w_lo"] + (spec["w_hi"] - spec["w_lo"]) * u[..., 3]
    return P0, phi0, chi0, W


def noise(seed, g, nchan):
    """Standard-normal (nQ, nU) [len(g)][nchan] by Box-Muller."""
    g = np.asarray(g, dtype=np.uint64)
    npair = (nchan + 1) // 2
    m = np.arange(npair, dtype=np.uint64)
    x = philox4x32_10(_ctr(m[None, :], np.broadcast_to(g[:, None], (g.size, npair)), 1), _key(seed))
    u = uniform24(x)
    ra, ta = np.sqrt(-2.0 * np.log(u[..., 0])), 2.0 * np.pi * u[..., 1]
    rb, tb = np.sqrt(-2.0 * np.log(u[..., 2])), 2.0 * np.pi * u[..., 3]
    nQ = np.empty((g.size, 2 * npair))
    nU = np.empty((g.size, 2 * npair))
    nQ[:, 0::2], nU[:, 0::2] = ra * np.cos(ta), ra * np.sin(ta)
    nQ[:, 1::2], nU[:, 1::2] = rb * np.cos(tb), rb * np.sin(tb)
    return nQ[:, :nchan], nU[:, :nchan]


def spectra(spec, seed, first_los, nlos, lambda2):
    """Q, U (FP32 values as float64 arrays [nlos][nchan]), class [nlos] and
    truth [nlos][4] = (phi0, P0) of components 0 and 1 (NaN where absent)."""
    lam = np.asarray(lambda2, dtype=np.float64)[None, :]
    g = np.arange(first_los, first_los + nlos, dtype=np.uint64)
    cls = classes(spec, seed, g)
    P = np.zeros((nlos, lam.size), dtype=np.complex128)
    truth = np.full((nlos, 4), np.nan)
    for c in (0, 1):
        P0, phi0, chi0, W = components(spec, seed, g, c)
        present = (cls >= 1) if c == 0 else (cls == 2)
        screen = P0[:, None] * np.exp(2j * (chi0[:, None] + phi0[:, None] * lam))
        slab = cls == 3
        x = W[:, None] * lam
        screen = np.where(slab[:, None], screen * (np.sin(x) / x), screen)
        P += np.where(present[:, None], screen, 0.0)
        truth[present, 2 * c] = phi0[present]
        truth[present, 2 * c + 1] = P0[present]
    nQ, nU = noise(seed, g, lam.size)
    Q = (P.real + spec["sigma"] * nQ).astype(np.float32).astype(np.float64)
    U = (P.imag + spec["sigma"] * nU).astype(np.float32).astype(np.float64)
    return Q, U, cls, truth


def labels(Q, U, lambda2, w, phi, det_threshold, fdf, peaks):
    """phi_label, det_label and the oracle peak record from the transform
    (`fdf`, `peaks`: the oracle's eq. (15) and peak search)."""
    Fq, Fu = fdf(Q, U, lambda2, w, phi)
    pk = peaks(Fq, Fu, phi)
    ok = pk["idx"] >= 0
    phi_label = np.where(ok, np.asarray(phi)[np.maximum(pk["idx"], 0)], 0.0)
    det = np.where(ok & (pk["amp"] >= det_threshold), 1.0, 0.0)
    return phi_label, det, pk, (Fq, Fu)
