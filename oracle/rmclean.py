"""FP64 RM-CLEAN -- test infrastructure only (see oracle/__init__.py).

The paper names RM-CLEAN as the deconvolution that needs the RMSF (Section
2.2, on eq. (12)) and leaves it unsupported (its footnote there, and Section 4).
This is the plain Hogbom-style iteration that deconvolution refers to, on a
uniform phi grid phi_k = phi_0 + k dphi:

  r <- F (the dirty spectrum of eq. (11)); C <- 0
  repeat at most max_iter times:
      p = the lowest index maximising |r_k|
      stop if |r_p| < cutoff
      c = gain r_p;  C_p <- C_p + c
      r_k <- r_k - c R(phi_k - phi_p)   for every k      (R of eq. (12))
  restored_k = r_k + sum_m C_m G(phi_k - phi_m),
  G(x) = exp(-4 ln2 x^2 / fwhm^2)  (a Gaussian restoring beam of peak 1).

R(phi_k - phi_p) = R((k - p) dphi) is read from the RMSF on the doubled grid
m dphi, m = -(N-1) .. N-1 (N = number of phi).  Besides the results, every
decision the loop takes is recorded with its margin, so that a comparison in
another precision can tell unique decisions from near-ties.
"""
from __future__ import annotations

import numpy as np


def rmsf_doubled(rmsf_fn, lambda2, w, dphi, nphi, lambda0_sq=float("nan")):
    """R on m dphi, m = -(nphi-1) .. nphi-1, as complex128 [2 nphi - 1]."""
    m = np.arange(-(nphi - 1), nphi, dtype=np.float64)
    re, im = rmsf_fn(lambda2, w, m * dphi, lambda0_sq)
    return re + 1j * im


def restoring_beam(x, fwhm):
    return np.exp(-4.0 * np.log(2.0) * (np.asarray(x, np.float64) / fwhm) ** 2)


def rmclean(Fq, Fu, R2, dphi, gain, cutoff, max_iter, fwhm):
    """RM-CLEAN of each LOS (rows of Fq + i Fu, float64 [nlos][N]).

    Returns dict: resid (complex [nlos][N]), cc (complex [nlos][N]),
    restored (complex [nlos][N]), niter (int [nlos]), and per LOS the
    smallest relative margin of its decisions: pick_margin (|r|^2 of the
    chosen phi over the runner-up, minus 1; inf when N = 1) and stop_margin
    (| |r_p| / cutoff - 1 | of the last comparison with the cutoff)."""
    F = np.asarray(Fq, np.float64) + 1j * np.asarray(Fu, np.float64)
    nlos, N = F.shape
    R2 = np.asarray(R2, np.complex128)
    assert R2.size == 2 * N - 1
    resid = F.copy()
    cc = np.zeros_like(F)
    niter = np.zeros(nlos, np.int64)
    pick_margin = np.full(nlos, np.inf)
    stop_margin = np.full(nlos, np.inf)
    k = np.arange(N)
    for l in range(nlos):
        r = resid[l]
        for it in range(max_iter):
            a2 = r.real ** 2 + r.imag ** 2
            p = int(np.argmax(a2))
            if N > 1:
                second = np.max(np.delete(a2, p))
                if second > 0:
                    pick_margin[l] = min(pick_margin[l], a2[p] / second - 1.0)
            amp = np.sqrt(a2[p])
            if cutoff > 0:
                stop_margin[l] = min(stop_margin[l], abs(amp / cutoff - 1.0))
            if amp < cutoff:
                break
            c = gain * r[p]
            cc[l, p] += c
            r -= c * R2[(N - 1) + k - p]
            niter[l] = it + 1
    beam = restoring_beam(dphi * (k[:, None] - k[None, :]), fwhm)     # [N][N]
    restored = resid + cc @ beam.T
    return dict(resid=resid, cc=cc, restored=restored, niter=niter, pick_margin=pick_margin,
                stop_margin=stop_margin)
