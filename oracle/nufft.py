"""FP64 NUFFT evaluation of eq. (11) on a uniform phi grid -- test
infrastructure only (see oracle/__init__.py).

The paper proposes an FFT in place of the direct sums of eqs. (15)-(16)
(Section 4).  With phi_k = phi_c + m dphi, m = k - floor(N/2), eq. (11) is a
type-1 non-uniform DFT in m:

  F_k = sum_j c_j exp(-i m x_j),   c_j = K w_j P_j exp(-2i a_j phi_c),
                                   x_j = 2 a_j dphi  (mod 2 pi),

evaluated here by its textbook steps (gridding with a kernel psi of width
`width` grid cells on n >= 2N uniform points over [0, 2 pi), an FFT, and
division by the kernel's Fourier transform):

  g_l  = sum_j c_j psi(x_l - x_j)          x_l = 2 pi l / n, distance taken
                                            periodically, psi(t) = 0 for
                                            |t| >= alpha = width pi / n
  G_m  = sum_l g_l exp(-i m x_l)           (numpy FFT)
  F_k  = (2 pi / n) G_m / psi_hat(m),      psi_hat(m) = int psi(t) e^{-imt} dt

psi(t) = exp(beta (sqrt(1 - (t/alpha)^2) - 1)), beta = 2.30 width (the
"exponential of semicircle" kernel of Barnett, Magland & af Klinteberg,
SIAM J. Sci. Comput. 2019), psi_hat by Gauss-Legendre quadrature.  The result
approximates eq. (11); its error falls by about a factor 7-10 per unit of
width (pinned against the direct sum in tests/test_oracle_nufft.py).
"""
from __future__ import annotations

import numpy as np


def kernel_params(width: int, n: int):
    alpha = width * np.pi / n
    return alpha, 2.30 * width


def psi(t, alpha, beta):
    z = np.asarray(t, np.float64) / alpha
    inside = np.abs(z) < 1.0
    return np.where(inside, np.exp(beta * (np.sqrt(np.clip(1.0 - z * z, 0.0, None)) - 1.0)), 0.0)


def psi_hat(m, alpha, beta, nodes=512):
    x, wq = np.polynomial.legendre.leggauss(nodes)
    t = alpha * x
    f = np.exp(beta * (np.sqrt(1.0 - x * x) - 1.0))
    return alpha * (np.cos(np.outer(np.asarray(m, np.float64), t)) @ (f * wq))


def grid_size(nphi: int) -> int:
    """Smallest power of two >= 2 nphi (and >= 16)."""
    n = 16
    while n < 2 * nphi:
        n *= 2
    return n


def fdf_nufft(Q, U, lambda2, w, phi, width=8, n=None):
    """F = Fq + i Fu [nlos][nphi] of LOS-major Q, U on the uniform grid phi."""
    Q, U = np.asarray(Q, np.float64), np.asarray(U, np.float64)
    lam, w, phi = (np.asarray(a, np.float64) for a in (lambda2, w, phi))
    N = phi.size
    if n is None:
        n = grid_size(N)
    K = 1.0 / w.sum()
    l0 = K * np.sum(w * lam)
    a = lam - l0
    kc = N // 2
    dphi = (phi[-1] - phi[0]) / (N - 1) if N > 1 else 0.0
    phic = phi[0] + kc * dphi
    keep = w > 0
    x = np.mod(2.0 * a * dphi, 2.0 * np.pi)
    c = (K * w * np.exp(-2j * a * phic))[None, :] * (Q + 1j * U)
    alpha, beta = kernel_params(width, n)
    xl = 2.0 * np.pi * np.arange(n) / n
    d = np.mod(xl[:, None] - x[None, :] + np.pi, 2.0 * np.pi) - np.pi     # periodic distance
    S = psi(d, alpha, beta)
    g = c[:, keep] @ S[:, keep].T
    G = np.fft.fft(g, axis=1)
    m = np.arange(N) - kc
    F = (2.0 * np.pi / n) * G[:, np.mod(m, n)] / psi_hat(m, alpha, beta)[None, :]
    return F.real.copy(), F.imag.copy()
