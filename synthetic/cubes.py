"""Synthetic Q/U cubes shaped like the workloads RM synthesis is run on.

Sky model (forward direction only):
  * a Faraday-thin screen at depth phi0 with intrinsic angle chi0 and
    polarised amplitude P0 gives P(lambda^2) = P0 exp(2i(chi0 + phi0 lambda^2))
    (eqs. (1) and (3), Section 2.1);
  * a Burn slab, i.e. a flat Faraday dispersion function of integrated
    amplitude P0 over [phic - W/2, phic + W/2], gives through eq. (4)
    P(lambda^2) = P0 exp(2i(chi0 + phic lambda^2)) sin(W lambda^2)/(W lambda^2);
  * every (LOS, channel, Stokes) sample also carries iid N(0, sigma^2) noise.

Channel frequencies are an inclusive linear spacing of the band; the
wavelength is c / nu with c = 299 792 458 m/s.  Nothing here evaluates the
Faraday-depth transform: that is the job of the oracle and of the GPU path.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

C_LIGHT = 299_792_458.0  # m / s

LOS_MAJOR = 0   # Q[l][j]
FREQ_MAJOR = 1  # Q[j][l]


def band_lambda2(f_lo_mhz: float, f_hi_mhz: float, nchan: int) -> np.ndarray:
    """lambda^2 [m^2] of `nchan` channels spaced linearly from f_lo to f_hi
    (both inclusive), in channel order (lowest frequency first)."""
    nu = np.linspace(f_lo_mhz * 1e6, f_hi_mhz * 1e6, nchan, dtype=np.float64)
    return (C_LIGHT / nu) ** 2


def phi_grid(lo: float, hi: float, step: float) -> np.ndarray:
    """Uniform Faraday-depth grid lo, lo+step, ..., hi [rad m^-2]."""
    n = int(round((hi - lo) / step)) + 1
    return lo + step * np.arange(n, dtype=np.float64)


def flag_channels(nchan: int, nflag: int, rng: np.random.Generator) -> np.ndarray:
    """Weights of 1 with `nflag` channels, drawn without replacement, set to 0."""
    w = np.ones(nchan, dtype=np.float64)
    if nflag > 0:
        w[rng.choice(nchan, size=nflag, replace=False)] = 0.0
    return w


def thin_spectrum(lambda2, P0, phi0, chi0) -> np.ndarray:
    """Complex P(lambda^2) of Faraday-thin screens; parameters broadcast to
    shape [n, 1] against lambda2 [nchan]."""
    lam = np.asarray(lambda2, dtype=np.float64)[None, :]
    P0 = np.asarray(P0, dtype=np.float64).reshape(-1, 1)
    phi0 = np.asarray(phi0, dtype=np.float64).reshape(-1, 1)
    chi0 = np.asarray(chi0, dtype=np.float64).reshape(-1, 1)
    return P0 * np.exp(2j * (chi0 + phi0 * lam))


def slab_spectrum(lambda2, P0, phic, W, chi0) -> np.ndarray:
    """Complex P(lambda^2) of Burn slabs of width W centred on phic."""
    lam = np.asarray(lambda2, dtype=np.float64)[None, :]
    W = np.asarray(W, dtype=np.float64).reshape(-1, 1)
    x = W * lam
    return thin_spectrum(lambda2, P0, phic, chi0) * (np.sin(x) / x)


def noise_sigma_F(sigma: float, w: np.ndarray) -> float:
    """Per-component noise of the Faraday spectrum for iid per-channel noise
    sigma and weights w: sigma * sqrt(sum w^2) / sum w."""
    w = np.asarray(w, dtype=np.float64)
    return float(sigma * np.sqrt(np.sum(w * w)) / np.sum(w))


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    f_lo: float          # MHz
    f_hi: float          # MHz
    nchan: int
    nflag: int           # channels with weight 0
    phi_lo: float
    phi_hi: float
    phi_step: float
    sigma: float         # noise per (LOS, channel, Stokes)
    layout: int          # LOS_MAJOR or FREQ_MAJOR
    n_thin1: float       # LOS with one thin component (count if >= 1, else fraction)
    n_thin2: float       # LOS with two thin components
    n_slab: float        # LOS with a Burn slab
    P0: tuple = (0.01, 0.1)
    phi0: tuple = (-80.0, 80.0)
    slab_W: tuple = (1.0, 5.0)
    seed: int = 1000
    note: str = ""

    @property
    def nlos(self) -> int:
        return self.nx * self.ny

    def lambda2(self) -> np.ndarray:
        return band_lambda2(self.f_lo, self.f_hi, self.nchan)

    def weights(self) -> np.ndarray:
        return flag_channels(self.nchan, self.nflag, np.random.default_rng(self.seed + 7))

    def phi(self) -> np.ndarray:
        return phi_grid(self.phi_lo, self.phi_hi, self.phi_step)

    def samples(self, nlos: Optional[int] = None) -> int:
        n = self.nlos if nlos is None else nlos
        return n * self.nchan * len(self.phi())


WORKLOADS = {
    # 64x64 LOS, 128 channels 120-168 MHz, phi -100..100 step 1; 20 thin sources.
    "c1": Workload("c1", 64, 64, 120.0, 168.0, 128, 0, -100.0, 100.0, 1.0, 1e-3,
                   LOS_MAJOR, 20, 0, 0, phi0=(-80.0, 80.0), seed=1001,
                   note="plain RM synthesis, FP32 in / FP64 oracle"),
    # LOFAR-HBA-like: 512^2 LOS, 800 channels, 40 flagged, phi -500..500 step 1.
    "c2": Workload("c2", 512, 512, 120.0, 168.0, 800, 40, -500.0, 500.0, 1.0, 5e-4,
                   FREQ_MAJOR, 0.005, 0.005, 0.005, phi0=(-400.0, 400.0), slab_W=(1.0, 5.0),
                   seed=1002, note="LOFAR-HBA-like cube, frequency-major"),
    # Split-precision stress case: 1024^2 LOS, 400 channels 700-1800 MHz,
    # phi -2000..2000 step 2; source statistics of c1.
    "c3": Workload("c3", 1024, 1024, 700.0, 1800.0, 400, 0, -2000.0, 2000.0, 2.0, 1e-3,
                   LOS_MAJOR, 20 / 4096, 0, 0, phi0=(-80.0, 80.0), seed=1003,
                   note="split-precision MFMA path vs plain FP32"),
    # Large low-frequency cube: 2048^2 LOS, 1024 channels 110-190 MHz,
    # phi -1000..1000 step 0.5, frequency-major.
    "c4": Workload("c4", 2048, 2048, 110.0, 190.0, 1024, 0, -1000.0, 1000.0, 0.5, 1e-4,
                   FREQ_MAJOR, 0.002, 0, 0, phi0=(-800.0, 800.0), seed=1004,
                   note="large low-frequency cube, FP16 split vs FP32"),
    # Gating inference cube: 2048^2 LOS, 288 channels 800-1088 MHz, phi -300..300 step 0.5;
    # 1 % of LOS with 1-2 thin components, 0.5 % with a slab, peak SNR 3-50 against the
    # noise of F (sigma_F = 1e-3 / sqrt(288) for 288 unit-weight channels).
    "c5": Workload("c5", 2048, 2048, 800.0, 1088.0, 288, 0, -300.0, 300.0, 0.5, 1e-3,
                   LOS_MAJOR, 0.005, 0.005, 0.005,
                   P0=(3e-3 / np.sqrt(288.0), 50e-3 / np.sqrt(288.0)),
                   phi0=(-300.0, 300.0), slab_W=(10.0, 100.0),
                   seed=1005, note="learned gating inference cube"),
}


def _count(spec: float, nlos: int) -> int:
    if spec >= 1:
        return min(int(spec), nlos)
    return int(round(spec * nlos))


def _draw_sources(wl: Workload, nlos: int, lambda2: np.ndarray, rng: np.random.Generator):
    """Pick the LOS that carry sources and build their complex spectra."""
    n1, n2, ns = _count(wl.n_thin1, nlos), _count(wl.n_thin2, nlos), _count(wl.n_slab, nlos)
    ntot = min(n1 + n2 + ns, nlos)
    los = rng.choice(nlos, size=ntot, replace=False)
    kinds = np.array([1] * n1 + [2] * n2 + [3] * ns)[:ntot]
    spec = np.zeros((ntot, lambda2.size), dtype=np.complex128)
    params = []
    for i, kind in enumerate(kinds):
        ncomp = 1 if kind != 2 else 2
        comps = []
        for _ in range(ncomp):
            P0 = rng.uniform(*wl.P0)
            phi0 = rng.uniform(*wl.phi0)
            chi0 = rng.uniform(0.0, np.pi)
            if kind == 3:
                W = rng.uniform(*wl.slab_W)
                spec[i] += slab_spectrum(lambda2, P0, phi0, W, chi0)[0]
                comps.append(("slab", P0, phi0, chi0, W))
            else:
                spec[i] += thin_spectrum(lambda2, P0, phi0, chi0)[0]
                comps.append(("thin", P0, phi0, chi0, 0.0))
        params.append(comps)
    order = np.argsort(los)
    return los[order], kinds[order], spec[order], [params[i] for i in order]


def make_cube(wl: Workload, nlos: Optional[int] = None, device: str = "cpu",
              layout: Optional[int] = None, seed: Optional[int] = None):
    """Build the workload's Q/U cube as float32 torch tensors on `device`.

    Returns a dict with Q, U (layout LOS-major [nlos][nchan] or frequency-major
    [nchan][nlos]), lambda2, weights, phi (float64 numpy), and the injected
    sources (src_los, src_kind, src_params).  The noise is drawn by torch's
    generator on `device` (seeded), the source parameters by numpy (seeded).
    """
    import torch

    nlos = wl.nlos if nlos is None else int(nlos)
    layout = wl.layout if layout is None else layout
    seed = wl.seed if seed is None else seed
    rng = np.random.default_rng(seed)
    lambda2, weights, phi = wl.lambda2(), wl.weights(), wl.phi()
    src_los, src_kind, spec, params = _draw_sources(wl, nlos, lambda2, rng)

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Q = torch.randn((nlos, wl.nchan), generator=g, device=device, dtype=torch.float32)
    Q.mul_(wl.sigma)
    U = torch.randn((nlos, wl.nchan), generator=g, device=device, dtype=torch.float32)
    U.mul_(wl.sigma)
    if src_los.size:
        idx = torch.as_tensor(src_los, device=device, dtype=torch.long)
        sq = torch.as_tensor(spec.real, device=device)
        su = torch.as_tensor(spec.imag, device=device)
        Q[idx] = (Q[idx].double() + sq).float()
        U[idx] = (U[idx].double() + su).float()
    if layout == FREQ_MAJOR:
        Q = Q.t().contiguous()
        U = U.t().contiguous()
    return dict(Q=Q, U=U, lambda2=lambda2, weights=weights, phi=phi, layout=layout,
                nlos=nlos, src_los=src_los, src_kind=src_kind, src_params=params,
                sigma=wl.sigma, seed=seed)


def make_small_cube(nlos: int, nchan: int, nphi: int, seed: int, f_lo=120.0, f_hi=168.0,
                    phi_max=100.0, nflag=0, sigma=1e-3, nsrc=0):
    """Small float64 numpy cube for CPU tests: LOS-major Q, U [nlos][nchan]
    with `nsrc` thin sources, plus lambda2, weights and a uniform phi grid."""
    rng = np.random.default_rng(seed)
    lambda2 = band_lambda2(f_lo, f_hi, nchan)
    w = flag_channels(nchan, nflag, rng)
    phi = np.linspace(-phi_max, phi_max, nphi)
    P = sigma * (rng.standard_normal((nlos, nchan)) + 1j * rng.standard_normal((nlos, nchan)))
    if nsrc:
        los = rng.choice(nlos, size=min(nsrc, nlos), replace=False)
        P[los] += thin_spectrum(lambda2, rng.uniform(0.01, 0.1, los.size),
                                rng.uniform(-0.8 * phi_max, 0.8 * phi_max, los.size),
                                rng.uniform(0, np.pi, los.size))
    return dict(Q=P.real.copy(), U=P.imag.copy(), lambda2=lambda2, weights=w, phi=phi)


def stratified_subsample(nlos: int, src_los: np.ndarray, n: int, seed: int) -> np.ndarray:
    """Sorted LOS indices: up to n/2 source LOS and the rest noise LOS, drawn
    without replacement (seeded)."""
    rng = np.random.default_rng(seed)
    n = min(n, nlos)
    nsrc = min(n // 2, src_los.size)
    pick_src = rng.choice(src_los, size=nsrc, replace=False) if nsrc else np.zeros(0, np.int64)
    mask = np.ones(nlos, dtype=bool)
    mask[src_los] = False
    noise_los = np.flatnonzero(mask)
    pick_noise = rng.choice(noise_los, size=min(n - nsrc, noise_los.size), replace=False)
    return np.sort(np.concatenate([pick_src, pick_noise]).astype(np.int64))
