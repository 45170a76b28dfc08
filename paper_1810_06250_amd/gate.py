"""Training and threshold calibration of the gate network.

Host orchestration over the C ABI (include/rmsynth_mlp.h): the training data
come from rmsynth_synth_training (spectra by the library's generator, labels
by its own transform and peak search), every step is rmsynth_mlp_train_step,
and inference is rmsynth_mlp_infer.  The only host arithmetic is the
learning-rate schedule and the choice of the score threshold from held-out
scores.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .rmsynth import Mlp, Plan, TrainSpec, make_training_data


def band_spec(sigma: float, weights, snr=(3.0, 50.0), phi=(-300.0, 300.0), slab_w=(10.0, 100.0),
              fractions=(0.25, 0.30, 0.20), det_snr: float = 6.0) -> TrainSpec:
    """Training mix of noise-only / one screen / two screens / slab lines of
    sight with polarised amplitude SNR x sigma_F, where sigma_F =
    sigma sqrt(sum w^2) / sum w is the noise of one component of F; a line of
    sight is a detection when its peak |F| reaches det_snr x sigma_F."""
    w = np.asarray(weights, dtype=np.float64)
    sig_f = sigma * math.sqrt(float(np.sum(w * w))) / float(np.sum(w))
    return TrainSpec(frac_noise=fractions[0], frac_thin1=fractions[1], frac_thin2=fractions[2],
                     p0_lo=snr[0] * sig_f, p0_hi=snr[1] * sig_f, phi_lo=phi[0], phi_hi=phi[1],
                     w_lo=slab_w[0], w_hi=slab_w[1], sigma=sigma, det_threshold=det_snr * sig_f)


@dataclass
class TrainReport:
    steps: int = 0
    seconds: float = 0.0
    losses: list = field(default_factory=list)   # (step, mean loss over the logging window)


def train(plan: Plan, net: Mlp, spec: TrainSpec, seed: int, n_train: int, epochs: int = 4,
          batch: int = 1024, lr: float = 1e-3, lr_final: float = 1e-5, log_every: int = 200,
          log: Optional[Callable[[str], None]] = None) -> TrainReport:
    """Train on lines of sight 0 .. n_train-1 of stream `seed` (resident in
    device memory), with a cosine learning-rate decay from lr to lr_final."""
    import torch
    data = make_training_data(plan, spec, seed, 0, n_train, labels=True)
    nb = n_train // batch
    total = epochs * nb
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    acc = torch.zeros(1, dtype=torch.float32, device="cuda")
    rep = TrainReport()
    t0 = time.perf_counter()
    step = 0
    for _ in range(epochs):
        for b in range(nb):
            sl = slice(b * batch, (b + 1) * batch)
            cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / max(total, 1)))
            net.train_step(data["Q"][sl], data["U"][sl], data["phi_label"][sl],
                           data["det_label"][sl], cur, loss)
            acc += loss
            step += 1
            if step % log_every == 0 or step == total:
                k = log_every if step % log_every == 0 else step % log_every
                mean = float(acc.item()) / k
                acc.zero_()
                rep.losses.append((step, mean))
                if log:
                    log(f"step {step}/{total} loss {mean:.4f} lr {cur:.2e}")
    torch.cuda.synchronize()
    rep.steps = step
    rep.seconds = time.perf_counter() - t0
    del data
    return rep


@dataclass
class Calibration:
    tau: float
    recall: float            # on held-out detections at tau
    gated_fraction: float    # held-out lines of sight at or above tau
    n_detected: int
    phi_rmse: float          # |phi_hat - phi_label| rms over held-out detections


def calibrate(plan: Plan, net: Mlp, spec: TrainSpec, seed: int, first_los: int, n_val: int,
              target_recall: float = 0.995) -> Calibration:
    """Largest score threshold whose recall on held-out detections (lines of
    sight first_los .. first_los + n_val - 1, disjoint from training) is at
    least target_recall."""
    data = make_training_data(plan, spec, seed, first_los, n_val, labels=True)
    phi_hat, score = net.infer(data["Q"], data["U"])
    s = score.cpu().numpy().astype(np.float64)
    det = data["det_label"].cpu().numpy() > 0.5
    ph = phi_hat.cpu().numpy().astype(np.float64)
    pl = data["phi_label"].cpu().numpy().astype(np.float64)
    pos = np.sort(s[det])
    if pos.size == 0:
        return Calibration(tau=1.0, recall=1.0, gated_fraction=float(np.mean(s >= 1.0)),
                           n_detected=0, phi_rmse=float("nan"))
    k = int(math.floor((1.0 - target_recall) * pos.size))
    tau = float(pos[k])
    recall = float(np.mean(s[det] >= tau))
    return Calibration(tau=tau, recall=recall, gated_fraction=float(np.mean(s >= tau)),
                       n_detected=int(det.sum()),
                       phi_rmse=float(np.sqrt(np.mean((ph[det] - pl[det]) ** 2))))


def main(argv=None):
    import argparse

    from synthetic import WORKLOADS

    ap = argparse.ArgumentParser(description="train the gate network on one band")
    ap.add_argument("--out", required=True)
    ap.add_argument("--n-train", type=int, default=1_000_000)
    ap.add_argument("--n-val", type=int, default=100_000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=2024)
    a = ap.parse_args(argv)
    wl = WORKLOADS["c5"]
    plan = Plan(wl.lambda2(), wl.weights(), wl.phi())
    spec = band_spec(wl.sigma, wl.weights())
    net = Mlp(wl.nchan, 256, 256, weights=wl.weights(), phi_scale=300.0, seed=a.seed)
    rep = train(plan, net, spec, a.seed, a.n_train, a.epochs, a.batch, a.lr, log=print)
    cal = calibrate(plan, net, spec, a.seed, a.n_train, a.n_val)
    print(f"trained {rep.steps} steps in {rep.seconds:.1f} s; tau {cal.tau:.4g} recall {cal.recall:.4f} "
          f"gated {cal.gated_fraction:.4f} phi rmse {cal.phi_rmse:.2f}")
    net.save(a.out)


if __name__ == "__main__":
    main()
