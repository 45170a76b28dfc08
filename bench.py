#!/usr/bin/env python3
"""Throughput of the RM-synthesis hot path on one MI355X.

One step = rmsynth_execute_peaks over the whole synthetic cube already
resident in HBM: the Faraday-depth transform of eq. (11) (phase generation,
split-bfloat16 MFMA contraction, epilogue writing Fq, Fu) with the per-LOS
peak search fused into its epilogue, then the per-tile merge.  Default
workload: 1024 x 1024 LOS, 400 channels 700-1800 MHz, phi -2000..2000 step 2
(2001 values), LOS-major.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]
                    [--precision bf16x3|fp16x3|fp32] [--no-cpu-baseline]
                    [--no-fp32-compare] [--no-extra] [--no-gate] [--gate-train N]

Beside the headline the line carries: the plain FP32 path timed the same way;
the FP64 oracle on the host cores (cpu_baseline) and every GPU path's error
against it; the peaks-only search (F never stored), the adjoint transform and
RM-CLEAN on the same cube; the other workloads (c1, c2, c4) with their own
errors against the oracle; and the learned gate on the c5 cube, judged by an
oracle census of its detected lines of sight.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MFMA_PEAK_TFLOPS = {"bf16x3": 2516.6, "fp16x3": 2516.6, "fp32": 157.3}
MFMA_FLOP_PER_SAMPLE = {"bf16x3": 24.0, "fp16x3": 24.0, "fp32": 8.0}
HBM_PEAK_GBS = 8000.0
METRIC = "LOS·chan·φ Gsamples/s + % MFMA peak, split-BF16 vs FP32 at ≤1e-5 rel err"

# The paper's own measurements (Table 1), quoted as context with the hardware
# it names (NVIDIA Tesla P100-SXM2-16GB against one thread of a vectorised CPU
# code on an Intel Xeon E5-2690 v4): cube sizes (LOS, channels, phi) and the
# seconds of the CPU run and of the GPU's compute phase (its FITS reorder and
# the file I/O excluded).
PAPER_TABLE1 = {
    "WSRT-SINGS": {"los": 512 * 512, "chan": 803, "phi": 401, "cpu_s": 122.0, "gpu_compute_s": 8.0},
    "LOFAR_LR": {"los": 540 * 540, "chan": 856, "phi": 7000, "cpu_s": 2370.0, "gpu_compute_s": 17.0},
    "LOFAR_HR": {"los": 4000 * 4000, "chan": 856, "phi": 7000, "cpu_s": 208892.0,
                 "gpu_compute_s": 827.0},
}


def paper_context():
    out = {"source": "the paper's Table 1 (other hardware and cubes: context, not a target)",
           "gpu": "NVIDIA Tesla P100-SXM2-16GB", "cpu": "Intel Xeon E5-2690 v4, 1 thread, vectorised"}
    for name, r in PAPER_TABLE1.items():
        n = r["los"] * r["chan"] * r["phi"]
        out[name] = {"samples": n, "cpu_gsamples_s": n / r["cpu_s"] / 1e9,
                     "gpu_compute_gsamples_s": n / r["gpu_compute_s"] / 1e9,
                     "gpu_vs_cpu_compute": r["cpu_s"] / r["gpu_compute_s"]}
    return out


# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counter runs scaled by a plain 1 GiB copy (FETCH x 2.0, WRITE x 1.0),
# keyed by (workload, precision, sha256 prefix of the kernel sources they were
# taken on).  A changed kernel source reports null until counters are retaken.
KERNEL_SRC = [os.path.join(ROOT, "paper_1810_06250_amd", "csrc", f)
              for f in ("synth_factored.hip", "common.h")]
TRAFFIC = {
    ("c3", "bf16x3", "c091c886c2c0df0f"): 2.0 * 2395509.8 * 1024 + 1.0 * 17044737.2 * 1024,
}


def measured_traffic(workload, precision):
    import hashlib
    try:
        h = hashlib.sha256()
        for f in KERNEL_SRC:
            h.update(open(f, "rb").read())
        digest = h.hexdigest()[:16]
    except OSError:
        return None
    return TRAFFIC.get((workload, precision, digest))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "fp16x3", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-compare", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-gate", action="store_true",
                    help="skip the learned-gate leg (c5 band: train, calibrate, gated search)")
    ap.add_argument("--gate-train", type=int, default=1_000_000)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (c1, c2, c4), the peaks-only search, the "
                         "NUFFT, the adjoint transform, RM-CLEAN and the irregular-grid leg")
    ap.add_argument("--no-gemm-ref", action="store_true",
                    help="skip timing the vendor bf16 GEMM used as a practical MFMA reference")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB "
                         "(a known-size reference for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def gemm_reference(n=16384, reps=5):
    """Throughput of a plain bf16 GEMM from the vendor library (torch.matmul,
    n x n x n): what the matrix cores sustain on this board for the plainest
    dense contraction, as context for the split kernel's MFMA rate."""
    import torch
    a = torch.randn(n, n, device="cuda", dtype=torch.bfloat16)
    b = torch.randn(n, n, device="cuda", dtype=torch.bfloat16)
    for _ in range(2):
        c = a @ b
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c = a @ b
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b, c
    torch.cuda.empty_cache()
    return 2.0 * n ** 3 / (ms * 1e-3) / 1e12, ms


def time_path(rs, plan, cube, prec, Fq, Fu, pk, steps, warmup, fused=False):
    """Run warmup + timed steps; returns wall ms/step and per-call event ms.
    fused: one rmsynth_execute_peaks per step (peaks reduced in the transform
    kernels' epilogue; the second time is then 0); otherwise rmsynth_execute
    then rmsynth_peaks."""
    import torch
    layout = cube["layout"]
    nlos = cube["nlos"]
    ws, nb = None, 0
    if fused:
        nb = rs.rmsynth_execute_peaks_workspace_size(plan.handle, nlos, layout, prec)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
    elif prec == rs.RMSYNTH_SPLIT_FP16:
        nb = rs.rmsynth_workspace_size(plan.handle, nlos, layout, prec)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")

    def first():
        if fused:
            rs.rmsynth_execute_peaks(plan.handle, cube["Q"], cube["U"], nlos, layout, prec, Fq, Fu,
                                     None, pk["idx"], pk["phi_pk"], pk["amp"], pk["q_pk"],
                                     pk["u_pk"], ws, nb)
        else:
            rs.rmsynth_execute(plan.handle, cube["Q"], cube["U"], nlos, layout, prec, Fq, Fu,
                               None, ws, nb)

    def second():
        if not fused:
            rs.rmsynth_peaks(plan.handle, Fq, Fu, nlos, pk["idx"], pk["phi_pk"], pk["amp"],
                             pk["q_pk"], pk["u_pk"])

    for _ in range(warmup):
        first()
        second()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record()
        first()
        e1.record()
        second()
        e2.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ex = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    pkms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    return wall, ex, pkms


def plan_uniform(phi):
    """The library takes the factored (fused-peaks) kernels on uniform grids."""
    phi = np.asarray(phi, dtype=np.float64)
    if phi.size < 2:
        return True
    d = (phi[-1] - phi[0]) / (phi.size - 1)
    scale = max(abs(phi[0]), abs(phi[-1]), abs(d))
    return bool(np.all(np.abs(phi - (phi[0] + d * np.arange(phi.size))) <= 1e-9 * scale))


def cpu_baseline_leg(cube, sub, gpu_out, seconds):
    """Time the FP64 oracle on host cores over a bounded sample of the same
    workload, and report the error of each GPU path on the stratified subsample."""
    import oracle
    import torch
    oracle.build(force=False)
    lam, w, phi = cube["lambda2"], cube["weights"], cube["phi"]
    subt = torch.as_tensor(sub, device="cuda")

    def rows(idx_t):
        if cube["layout"] == 0:
            q, u = cube["Q"][idx_t], cube["U"][idx_t]
        else:
            q, u = cube["Q"][:, idx_t].t(), cube["U"][:, idx_t].t()
        return q.double().cpu().numpy(), u.double().cpu().numpy()

    Q64, U64 = rows(subt)
    t0 = time.perf_counter()
    rq, ru = oracle.fdf(Q64, U64, lam, w, phi, layout=0)
    done_los = len(sub)
    elapsed = time.perf_counter() - t0
    # keep going on further chunks of the cube until the time budget is used
    chunk = len(sub)
    start = 0
    while elapsed < seconds and start + chunk <= cube["nlos"]:
        q, u = rows(torch.arange(start, start + chunk, device="cuda"))
        t1 = time.perf_counter()
        oracle.fdf(q, u, lam, w, phi, layout=0)
        elapsed += time.perf_counter() - t1
        done_los += chunk
        start += chunk
    samples = done_los * len(lam) * len(phi)
    ref = oracle.peaks(rq, ru, phi)
    errors = {}
    for name, (Fq, Fu, idx) in gpu_out.items():
        gq, gu = Fq[subt].cpu().numpy(), Fu[subt].cpu().numpy()
        e = oracle.per_los_error(gq, gu, rq, ru)
        nun, mism, bad = oracle.peak_agreement(idx[subt].cpu().numpy(), rq, ru, ref)
        errors[name] = {"max_per_los_rel_err": float(e.max()), "median_per_los_rel_err": float(np.median(e)),
                        "peaks_unambiguous": nun, "peak_mismatches": mism, "ambiguous_invalid": bad,
                        "subsample_los": int(len(sub))}
    return ({"value": samples / elapsed / 1e9, "unit": "Gsamples/s", "cores": oracle.threads(),
             "kind": "oracle",
             "sample": f"{done_los} LOS x {len(lam)} channels x {len(phi)} phi "
                       f"(stratified 2048 source + 2048 noise LOS, then contiguous chunks), "
                       f"FP64 table-mode C triple loop, {elapsed:.1f} s"}, errors)


def _timed(fn, steps, warmup):
    """Wall ms per call (K calls between two synchronisations) and the mean
    HIP-event ms per call on torch's current stream (the library's stream)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, float(np.mean([a.elapsed_time(b) for a, b in ev]))


def _search_outputs(nlos, device="cuda"):
    import torch
    out = {"idx": torch.empty(nlos, dtype=torch.int32, device=device)}
    for k in ("phi_pk", "amp", "q_pk", "u_pk", "phi_fit", "amp_fit"):
        out[k] = torch.empty(nlos, dtype=torch.float32, device=device)
    return out


def search_leg(rs, plan, cube, prec, steps, warmup, ref_pk=None):
    """The peaks-only search (rmsynth_search: transform, peaks and sub-grid
    peak, F never stored) over the whole cube."""
    import torch
    nlos, layout = cube["nlos"], cube["layout"]
    nchan, nphi = len(cube["lambda2"]), len(cube["phi"])
    out = _search_outputs(nlos)
    nb = rs.rmsynth_search_workspace_size(plan.handle, nlos, layout, prec)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")

    def run():
        rs.rmsynth_search(plan.handle, cube["Q"], cube["U"], nlos, layout, prec, out["idx"],
                          out["phi_pk"], out["amp"], out["q_pk"], out["u_pk"], out["phi_fit"],
                          out["amp_fit"], ws, nb)

    wall, ev = _timed(run, steps, warmup)
    samples = nlos * nchan * nphi
    res = {"call": "rmsynth_search (transform + peaks + sub-grid peak; F not stored)",
           "ms_per_step": wall, "event_ms": ev, "gsamples_s": samples / (wall * 1e-3) / 1e9,
           "workspace_bytes": nb}
    if prec != rs.RMSYNTH_FP32:
        res["frac_of_mfma_peak"] = 24.0 * samples / (ev * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["bf16x3"]
    if ref_pk is not None:
        res["identical_to_execute_peaks"] = bool(all(torch.equal(out[k], ref_pk[k])
                                                     for k in ("idx", "amp", "q_pk", "u_pk")))
    del ws
    return res, out


def oracle_errors(cube, sub, paths):
    """Per-LOS error and peak agreement of GPU outputs on a subsample, against
    the FP64 oracle on the exact FP32 inputs."""
    import oracle
    import torch
    oracle.build(force=False)
    lam, w, phi = cube["lambda2"], cube["weights"], cube["phi"]
    subt = torch.as_tensor(sub, device="cuda")
    if cube["layout"] == 0:
        q, u = cube["Q"][subt], cube["U"][subt]
    else:
        q, u = cube["Q"][:, subt].t(), cube["U"][:, subt].t()
    rq, ru = oracle.fdf(q.double().cpu().numpy(), u.double().cpu().numpy(), lam, w, phi)
    ref = oracle.peaks(rq, ru, phi)
    out = {}
    for name, (Fq, Fu, idx) in paths.items():
        e = oracle.per_los_error(Fq[subt].cpu().numpy(), Fu[subt].cpu().numpy(), rq, ru)
        nun, mism, bad = oracle.peak_agreement(idx[subt].cpu().numpy(), rq, ru, ref)
        out[name] = {"max_per_los_rel_err": float(e.max()), "median_per_los_rel_err": float(np.median(e)),
                     "peaks_unambiguous": nun, "peak_mismatches": mism, "ambiguous_invalid": bad}
    return out, (rq, ru, ref)


def config_leg(rs, name, precs, steps, nsub):
    """One more workload: every path in precs timed as one step (transform +
    peaks, fused where the library fuses them; the split paths also as the
    peaks-only search), errors against the oracle on a stratified subsample."""
    import torch
    from synthetic import WORKLOADS, make_cube, stratified_subsample
    wl = WORKLOADS[name]
    log(f"{name}: generating {wl.nlos} LOS x {wl.nchan} ch x {len(wl.phi())} phi")
    cube = make_cube(wl, device="cuda")
    plan = rs.Plan(cube["lambda2"], cube["weights"], cube["phi"])
    nlos, nchan, nphi = cube["nlos"], len(cube["lambda2"]), len(cube["phi"])
    samples = nlos * nchan * nphi
    Fq = torch.empty((nlos, nphi), dtype=torch.float32, device="cuda")
    Fu = torch.empty_like(Fq)
    sub = stratified_subsample(nlos, cube["src_los"], nsub, seed=wl.seed + 11)
    res = {"workload": f"{name}: {wl.nx}x{wl.ny} LOS, {nchan} channels {wl.f_lo:g}-{wl.f_hi:g} MHz, "
                       f"phi {wl.phi_lo:g}..{wl.phi_hi:g} step {wl.phi_step:g} ({nphi}), "
                       f"{'LOS-major' if cube['layout'] == 0 else 'frequency-major'}",
           "samples": samples, "paths": {}}
    for prec_name in precs:
        prec = rs.PRECISIONS[prec_name]
        pk = dict(idx=torch.empty(nlos, dtype=torch.int32, device="cuda"),
                  phi_pk=torch.empty(nlos, device="cuda"), amp=torch.empty(nlos, device="cuda"),
                  q_pk=torch.empty(nlos, device="cuda"), u_pk=torch.empty(nlos, device="cuda"))
        fused = prec_name != "fp32" and plan_uniform(cube["phi"])
        n = steps if prec_name != "fp32" else max(2, steps // 3)
        # Short launches: enough untimed ones for the clock to settle after
        # the host-side work before this leg.
        warm = 5 if samples < 10 ** 12 else 1
        log(f"{name}: {prec_name}, {warm} warmup + {n} steps")
        wall, ex, pkms = time_path(rs, plan, cube, prec, Fq, Fu, pk, n, warm, fused=fused)
        flop = MFMA_FLOP_PER_SAMPLE[prec_name] * samples
        r = {"step": "rmsynth_execute_peaks" if fused else "rmsynth_execute + rmsynth_peaks",
             "ms_per_step": wall, "us_per_step": wall * 1e3, "gsamples_s": samples / (wall * 1e-3) / 1e9,
             "transform_ms": ex, "frac_of_peak": flop / (ex * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[prec_name]}
        errs, _ = oracle_errors(cube, sub, {prec_name: (Fq, Fu, pk["idx"])})
        r["errors_vs_oracle"] = errs[prec_name]
        r["errors_vs_oracle"]["subsample_los"] = int(len(sub))
        if prec_name != "fp32" and fused:
            sres, sout = search_leg(rs, plan, cube, prec, max(2, n // 2), warm, ref_pk=pk)
            r["peaks_only_search"] = sres
            del sout
        res["paths"][prec_name] = r
        del pk
        torch.cuda.empty_cache()
    if "fp32" in res["paths"]:
        for p_ in res["paths"]:
            if p_ != "fp32":
                res["paths"][p_]["speedup_vs_fp32_step"] = (res["paths"]["fp32"]["ms_per_step"] /
                                                             res["paths"][p_]["ms_per_step"])
    plan.close()
    del Fq, Fu, cube
    torch.cuda.empty_cache()
    return res


def adjoint_leg(rs, plan, Fq, Fu, lam, phi, steps):
    """Spectrum synthesis (rmsynth_adjoint) of the whole c3 grid of components
    (the main step's F used as C), timed per precision, with the error
    against the FP64 oracle on 256 LOS."""
    import torch
    import oracle
    nlos, nphi = Fq.shape
    nchan = len(lam)
    Pq = torch.empty((nlos, nchan), dtype=torch.float32, device="cuda")
    Pu = torch.empty_like(Pq)
    info = plan.info
    res = {"call": "rmsynth_adjoint: P_lj = sum_k C_lk exp(+2i phi_k (lambda_j^2 - lambda0^2))",
           "shape": f"{nlos} LOS x {nphi} phi -> {nchan} channels", "samples": nlos * nphi * nchan}
    sel = np.linspace(0, nlos - 1, 256).astype(np.int64)
    selt = torch.as_tensor(sel, device="cuda")
    cq, cu = Fq[selt].cpu().numpy(), Fu[selt].cpu().numpy()
    for prec_name in ("bf16x3", "fp32"):
        prec = rs.PRECISIONS[prec_name]

        def run():
            rs.rmsynth_adjoint(plan.handle, Fq, Fu, nlos, prec, Pq, Pu)

        wall, ev = _timed(run, steps, 1)
        rq, ru = oracle.adjoint(cq, cu, lam, np.ones(nchan), phi, lambda0_sq=info["lambda0_sq"])
        e = oracle.per_los_error(Pq[selt].cpu().numpy(), Pu[selt].cpu().numpy(), rq, ru)
        flop = MFMA_FLOP_PER_SAMPLE[prec_name] * nlos * nphi * nchan
        res[prec_name] = {"ms": wall, "event_ms": ev, "gsamples_s": nlos * nphi * nchan / (ev * 1e-3) / 1e9,
                          "frac_of_peak": flop / (ev * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[prec_name],
                          "max_per_los_rel_err_256": float(e.max())}
    del Pq, Pu
    torch.cuda.empty_cache()
    return res


def nufft_leg(rs, plan, cube, sub, steps):
    """F of the whole cube by the non-uniform FFT (rmsynth_execute_nufft),
    timed, with its error against the FP64 direct sum on the stratified
    subsample (LOS-major cubes only)."""
    import torch
    nlos, nphi = cube["nlos"], len(cube["phi"])
    samples = nlos * len(cube["lambda2"]) * nphi
    Fq = torch.empty((nlos, nphi), dtype=torch.float32, device="cuda")
    Fu = torch.empty_like(Fq)

    def run():
        rs.rmsynth_execute_nufft(plan.handle, cube["Q"], cube["U"], nlos, Fq, Fu)

    wall, ev = _timed(run, steps, 1)
    pk = plan.peaks(Fq, Fu)
    errs, _ = oracle_errors(cube, sub, {"nufft": (Fq, Fu, pk["idx"])})
    res = {"call": "rmsynth_execute_nufft (gridding, 8-cell kernel, 2x power-of-two grid, FFT in LDS, "
                   "deconvolution; F stored)",
           "ms": wall, "event_ms": ev, "gsamples_s": samples / (ev * 1e-3) / 1e9,
           "equivalent_dense_tflops_24": 24.0 * samples / (ev * 1e-3) / 1e12,
           "errors_vs_oracle": errs["nufft"]}
    del Fq, Fu, pk
    torch.cuda.empty_cache()
    return res


def nonuniform_leg(rs, cube, sub, steps):
    """The same cube on an irregular phi grid (each phi of the workload moved by
    up to +-0.2 of its step, seeded): the split precisions then read the
    plan's phase table (with the fused peaks: one rmsynth_execute_peaks per
    step), FP32 generates the phases per element (rmsynth_execute +
    rmsynth_peaks).  Errors against the FP64 oracle on the stratified
    subsample."""
    import torch
    phi = np.asarray(cube["phi"], dtype=np.float64)
    step = float(phi[1] - phi[0])
    rng = np.random.default_rng(1810)
    phi2 = phi + rng.uniform(-0.2 * step, 0.2 * step, phi.size)
    cube2 = dict(cube, phi=phi2)
    plan = rs.Plan(cube["lambda2"], cube["weights"], phi2)
    nlos, nphi = cube["nlos"], phi2.size
    samples = nlos * len(cube["lambda2"]) * nphi
    Fq = torch.empty((nlos, nphi), dtype=torch.float32, device="cuda")
    Fu = torch.empty_like(Fq)
    res = {"phi_grid": f"the workload's grid, each phi moved by U(-0.2, 0.2) x {step:g} (seed 1810)",
           "paths": {}}
    for prec_name in ("bf16x3", "fp16x3", "fp32"):
        prec = rs.PRECISIONS[prec_name]
        pk = dict(idx=torch.empty(nlos, dtype=torch.int32, device="cuda"),
                  phi_pk=torch.empty(nlos, device="cuda"), amp=torch.empty(nlos, device="cuda"),
                  q_pk=torch.empty(nlos, device="cuda"), u_pk=torch.empty(nlos, device="cuda"))
        n = steps if prec_name != "fp32" else max(2, steps // 2)
        log(f"non-uniform grid: {prec_name}, {n} steps")
        fused = prec_name != "fp32"
        wall, ex, pkms = time_path(rs, plan, cube, prec, Fq, Fu, pk, n, 1, fused=fused)
        flop = MFMA_FLOP_PER_SAMPLE[prec_name] * samples
        errs, _ = oracle_errors(cube2, sub, {prec_name: (Fq, Fu, pk["idx"])})
        res["paths"][prec_name] = {
            "step": "rmsynth_execute_peaks" if fused else "rmsynth_execute + rmsynth_peaks",
            "ms_per_step": wall, "transform_ms": ex,
            "peaks_ms": pkms, "gsamples_s": samples / (wall * 1e-3) / 1e9,
            "frac_of_peak": flop / (ex * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[prec_name],
            "errors_vs_oracle": errs[prec_name]}
        del pk
    for p_ in ("bf16x3", "fp16x3"):
        res["paths"][p_]["speedup_vs_fp32_step"] = (res["paths"]["fp32"]["ms_per_step"] /
                                                     res["paths"][p_]["ms_per_step"])
    plan.close()
    del Fq, Fu
    torch.cuda.empty_cache()
    return res


def rmclean_leg(rs, plan, Fq, Fu, lam, w, phi, sigma_f, src_los, steps):
    """RM-CLEAN (rmsynth_rmclean) of every LOS of the c3 spectrum (gain 0.1,
    cutoff 5 sigma_F, at most 1000 iterations), timed, and compared with the
    FP64 oracle's iteration on 48 source LOS."""
    import torch
    import oracle
    from oracle import rmclean as orc
    nlos, N = Fq.shape
    cutoff = 5.0 * sigma_f
    o = {k: torch.empty_like(Fq) for k in ("rq", "ru", "cq", "cu", "Rq", "Ru")}
    niter = torch.empty(nlos, dtype=torch.int32, device="cuda")
    nb = rs.rmsynth_rmclean_workspace_size(plan.handle)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")

    def run():
        rs.rmsynth_rmclean(plan.handle, Fq, Fu, nlos, 0.1, cutoff, 1000, float("nan"), o["rq"], o["ru"],
                           o["cq"], o["cu"], o["Rq"], o["Ru"], niter, ws, nb)

    wall, ev = _timed(run, steps, 1)
    it = niter.cpu().numpy()
    sel = np.sort(np.random.default_rng(7).choice(src_los, size=min(48, len(src_los)), replace=False))
    selt = torch.as_tensor(sel, device="cuda")
    dphi = (phi[-1] - phi[0]) / (N - 1)
    R2 = orc.rmsf_doubled(oracle.rmsf, lam, w, dphi, N)
    fwhm = plan.info["fwhm_est"]
    ref = orc.rmclean(Fq[selt].double().cpu().numpy(), Fu[selt].double().cpu().numpy(), R2, dphi,
                      0.1, cutoff, 1000, fwhm)
    clear = (ref["pick_margin"] > 1e-4) & (ref["stop_margin"] > 1e-4)
    g_it = it[sel]
    scale = np.hypot(Fq[selt].cpu().numpy(), Fu[selt].cpu().numpy()).max(axis=1)
    d = np.abs(o["Rq"][selt].cpu().numpy() + 1j * o["Ru"][selt].cpu().numpy() - ref["restored"]).max(axis=1)
    res = {"call": "rmsynth_rmclean (Hogbom, gain 0.1, cutoff 5 sigma_F, max 1000 iterations, "
                   "restored with a Gaussian beam of the plan's FWHM)",
           "los": nlos, "nphi": N, "ms": wall, "event_ms": ev,
           "los_cleaned": int(np.sum(it > 0)), "iterations_total": int(it[it > 0].sum()),
           "iterations_max": int(it.max()),
           "ns_per_los_iteration_phi": ev * 1e6 / max(1, int(it[it > 0].sum()) * N),
           "oracle_check": {"los": int(len(sel)), "clear_decisions": int(clear.sum()),
                            "niter_equal_on_clear": bool(np.all(g_it[clear] == ref["niter"][clear])),
                            "max_restored_err_rel": float(np.max((d / scale)[clear])) if clear.any() else None}}
    del o, ws
    torch.cuda.empty_cache()
    return res


def _event_ms(fn, reps=3):
    """Best of `reps` runs of fn() between HIP events on torch's stream (after one warm run)."""
    import torch
    out = fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        out = fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return out, best


def gate_leg(rs, n_train):
    """Learned gate on the c5 band: train the network on n_train lines of sight
    the library synthesises and labels, calibrate the score threshold for
    99.5 % recall on 100 000 held-out lines of sight, then run the gated peak
    search on the 2048 x 2048 c5 cube and compare it with the ungated search
    (FP32 transform then peaks; fused split-bf16 transform and peaks), with a non-learned gate (FP32 transform
    on a coarse grid of step FWHM/4, threshold 0.8 x the detection level, then
    the fine transform on the survivors) and, on detected lines of sight, with
    the FP64 oracle."""
    import torch
    import oracle
    from paper_1810_06250_amd import gate
    from synthetic import WORKLOADS, make_cube
    wl = WORKLOADS["c5"]
    lam, w, phi = wl.lambda2(), wl.weights(), wl.phi()
    plan = rs.Plan(lam, w, phi)
    spec = gate.band_spec(wl.sigma, w)
    net = rs.Mlp(wl.nchan, 256, 256, weights=w, phi_scale=300.0, seed=2024)
    log(f"gate: training on {n_train} LOS")
    t0 = time.perf_counter()
    rep = gate.train(plan, net, spec, seed=2024, n_train=n_train, epochs=4, batch=1024, lr=1e-3)
    train_s = time.perf_counter() - t0
    cal = gate.calibrate(plan, net, spec, seed=2024, first_los=n_train, n_val=100_000,
                         target_recall=0.995)
    log(f"gate: tau {cal.tau:.4g}, held-out recall {cal.recall:.4f}")
    cube = make_cube(wl, device="cuda")
    Q, U = cube["Q"], cube["U"]
    nlos = cube["nlos"]

    def ungated(prec):
        Fq, Fu, _ = plan.execute(Q, U, rs.RMSYNTH_LOS_MAJOR, prec)
        return plan.peaks(Fq, Fu)

    full, t32 = _event_ms(lambda: ungated(rs.RMSYNTH_FP32))
    # The split-bf16 comparison uses the fused transform + peak search.
    _, tbf = _event_ms(lambda: plan.execute_peaks(Q, U, rs.RMSYNTH_LOS_MAJOR,
                                                  rs.RMSYNTH_SPLIT_BF16)[3])
    torch.cuda.empty_cache()
    g, tg = _event_ms(lambda: net.gate(plan, Q, U, cal.tau))
    gs, tgs = _event_ms(lambda: net.gate(plan, Q, U, cal.tau, precision=rs.RMSYNTH_SPLIT_BF16))
    _, tinf = _event_ms(lambda: net.infer(Q, U))
    thr = spec.det_threshold
    step_c = plan.info["fwhm_est"] / 4.0
    planc = rs.Plan(lam, w, np.arange(phi[0], phi[-1] + 1e-9, step_c))

    def coarse():
        Fq, Fu, _ = planc.execute(Q, U, rs.RMSYNTH_LOS_MAJOR, rs.RMSYNTH_FP32)
        pk = planc.peaks(Fq, Fu)
        sel = torch.nonzero(pk["amp"] >= 0.8 * thr).squeeze(1)
        Fq2, Fu2, _ = plan.execute(Q.index_select(0, sel).contiguous(),
                                   U.index_select(0, sel).contiguous())
        return sel, plan.peaks(Fq2, Fu2)

    (csel, cpk), tc = _event_ms(coarse)

    # The same non-learned gate with its fastest coarse stage: the fused
    # split-bf16 peaks-only search on the coarse grid (no F stored).
    cws_n = rs.rmsynth_search_workspace_size(planc.handle, nlos, rs.RMSYNTH_LOS_MAJOR,
                                             rs.RMSYNTH_SPLIT_BF16)
    cws = torch.empty(cws_n, dtype=torch.uint8, device="cuda")
    cout = _search_outputs(nlos)

    def coarse_best():
        rs.rmsynth_search(planc.handle, Q, U, nlos, rs.RMSYNTH_LOS_MAJOR, rs.RMSYNTH_SPLIT_BF16,
                          cout["idx"], None, cout["amp"], None, None, None, None, cws, cws_n)
        sel = torch.nonzero(cout["amp"] >= 0.8 * thr).squeeze(1)
        Fq2, Fu2, _ = plan.execute(Q.index_select(0, sel).contiguous(),
                                   U.index_select(0, sel).contiguous())
        return sel, plan.peaks(Fq2, Fu2)

    (bsel, bpk), tcb = _event_ms(coarse_best)
    del cws, cout
    idx = full["idx"].cpu().numpy()
    amp = full["amp"].cpu().numpy()
    det = amp >= thr
    gidx = g["idx"].cpu().numpy()
    gsidx = gs["idx"].cpu().numpy()
    gated = g["gated"].cpu().numpy().astype(bool)
    csel = csel.cpu().numpy()
    cidx = np.full(nlos, -1, np.int64)
    cidx[csel] = cpk["idx"].cpu().numpy()
    bsel = bsel.cpu().numpy()
    bidx = np.full(nlos, -1, np.int64)
    bidx[bsel] = bpk["idx"].cpu().numpy()

    # Census by the FP64 oracle: every injected LOS, every LOS the ungated GPU
    # search detects and 4096 random LOS.  "Detected" is the oracle's peak
    # |F| reaching the threshold; a gate matches on such a LOS when its index
    # passes the oracle's peak rule (exact where the peak is unambiguous).
    rng = np.random.default_rng(wl.seed + 5)
    census = np.union1d(np.union1d(cube["src_los"], np.flatnonzero(det)),
                        rng.choice(nlos, size=4096, replace=False))
    log(f"gate: oracle census on {census.size} LOS")
    oracle.build(force=False)
    t_or = time.perf_counter()
    ct = torch.as_tensor(census, device="cuda")
    rq, ru = oracle.fdf(Q[ct].double().cpu().numpy(), U[ct].double().cpu().numpy(), lam, w, phi)
    ref = oracle.peaks(rq, ru, phi)
    t_or = time.perf_counter() - t_or
    odet = ref["amp"] >= thr

    def match_rate(ix):
        rows = np.flatnonzero(odet)
        sub = {k: v[rows] for k, v in ref.items()}
        n_u, mism, bad = oracle.peak_agreement(ix[census][rows], rq[rows], ru[rows], sub)
        return float(1.0 - (mism + bad) / max(1, rows.size)), int(rows.size)

    m_gate, n_odet = match_rate(gidx)
    m_gate_s, _ = match_rate(gsidx)
    m_full, _ = match_rate(idx)
    m_coarse, _ = match_rate(cidx)
    m_best, _ = match_rate(bidx)
    res = {
        "workload": "c5: 2048x2048 LOS, 288 channels 800-1088 MHz, phi -300..300 step 0.5 (1201), "
                    "1 % thin (1-2), 0.5 % slab, SNR 3-50",
        "network": "288x2 -> 256 -> 256 -> 2, FP16 MFMA, FP32 accumulate",
        "train_los": n_train, "train_steps": rep.steps, "train_s": train_s,
        "train_loss_first_last": [rep.losses[0][1], rep.losses[-1][1]],
        "tau": cal.tau, "heldout_recall": cal.recall,
        "detection_threshold": thr,
        "oracle_census": {"los": int(census.size), "oracle_detected": n_odet,
                          "oracle_s": t_or, "oracle_gsamples_s": census.size * len(lam) * len(phi) / t_or / 1e9,
                          "rule": "oracle |F|max >= 6 sigma_F; index agrees under the oracle's "
                                  "peak rule (exact where the margin exceeds 2e-5)"},
        "match_on_oracle_detected": m_gate,
        "search_bf16_fallback": {"gated_ms": tgs, "match_on_oracle_detected": m_gate_s,
                                 "call": "rmsynth_gate_search (gated LOS through the fused "
                                         "split-bf16 peaks-only search)"},
        "ungated_fp32_match_on_oracle_detected": m_full,
        "gpu_detected_los": int(det.sum()),
        "match_on_gpu_detected": float(np.mean((gidx == idx)[det])),
        "gated_fraction": float(gated.mean()),
        "gated_ms": tg, "infer_ms": tinf, "ungated_fp32_ms": t32, "ungated_bf16x3_ms": tbf,
        "coarse_gate": {"fp32_coarse_ms": tc, "kept_fraction": float(len(csel) / nlos),
                        "match_on_oracle_detected": m_coarse,
                        "search_bf16_coarse_ms": tcb, "search_bf16_kept_fraction": float(len(bsel) / nlos),
                        "search_bf16_match_on_oracle_detected": m_best},
        "speedup_vs_ungated_fp32": t32 / min(tg, tgs), "speedup_vs_ungated_bf16x3": tbf / min(tg, tgs),
        "speedup_vs_coarse_gate_best": min(tc, tcb) / min(tg, tgs),
    }
    del rq, ru
    plan.close()
    planc.close()
    net.close()
    del cube, Q, U, full, g
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this RM-synthesis build measures one GPU only; "
                                   "run with --gpus 1 (LOS sharding across GPUs is a design note)"}))
        return 2
    import torch
    import paper_1810_06250_amd as rs
    from synthetic import WORKLOADS, make_cube, stratified_subsample

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy_mib} MiB read + written")
        del src, dst

    wl = WORKLOADS[args.workload]
    log(f"generating {args.workload}: {wl.nlos} LOS x {wl.nchan} ch x {len(wl.phi())} phi")
    cube = make_cube(wl, device="cuda")
    plan = rs.Plan(cube["lambda2"], cube["weights"], cube["phi"])
    nlos, nchan, nphi = cube["nlos"], len(cube["lambda2"]), len(cube["phi"])
    samples = nlos * nchan * nphi

    def alloc():
        Fq = torch.empty((nlos, nphi), dtype=torch.float32, device="cuda")
        Fu = torch.empty_like(Fq)
        pk = dict(idx=torch.empty(nlos, dtype=torch.int32, device="cuda"),
                  phi_pk=torch.empty(nlos, device="cuda"), amp=torch.empty(nlos, device="cuda"),
                  q_pk=torch.empty(nlos, device="cuda"), u_pk=torch.empty(nlos, device="cuda"))
        return Fq, Fu, pk

    prec_id = rs.PRECISIONS[args.precision]
    Fq, Fu, pk = alloc()
    fused = args.precision != "fp32" and plan_uniform(cube["phi"])
    log(f"timing {args.precision}: {args.warmup} warmup + {args.steps} steps"
        f"{' (transform with fused peaks)' if fused else ''}")
    wall, ex_ms, pk_ms = time_path(rs, plan, cube, prec_id, Fq, Fu, pk, args.steps, args.warmup,
                                   fused=fused)
    gpu_out = {args.precision: (Fq, Fu, pk["idx"])}

    fp32 = None
    if args.precision != "fp32" and not args.no_fp32_compare:
        Fq2, Fu2, pk2 = alloc()
        steps32 = max(3, args.steps // 4)
        log(f"timing fp32 path: 1 warmup + {steps32} steps")
        w32, ex32, pk32 = time_path(rs, plan, cube, rs.RMSYNTH_FP32, Fq2, Fu2, pk2, steps32, 1)
        gpu_out["fp32"] = (Fq2, Fu2, pk2["idx"])
        fp32 = {"value": samples / (w32 * 1e-3) / 1e9, "unit": "Gsamples/s", "ms_per_step": w32,
                "execute_ms": ex32, "peaks_ms": pk32,
                "mfma_tflops": 8.0 * samples / (ex32 * 1e-3) / 1e12,
                "frac_fp32_peak": 8.0 * samples / (ex32 * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["fp32"]}

    achieved = MFMA_FLOP_PER_SAMPLE[args.precision] * samples / (ex_ms * 1e-3) / 1e12
    peak = MFMA_PEAK_TFLOPS[args.precision]
    res = {
        "metric": METRIC,
        "value": samples / (wall * 1e-3) / 1e9,
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16", "fp16x3": "f16", "fp32": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.nx}x{wl.ny} LOS, {nchan} channels "
                               f"{wl.f_lo:g}-{wl.f_hi:g} MHz, phi {wl.phi_lo:g}..{wl.phi_hi:g} "
                               f"step {wl.phi_step:g} ({nphi}), "
                               f"{'LOS-major' if cube['layout'] == 0 else 'frequency-major'}",
                   "nlos": nlos, "nchan": nchan, "nphi": nphi, "samples": samples,
                   "precision": args.precision,
                   "step": ("rmsynth_execute_peaks (transform, peak reduction fused into its "
                            "epilogue, per-tile merge)") if fused else
                           "rmsynth_execute + rmsynth_peaks"},
        "kernels": ({"execute_peaks_ms": ex_ms, "fused_peaks": True} if fused else
                    {"execute_ms": ex_ms, "peaks_ms": pk_ms,
                     "peaks_hbm_gbs": 8.0 * nlos * nphi / (pk_ms * 1e-3) / 1e9}),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(args.workload, args.precision),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                     "per_unit": f"{MFMA_FLOP_PER_SAMPLE[args.precision]:g} MFMA flop per "
                                 f"LOS*channel*phi sample x {samples} samples per launch"},
        "effective_fp32_tflops": 8.0 * samples / (ex_ms * 1e-3) / 1e12,
    }
    if fp32 is not None:
        res["fp32_path"] = fp32
        res["speedup_vs_fp32_execute"] = fp32["execute_ms"] / ex_ms
        res["speedup_vs_fp32_step"] = fp32["ms_per_step"] / wall
    res["paper_context"] = paper_context()
    if not args.no_cpu_baseline:
        sub = stratified_subsample(nlos, cube["src_los"], 4096, seed=wl.seed + 11)
        log("cpu_baseline: FP64 oracle on host cores")
        cb, errors = cpu_baseline_leg(cube, sub, gpu_out, args.cpu_seconds)
        res["cpu_baseline"] = cb
        res["errors_vs_oracle"] = errors
    if not args.no_extra:
        from synthetic import noise_sigma_F
        if args.precision != "fp32" and fused:
            log("peaks-only search on the same cube")
            res["peaks_only_search"], _ = search_leg(rs, plan, cube, prec_id, max(3, args.steps // 2),
                                                     1, ref_pk=pk)
        if fp32 is not None:
            del Fq2, Fu2, pk2
            fp32 = None
        torch.cuda.empty_cache()
        if cube["layout"] == 0 and args.workload != "c4":
            log("NUFFT evaluation of the cube")
            sub = stratified_subsample(nlos, cube["src_los"], 4096, seed=wl.seed + 11)
            res["nufft"] = nufft_leg(rs, plan, cube, sub, 5)
        log("adjoint transform of the cube's F")
        res["adjoint"] = adjoint_leg(rs, plan, Fq, Fu, cube["lambda2"], cube["phi"], 3)
        log("RM-CLEAN of the cube's F")
        res["rmclean"] = rmclean_leg(rs, plan, Fq, Fu, cube["lambda2"], cube["weights"], cube["phi"],
                                     noise_sigma_F(wl.sigma, cube["weights"]), cube["src_los"], 3)
        if cube["layout"] == 0 and args.workload != "c4":
            log("the cube on an irregular phi grid")
            sub = stratified_subsample(nlos, cube["src_los"], 2048, seed=wl.seed + 13)
            res["nonuniform_phi"] = nonuniform_leg(rs, cube, sub, 4)
    del Fq, Fu, pk, gpu_out, cube
    if fp32 is not None:
        del Fq2, Fu2, pk2
    torch.cuda.empty_cache()
    if not args.no_extra:
        res["configs"] = {}
        for name, precs, steps, nsub in (("c1", ["fp32", "bf16x3"], 20, 4096),
                                         ("c2", ["bf16x3", "fp16x3", "fp32"], 10, 2048),
                                         ("c4", ["fp16x3", "fp32"], 3, 2048)):
            if name == args.workload:
                continue
            res["configs"][name] = config_leg(rs, name, precs, steps, nsub)
    if not args.no_gate:
        res["learned_gate"] = gate_leg(rs, args.gate_train)
    if not args.no_gemm_ref and args.precision == "bf16x3":
        log("reference: vendor bf16 GEMM 16384^3")
        tf, ms = gemm_reference()
        res["mfma_reference"] = {
            "kind": "torch.matmul bf16, 16384 x 16384 x 16384 (vendor GEMM library), same run",
            "ms": ms, "tflops": tf, "frac_of_peak": tf / MFMA_PEAK_TFLOPS["bf16x3"],
            "split_kernel_vs_reference": achieved / tf}
    print(json.dumps(res), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
