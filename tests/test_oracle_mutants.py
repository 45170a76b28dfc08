"""The oracle's pins must be sensitive: plant a plausible mistake in a copy
of the C oracle (on the CPU), rebuild it, and check that the pin suite fails.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "sign_of_imaginary_part": ("im += y * c - x * s;", "im += y * c + x * s;"),
    "sign_of_real_part": ("re += x * c + y * s;", "re += x * c - y * s;"),
    "dropped_weight": ("double x = w[j] * Q[at];", "double x = Q[at];"),
    "transposed_operand": ("? (size_t)l * nchan + j", "? (size_t)j * nlos + l"),
    "theta_missing_factor_2": (
        "double theta = 2.0 * phi[k] * (lambda2[j] - lambda0_sq);\n                ctab",
        "double theta = phi[k] * (lambda2[j] - lambda0_sq);\n                ctab"),
    "unweighted_lambda0": ("swl += w[j] * lambda2[j];", "swl += lambda2[j];"),
    "wrong_K": ("double K = 1.0 / sw;", "double K = 1.0 / (sw + 1.0);"),
    "rmsf_conjugated": ("im -= w[j] * sin(theta);", "im += w[j] * sin(theta);"),
    "peak_tie_to_highest": ("if (a > m1) { m1 = a; best = k; }",
                            "if (a >= m1) { m1 = a; best = k; }"),
    "flagged_channels_used": ("if (!(w[j] > 0.0)) continue;          /* flagged channel */", ""),
    "adjoint_conjugated": ("re += x * c - y * s;\n                im += y * c + x * s;",
                           "re += x * c + y * s;\n                im += y * c - x * s;"),
    "adjoint_without_lambda0": ("double theta = 2.0 * phi[k] * (lambda2[j] - lambda0_sq);\n                double c = cos(theta), s = sin(theta);",
                                "double theta = 2.0 * phi[k] * lambda2[j];\n                double c = cos(theta), s = sin(theta);"),
    "adjoint_missing_factor_2": ("double theta = 2.0 * phi[k] * (lambda2[j] - lambda0_sq);\n                double c = cos(theta), s = sin(theta);",
                                 "double theta = phi[k] * (lambda2[j] - lambda0_sq);\n                double c = cos(theta), s = sin(theta);"),
    "adjoint_parts_swapped": ("Pre[(size_t)l * nchan + j] = re;\n            Pim[(size_t)l * nchan + j] = im;",
                              "Pre[(size_t)l * nchan + j] = im;\n            Pim[(size_t)l * nchan + j] = re;"),
    "cos_sin_swapped": ("c = ctab[(size_t)k * nchan + j];\n                    s = stab[(size_t)k * nchan + j];",
                        "s = ctab[(size_t)k * nchan + j];\n                    c = stab[(size_t)k * nchan + j];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    src = open(os.path.join(ROOT, "oracle", "rmsynth_oracle.c")).read()
    a, b = MUTANTS[name]
    assert a in src, f"mutation site for {name} not found"
    for sub in ("tests", "synthetic", "oracle"):
        shutil.copytree(os.path.join(ROOT, sub), tmp_path / sub,
                        ignore=shutil.ignore_patterns("__pycache__", "*.so", "test_oracle_mutants.py"))
    (tmp_path / "oracle" / "rmsynth_oracle.c").write_text(src.replace(a, b))
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o",
                    str(tmp_path / "oracle" / "liboracle.so"),
                    str(tmp_path / "oracle" / "rmsynth_oracle.c"), "-lm"], check=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_oracle_adjoint.py"], cwd=tmp_path,
                       capture_output=True, text=True)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"


# Plausible mistakes in the comparison rules and the sub-grid peak of
# oracle/oracle.py; each must make tests/test_oracle_compare.py or
# tests/test_oracle_fit.py fail.
PY_MUTANTS = {
    "error_reduced_over_los": ("num = np.sqrt(dq * dq + du * du).max(axis=1)",
                               "num = np.sqrt(dq * dq + du * du).max(axis=0)"),
    "reference_reduced_over_los": ("den = np.hypot(Fq_ref, Fu_ref).max(axis=1)",
                                   "den = np.hypot(Fq_ref, Fu_ref).max(axis=0)"),
    "error_without_imaginary_part": ("num = np.sqrt(dq * dq + du * du)", "num = np.sqrt(dq * dq)"),
    "floor_ignored": ("den = np.maximum(den, floor)", "den = den"),
    "floor_replaces_reference": ("den = np.maximum(den, floor)", "den = floor"),
    "floor_inverted": ("den = np.maximum(den, floor)", "den = np.minimum(den, floor)"),
    "scale_unsquared_weights": ("P2 @ (w[keep] ** 2)", "P2 @ w[keep]"),
    "scale_without_K": ("np.sqrt(P2 @ (w[keep] ** 2)) / w.sum()", "np.sqrt(P2 @ (w[keep] ** 2))"),
    "scale_transposed_layout": ("if layout == 1:\n        Q, U = Q.T, U.T",
                                "if layout == 0:\n        Q, U = Q.T, U.T"),
    "ambiguity_mask_inverted": ('(ref_peaks["margin"] > margin_thr)', '(ref_peaks["margin"] <= margin_thr)'),
    "margin_at_threshold_unambiguous": ('(ref_peaks["margin"] > margin_thr)',
                                        '(ref_peaks["margin"] >= margin_thr)'),
    "result_order_swapped": ("return int(unamb.sum()), mism, bad", "return mism, int(unamb.sum()), bad"),
    "acceptance_band_ten_times_wider": ("(1.0 - margin_thr) * ref_peaks",
                                        "(1.0 - 10.0 * margin_thr) * ref_peaks"),
    "out_of_range_index_accepted": ("if k < 0 or k >= Fq_ref.shape[1]:", "if k < -1 or k > Fq_ref.shape[1]:"),
    "flag_disagreement_ignored": ("bad = int(np.sum(flagged & (idx_gpu != -1)))", "bad = 0"),
    "fit_offset_sign": ("t = -B / (2.0 * A)", "t = B / (2.0 * A)"),
    "fit_neighbours_swapped": ("s0, s2 = (y0 - y1) / d0, (y2 - y1) / d2", "s0, s2 = (y2 - y1) / d0, (y0 - y1) / d2"),
    "fit_top_without_correction": ("top = y1 - B * B / (4.0 * A)", "top = y1"),
    "fit_on_squared_amplitude": ("np.where(inside, np.hypot(Fq[rows, kc], Fu[rows, kc]), np.nan)",
                                 "np.where(inside, Fq[rows, kc] ** 2 + Fu[rows, kc] ** 2, np.nan)"),
    "fit_edges_wrapped": ("inside = have & (kk >= 0) & (kk < nphi)\n        kc = np.clip(kk, 0, nphi - 1)",
                          "inside = have\n        kc = kk % nphi"),
    "threshold_argument_ignored": ("def peak_agreement(idx_gpu, Fq_ref, Fu_ref, ref_peaks, margin_thr=2e-5):",
                                   "def peak_agreement(idx_gpu, Fq_ref, Fu_ref, ref_peaks, margin_thr=2e-5):\n"
                                   "    margin_thr = 2e-5"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_comparison_pins_catch_planted_mistake(tmp_path, name):
    src = open(os.path.join(ROOT, "oracle", "oracle.py")).read()
    a, b = PY_MUTANTS[name]
    assert src.count(a) == 1, f"mutation site for {name} not found exactly once"
    for sub in ("tests", "synthetic", "oracle"):
        shutil.copytree(os.path.join(ROOT, sub), tmp_path / sub,
                        ignore=shutil.ignore_patterns("__pycache__", "test_oracle_mutants.py"))
    (tmp_path / "oracle" / "oracle.py").write_text(src.replace(a, b))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_compare.py", "tests/test_oracle_fit.py"], cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode != 0, f"comparison pins did not catch mutant {name}:\n{r.stdout[-2000:]}"


# Plausible mistakes in the RM-CLEAN and NUFFT oracles; each must make the
# module's own pins fail.
MOD_MUTANTS = {
    "clean_gain_ignored": ("oracle/rmclean.py", "c = gain * r[p]", "c = r[p]", "tests/test_oracle_rmclean.py"),
    "clean_rmsf_mirrored": ("oracle/rmclean.py", "r -= c * R2[(N - 1) + k - p]", "r -= c * R2[(N - 1) - k + p]",
                            "tests/test_oracle_rmclean.py"),
    "clean_component_not_accumulated": ("oracle/rmclean.py", "cc[l, p] += c", "cc[l, p] = c",
                                        "tests/test_oracle_rmclean.py"),
    "clean_stop_test_inclusive": ("oracle/rmclean.py", "if amp < cutoff:", "if amp <= cutoff:",
                                  "tests/test_oracle_rmclean.py"),
    "clean_restored_without_residual": ("oracle/rmclean.py", "restored = resid + cc @ beam.T",
                                        "restored = cc @ beam.T", "tests/test_oracle_rmclean.py"),
    "clean_beam_width_halved": ("oracle/rmclean.py", "(np.asarray(x, np.float64) / fwhm) ** 2",
                                "(np.asarray(x, np.float64) / (0.5 * fwhm)) ** 2", "tests/test_oracle_rmclean.py"),
    "nufft_phase_centre_dropped": ("oracle/nufft.py", "np.exp(-2j * a * phic)", "np.exp(-2j * a * 0.0)",
                                   "tests/test_oracle_nufft.py"),
    "nufft_no_deconvolution": ("oracle/nufft.py", "/ psi_hat(m, alpha, beta)[None, :]", "/ alpha",
                               "tests/test_oracle_nufft.py"),
    "nufft_non_periodic_distance": ("oracle/nufft.py",
                                    "d = np.mod(xl[:, None] - x[None, :] + np.pi, 2.0 * np.pi) - np.pi",
                                    "d = xl[:, None] - x[None, :]", "tests/test_oracle_nufft.py"),
    "nufft_mode_sign": ("oracle/nufft.py", "G[:, np.mod(m, n)]", "G[:, np.mod(-m, n)]",
                        "tests/test_oracle_nufft.py"),
}


@pytest.mark.parametrize("name", sorted(MOD_MUTANTS))
def test_module_pins_catch_planted_mistake(tmp_path, name):
    rel, a, b, tests = MOD_MUTANTS[name]
    src = open(os.path.join(ROOT, rel)).read()
    assert src.count(a) == 1, f"mutation site for {name} not found exactly once"
    for sub in ("tests", "synthetic", "oracle"):
        shutil.copytree(os.path.join(ROOT, sub), tmp_path / sub,
                        ignore=shutil.ignore_patterns("__pycache__", "test_oracle_mutants.py"))
    (tmp_path / rel).write_text(src.replace(a, b))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", tests],
                       cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
