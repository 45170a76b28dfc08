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
                        "tests/test_oracle_pins.py"], cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
