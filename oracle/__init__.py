"""FP64 CPU oracle for RM synthesis -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    build,
    lib_path,
    plan,
    plan_info,
    cost_flop,
    threads,
    fdf,
    rmsf,
    adjoint,
    peaks,
    peak_angle,
    peak_fit,
    peak_fit_from_spectra,
    fdf_bruteforce,
    per_los_error,
    incoherent_scale,
    peak_agreement,
)
