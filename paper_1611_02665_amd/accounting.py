"""Algorithmic byte and flop accounting of the evaluation kernels.

The paper counts, per random position, 64N stride-one coefficient reads and
10N output writes for the SoA VGH kernel (section "Performance Summary and
Roofline analysis"; also "Baseline and miniQMC": 64 input streams), and a
tile working set of 4 N_g N_b bytes in single precision (section
"Experiments and Results", tiling subsection).  These are the bytes the
method must move; cache reuse across positions is not credited.
"""

from __future__ import annotations

import math

NOUT = {"v": 1, "vgl": 5, "vgh": 10}
ELEM_BYTES = {"f32": 4, "f16": 2, "bf16": 2}

# FP32 fused multiply-adds per orbital-eval in the z-then-y-then-x factorised
# reduction the kernels use (informational; the path is HBM-bound).
FMA_PER_EVAL = {"v": 64 + 16 + 4, "vgl": 192 + 80 + 24, "vgh": 192 + 96 + 40}


def bytes_per_eval(kind: str, dtype: str = "f32") -> int:
    """64 coefficient reads + n_out FP32 writes per (position, spline)."""
    return 64 * ELEM_BYTES[dtype] + 4 * NOUT[kind]


def batch_bytes(kind: str, dtype: str, npos: int, nsplines: int) -> int:
    """Algorithmic HBM bytes of one call: per-eval bytes plus 24 B of FP64
    position per position (scales of reduced-precision tables excluded)."""
    return npos * nsplines * bytes_per_eval(kind, dtype) + 24 * npos


def tile_working_set_bytes(grid_points: int, nb: int, elem_bytes: int = 4) -> int:
    """Input working set of one spline tile: elem_bytes * N_g * N_b."""
    return elem_bytes * grid_points * nb


def unique_row_fraction(npos: int, padded_points: int) -> float:
    """Expected fraction of distinct table rows among 64*npos random row
    reads: (1 - exp(-lam)) / lam with lam = 64 npos / padded points."""
    lam = 64.0 * npos / padded_points
    return (1.0 - math.exp(-lam)) / lam if lam > 0 else 1.0


def roofline_evals_per_s(kind: str, dtype: str, peak_bytes_per_s: float = 8.0e12) -> float:
    return peak_bytes_per_s / bytes_per_eval(kind, dtype)
