"""Randomised GPU parity: shapes, N, dtype, kind, cell and tile drawn at
random (seeded), each case against the oracle on the coefficients the kernel
reads.  It covers combinations the hand-written cases do not."""

import numpy as np
import pytest

import oracle
from helpers import assert_canary, assert_close, dequantized, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_02665_amd import binding as B  # noqa: E402

NOUT = {"v": 1, "vgl": 5, "vgh": 10}


def _random_case(rng):
    dims = tuple(int(x) for x in rng.integers(1, 10, 3))
    n = int(rng.integers(1, 700))
    dtype = ["f32", "f16", "bf16"][rng.integers(0, 3)]
    kind = ["v", "vgl", "vgh"][rng.integers(0, 3)]
    if rng.random() < 0.5:
        cell = np.diag(rng.uniform(0.4, 2.5, 3))
    else:
        while True:
            cell = np.diag(rng.uniform(0.6, 2.0, 3)) + 0.3 * rng.standard_normal((3, 3))
            if abs(np.linalg.det(cell)) > 0.2:
                break
    vw = int(rng.choice([1, 2, 4] if dtype == "f32" else [2, 4, 8]))
    split = int(rng.choice([1, 1, 2, 4]))
    if split > 1:
        wx = int(rng.choice([w for w in (1, 2, 4) if w * split <= 8]))
        tile = (vw, wx, 1, 0, int(rng.integers(0, 3)), split)
        if split * wx * NOUT[kind] * vw * 256 > 65536:
            tile = (vw, 1, 1, 0, tile[4], 2)
    else:
        wx = int(rng.choice([1, 2, 4, 8]))
        wy = int(rng.choice([w for w in (1, 2, 4, 8) if w * wx <= 8]))
        tile = (vw, wx, wy, int(rng.choice([0, 0, 7, 64])), int(rng.integers(0, 3)), 1)
    npos = int(rng.integers(1, 300))
    return dims, n, dtype, kind, cell, tile, npos


@pytest.mark.parametrize("case", range(150))
def test_random_configuration(case):
    rng = np.random.default_rng(1000 + case)
    dims, n, dtype, kind, cell, tile, npos = _random_case(rng)
    coef = rng.uniform(-1, 1, dims + (n,)).astype(np.float32)
    frac = rng.uniform(-2.0, 3.0, (3, npos))
    pos = np.ascontiguousarray(cell.T @ frac)
    ldo = n + int(rng.integers(0, 5))
    h = B.spline_table_create_lattice(*dims, n, coef, cell, dtype)
    try:
        gpu, raw = run_gpu(B, h, kind, pos, n, ldo=ldo, tile=tile)
    finally:
        B.spline_table_destroy(h)
    assert_canary(raw, n)
    ref = oracle.evaluate_lattice(kind, dequantized(coef, dtype), pos, cell)
    label = f"case {case}: {dims} N={n} {dtype} {kind} tile {tile} npos {npos}"
    # a component whose values all vanish (n_d = 1 makes its derivatives 0)
    # is normalised by the natural scale max|V| * (1/Delta)^order
    inv_delta = float(np.max(np.abs(np.linalg.inv(cell)) * np.array(dims)[None, :]))
    assert_close(kind, gpu, ref, label=label, inv_delta=inv_delta)
