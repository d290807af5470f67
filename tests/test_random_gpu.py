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
        tile = (vw, wx, wy, int(rng.choice([0, 0, 7, 64])), int(rng.integers(0, 5)), 1)
    npos = int(rng.integers(1, 300))
    return dims, n, dtype, kind, cell, tile, npos


@pytest.mark.parametrize("case", range(600))
def test_random_configuration(case):
    rng = np.random.default_rng(1000 + case)
    dims, n, dtype, kind, cell, tile, npos = _random_case(rng)
    coef = rng.uniform(-1, 1, dims + (n,)).astype(np.float32)
    frac = rng.uniform(-2.0, 3.0, (3, npos))
    pos = np.ascontiguousarray(cell.T @ frac)
    ldo = n + int(rng.integers(0, 5))
    # the table layout comes from a generator of its own, so the cases above
    # stay what they were; both layouts must give the oracle's values
    flags = B.BSPL_LAYOUT_BLOCKED if np.random.default_rng(7000 + case).random() < 0.5 else 0
    h = B.spline_table_create_lattice(*dims, n, coef, cell, dtype, flags)
    try:
        gpu, raw = run_gpu(B, h, kind, pos, n, ldo=ldo, tile=tile)
    finally:
        B.spline_table_destroy(h)
    assert_canary(raw, n)
    ref = oracle.evaluate_lattice(kind, dequantized(coef, dtype), pos, cell)
    label = f"case {case}: {dims} N={n} {dtype} {kind} tile {tile} npos {npos} flags {flags}"
    # a component whose values all vanish (n_d = 1 makes its derivatives 0)
    # is normalised by the natural scale max|V| * (1/Delta)^order
    inv_delta = float(np.max(np.abs(np.linalg.inv(cell)) * np.array(dims)[None, :]))
    assert_close(kind, gpu, ref, label=label, inv_delta=inv_delta)


def _random_cell(rng):
    if rng.random() < 0.5:
        return np.diag(rng.uniform(0.4, 2.5, 3))
    while True:
        cell = np.diag(rng.uniform(0.6, 2.0, 3)) + 0.3 * rng.standard_normal((3, 3))
        if abs(np.linalg.det(cell)) > 0.2:
            return cell


@pytest.mark.parametrize("case", range(120))
def test_random_plan(case):
    """A batch plan over 1-5 random tables (some empty), replayed twice."""
    rng = np.random.default_rng(5000 + case)
    dtype = ["f32", "f16", "bf16"][rng.integers(0, 3)]
    kind = ["v", "vgl", "vgh"][rng.integers(0, 3)]
    nt = int(rng.integers(1, 6))
    vw = int(rng.choice([1, 2, 4] if dtype == "f32" else [2, 4, 8]))
    wx = int(rng.choice([1, 2, 4]))
    wy = int(rng.choice([w for w in (1, 2) if w * wx <= 8]))
    tile = (vw, wx, wy, int(rng.choice([0, 64, 256])), int(rng.integers(0, 5)), 1)
    dev = torch.device("cuda")
    lay = np.random.default_rng(8000 + case)  # table layouts, apart from the cases' draws
    tabs, coefs, cells, poss, outs, npos, ldos = [], [], [], [], [], [], []
    try:
        for _ in range(nt):
            dims = tuple(int(x) for x in rng.integers(1, 8, 3))
            n = int(rng.integers(1, 400))
            m = int(rng.integers(0, 120)) if rng.random() > 0.15 else 0
            cell = _random_cell(rng)
            coef = rng.uniform(-1, 1, dims + (n,)).astype(np.float32)
            flags = B.BSPL_LAYOUT_BLOCKED if lay.random() < 0.5 else 0
            tabs.append(B.spline_table_create_lattice(*dims, n, coef, cell, dtype, flags))
            coefs.append(coef)
            cells.append(cell)
            pos = np.ascontiguousarray(cell.T @ rng.uniform(-1.0, 2.0, (3, max(m, 1))))[:, :m]
            poss.append(np.ascontiguousarray(pos))
            npos.append(m)
            ldos.append(n + int(rng.integers(0, 3)))
            o = {"v": torch.full((max(m, 1), ldos[-1]), 9.0, device=dev)}
            if kind != "v":
                o["g"] = torch.full((max(m, 1), 3, ldos[-1]), 9.0, device=dev)
                o["l" if kind == "vgl" else "h"] = torch.full(
                    (max(m, 1), ldos[-1]) if kind == "vgl" else (max(m, 1), 6, ldos[-1]), 9.0,
                    device=dev)
            outs.append(o)
        pd = [torch.from_numpy(p).to(dev) if p.shape[1] else None for p in poss]
        lhk = "l" if kind == "vgl" else "h"
        plan = B.spline_batch_plan_create(
            tabs, npos, kind, pd, [o["v"] for o in outs],
            [o.get("g") for o in outs] if kind != "v" else None,
            [o.get(lhk) for o in outs] if kind != "v" else None, ldos, tile=tile)
        try:
            for _ in range(2):
                B.spline_batch_execute(plan)
                torch.cuda.synchronize()
            for i in range(nt):
                if npos[i] == 0:
                    continue
                raw = {k: t.cpu().numpy() for k, t in outs[i].items()}
                n = coefs[i].shape[-1]
                assert_canary(raw, n, value=9.0)
                got = {k: a[..., :n].astype(np.float64) for k, a in raw.items()}
                ref = oracle.evaluate_lattice(kind, dequantized(coefs[i], dtype), poss[i],
                                              cells[i])
                inv_delta = float(np.max(np.abs(np.linalg.inv(cells[i]))
                                         * np.array(coefs[i].shape[:3])[None, :]))
                assert_close(kind, got, ref, inv_delta=inv_delta,
                             label=f"case {case} table {i} {dtype} {kind} tile {tile}")
        finally:
            B.spline_batch_plan_destroy(plan)
    finally:
        for t in tabs:
            B.spline_table_destroy(t)


@pytest.mark.parametrize("case", range(90))
def test_random_ratio(case):
    rng = np.random.default_rng(9000 + case)
    dims = tuple(int(x) for x in rng.integers(1, 9, 3))
    n = int(rng.integers(1, 600))
    dtype = ["f32", "f16", "bf16"][rng.integers(0, 3)]
    kind = ["v", "vgl", "vgh"][rng.integers(0, 3)]
    cell = _random_cell(rng)
    npos = int(rng.integers(1, 150))
    vw = int(rng.choice([1, 2, 4] if dtype == "f32" else [2, 4, 8]))
    tile = (vw, int(rng.choice([1, 2, 4, 8])), 1, int(rng.choice([0, 0, 37])), 0, 1)
    coef = rng.uniform(-1, 1, dims + (n,)).astype(np.float32)
    pos = np.ascontiguousarray(cell.T @ rng.uniform(-1.0, 2.0, (3, npos)))
    ld = n + int(rng.integers(0, 4))
    flags = B.BSPL_LAYOUT_BLOCKED if np.random.default_rng(9500 + case).random() < 0.5 else 0
    ainv = rng.standard_normal((npos, ld)).astype(np.float32)
    full = oracle.evaluate_lattice(kind, dequantized(coef, dtype).astype(np.float64), pos, cell)
    comps = [full["v"]]
    if kind != "v":
        comps += [full["g"][:, c] for c in range(3)]
    if kind == "vgl":
        comps.append(full["l"])
    if kind == "vgh":
        comps += [full["h"][:, c] for c in range(6)]
    a = ainv[:, :n].astype(np.float64)
    ref = np.stack([(x * a).sum(axis=1) for x in comps], axis=1)
    scale = np.array([np.abs(x * a).sum(axis=1).max() for x in comps]) + 1e-300
    dev = torch.device("cuda")
    h = B.spline_table_create_lattice(*dims, n, coef, cell, dtype, flags)
    try:
        out = torch.full((npos, ref.shape[1]), 7.0, dtype=torch.float64, device=dev)
        B.spline_eval_ratio(h, kind, npos, torch.from_numpy(pos).to(dev),
                            torch.from_numpy(ainv).to(dev), ld, out, tile=tile)
        torch.cuda.synchronize()
    finally:
        B.spline_table_destroy(h)
    err = np.abs(out.cpu().numpy() - ref).max(axis=0) / scale
    # components that vanish (an axis of one cell) are compared to the value's scale
    vanish = scale < 1e-6 * scale[0]
    err[vanish] = np.abs(out.cpu().numpy() - ref).max(axis=0)[vanish] / scale[0]
    assert np.all(err <= 1e-5), (case, dims, n, dtype, kind, tile, err)
