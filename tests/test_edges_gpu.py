"""Edge cases across the features: non-finite positions on every path
(general cells, latency mode, ordering, fused ratios, plans), plans with
empty tables and with the maximum of 16 tables."""

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_close, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_02665_amd import binding as B  # noqa: E402

HEX = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3) / 2, 0.0], [0.0, 0.0, 1.6]])
# columns: finite, NaN x, -inf y, inf x, far (no fraction bits), finite
BAD = np.array([[0.1, np.nan, 0.3, np.inf, 1e300, 0.7],
                [0.2, 0.2, -np.inf, 0.1, 0.5, 0.4],
                [0.3, 0.3, 0.3, 0.1, 0.5, 0.9]])


def _check_bad(gpu, label):
    for key, a in gpu.items():
        assert np.all(np.isfinite(a[[0, 5]])), (label, key)
        assert np.all(np.isnan(a[1:4])), (label, key)
        assert np.all(np.isfinite(a[4])), (label, key)


@pytest.fixture(scope="module")
def tables():
    coef = synth.coef_table(7, 8, 9, 200, stream=170)
    box = B.spline_table_create(7, 8, 9, 200, coef, "f32")
    hexa = B.spline_table_create_lattice(7, 8, 9, 200, coef, HEX, "f16")
    yield coef, box, hexa
    B.spline_table_destroy(box)
    B.spline_table_destroy(hexa)


@pytest.mark.parametrize("tile", [(1, 2, 1, 0, 0, 1), (1, 2, 1, 0, 1, 1), (2, 1, 1, 0, 2, 1),
                                  (1, 1, 1, 0, 0, 4), (2, 2, 1, 0, 1, 2)])
def test_non_finite_positions_every_path(tables, tile):
    coef, box, hexa = tables
    for name, h in (("box", box), ("hex", hexa)):
        t = tile if name == "box" or tile[0] > 1 else (2,) + tile[1:]  # FP16 has vw >= 2
        for kind in ("v", "vgl", "vgh"):
            gpu, _ = run_gpu(B, h, kind, BAD, 200, tile=t)
            _check_bad(gpu, f"{name} {kind} {t}")
    # the finite positions are right
    gpu, _ = run_gpu(B, box, "vgh", BAD[:, [0, 5]].copy(), 200, tile=tile)
    assert_close("vgh", gpu, oracle.evaluate("vgh", coef, BAD[:, [0, 5]]))


def test_non_finite_positions_in_ratios(tables):
    coef, box, hexa = tables
    dev = torch.device("cuda")
    p = torch.from_numpy(BAD.copy()).to(dev)
    a = torch.ones((6, 200), device=dev)
    for h in (box, hexa):
        out = torch.zeros((6, 10), dtype=torch.float64, device=dev)
        B.spline_eval_ratio(h, "vgh", 6, p, a, 200, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert np.all(np.isfinite(o[[0, 4, 5]])) and np.all(np.isnan(o[1:4]))


def test_plan_with_empty_and_non_finite_tables(tables):
    """A table with no positions contributes nothing and its buffers may be
    NULL; non-finite positions give NaN rows inside a plan too."""
    coef, box, _ = tables
    dev = torch.device("cuda")
    p0 = torch.from_numpy(BAD.copy()).to(dev)
    v0 = torch.full((6, 200), 3.0, device=dev)
    g0 = torch.full((6, 3, 200), 3.0, device=dev)
    h0 = torch.full((6, 6, 200), 3.0, device=dev)
    plan = B.spline_batch_plan_create([box, box], [6, 0], "vgh", [p0, None], [v0, None],
                                      [g0, None], [h0, None], [200, 200], tile=(1, 2, 1, 0, 1, 1))
    try:
        B.spline_batch_execute(plan)
        torch.cuda.synchronize()
        _check_bad({"v": v0.cpu().numpy(), "g": g0.cpu().numpy(), "h": h0.cpu().numpy()}, "plan")
    finally:
        B.spline_batch_plan_destroy(plan)
    # every table empty: creation and replay are no-ops
    plan = B.spline_batch_plan_create([box], [0], "v", [None], [None], ldo=[200],
                                      tile=(1, 1, 1, 0, 0, 1))
    B.spline_batch_execute(plan)
    B.spline_batch_plan_destroy(plan)


def test_plan_with_sixteen_tables():
    shapes = [(4 + i % 5, 5 + i % 3, 6 + i % 4, 40 + 17 * i) for i in range(16)]
    npos = [5 + 9 * i for i in range(16)]
    coefs = [synth.coef_table(*s, stream=180 + i) for i, s in enumerate(shapes)]
    hs = [B.spline_table_create(*s, c, "f32") for s, c in zip(shapes, coefs)]
    dev = torch.device("cuda")
    try:
        pos = [synth.positions(n, stream=200 + i) * 2 - 0.5 for i, n in enumerate(npos)]
        pd = [torch.from_numpy(p).to(dev) for p in pos]
        outs = [(torch.empty(n, s[3], device=dev), torch.empty(n, 3, s[3], device=dev),
                 torch.empty(n, s[3], device=dev)) for n, s in zip(npos, shapes)]
        plan = B.spline_batch_plan_create(hs, npos, "vgl", pd, [o[0] for o in outs],
                                          [o[1] for o in outs], [o[2] for o in outs],
                                          [s[3] for s in shapes], tile=(1, 2, 2, 512, 0, 1))
        try:
            B.spline_batch_execute(plan)
            torch.cuda.synchronize()
            for i in range(16):
                got = {"v": outs[i][0].cpu().numpy().astype(np.float64),
                       "g": outs[i][1].cpu().numpy().astype(np.float64),
                       "l": outs[i][2].cpu().numpy().astype(np.float64)}
                assert_close("vgl", got, oracle.evaluate("vgl", coefs[i], pos[i]),
                             label=f"table {i}")
        finally:
            B.spline_batch_plan_destroy(plan)
        with pytest.raises(B.BsplineError):
            B.spline_batch_plan_create(hs + [hs[0]], npos + [1], "v", pd + [pd[0]],
                                       [o[0] for o in outs] + [outs[0][0]],
                                       ldo=[s[3] for s in shapes] + [shapes[0][3]])
    finally:
        for h in hs:
            B.spline_table_destroy(h)


def _degenerate_position_sets(cell):
    """Position sets that stress the ordering pre-pass's counting sort:
    every position in one bin (two chunks, ragged tail), grid points and
    bin boundaries with far periodic images, two tight clusters, and
    non-finite coordinates (which all share bin 0)."""
    rng = np.random.default_rng(190)
    same = np.tile(np.array([[0.37], [0.52], [0.91]]), (1, 5000))
    k = np.arange(4200)
    grid_pts = np.stack([(k % 16) / 16.0, ((k // 16) % 16) / 16.0, (k // 256) / 16.0])
    grid_pts = grid_pts + rng.integers(-10**6, 10**6, (3, 1)) * np.array([[1.0], [-1.0], [1.0]])
    grid_pts[:, ::7] *= -1.0
    clusters = np.concatenate([0.2 + 1e-6 * rng.standard_normal((3, 2100)),
                               0.8 + 1e-6 * rng.standard_normal((3, 2100))], axis=1)
    mixed = rng.uniform(-3.0, 4.0, (3, 4500))
    mixed[0, ::11] = np.nan
    mixed[1, 5::13] = np.inf
    mixed[2, 7::17] = -np.inf
    with np.errstate(invalid="ignore"):  # inf * 0 in the map: that position stays non-finite
        return {name: np.ascontiguousarray(cell.T @ f) for name, f in
                (("one bin", same), ("grid points", grid_pts), ("clusters", clusters),
                 ("non-finite", mixed))}


@pytest.mark.parametrize("cell", ["box", "hex"])
def test_ordering_degenerate_distributions(cell):
    """Orders 1 to 4 give the same bits as input order on position sets that
    pile every position into one bin or sit on bin boundaries; a position
    the permutation dropped would keep its canary and fail the comparison."""
    coef = synth.coef_table(9, 10, 11, 130, stream=191)
    A = np.eye(3) if cell == "box" else HEX
    h = B.spline_table_create_lattice(9, 10, 11, 130, coef, A, "f32")
    try:
        for name, pos in _degenerate_position_sets(A).items():
            for kind in ("v", "vgh"):
                outs = [run_gpu(B, h, kind, pos, 130, tile=(1, 2, 1, 0, order, 1))[1]
                        for order in (0, 1, 2, 3, 4)]
                for o in outs[1:]:
                    for key in o:
                        assert np.array_equal(o[key], outs[0][key], equal_nan=True), \
                            (cell, name, kind, key)
                assert not np.any(outs[0]["v"][:, :130] == 12345.0), (cell, name, kind)
        finite = _degenerate_position_sets(A)["grid points"][:, :64]
        gpu, _ = run_gpu(B, h, "vgh", finite, 130, tile=(1, 2, 1, 0, 1, 1))
        assert_close("vgh", gpu, oracle.evaluate_lattice("vgh", coef, finite, A),
                     label=f"{cell} grid points, ordered")
    finally:
        B.spline_table_destroy(h)


def test_table_larger_than_device_memory_is_enomem():
    """A 449 GB table (603^3 x 512 FP32 rows) cannot be allocated on a 288 GB
    device: creation returns ENOMEM before it reads any coefficient, and the
    library keeps working afterwards."""
    info = B.spline_layout_query(600, 600, 600, 512, "f32")
    free, total = torch.cuda.mem_get_info()
    assert info["table_bytes"] > total
    dev = torch.device("cuda")
    dummy = torch.zeros(16, device=dev)  # never read: the table allocation fails first
    with pytest.raises(B.BsplineError) as e:
        B.spline_table_create(600, 600, 600, 512, dummy, "f32", flags=B.BSPL_COEFS_DEVICE)
    assert e.value.status == B.BSPL_ENOMEM
    assert "hipMalloc(table)" in B.spline_last_error()
    coef = synth.coef_table(4, 5, 6, 70, stream=195)
    h = B.spline_table_create(4, 5, 6, 70, coef, "f32")
    try:
        pos = synth.positions(20, stream=196)
        gpu, _ = run_gpu(B, h, "vgh", pos, 70)
        assert_close("vgh", gpu, oracle.evaluate("vgh", coef, pos))
    finally:
        B.spline_table_destroy(h)
