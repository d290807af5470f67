"""Spline-blocked tables (BSPL_LAYOUT_BLOCKED, the paper's AoSoA table of
sub-tables along N) against plain tables on the GPU.

Both layouts hold the same coefficients and every output is computed by the
same arithmetic, so the evaluations must agree bit for bit: on every kind,
dtype, vector width, order, latency-mode split and persistent grid, in
fused ratios, general cells, batch plans that mix the layouts, tables built
from grid values or padded input, and a table whose blocks lie beyond 4 GiB.
A blocked evaluation is also compared with the oracle directly."""

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_canary, assert_close, dequantized, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_02665_amd import binding as B  # noqa: E402

HEX = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3) / 2, 0.0], [0.0, 0.0, 1.6]])
# three blocks with a ragged last one: 600 = 2 x 256 + 88 (F32), 1100 = 2 x 512 + 76
NSPL = {"f32": 600, "f16": 1100, "bf16": 1100}
VWS = {"f32": (1, 2, 4), "f16": (2, 4, 8), "bf16": (2, 4, 8)}


def _pair(coef, dtype, flags=0, lattice=None):
    n = coef.shape[-1]
    dims = coef.shape[:3] if not flags & B.BSPL_COEFS_PADDED else tuple(d - 3 for d in coef.shape[:3])
    if lattice is None:
        mk = lambda f: B.spline_table_create(*dims, n, coef, dtype, flags=flags | f)  # noqa: E731
    else:
        mk = lambda f: B.spline_table_create_lattice(*dims, n, coef, lattice, dtype,  # noqa: E731
                                                     flags | f)
    return mk(0), mk(B.BSPL_LAYOUT_BLOCKED)


def _same(a, b, label):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), f"{label}: {k} differs"


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_blocked_bit_identical_to_plain(dtype):
    n = NSPL[dtype]
    coef = synth.coef_table(7, 8, 9, n, stream=300)
    plain, blocked = _pair(coef, dtype)
    try:
        info = B.spline_table_info(blocked)
        assert info["block_splines"] == (256 if dtype == "f32" else 512)
        assert B.spline_table_info(plain)["block_splines"] == 0
        pos = synth.positions(300, stream=301) * 2.5 - 0.7
        tiles = []
        for vw in VWS[dtype]:
            # latency mode: split 4, or 2 where 4 partial sums of VGH exceed 64 KiB
            tiles += [(vw, 1, 1, 0, 0, 1), (vw, 2, 2, 0, 1, 1), (vw, 4, 1, 37, 2, 1),
                      (vw, 1, 1, 0, 0, 4 if vw <= 4 else 2)]
        for kind in ("v", "vgl", "vgh"):
            for tile in tiles:
                ldo = n + 3
                a = run_gpu(B, plain, kind, pos, n, ldo=ldo, tile=tile)[1]
                b = run_gpu(B, blocked, kind, pos, n, ldo=ldo, tile=tile)[1]
                assert_canary(b, n)
                _same(a, b, f"{dtype} {kind} tile {tile}")
        gpu, _ = run_gpu(B, blocked, "vgh", pos[:, :80].copy(), n)
        assert_close("vgh", gpu, oracle.evaluate("vgh", dequantized(coef, dtype), pos[:, :80]),
                     label=f"blocked {dtype} vs oracle")
    finally:
        B.spline_table_destroy(plain)
        B.spline_table_destroy(blocked)


def test_blocked_general_cell_and_ratio():
    n = 777  # 4 blocks, the last one 9 splines wide
    coef = synth.coef_table(6, 7, 8, n, stream=302)
    plain, blocked = _pair(coef, "f32", lattice=HEX)
    dev = torch.device("cuda")
    try:
        pos = np.ascontiguousarray(HEX.T @ (synth.positions(200, stream=303) * 3 - 1))
        for kind in ("vgl", "vgh"):
            _same(run_gpu(B, plain, kind, pos, n)[1], run_gpu(B, blocked, kind, pos, n)[1],
                  f"hexagonal {kind}")
        p = torch.from_numpy(pos).to(dev)
        ainv = torch.from_numpy(np.random.default_rng(304).standard_normal((200, n + 5))
                                .astype(np.float32)).to(dev)
        outs = []
        for h in (plain, blocked):
            o = torch.zeros((200, 10), dtype=torch.float64, device=dev)
            B.spline_eval_ratio(h, "vgh", 200, p, ainv, n + 5, o, tile=(2, 4, 1, 0, 0))
            torch.cuda.synchronize()
            outs.append(o.cpu().numpy())
        assert np.array_equal(outs[0], outs[1])
    finally:
        B.spline_table_destroy(plain)
        B.spline_table_destroy(blocked)


def test_blocked_grid_values_and_padded_input():
    """The interpolating fit and padded input feed both layouts alike."""
    n = 530
    values = synth.coef_table(8, 6, 7, n, stream=305)
    pos = synth.positions(120, stream=306) * 2 - 0.5
    for flags, src in ((B.BSPL_COEFS_GRID_VALUES, values),
                       (B.BSPL_COEFS_PADDED, synth.coef_table(11, 9, 10, n, stream=307))):
        plain, blocked = _pair(src, "f32", flags=flags)
        try:
            _same(run_gpu(B, plain, "vgh", pos, n)[1], run_gpu(B, blocked, "vgh", pos, n)[1],
                  f"flags {flags:#x}")
        finally:
            B.spline_table_destroy(plain)
            B.spline_table_destroy(blocked)


@pytest.mark.parametrize("tile", [(1, 2, 1, 0, 1, 1), (4, 1, 2, 96, 0, 1), (2, 4, 1, 0, 2, 1)])
def test_batch_plan_mixing_layouts(tile):
    """One plan over blocked and plain tables of uneven N equals the single
    evaluations of each table."""
    shapes = [(5, 6, 7, 700), (6, 5, 4, 300), (4, 4, 5, 1030)]
    npos = [90, 61, 128]
    flags = [B.BSPL_LAYOUT_BLOCKED, 0, B.BSPL_LAYOUT_BLOCKED]
    coefs = [synth.coef_table(*s, stream=310 + i) for i, s in enumerate(shapes)]
    hs = [B.spline_table_create(*s, c, "f32", flags=f) for s, c, f in zip(shapes, coefs, flags)]
    dev = torch.device("cuda")
    try:
        pos = [synth.positions(m, stream=320 + i) * 2 - 0.5 for i, m in enumerate(npos)]
        pd = [torch.from_numpy(p).to(dev) for p in pos]
        outs = [(torch.full((m, s[3]), 5.0, device=dev), torch.full((m, 3, s[3]), 5.0, device=dev),
                 torch.full((m, 6, s[3]), 5.0, device=dev)) for m, s in zip(npos, shapes)]
        plan = B.spline_batch_plan_create(hs, npos, "vgh", pd, [o[0] for o in outs],
                                          [o[1] for o in outs], [o[2] for o in outs],
                                          [s[3] for s in shapes], tile=tile)
        try:
            B.spline_batch_execute(plan)
            torch.cuda.synchronize()
        finally:
            B.spline_batch_plan_destroy(plan)
        for i in range(3):
            got = {"v": outs[i][0].cpu().numpy(), "g": outs[i][1].cpu().numpy(),
                   "h": outs[i][2].cpu().numpy()}
            single = run_gpu(B, hs[i], "vgh", pos[i], shapes[i][3], tile=tile)[1]
            _same(got, single, f"table {i} in the plan")
    finally:
        for h in hs:
            B.spline_table_destroy(h)


def test_layout_select_records_both_layouts(tmp_path):
    """The selector tunes both layouts once, records them in the wisdom file
    and answers the second time from the cache."""
    wisdom = str(tmp_path / "wisdom.txt")
    shape, n, npos = (20, 20, 20), 1024, 256
    first = B.spline_layout_select(*shape, n, "f32", "vgh", npos, wisdom)
    assert first in (0, B.BSPL_LAYOUT_BLOCKED)
    lines = open(wisdom).read().splitlines()
    assert any(x.startswith("single|") for x in lines)
    assert any(x.startswith("single-blocked|") for x in lines)
    assert all(len(x.split()) == 8 for x in lines)  # key, six tile fields, time
    assert B.spline_layout_select(*shape, n, "f32", "vgh", npos, wisdom) == first
    assert open(wisdom).read().splitlines() == lines  # nothing re-tuned
    # a blocked table of that shape takes its tuned tile from the cache
    h = B.spline_table_create(*shape, n, synth.coef_table(*shape, n, stream=330), "f32",
                              flags=B.BSPL_LAYOUT_BLOCKED)
    try:
        key = [x for x in lines if x.startswith("single-blocked|")][0].split()
        assert B.spline_tile_select(h, "vgh", npos).as_tuple() == tuple(int(v) for v in key[1:7])
    finally:
        B.spline_table_destroy(h)


def test_blocked_table_beyond_4_gib():
    """96^3 x 4096 FP16: blocks of 99^3 KB each, so blocks 5-7 start beyond
    4 GiB; 256 positions agree bit for bit with the plain table."""
    grid, n = (96, 96, 96), 4096
    dev = torch.device("cuda")
    src = synth.coef_table_torch(torch, *grid, n, device=dev, stream=synth.table_stream(0))
    hs = [B.spline_table_create(*grid, n, src, "f16", flags=B.BSPL_COEFS_DEVICE | f)
          for f in (0, B.BSPL_LAYOUT_BLOCKED)]
    del src
    torch.cuda.empty_cache()
    try:
        info = B.spline_table_info(hs[1])
        assert info["block_bytes"] == 99 ** 3 * 1024 and info["table_bytes"] > 4 << 30
        pos = synth.positions(256, stream=331)
        outs = []
        for h in hs:
            p = torch.from_numpy(pos).to(dev)
            v = torch.empty(256, n, device=dev)
            g = torch.empty(256, 3, n, device=dev)
            hh = torch.empty(256, 6, n, device=dev)
            B.spline_eval(h, "vgh", 256, p, v, g, hh, n, tile=(2, 4, 1, 0, 0, 1))
            torch.cuda.synchronize()
            outs.append([x.cpu().numpy() for x in (v, g, hh)])
        for a, b in zip(*outs):
            assert np.array_equal(a, b)
    finally:
        for h in hs:
            B.spline_table_destroy(h)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("kind", ["v", "vgl", "vgh"])
def test_blocked_ratio_reduced_precision(dtype, kind):
    """Fused ratios on FP16/BF16 blocked tables (two blocks, ragged) equal
    those on plain tables bit for bit, for every kind and two tiles."""
    n = 900
    coef = synth.coef_table(5, 6, 7, n, stream=340)
    plain, blocked = _pair(coef, dtype)
    dev = torch.device("cuda")
    try:
        pos = torch.from_numpy(synth.positions(90, stream=341) * 2 - 0.5).to(dev)
        ainv = torch.from_numpy(np.random.default_rng(342).standard_normal((90, n))
                                .astype(np.float32)).to(dev)
        nc = {"v": 1, "vgl": 5, "vgh": 10}[kind]
        for tile in ((2, 4, 1, 0, 0), (8, 1, 1, 0, 0)):
            outs = []
            for h in (plain, blocked):
                o = torch.full((90, nc), 3.0, dtype=torch.float64, device=dev)
                B.spline_eval_ratio(h, kind, 90, pos, ainv, n, o, tile=tile)
                torch.cuda.synchronize()
                outs.append(o.cpu().numpy())
            assert np.array_equal(outs[0], outs[1]), (dtype, kind, tile)
    finally:
        B.spline_table_destroy(plain)
        B.spline_table_destroy(blocked)
