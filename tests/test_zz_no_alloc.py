"""spline_eval_noalloc (the evaluation that allocates nothing) against
spline_eval, through the C ABI.

The two entry points run the same kernels with the same decomposition; the
only difference is where an ordered tile's permutation lives (a static
device array instead of stream-ordered scratch memory).  Their outputs must
therefore agree bit for bit, which is stricter than the 1e-5 FP32 bar; the
FP32 case is also checked against the FP64 oracle at that bar.  Each case
makes two calls in a row, the second with fewer positions, so the second
call runs on the array the first call left behind.
"""

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_02665_amd import binding as B  # noqa: E402

NCOMP = {"v": 1, "vgl": 5, "vgh": 10}


def _outputs(kind, npos, ldo, dev):
    v = torch.full((npos, ldo), 12345.0, device=dev)
    g = torch.full((npos, 3, ldo), 12345.0, device=dev) if kind != "v" else None
    lh = None
    if kind == "vgl":
        lh = torch.full((npos, ldo), 12345.0, device=dev)
    elif kind == "vgh":
        lh = torch.full((npos, 6, ldo), 12345.0, device=dev)
    return v, g, lh


def _run(fn, table, kind, pos_dev, ldo, tile):
    npos = pos_dev.shape[1]
    v, g, lh = _outputs(kind, npos, ldo, pos_dev.device)
    fn(table, kind, npos, pos_dev, v, g, lh, ldo, tile=tile)
    torch.cuda.synchronize()
    out = {"v": v.cpu().numpy()}
    if g is not None:
        out["g"] = g.cpu().numpy()
    if kind == "vgl":
        out["l"] = lh.cpu().numpy()
    if kind == "vgh":
        out["h"] = lh.cpu().numpy()
    return out


CASES = [
    # dtype, kind, tile (vw, wx, wy, grid, order, split)
    ("f32", "vgh", (1, 4, 1, 0, 1, 1)),
    ("f32", "vgl", (2, 2, 2, 0, 2, 1)),
    ("f16", "vgh", (2, 4, 1, 0, 1, 1)),
    ("bf16", "v", (4, 1, 4, 0, 2, 1)),
    ("f32", "vgh", (1, 2, 1, 0, 0, 1)),   # unordered: no scratch at all
    ("f32", "vgh", (1, 2, 1, 0, 0, 4)),   # latency mode
    ("f16", "vgh", (2, 2, 1, 0, 4, 1)),   # sorted, spline-tile-major: uses the array
    ("f32", "vgl", (1, 2, 2, 0, 3, 1)),   # input order, spline-tile-major: no scratch
    ("f32", "vgh", None),                 # built-in default tile
]


@pytest.mark.parametrize("dtype,kind,tile", CASES)
def test_noalloc_matches_spline_eval(dtype, kind, tile):
    nx, ny, nz, n = 20, 17, 23, 300
    coef = synth.coef_table(nx, ny, nz, n, stream=synth.table_stream(7))
    dev = torch.device("cuda")
    table = B.spline_table_create(nx, ny, nz, n, coef, dtype)
    try:
        ldo = n + 5
        for call, npos in enumerate((9000, 1300)):  # second call: fewer positions
            pos = synth.positions(npos, stream=synth.position_stream(40 + call))
            p = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
            want = _run(B.spline_eval, table, kind, p, ldo, tile)
            got = _run(B.spline_eval_noalloc, table, kind, p, ldo, tile)
            for k in want:
                assert np.array_equal(got[k].view(np.uint32), want[k].view(np.uint32)), \
                    f"call {call} ({npos} positions), {k}: noalloc differs from spline_eval"
                assert np.all(got[k][..., n:] == 12345.0), f"{k}: columns [N, ldo) written"
            if dtype == "f32" and call == 1:
                ref = oracle.evaluate(kind, coef, pos)
                gpu = {k: a[..., :n].astype(np.float64) for k, a in got.items()}
                assert_close(kind, gpu, ref, label=f"noalloc {kind} {tile}")
    finally:
        B.spline_table_destroy(table)


def test_noalloc_limit_and_errors():
    """An ordered tile beyond the static array is EUNSUPPORTED before any
    launch.  The buffers are real and large enough for the request, so even
    a missing check could only compute, never read out of bounds."""
    n = 64
    coef = synth.coef_table(8, 8, 8, n, stream=synth.table_stream(8))
    dev = torch.device("cuda")
    table = B.spline_table_create(8, 8, 8, n, coef, "f32")
    try:
        npos = B.NOALLOC_MAX_POSITIONS + 1
        p = torch.rand(3, npos, dtype=torch.float64, device=dev)
        v = torch.full((npos, n), 7.0, device=dev)
        with pytest.raises(B.BsplineError) as e:
            B.spline_eval_noalloc(table, "v", npos, p, v, None, None, n, tile=(1, 1, 1, 0, 1, 1))
        assert e.value.status == B.BSPL_EUNSUPPORTED
        torch.cuda.synchronize()
        assert bool((v == 7.0).all()), "outputs written after the limit error"
        with pytest.raises(B.BsplineError) as e:  # sorted and spline-tile-major
            B.spline_eval_noalloc(table, "v", npos, p, v, None, None, n, tile=(1, 1, 1, 0, 4, 1))
        assert e.value.status == B.BSPL_EUNSUPPORTED
        torch.cuda.synchronize()
        assert bool((v == 7.0).all()), "outputs written after the limit error"
        # unsorted tiles need no scratch: the same size evaluates
        for order in (0, 3):
            v.fill_(7.0)
            B.spline_eval_noalloc(table, "v", npos, p, v, None, None, n,
                                  tile=(1, 1, 1, 0, order, 1))
            torch.cuda.synchronize()
            assert bool(torch.isfinite(v).all()) and not bool((v == 7.0).any())
        # exactly the limit is accepted with an ordered tile
        m = B.NOALLOC_MAX_POSITIONS
        w = torch.empty((m, n), device=dev)
        B.spline_eval_noalloc(table, "v", m, p[:, :m].contiguous(), w, None, None, n,
                              tile=(1, 1, 1, 0, 1, 1))
        ref = torch.empty((m, n), device=dev)
        B.spline_eval(table, "v", m, p[:, :m].contiguous(), ref, None, None, n,
                      tile=(1, 1, 1, 0, 1, 1))
        torch.cuda.synchronize()
        assert torch.equal(w, ref)
        # argument errors as spline_eval
        with pytest.raises(B.BsplineError) as e:
            B.spline_eval_noalloc(None, "v", 10, p, v, None, None, n)
        assert e.value.status == B.BSPL_EINVAL
        with pytest.raises(B.BsplineError) as e:
            B.spline_eval_noalloc(table, "vgh", 10, p, v, None, None, n)
        assert e.value.status == B.BSPL_EINVAL
        with pytest.raises(B.BsplineError) as e:
            B.spline_eval_noalloc(table, "v", 10, p, v, None, None, n - 1)
        assert e.value.status == B.BSPL_EINVAL
        B.spline_eval_noalloc(table, "v", 0, None, None, None, None, n)  # no-op
    finally:
        B.spline_table_destroy(table)
