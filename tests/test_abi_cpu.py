"""C ABI checks that need no GPU: exported symbols, layout arithmetic,
status codes and argument validation (which happens before any HIP call)."""

import ctypes
import os
import re

import pytest

from paper_1611_02665_amd import binding as B

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include")
HEADER = os.path.join(INCLUDE, "bspline.h")


def _declared_functions():
    """Every spline_* function declared in include/*.h."""
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(spline_\w+)\s*\(", text))
    return sorted(names)


def test_every_declared_function_is_exported_and_bound():
    names = _declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(B.lib, n), f"{n} missing from libbspline.so"
        assert n in B.EXPORTED, f"{n} has no binding"
    assert sorted(B.EXPORTED) == names


def test_status_strings():
    for s in range(6):
        assert B.spline_status_string(s).startswith("BSPL_")
    assert "unknown" in B.spline_status_string(99)


@pytest.mark.parametrize("shape,dtype,np_,nbytes", [
    ((16, 16, 16, 64), "f32", 64, 19**3 * 64 * 4),
    ((48, 48, 48, 2048), "f32", 2048, 1_086_676_992),
    ((48, 48, 48, 2048), "f16", 2048, 543_338_496),
    ((48, 48, 48, 2048), "bf16", 2048, 543_338_496),
    ((96, 96, 96, 4096), "f32", 4096, 15_897_378_816),
    ((96, 96, 96, 4096), "f16", 4096, 7_948_689_408),
    ((64, 64, 64, 2048), "f32", 2048, 67**3 * 2048 * 4),
    ((3, 4, 5, 33), "f32", 64, 6 * 7 * 8 * 64 * 4),
    ((3, 4, 5, 33), "f16", 64, 6 * 7 * 8 * 64 * 2),
    ((48, 48, 60, 128), "f32", 128, 51 * 51 * 63 * 128 * 4),
])
def test_layout_query(shape, dtype, np_, nbytes):
    info = B.spline_layout_query(*shape, dtype)
    assert info["n_padded"] == np_
    assert info["row_bytes"] % 128 == 0
    assert (info["px"], info["py"], info["pz"]) == tuple(s + 3 for s in shape[:3])
    assert info["table_bytes"] == nbytes
    assert info["data"] is None and info["scales"] is None


@pytest.mark.parametrize("shape,dtype,bs,np_", [
    ((48, 48, 48, 2048), "f32", 256, 2048),
    ((48, 48, 48, 1152), "f32", 256, 1280),   # ragged last block: 4.5 -> 5 blocks
    ((48, 48, 48, 2048), "f16", 512, 2048),
    ((7, 8, 9, 600), "bf16", 512, 1024),
    ((96, 96, 96, 4096), "f16", 512, 4096),
])
def test_layout_query_blocked(shape, dtype, bs, np_):
    """Spline-blocked tables: [n_padded/B][px][py][pz][B], a 1 KB z row,
    blocks of px*py*pz rows; the same bytes as the plain table when N needs
    no extra padding."""
    info = B.spline_layout_query(*shape, dtype, B.BSPL_LAYOUT_BLOCKED)
    eb = 4 if dtype == "f32" else 2
    pts = (shape[0] + 3) * (shape[1] + 3) * (shape[2] + 3)
    assert info["block_splines"] == bs and info["n_padded"] == np_
    assert info["row_bytes"] == bs * eb == 1024
    assert info["block_bytes"] == pts * 1024
    assert info["table_bytes"] == (np_ // bs) * info["block_bytes"] == pts * np_ * eb
    plain = B.spline_layout_query(*shape, dtype)
    assert plain["block_splines"] == 0 and plain["block_bytes"] == 0
    if np_ == plain["n_padded"]:
        assert info["table_bytes"] == plain["table_bytes"]


def test_layout_query_blocked_single_block_is_plain():
    for dtype, n in (("f32", 256), ("f32", 200), ("f16", 512), ("bf16", 64)):
        info = B.spline_layout_query(7, 8, 9, n, dtype, B.BSPL_LAYOUT_BLOCKED)
        assert info == B.spline_layout_query(7, 8, 9, n, dtype)


def test_layout_select_validates_and_skips_single_block_shapes():
    out = ctypes.c_uint(99)
    f = B.lib.spline_layout_select
    assert f(8, 8, 8, 2048, 0, 2, 64, None, None, None) == B.BSPL_EINVAL  # NULL layout
    assert f(8, 8, 8, 2048, 0, 5, 64, None, ctypes.byref(out), None) == B.BSPL_EINVAL
    assert f(8, 8, 8, 2048, 0, 2, 0, None, ctypes.byref(out), None) == B.BSPL_EINVAL
    assert f(8, 8, 8, 2048, 9, 2, 64, None, ctypes.byref(out), None) == B.BSPL_EINVAL
    # at most one block: the layouts coincide, decided without the device
    assert B.spline_layout_select(8, 8, 8, 256, "f32", "vgh", 64) == 0
    assert B.spline_layout_select(8, 8, 8, 512, "f16", "vgh", 64) == 0


def test_layout_query_rejects():
    with pytest.raises(B.BsplineError) as e:
        B.spline_layout_query(0, 4, 4, 8)
    assert e.value.status == B.BSPL_EINVAL
    with pytest.raises(B.BsplineError) as e:
        B.spline_layout_query(4, 4, 4, 8, 7)
    assert e.value.status == B.BSPL_EINVAL
    with pytest.raises(B.BsplineError) as e:
        B.spline_layout_query(4, 4, 4, -1)
    assert e.value.status == B.BSPL_EINVAL
    # a single cell's 4x4x4 row block would span more than 4 GiB
    with pytest.raises(B.BsplineError) as e:
        B.spline_layout_query(4096, 4096, 4096, 4096)
    assert e.value.status == B.BSPL_EUNSUPPORTED


def test_create_validates_before_touching_the_device():
    h = ctypes.c_void_p(1234)
    coefs = (ctypes.c_float * 8)()
    assert B.lib.spline_table_create(None, 1, 1, 1, 8, coefs, 0, None, 0, None) == B.BSPL_EINVAL
    assert B.lib.spline_table_create(ctypes.byref(h), 1, 1, 1, 8, None, 0, None, 0, None) \
        == B.BSPL_EINVAL
    assert h.value is None  # *out is cleared on failure
    assert B.lib.spline_table_create(ctypes.byref(h), 0, 1, 1, 8, coefs, 0, None, 0, None) \
        == B.BSPL_EINVAL
    assert B.lib.spline_table_create(ctypes.byref(h), 1, 1, 1, 8, coefs, 5, None, 0, None) \
        == B.BSPL_EINVAL
    assert B.lib.spline_table_create(ctypes.byref(h), 1, 1, 1, 8, coefs, 0, None, 0x80, None) \
        == B.BSPL_EINVAL
    bad_box = (ctypes.c_double * 3)(1.0, -1.0, 1.0)
    assert B.lib.spline_table_create(ctypes.byref(h), 1, 1, 1, 8, coefs, 0, bad_box, 0, None) \
        == B.BSPL_EINVAL
    assert "box" in B.spline_last_error()
    nan_box = (ctypes.c_double * 3)(1.0, float("nan"), 1.0)
    assert B.lib.spline_table_create(ctypes.byref(h), 1, 1, 1, 8, coefs, 0, nan_box, 0, None) \
        == B.BSPL_EINVAL


def test_create_lattice_validates_before_touching_the_device():
    h = ctypes.c_void_p(1234)
    coefs = (ctypes.c_float * 8)()
    f = B.lib.spline_table_create_lattice
    assert f(ctypes.byref(h), 1, 1, 1, 8, coefs, 0, None, 0, None) == B.BSPL_EINVAL
    assert h.value is None
    assert "lattice" in B.spline_last_error()
    # a2 = 2 a1: the cell vectors span a plane only
    flat = (ctypes.c_double * 9)(1.0, 0.5, 0.0, 2.0, 1.0, 0.0, 0.0, 0.0, 1.0)
    assert f(ctypes.byref(h), 1, 1, 1, 8, coefs, 0, flat, 0, None) == B.BSPL_EINVAL
    assert "linearly dependent" in B.spline_last_error()
    zero = (ctypes.c_double * 9)()
    assert f(ctypes.byref(h), 1, 1, 1, 8, coefs, 0, zero, 0, None) == B.BSPL_EINVAL
    inf = (ctypes.c_double * 9)(1.0, 0.0, 0.0, 0.0, float("inf"), 0.0, 0.0, 0.0, 1.0)
    assert f(ctypes.byref(h), 1, 1, 1, 8, coefs, 0, inf, 0, None) == B.BSPL_EINVAL
    assert "not finite" in B.spline_last_error()
    ok = (ctypes.c_double * 9)(1.0, 0.0, 0.0, -0.5, 0.8, 0.0, 0.0, 0.0, 1.6)
    # valid cell, but bad sizes / dtype are still rejected first
    assert f(ctypes.byref(h), 0, 1, 1, 8, coefs, 0, ok, 0, None) == B.BSPL_EINVAL
    assert f(ctypes.byref(h), 1, 1, 1, 8, coefs, 9, ok, 0, None) == B.BSPL_EINVAL
    assert f(None, 1, 1, 1, 8, coefs, 0, ok, 0, None) == B.BSPL_EINVAL


def test_fit_validates_before_touching_the_device():
    buf = (ctypes.c_float * 8)()
    f = B.lib.spline_fit_interpolating
    assert f(0, 2, 2, 1, buf, buf, None) == B.BSPL_EINVAL
    assert f(2, 2, 2, 0, buf, buf, None) == B.BSPL_EINVAL
    assert f(2, 2, 2, 1, None, buf, None) == B.BSPL_EINVAL
    assert f(2, 2, 2, 1, buf, None, None) == B.BSPL_EINVAL
    assert f(1 << 30, 1 << 30, 1 << 30, 1 << 20, buf, buf, None) == B.BSPL_EUNSUPPORTED
    # grid values are unpadded: the two flags exclude each other
    h = ctypes.c_void_p(7)
    assert B.lib.spline_table_create(ctypes.byref(h), 1, 1, 1, 8, buf, 0, None,
                                     B.BSPL_COEFS_PADDED | B.BSPL_COEFS_GRID_VALUES,
                                     None) == B.BSPL_EINVAL
    assert h.value is None
    assert "GRID_VALUES" in B.spline_last_error()


def test_table_info_struct_matches_header():
    text = open(HEADER).read()
    body = text[text.index("typedef struct {\n    int32_t nx, ny, nz;"):]
    body = body[:body.index("} bspl_table_info;")]
    fields = []
    for m in re.finditer(r"^\s+(?:const )?\w+\*? ?\*?\s*([\w, \[\]0-9]+);", body, re.M):
        for name in m.group(1).split(","):
            fields.append(re.sub(r"\[\d+\]", "", name).strip())
    assert fields == [f for f, _ in B.bspl_table_info._fields_]


def test_tile_struct_matches_header():
    text = open(HEADER).read()
    body = text[text.index("typedef struct {\n    int32_t vw;"):]
    body = body[:body.index("} bspl_tile;")]
    fields = re.findall(r"int32_t (\w+);", body)
    assert fields == [f for f, _ in B.bspl_tile._fields_]


def test_null_handles():
    assert B.lib.spline_table_destroy(None) == B.BSPL_OK
    assert B.lib.spline_batch_plan_destroy(None) == B.BSPL_OK
    info = B.bspl_table_info()
    assert B.lib.spline_table_info(None, ctypes.byref(info)) == B.BSPL_EINVAL
    for fn in ("spline_eval_v",):
        assert getattr(B.lib, fn)(None, 1, None, None, 1, None) == B.BSPL_EINVAL
    assert B.lib.spline_eval_vgh(None, 1, None, None, None, None, 1, None) == B.BSPL_EINVAL
    assert B.lib.spline_eval_vgl(None, 1, None, None, None, None, 1, None) == B.BSPL_EINVAL
    assert B.lib.spline_eval(None, 2, 1, None, None, None, None, 1, None, None) == B.BSPL_EINVAL
    t = B.bspl_tile()
    assert B.lib.spline_tile_select(None, 0, 1, ctypes.byref(t)) == B.BSPL_EINVAL
    assert B.lib.spline_autotune(None, 0, 1, None, None, None) == B.BSPL_EINVAL
    assert B.lib.spline_batch_execute(None, None) == B.BSPL_EINVAL
    assert B.lib.spline_batch_launch(None, None) == B.BSPL_EINVAL
    assert B.lib.spline_batch_rebind(None, 0, None, None, None, None) == B.BSPL_EINVAL
    assert B.lib.spline_batch_plan_tile(None, ctypes.byref(t)) == B.BSPL_EINVAL
    assert B.lib.spline_eval_noalloc(None, 2, 1, None, None, None, None, 1, None,
                                     None) == B.BSPL_EINVAL


def test_stream_probe_argument_checks():
    """The bandwidth probe validates everything before its launch."""
    f = B.lib.spline_stream_probe
    assert f(None, None, 0, 1, 0, 0, 0, None) == B.BSPL_OK        # nothing to move
    assert f(None, None, -1, 1, 0, 0, 0, None) == B.BSPL_EINVAL
    assert f(None, None, 10, 1, 0, 0, 0, None) == B.BSPL_EINVAL   # NULL buffers
    assert f(None, None, 0, 3, 0, 0, 0, None) == B.BSPL_EINVAL    # per_lane not 1, 2, 4
    assert f(None, None, 0, 1, -1, 0, 0, None) == B.BSPL_EINVAL
    assert f(None, None, 0, 1, 0, 0x8, 0, None) == B.BSPL_EINVAL
    for fl in (B.BSPL_PROBE_CHUNKED, B.BSPL_PROBE_RANDOM):
        assert f(1, 1, 100, 1, 0, fl, 0, None) == B.BSPL_EINVAL   # not a multiple of 64
    assert f(1, 1, 1 << 62, 1, 0, 0, 0, None) == B.BSPL_EUNSUPPORTED

def test_batch_plan_argument_checks():
    h = ctypes.c_void_p()
    z64 = (ctypes.c_int64 * 17)()
    zp = (ctypes.c_void_p * 17)()
    args = (zp, z64, 2, zp, zp, zp, zp, z64, None, None, None)
    assert B.lib.spline_batch_plan_create(ctypes.byref(h), 0, *args) == B.BSPL_EINVAL
    assert B.lib.spline_batch_plan_create(ctypes.byref(h), 17, *args) == B.BSPL_EINVAL
    assert B.lib.spline_batch_plan_create(None, 1, *args) == B.BSPL_EINVAL
    # NULL table pointer inside the array
    assert B.lib.spline_batch_plan_create(ctypes.byref(h), 1, *args) == B.BSPL_EINVAL
    assert "table 0" in B.spline_last_error()


def test_wisdom_files(tmp_path):
    missing = str(tmp_path / "missing.txt")
    with pytest.raises(B.BsplineError) as e:
        B.spline_wisdom_load(missing)
    assert e.value.status == B.BSPL_EIO
    p = tmp_path / "w.txt"
    p.write_text("# comment\nsingle|gfx950|f32|vgh|N64|16x16x16|p1024 2 2 1 0 1 1 12.5\n"
                 "single|gfx950|f32|vgh|N64|16x16x16|p1 1 2 1 0 0 4\n"
                 "garbage line\nsingle|gfx950|f32|v|N64|16x16x16|p8 1 1 1 0\n")
    B.spline_wisdom_load(str(p))
    out = str(tmp_path / "out.txt")
    B.spline_wisdom_save(out)
    text = open(out).read()
    # a line's time survives a load and save; a line without one stays without
    assert "single|gfx950|f32|vgh|N64|16x16x16|p1024 2 2 1 0 1 1 12.500\n" in text
    assert "single|gfx950|f32|vgh|N64|16x16x16|p1 1 2 1 0 0 4\n" in text
    assert "|v|" not in text  # a line with too few fields is skipped
    with pytest.raises(B.BsplineError) as e:
        B.spline_wisdom_save(str(tmp_path / "no" / "such" / "dir.txt"))
    assert e.value.status == B.BSPL_EIO


def test_missing_library_fails_loudly(tmp_path):
    """Without the compiled library the binding refuses to import: there is
    no CPU fallback to silently run instead."""
    import shutil
    import subprocess
    import sys
    pkg = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1611_02665_amd")
    copy = tmp_path / "paper_1611_02665_amd"
    copy.mkdir()
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            shutil.copy(os.path.join(pkg, f), copy / f)
    r = subprocess.run([sys.executable, "-c", "import paper_1611_02665_amd.binding"],
                       cwd=tmp_path, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libbspline.so is missing" in r.stderr


def test_launch_query_limits_without_a_device():
    """The size limits spline_eval checks before any HIP call, on a layout
    from the host-only query: npos >= 2^31, more than 2^31 - 1 work blocks
    and split launches beyond 2^32 - 1 work-items are EUNSUPPORTED; grids
    beyond one dispatch become persistent grids."""
    lay = B.spline_layout_query(4, 4, 4, 700, "f32")
    # 700 splines at vw = 1: 11 tiles of 64; wx = 1 -> 11 blocks per position
    for npos, tile in (((1 << 31), None), ((1 << 31), (1, 1, 1, 0, 0, 1)),
                       ((1 << 31) - 1, (1, 1, 1, 0, 0, 1)), ((1 << 31) - 1, None)):
        with pytest.raises(B.BsplineError) as e:
            B.spline_launch_query(lay, "vgh", npos, tile)
        assert e.value.status == B.BSPL_EUNSUPPORTED, (npos, tile)
    # the largest batch that fits: 2^31 - 1 blocks of one tile x one position
    npos = (2**31 - 1) // 11
    q = B.spline_launch_query(lay, "vgh", npos, (1, 1, 1, 0, 0, 1))
    assert q["units"] == 11 * npos and q["threads"] == 64
    assert q["workgroups"] * 64 <= 2**32 - 1 < q["units"] * 64  # persistent grid
    # eight wavefronts per workgroup: at most 2^32 / 512 workgroups
    q = B.spline_launch_query(lay, "vgh", npos, (1, 1, 8, 0, 0, 1))
    assert q["threads"] == 512 and q["workgroups"] == (2**32 - 1) // 512
    # a requested persistent grid below the cap is kept
    q = B.spline_launch_query(lay, "v", 1000, (1, 2, 1, 512, 0, 1))
    assert q == {"units": 6 * 1000, "workgroups": 512, "threads": 128}
    # split tiles have no striding loop: their work-items are bounded
    q = B.spline_launch_query(lay, "vgh", 1000, (1, 1, 1, 0, 0, 4))
    assert q == {"units": 11 * 1000, "workgroups": 11 * 1000, "threads": 256}
    with pytest.raises(B.BsplineError) as e:
        B.spline_launch_query(lay, "vgh", (2**32 // 256) // 11 + 1, (1, 1, 1, 0, 0, 4))
    assert e.value.status == B.BSPL_EUNSUPPORTED
    # the default tile (NULL): split 4 for a handful of positions, else wx up to 4
    assert B.spline_launch_query(lay, "vgh", 8)["threads"] == 256
    q = B.spline_launch_query(lay, "vgh", 100)
    assert q == {"units": 3 * 100, "workgroups": 300, "threads": 256}
    # npos = 0: nothing to launch
    assert B.spline_launch_query(lay, "v", 0, (1, 1, 1, 0, 0, 1))["workgroups"] == 0
    # orders 3 and 4 (spline-tile-major) are valid tiles; order 5 is not, and
    # split units keep orders 0..2
    for order in (3, 4):
        q = B.spline_launch_query(lay, "vgh", 10, (1, 1, 1, 0, order, 1))
        assert q["units"] == 11 * 10
    for bad in ((3, 1, 1, 0, 0, 1), (1, 1, 1, 0, 5, 1), (1, 4, 1, 0, 0, 4),
                (1, 1, 1, 0, 3, 4), (1, 1, 1, 0, -1, 1)):
        with pytest.raises(B.BsplineError) as e:
            B.spline_launch_query(lay, "vgh", 10, bad)
        assert e.value.status == B.BSPL_EINVAL, bad
    for kind, npos in ((7, 10), ("vgh", -1)):
        with pytest.raises(B.BsplineError) as e:
            B.spline_launch_query(lay, kind, npos)
        assert e.value.status == B.BSPL_EINVAL
    assert B.lib.spline_launch_query(None, B.BSPL_V, 1, None, None, None, None) == B.BSPL_EINVAL
    # FP16 tables take their own vector widths (2, 4, 8)
    lay16 = B.spline_layout_query(48, 48, 48, 2048, "f16")
    assert B.spline_launch_query(lay16, "vgh", 4096, (2, 4, 2, 0, 1, 1))["units"] == 4 * 2048
    with pytest.raises(B.BsplineError):
        B.spline_launch_query(lay16, "vgh", 4096, (1, 4, 2, 0, 1, 1))
