"""ctypes binding of ``libbspline.so`` (argument marshalling only).

Every function keeps the C name.  Pointer arguments accept a torch tensor
(its ``data_ptr()``), a plain integer address, or ``None`` (NULL).  Streams
default to torch's current stream on the current device.  A non-OK status
raises :class:`BsplineError`.  There is no fallback: if the library has not
been built, importing this module fails.
"""

from __future__ import annotations

import ctypes
import os

try:  # load torch's HIP runtime first so that libbspline binds to the same one
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - the CPU-only checks need no torch
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbspline.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "or python -m paper_1611_02665_amd.build")

BSPL_OK, BSPL_EINVAL, BSPL_ENOMEM, BSPL_EDEVICE, BSPL_EUNSUPPORTED, BSPL_EIO = range(6)
BSPL_F32, BSPL_F16, BSPL_BF16 = 0, 1, 2
BSPL_V, BSPL_VGL, BSPL_VGH = 0, 1, 2
BSPL_COEFS_PADDED = 0x1
BSPL_COEFS_DEVICE = 0x2
BSPL_COEFS_GRID_VALUES = 0x4
BSPL_LAYOUT_BLOCKED = 0x8
MAX_TABLES = 16
NOALLOC_MAX_POSITIONS = 1 << 20
BSPL_PROBE_NT_STORES = 0x1
BSPL_PROBE_CHUNKED = 0x2
BSPL_PROBE_RANDOM = 0x4

DTYPES = {"f32": BSPL_F32, "f16": BSPL_F16, "bf16": BSPL_BF16}
KINDS = {"v": BSPL_V, "vgl": BSPL_VGL, "vgh": BSPL_VGH}
NCOMP = {BSPL_V: 1, BSPL_VGL: 5, BSPL_VGH: 10}


class bspl_table_info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("px", ctypes.c_int32), ("py", ctypes.c_int32), ("pz", ctypes.c_int32),
                ("n_splines", ctypes.c_int64), ("n_padded", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("elem_bytes", ctypes.c_int32),
                ("row_bytes", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("box", ctypes.c_double * 3), ("lattice", ctypes.c_double * 9),
                ("data", ctypes.c_void_p),
                ("scales", ctypes.c_void_p),
                ("block_splines", ctypes.c_int64), ("block_bytes", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["box"] = tuple(self.box)
        d["lattice"] = tuple(self.lattice)
        return d


class bspl_tile(ctypes.Structure):
    _fields_ = [("vw", ctypes.c_int32), ("wx", ctypes.c_int32), ("wy", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("order", ctypes.c_int32), ("split", ctypes.c_int32)]

    def as_tuple(self):
        return (self.vw, self.wx, self.wy, self.grid, self.order, self.split)

    def __repr__(self):
        return (f"bspl_tile(vw={self.vw}, wx={self.wx}, wy={self.wy}, grid={self.grid}, "
                f"order={self.order}, split={self.split})")


lib = ctypes.CDLL(LIB_PATH)

_vp, _i64, _int, _u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint
_P = ctypes.POINTER
_SIGS = {
    "spline_status_string": (ctypes.c_char_p, [_int]),
    "spline_last_error": (ctypes.c_char_p, []),
    "spline_layout_query": (_int, [_int, _int, _int, _i64, _int, ctypes.c_uint,
                                   _P(bspl_table_info)]),
    "spline_layout_select": (_int, [_int, _int, _int, _i64, _int, _int, _i64, ctypes.c_char_p,
                                    _P(ctypes.c_uint), _vp]),
    "spline_table_create": (_int, [_P(_vp), _int, _int, _int, _i64, _vp, _int,
                                   _P(ctypes.c_double), _u32, _vp]),
    "spline_fit_interpolating": (_int, [_int, _int, _int, _i64, _vp, _vp, _vp]),
    "spline_table_create_lattice": (_int, [_P(_vp), _int, _int, _int, _i64, _vp, _int,
                                           _P(ctypes.c_double), _u32, _vp]),
    "spline_table_destroy": (_int, [_vp]),
    "spline_table_info": (_int, [_vp, _P(bspl_table_info)]),
    "spline_eval_v": (_int, [_vp, _i64, _vp, _vp, _i64, _vp]),
    "spline_eval_vgl": (_int, [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp]),
    "spline_eval_vgh": (_int, [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp]),
    "spline_eval": (_int, [_vp, _int, _i64, _vp, _vp, _vp, _vp, _i64, _P(bspl_tile), _vp]),
    "spline_eval_noalloc": (_int, [_vp, _int, _i64, _vp, _vp, _vp, _vp, _i64, _P(bspl_tile),
                                   _vp]),
    "spline_eval_ratio": (_int, [_vp, _int, _i64, _vp, _vp, _i64, _vp, _P(bspl_tile), _vp]),
    "spline_launch_query": (_int, [_P(bspl_table_info), _int, _i64, _P(bspl_tile), _P(_i64),
                                   _P(_i64), _P(ctypes.c_int32)]),
    "spline_tile_select": (_int, [_vp, _int, _i64, _P(bspl_tile)]),
    "spline_autotune": (_int, [_vp, _int, _i64, ctypes.c_char_p, _P(bspl_tile), _vp]),
    "spline_wisdom_load": (_int, [ctypes.c_char_p]),
    "spline_wisdom_save": (_int, [ctypes.c_char_p]),
    "spline_batch_plan_create": (_int, [_P(_vp), _int, _P(_vp), _P(_i64), _int, _P(_vp),
                                        _P(_vp), _P(_vp), _P(_vp), _P(_i64), _P(bspl_tile),
                                        ctypes.c_char_p, _vp]),
    "spline_batch_execute": (_int, [_vp, _vp]),
    "spline_batch_launch": (_int, [_vp, _vp]),
    "spline_batch_rebind": (_int, [_vp, _int, _vp, _vp, _vp, _vp]),
    "spline_batch_plan_tile": (_int, [_vp, _P(bspl_tile)]),
    "spline_batch_plan_destroy": (_int, [_vp]),
    "spline_stream_probe": (_int, [_vp, _vp, _i64, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_uint64, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class BsplineError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.spline_status_string(status).decode()
        detail = lib.spline_last_error().decode()
        super().__init__(f"{where}: {msg}" + (f" ({detail})" if detail else ""))


def _check(status: int, where: str) -> None:
    if status != BSPL_OK:
        raise BsplineError(status, where)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    dp = getattr(x, "data_ptr", None)
    if dp is not None:
        return dp()
    if hasattr(x, "ctypes"):  # numpy array on the host
        return x.ctypes.data
    raise TypeError(f"cannot take an address of {type(x)!r}")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _enum(x, table):
    return table[x] if isinstance(x, str) else int(x)


def spline_status_string(status: int) -> str:
    return lib.spline_status_string(status).decode()


def spline_last_error() -> str:
    return lib.spline_last_error().decode()


def spline_layout_query(nx, ny, nz, n_splines, dtype="f32", flags=0) -> dict:
    info = bspl_table_info()
    _check(lib.spline_layout_query(nx, ny, nz, n_splines, _enum(dtype, DTYPES), flags,
                                   ctypes.byref(info)), "spline_layout_query")
    return info.as_dict()


def spline_layout_select(nx, ny, nz, n_splines, dtype, kind, npos, wisdom_path=None,
                         stream=None) -> int:
    """0 (plain) or BSPL_LAYOUT_BLOCKED, whichever runs this shape faster."""
    out = ctypes.c_uint(0)
    wp = wisdom_path.encode() if wisdom_path else None
    _check(lib.spline_layout_select(nx, ny, nz, n_splines, _enum(dtype, DTYPES),
                                    _enum(kind, KINDS), npos, wp, ctypes.byref(out),
                                    _stream(stream)), "spline_layout_select")
    return out.value


def spline_table_create(nx, ny, nz, n_splines, coefs, dtype="f32", box=None, flags=0,
                        stream=None) -> int:
    """Returns the table handle (an integer address).  ``coefs`` is a host
    numpy float32 array, or a device tensor with ``BSPL_COEFS_DEVICE``."""
    h = ctypes.c_void_p()
    bx = (ctypes.c_double * 3)(*box) if box is not None else None
    _check(lib.spline_table_create(ctypes.byref(h), nx, ny, nz, n_splines, _ptr(coefs),
                                   _enum(dtype, DTYPES), bx, flags, _stream(stream)),
           "spline_table_create")
    return h.value


def spline_table_create_lattice(nx, ny, nz, n_splines, coefs, lattice, dtype="f32", flags=0,
                                stream=None) -> int:
    """Table on a general cell; ``lattice`` holds the cell vectors as rows."""
    h = ctypes.c_void_p()
    lat = (ctypes.c_double * 9)(*[float(x) for x in list(lattice[0]) + list(lattice[1])
                                  + list(lattice[2])]) if len(lattice) == 3 else \
        (ctypes.c_double * 9)(*[float(x) for x in lattice])
    _check(lib.spline_table_create_lattice(ctypes.byref(h), nx, ny, nz, n_splines, _ptr(coefs),
                                           _enum(dtype, DTYPES), lat, flags, _stream(stream)),
           "spline_table_create_lattice")
    return h.value


def spline_fit_interpolating(nx, ny, nz, n_splines, values, coefs, stream=None) -> None:
    """Device arrays [nx][ny][nz][n_splines]; coefs may be values (in place)."""
    _check(lib.spline_fit_interpolating(nx, ny, nz, n_splines, _ptr(values), _ptr(coefs),
                                        _stream(stream)), "spline_fit_interpolating")


def spline_table_destroy(table) -> None:
    _check(lib.spline_table_destroy(table), "spline_table_destroy")


def spline_table_info(table) -> dict:
    info = bspl_table_info()
    _check(lib.spline_table_info(table, ctypes.byref(info)), "spline_table_info")
    return info.as_dict()


def spline_eval_v(table, npos, pos, v, ldo, stream=None) -> None:
    _check(lib.spline_eval_v(table, npos, _ptr(pos), _ptr(v), ldo, _stream(stream)),
           "spline_eval_v")


def spline_eval_vgl(table, npos, pos, v, g, l, ldo, stream=None) -> None:
    _check(lib.spline_eval_vgl(table, npos, _ptr(pos), _ptr(v), _ptr(g), _ptr(l), ldo,
                               _stream(stream)), "spline_eval_vgl")


def spline_eval_vgh(table, npos, pos, v, g, h, ldo, stream=None) -> None:
    _check(lib.spline_eval_vgh(table, npos, _ptr(pos), _ptr(v), _ptr(g), _ptr(h), ldo,
                               _stream(stream)), "spline_eval_vgh")


def _tile(tile):
    if tile is None:
        return None
    if isinstance(tile, bspl_tile):
        return ctypes.byref(tile)
    return ctypes.byref(bspl_tile(*tile))


def spline_eval(table, kind, npos, pos, v, g=None, lh=None, ldo=None, tile=None,
                stream=None) -> None:
    _check(lib.spline_eval(table, _enum(kind, KINDS), npos, _ptr(pos), _ptr(v), _ptr(g),
                           _ptr(lh), ldo, _tile(tile), _stream(stream)), "spline_eval")


def spline_eval_noalloc(table, kind, npos, pos, v, g=None, lh=None, ldo=None, tile=None,
                        stream=None) -> None:
    _check(lib.spline_eval_noalloc(table, _enum(kind, KINDS), npos, _ptr(pos), _ptr(v), _ptr(g),
                                   _ptr(lh), ldo, _tile(tile), _stream(stream)),
           "spline_eval_noalloc")


def spline_eval_ratio(table, kind, npos, pos, ainv, ld_ainv, out, tile=None, stream=None) -> None:
    _check(lib.spline_eval_ratio(table, _enum(kind, KINDS), npos, _ptr(pos), _ptr(ainv), ld_ainv,
                                 _ptr(out), _tile(tile), _stream(stream)), "spline_eval_ratio")


def spline_launch_query(layout: dict, kind, npos, tile=None) -> dict:
    """Host-only launch shape of an evaluation on a table of this layout (a
    dict from spline_layout_query or spline_table_info): work blocks,
    workgroups launched and threads per workgroup."""
    info = bspl_table_info()
    for k, _ in bspl_table_info._fields_:
        val = layout[k]
        if k in ("box", "lattice"):
            getattr(info, k)[:] = list(val)
        else:
            setattr(info, k, val)
    units, wgs, thr = _i64(), _i64(), ctypes.c_int32()
    _check(lib.spline_launch_query(ctypes.byref(info), _enum(kind, KINDS), npos, _tile(tile),
                                   ctypes.byref(units), ctypes.byref(wgs), ctypes.byref(thr)),
           "spline_launch_query")
    return {"units": units.value, "workgroups": wgs.value, "threads": thr.value}


def spline_tile_select(table, kind, npos) -> bspl_tile:
    t = bspl_tile()
    _check(lib.spline_tile_select(table, _enum(kind, KINDS), npos, ctypes.byref(t)),
           "spline_tile_select")
    return t


def spline_autotune(table, kind, npos, wisdom_path=None, stream=None) -> bspl_tile:
    t = bspl_tile()
    wp = wisdom_path.encode() if wisdom_path else None
    _check(lib.spline_autotune(table, _enum(kind, KINDS), npos, wp, ctypes.byref(t),
                               _stream(stream)), "spline_autotune")
    return t


def spline_wisdom_load(path) -> None:
    _check(lib.spline_wisdom_load(path.encode()), "spline_wisdom_load")


def spline_wisdom_save(path) -> None:
    _check(lib.spline_wisdom_save(path.encode()), "spline_wisdom_save")


def spline_batch_plan_create(tables, npos, kind, pos, v, g=None, lh=None, ldo=None,
                             tile=None, wisdom_path=None, stream=None) -> int:
    n = len(tables)
    arr = lambda ty, xs: (ty * n)(*xs)  # noqa: E731
    g = g if g is not None else [None] * n
    lh = lh if lh is not None else [None] * n
    h = ctypes.c_void_p()
    wp = wisdom_path.encode() if wisdom_path else None
    _check(lib.spline_batch_plan_create(
        ctypes.byref(h), n, arr(_vp, tables), arr(_i64, npos), _enum(kind, KINDS),
        arr(_vp, [_ptr(x) for x in pos]), arr(_vp, [_ptr(x) for x in v]),
        arr(_vp, [_ptr(x) for x in g]), arr(_vp, [_ptr(x) for x in lh]),
        arr(_i64, ldo), _tile(tile), wp, _stream(stream)), "spline_batch_plan_create")
    return h.value


def spline_batch_execute(plan, stream=None) -> None:
    _check(lib.spline_batch_execute(plan, _stream(stream)), "spline_batch_execute")


def spline_batch_launch(plan, stream=None) -> None:
    _check(lib.spline_batch_launch(plan, _stream(stream)), "spline_batch_launch")


def spline_batch_rebind(plan, i, pos, v, g=None, lh=None) -> None:
    _check(lib.spline_batch_rebind(plan, i, _ptr(pos), _ptr(v), _ptr(g), _ptr(lh)),
           "spline_batch_rebind")


def spline_batch_plan_tile(plan) -> bspl_tile:
    t = bspl_tile()
    _check(lib.spline_batch_plan_tile(plan, ctypes.byref(t)), "spline_batch_plan_tile")
    return t


def spline_batch_plan_destroy(plan) -> None:
    _check(lib.spline_batch_plan_destroy(plan), "spline_batch_plan_destroy")


def spline_stream_probe(src, dst, units, per_lane=1, grid=0, flags=0, salt=0,
                        stream=None) -> None:
    """Measurement helper (bspline_probe.h): 6 reads of 16 bytes per 16-byte
    write; src holds 6 * units words, dst units words."""
    _check(lib.spline_stream_probe(_ptr(src), _ptr(dst), units, per_lane, grid, flags, salt,
                                   _stream(stream)), "spline_stream_probe")
