"""Python access to the FP64 CPU oracle (``bspline_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never calls it, and it shares no code with the GPU library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bspline_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

V, VGL, VGH = 0, 1, 2
KINDS = {"v": V, "vgl": VGL, "vgh": VGH}

_lib = None


def compile_source(src: str, out: str) -> str:
    """Compile an oracle source file with gcc (plain -O2, OpenMP)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-I", _HERE, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle library next to its source."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


def _bind(path: str):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_basis.argtypes = [ctypes.c_double, dp, dp, dp]
    lib.oracle_weights.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp, dp]
    lib.oracle_locate.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int), dp]
    lib.oracle_locate.restype = ctypes.c_int
    lib.oracle_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                dp, ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int64]
    lib.oracle_eval.restype = ctypes.c_int
    lib.oracle_eval_bruteforce.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int64, dp, dp, ctypes.c_int64, dp,
                                           dp, dp, dp, dp, ctypes.c_int64]
    lib.oracle_eval_bruteforce.restype = ctypes.c_int
    lib.oracle_eval_ratio.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, dp,
                                      ctypes.c_int64, dp, dp, ctypes.c_int64, dp]
    lib.oracle_eval_ratio.restype = ctypes.c_int
    lib.oracle_eval_lattice.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp, dp, dp,
                                        ctypes.c_int64]
    lib.oracle_eval_lattice.restype = ctypes.c_int
    lib.oracle_fit_interpolating.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int64, dp, dp]
    lib.oracle_fit_interpolating.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _bind(_LIB)
    return _lib


class Oracle:
    """The oracle's functions bound to one compiled library file."""

    def __init__(self, path: str | None = None):
        self._path = path

    def _l(self):
        return _bind(self._path) if self._path else _load()

    def weights(self, t, delta=1.0):
        return weights(t, delta, _lib_=self._l())

    def evaluate(self, kind, coef, pos, box=(1.0, 1.0, 1.0), padded=False):
        return evaluate(kind, coef, pos, box, padded, _lib_=self._l())

    def evaluate_bruteforce(self, coef, pos, box=(1.0, 1.0, 1.0)):
        return evaluate_bruteforce(coef, pos, box, _lib_=self._l())

    def evaluate_ratio(self, kind, coef, pos, ainv, box=(1.0, 1.0, 1.0)):
        return evaluate_ratio(kind, coef, pos, ainv, box, _lib_=self._l())

    def evaluate_lattice(self, kind, coef, pos, lattice, padded=False):
        return evaluate_lattice(kind, coef, pos, lattice, padded, _lib_=self._l())

    def fit_interpolating(self, values):
        return fit_interpolating(values, _lib_=self._l())


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def basis(s: float):
    lib = _load()
    b, db, d2b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.oracle_basis(float(s), ctypes.byref(b), ctypes.byref(db), ctypes.byref(d2b))
    return b.value, db.value, d2b.value


def weights(t: float, delta: float = 1.0, _lib_=None):
    lib = _lib_ or _load()
    w, dw, d2w = (np.zeros(4) for _ in range(3))
    lib.oracle_weights(float(t), float(delta), _dp(w), _dp(dw), _dp(d2w))
    return w, dw, d2w


def locate(x: float, box_len: float, n: int):
    lib = _load()
    i0, t = ctypes.c_int(), ctypes.c_double()
    rc = lib.oracle_locate(float(x), float(box_len), int(n), ctypes.byref(i0), ctypes.byref(t))
    if rc != 0:
        raise ValueError("position has no fraction bits or is not finite")
    return i0.value, t.value


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def _outputs(kind, npos, ncoef):
    v = np.empty((npos, ncoef))
    g = np.empty((npos, 3, ncoef)) if kind >= VGL else None
    l = np.empty((npos, ncoef)) if kind == VGL else None
    h = np.empty((npos, 6, ncoef)) if kind == VGH else None
    return v, g, l, h


def evaluate(kind, coef: np.ndarray, pos: np.ndarray, box=(1.0, 1.0, 1.0),
             padded: bool = False, _lib_=None) -> dict:
    """Evaluate V / VGL / VGH for all positions and all spline columns.

    ``coef`` is ``[nx][ny][nz][N]`` (periodic, unpadded) or, with
    ``padded=True``, ``[nx+3][ny+3][nz+3][N]``; float32 or float64.
    ``pos`` is ``[3][npos]`` float64.  Returns FP64 arrays ``v [npos][N]``,
    ``g [npos][3][N]``, ``l [npos][N]``, ``h [npos][6][N]`` as the kind asks.
    """
    kind = KINDS.get(kind, kind)
    lib = _lib_ or _load()
    coef = np.ascontiguousarray(coef)
    if coef.dtype == np.float32:
        cdt = 1
    else:
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        cdt = 0
    nx, ny, nz, ncoef = coef.shape
    if padded:
        nx, ny, nz = nx - 3, ny - 3, nz - 3
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    npos = pos.shape[1]
    v, g, l, h = _outputs(kind, npos, ncoef)
    bx = np.asarray(box, dtype=np.float64)
    rc = lib.oracle_eval(kind, nx, ny, nz, ncoef, coef.ctypes.data_as(ctypes.c_void_p), cdt,
                         1 if padded else 0, _dp(bx), npos, _dp(pos),
                         _dp(v), _dp(g), _dp(l), _dp(h), ncoef)
    if rc != 0:
        raise ValueError("oracle_eval rejected its arguments")
    out = {"v": v}
    if g is not None:
        out["g"] = g
    if l is not None:
        out["l"] = l
    if h is not None:
        out["h"] = h
    return out


def evaluate_bruteforce(coef: np.ndarray, pos: np.ndarray, box=(1.0, 1.0, 1.0),
                        _lib_=None) -> dict:
    """Brute-force V, G, L, H over all grid points and periodic images."""
    lib = _lib_ or _load()
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    nx, ny, nz, ncoef = coef.shape
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    npos = pos.shape[1]
    v = np.empty((npos, ncoef))
    g = np.empty((npos, 3, ncoef))
    l = np.empty((npos, ncoef))
    h = np.empty((npos, 6, ncoef))
    bx = np.asarray(box, dtype=np.float64)
    rc = lib.oracle_eval_bruteforce(nx, ny, nz, ncoef, _dp(coef), _dp(bx), npos, _dp(pos),
                                    _dp(v), _dp(g), _dp(l), _dp(h), ncoef)
    if rc != 0:
        raise ValueError("oracle_eval_bruteforce rejected its arguments")
    return {"v": v, "g": g, "l": l, "h": h}


def evaluate_ratio(kind, coef: np.ndarray, pos: np.ndarray, ainv: np.ndarray,
                   box=(1.0, 1.0, 1.0), _lib_=None) -> np.ndarray:
    """Determinant ratios ``[npos][ncomp]``: sum_n X_{c,n}(r_p) * ainv[p][n]."""
    kind = KINDS.get(kind, kind)
    lib = _lib_ or _load()
    coef = np.ascontiguousarray(coef)
    if coef.dtype == np.float32:
        cdt = 1
    else:
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        cdt = 0
    nx, ny, nz, ncoef = coef.shape
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    npos = pos.shape[1]
    ainv = np.ascontiguousarray(ainv, dtype=np.float64)
    if ainv.shape[0] != npos or ainv.shape[1] < ncoef:
        raise ValueError("ainv must be [npos][>= N]")
    ncomp = {V: 1, VGL: 5, VGH: 10}[kind]
    out = np.empty((npos, ncomp))
    bx = np.asarray(box, dtype=np.float64)
    rc = lib.oracle_eval_ratio(kind, nx, ny, nz, ncoef, coef.ctypes.data_as(ctypes.c_void_p), cdt,
                               _dp(bx), npos, _dp(pos), _dp(ainv), ainv.shape[1], _dp(out))
    if rc != 0:
        raise ValueError("oracle_eval_ratio rejected its arguments")
    return out


def evaluate_lattice(kind, coef: np.ndarray, pos: np.ndarray, lattice, padded: bool = False,
                     _lib_=None) -> dict:
    """V / VGL / VGH on a general cell; ``lattice`` rows are the cell vectors."""
    kind = KINDS.get(kind, kind)
    lib = _lib_ or _load()
    coef = np.ascontiguousarray(coef)
    if coef.dtype == np.float32:
        cdt = 1
    else:
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        cdt = 0
    nx, ny, nz, ncoef = coef.shape
    if padded:
        nx, ny, nz = nx - 3, ny - 3, nz - 3
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    npos = pos.shape[1]
    v, g, l, h = _outputs(kind, npos, ncoef)
    lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
    rc = lib.oracle_eval_lattice(kind, nx, ny, nz, ncoef, coef.ctypes.data_as(ctypes.c_void_p),
                                 cdt, 1 if padded else 0, _dp(lat), npos, _dp(pos), _dp(v),
                                 _dp(g), _dp(l), _dp(h), ncoef)
    if rc != 0:
        raise ValueError("oracle_eval_lattice rejected its arguments")
    out = {"v": v}
    if g is not None:
        out["g"] = g
    if l is not None:
        out["l"] = l
    if h is not None:
        out["h"] = h
    return out


def fit_interpolating(values: np.ndarray, _lib_=None) -> np.ndarray:
    """Periodic coefficients [nx][ny][nz][N] whose spline equals ``values``
    (same shape) at the grid points."""
    lib = _lib_ or _load()
    values = np.ascontiguousarray(values, dtype=np.float64)
    nx, ny, nz, n = values.shape
    out = np.empty_like(values)
    if lib.oracle_fit_interpolating(nx, ny, nz, n, _dp(values), _dp(out)) != 0:
        raise ValueError("oracle_fit_interpolating rejected its arguments")
    return out
