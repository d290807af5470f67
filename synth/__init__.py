"""Seeded synthetic inputs shared by the oracle checks and the GPU path.

This module only draws random numbers: it holds none of the B-spline
arithmetic.  Both sides of every comparison take their coefficient tables and
electron positions from here, so that they see bit-identical inputs.

Generator: a counter-based hash built from the SplitMix64 output function
(Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014; constants as published by Vigna for splitmix64).  Value ``i`` of
stream ``s`` under seed ``seed`` is

    key   = mix64(mix64(seed) ^ ((s + 1) * GAMMA))
    h(i)  = mix64(key + (i + 1) * GAMMA)          (all arithmetic mod 2**64)

Coefficients take the top 24 bits ``k`` of ``h`` and map them to
``(2k + 1 - 2**24) / 2**24``: symmetric in (-1, 1) and exact in FP32.
Positions take the top 53 bits and map them to ``k * 2**-53`` in [0, 1), FP64.

Workload recipe (paper's miniQMC: random positions on a fixed read-only
table, grid 48^3, N = 128 ... 4096 splines):
  * table ``t`` of a workload draws its unpadded coefficients from stream
    ``2t``; the flat counter is ``((ix*ny + iy)*nz + iz)*N + n``;
  * position batch ``b`` of table ``t`` draws from stream ``2t + 1`` with
    counter ``(b * 2**32 + p) * 4 + d`` for coordinate ``d`` of position ``p``.
"""

from __future__ import annotations

import numpy as np

SEED = 161102665

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to a uint64 array."""
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = mix64(np.array([seed], dtype=np.uint64))
        k = mix64(s ^ (np.array([stream + 1], dtype=np.uint64) * _GAMMA))
    return k[0]


def hash_at(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Raw 64-bit hash of counters ``idx`` (uint64 array) in one stream."""
    key = stream_key(seed, stream)
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + (idx + np.uint64(1)) * _GAMMA)


def unit_symmetric_f32(h: np.ndarray) -> np.ndarray:
    """Top 24 bits of ``h`` -> (2k+1-2^24)/2^24, exactly representable in FP32."""
    k = (h >> np.uint64(40)).astype(np.int64)
    return ((2 * k + 1 - (1 << 24)).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def unit_f64(h: np.ndarray) -> np.ndarray:
    """Top 53 bits of ``h`` -> k * 2^-53 in [0, 1)."""
    return (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def coef_values(seed: int, stream: int, flat_index: np.ndarray) -> np.ndarray:
    """Coefficients at arbitrary flat unpadded indices (FP32)."""
    return unit_symmetric_f32(hash_at(seed, stream, flat_index))


def coef_table(nx: int, ny: int, nz: int, nsplines: int, *, seed: int = SEED,
               stream: int = 0, splines=None, chunk: int = 1 << 24) -> np.ndarray:
    """Unpadded periodic coefficient table ``[nx][ny][nz][Ns]`` (FP32).

    ``splines`` selects a subset of spline columns (their values are those of
    the full ``nsplines``-wide table), so that sampled checks on very large
    tables need not materialise every column.
    """
    cols = np.arange(nsplines, dtype=np.uint64) if splines is None \
        else np.asarray(splines, dtype=np.uint64)
    if cols.size and int(cols.max()) >= nsplines:
        raise ValueError("spline index out of range")
    ncell = nx * ny * nz
    out = np.empty((ncell, cols.size), dtype=np.float32)
    rows_per = max(1, chunk // max(1, cols.size))
    for r0 in range(0, ncell, rows_per):
        r1 = min(ncell, r0 + rows_per)
        cell = np.arange(r0, r1, dtype=np.uint64)[:, None]
        with np.errstate(over="ignore"):
            flat = cell * np.uint64(nsplines) + cols[None, :]
        out[r0:r1] = coef_values(seed, stream, flat)
    return out.reshape(nx, ny, nz, cols.size)


def positions(npos: int, *, seed: int = SEED, stream: int = 1, batch: int = 0,
              box=(1.0, 1.0, 1.0)) -> np.ndarray:
    """``[3][npos]`` FP64 positions uniform in the box [0,Lx)x[0,Ly)x[0,Lz)."""
    if npos >= 1 << 32:
        raise ValueError("npos must be < 2**32")
    p = np.arange(npos, dtype=np.uint64)
    out = np.empty((3, npos), dtype=np.float64)
    base = (np.uint64(batch) << np.uint64(32)) + p
    for d in range(3):
        with np.errstate(over="ignore"):
            ctr = base * np.uint64(4) + np.uint64(d)
        out[d] = unit_f64(hash_at(seed, stream, ctr)) * float(box[d])
    return out


def table_stream(t: int) -> int:
    return 2 * t


def position_stream(t: int) -> int:
    return 2 * t + 1


# --------------------------------------------------------------------------
# The same generator with torch integer ops, so that very large tables can be
# drawn directly in device memory.  Bit-identical to the numpy version (the
# arithmetic is modulo 2**64 in both; shifts are made logical by masking).

def _i64(u: int) -> int:
    u &= (1 << 64) - 1
    return u - (1 << 64) if u >= 1 << 63 else u


def _lsr(torch, z, s: int):
    return (z >> s) & ((1 << (64 - s)) - 1)


def mix64_torch(torch, z):
    z = (z ^ _lsr(torch, z, 30)) * _i64(0xBF58476D1CE4E5B9)
    z = (z ^ _lsr(torch, z, 27)) * _i64(0x94D049BB133111EB)
    return z ^ _lsr(torch, z, 31)


def coef_table_torch(torch, nx: int, ny: int, nz: int, nsplines: int, *, device,
                     seed: int = SEED, stream: int = 0, chunk: int = 1 << 26):
    """Unpadded ``[nx][ny][nz][N]`` FP32 table drawn on ``device``; equal bit
    for bit to :func:`coef_table`."""
    key = _i64(int(stream_key(seed, stream)))
    gamma = _i64(0x9E3779B97F4A7C15)
    total = nx * ny * nz * nsplines
    out = torch.empty(total, dtype=torch.float32, device=device)
    for i0 in range(0, total, chunk):
        i1 = min(total, i0 + chunk)
        idx = torch.arange(i0 + 1, i1 + 1, dtype=torch.int64, device=device)
        h = mix64_torch(torch, idx * gamma + key)
        k = _lsr(torch, h, 40)
        out[i0:i1] = (2 * k + 1 - (1 << 24)).to(torch.float64).mul_(2.0 ** -24).to(torch.float32)
        del idx, h, k
    return out.view(nx, ny, nz, nsplines)
