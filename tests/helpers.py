"""Shared helpers for the GPU parity tests (test infrastructure)."""

from __future__ import annotations

import numpy as np

COMPONENTS = {
    "v": [("v", None)],
    "vgl": [("v", None), ("g", 0), ("g", 1), ("g", 2), ("l", None)],
    "vgh": [("v", None), ("g", 0), ("g", 1), ("g", 2)] + [("h", k) for k in range(6)],
}
COMP_NAMES = {("v", None): "v", ("l", None): "l",
              **{("g", k): "g" + "xyz"[k] for k in range(3)},
              **{("h", k): "h" + ["xx", "xy", "xz", "yy", "yz", "zz"][k] for k in range(6)}}

FP32_TOL = 1e-5  # per-component max error over max |reference| (FP32 tables)


def run_gpu(B, table, kind, pos, nsplines, ldo=None, tile=None, canary=True, torch=None,
            stream=None):
    """Evaluate ``kind`` on the GPU; returns (outputs as float64 numpy arrays
    trimmed to nsplines, raw float32 outputs including the [N, ldo) columns)."""
    import torch as _t
    torch = torch or _t
    dev = torch.device("cuda")
    ldo = ldo or nsplines
    npos = pos.shape[1]
    p = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    fill = float("nan") if not canary else 12345.0
    v = torch.full((npos, ldo), fill, device=dev)
    g = torch.full((npos, 3, ldo), fill, device=dev) if kind != "v" else None
    lh = None
    if kind == "vgl":
        lh = torch.full((npos, ldo), fill, device=dev)
    elif kind == "vgh":
        lh = torch.full((npos, 6, ldo), fill, device=dev)
    B.spline_eval(table, kind, npos, p, v, g, lh, ldo, tile=tile, stream=stream)
    torch.cuda.synchronize()
    raw = {"v": v.cpu().numpy()}
    if g is not None:
        raw["g"] = g.cpu().numpy()
    if kind == "vgl":
        raw["l"] = lh.cpu().numpy()
    if kind == "vgh":
        raw["h"] = lh.cpu().numpy()
    out = {k: a[..., :nsplines].astype(np.float64) for k, a in raw.items()}
    return out, raw


def component(arr_dict, key, k):
    a = arr_dict[key]
    return a if k is None else a[:, k]


ORDER = {"v": 0, "g": 1, "l": 2, "h": 2}


def normalized_errors(kind, gpu, ref, inv_delta=None):
    """Per component: max |gpu - ref| / max |ref| over all positions and splines.

    A component whose reference vanishes identically (a constant function on
    a degenerate grid) has no scale of its own; given ``inv_delta`` (the
    largest n_d / L_d), it is normalised by the natural scale
    max|V| * inv_delta^order instead."""
    errs = {}
    vmax = np.abs(ref["v"]).max() if "v" in ref else 0.0
    for key, k in COMPONENTS[kind]:
        r = component(ref, key, k)
        g = component(gpu, key, k)
        scale = np.abs(r).max()
        if inv_delta is not None:
            natural = vmax * inv_delta ** ORDER[key]
            if scale < 1e-6 * natural:
                scale = natural
        errs[COMP_NAMES[(key, k)]] = float(np.abs(g - r).max() / (scale if scale > 0 else 1.0))
    return errs


def assert_close(kind, gpu, ref, tol=FP32_TOL, label="", inv_delta=None):
    errs = normalized_errors(kind, gpu, ref, inv_delta)
    bad = {k: e for k, e in errs.items() if not e <= tol}
    assert not bad, f"{label} normalised errors above {tol}: {bad} (all: {errs})"
    return errs


def assert_canary(raw, nsplines, value=12345.0):
    for k, a in raw.items():
        tail = a[..., nsplines:]
        assert np.all(tail == value), f"{k}: columns [N, ldo) were written"


def quantize_f16(coef):
    """Per-spline power-of-two scales and RNE FP16 codes, restated on the
    host: s_n = 2^ceil(log2 max|c_n|) (1 if all zero), q = fp16(c / s_n)."""
    m = np.abs(coef.reshape(-1, coef.shape[-1])).max(axis=0).astype(np.float64)
    s = np.ones_like(m)
    nz = m > 0
    s[nz] = 2.0 ** np.ceil(np.log2(m[nz]))
    q = (coef / s.astype(np.float32)).astype(np.float16)
    return q, s.astype(np.float32)


def quantize_bf16(coef):
    """Same scales; bf16 codes by round-to-nearest-even on the FP32 bits."""
    m = np.abs(coef.reshape(-1, coef.shape[-1])).max(axis=0).astype(np.float64)
    s = np.ones_like(m)
    nz = m > 0
    s[nz] = 2.0 ** np.ceil(np.log2(m[nz]))
    x = (coef / s.astype(np.float32)).astype(np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)
    return r, s.astype(np.float32)


def bf16_to_f32(codes):
    return (codes.astype(np.uint32) << 16).view(np.float32)


def dequantized(coef, dtype):
    if dtype == "f16":
        q, s = quantize_f16(coef)
        return q.astype(np.float32) * s
    if dtype == "bf16":
        q, s = quantize_bf16(coef)
        return bf16_to_f32(q) * s
    return coef


def padded_layout(coef, np_):
    """Periodic +3 padding (padded index i holds coefficient (i-1) mod n) and
    zero row padding to np_ columns, restated on the host."""
    nx, ny, nz, n = coef.shape
    ix = (np.arange(nx + 3) - 1) % nx
    iy = (np.arange(ny + 3) - 1) % ny
    iz = (np.arange(nz + 3) - 1) % nz
    p = coef[ix][:, iy][:, :, iz]
    out = np.zeros((nx + 3, ny + 3, nz + 3, np_), dtype=coef.dtype)
    out[..., :n] = p
    return out


def smooth_grid_values(dims, n, seed):
    """Band-limited periodic orbitals sampled on the grid: each of the n
    columns is a sum of three random Fourier modes with |k_d| <= 2 (the
    smooth data interpolation tables are built from)."""
    rng = np.random.default_rng(seed)
    idx = np.meshgrid(*[np.arange(d) / d for d in dims], indexing="ij")
    out = np.zeros(tuple(dims) + (n,))
    for s in range(n):
        for _ in range(3):
            k = rng.integers(-2, 3, 3)
            ph = rng.uniform(0, 2 * np.pi)
            out[..., s] += rng.uniform(-1, 1) * np.cos(
                2 * np.pi * (k[0] * idx[0] + k[1] * idx[1] + k[2] * idx[2]) + ph)
    return out.astype(np.float32)
