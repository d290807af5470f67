"""GPU parity of the interpolating-coefficient fit, through the C ABI.

Reference: the oracle's dense per-axis solve of the interpolation condition
(c[i-1] + 4 c[i] + c[i+1]) / 6 = f[i] in FP64.  Tolerance: per table,
max |gpu - oracle| / max |oracle| <= 1e-5.  The GPU keeps FP64 recursion
state but stores FP32 between its passes.  Each axis system has an inverse
of infinity-norm 3 (its symbol (4 + 2 cos t)/6 is smallest, 1/3, at t = pi),
so the roundings of the stored intermediate and output of one pass cost a
few FP32 ulp of the result; three passes stay near 1e-6, inside the bound.
"""

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_close, run_gpu, smooth_grid_values

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_02665_amd import binding as B  # noqa: E402

FIT_TOL = 1e-5
HEX = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3) / 2, 0.0], [0.0, 0.0, 1.6]])


def _gpu_fit(values, in_place=False):
    dev = torch.device("cuda")
    v = torch.from_numpy(np.ascontiguousarray(values, np.float32)).to(dev)
    c = v if in_place else torch.full_like(v, float("nan"))
    nx, ny, nz, n = values.shape
    B.spline_fit_interpolating(nx, ny, nz, n, v, c)
    torch.cuda.synchronize()
    return c.cpu().numpy()


def _rel_err(got, ref):
    return float(np.abs(got.astype(np.float64) - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("shape", [(7, 9, 5, 300), (1, 2, 3, 5), (2, 1, 40, 64),
                                   (100, 3, 2, 70), (33, 31, 32, 17), (48, 48, 60, 128),
                                   (300, 2, 1, 5), (2, 3, 260, 70)])
def test_fit_matches_oracle(shape):
    """Random values (axes of 1 and 2 points, axes shorter and longer than
    the 32-term periodic start, ragged N; axes of 300 and 260 points take
    the global-memory passes, shorter ones the LDS-staged passes)."""
    values = synth.coef_table(*shape, stream=101)
    ref = oracle.fit_interpolating(values.astype(np.float64))
    got = _gpu_fit(values)
    assert _rel_err(got, ref) <= FIT_TOL, (shape, _rel_err(got, ref))


def test_fit_smooth_values():
    values = smooth_grid_values((12, 10, 14), 9, seed=102)
    ref = oracle.fit_interpolating(values.astype(np.float64))
    assert _rel_err(_gpu_fit(values), ref) <= FIT_TOL


def test_fit_in_place_equals_out_of_place():
    values = synth.coef_table(9, 8, 11, 130, stream=103)
    a = _gpu_fit(values)
    b = _gpu_fit(values, in_place=True)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("where", ["host", "device"])
@pytest.mark.parametrize("cell", ["box", "hex"])
def test_table_from_grid_values(where, cell):
    """A table created from grid values reproduces them at the grid points
    and matches the oracle's spline on the oracle's fit elsewhere."""
    dims, n = (8, 7, 9), 200
    values = synth.coef_table(*dims, n, stream=104)
    flags = B.BSPL_COEFS_GRID_VALUES
    src = values
    if where == "device":
        src = torch.from_numpy(values).cuda()
        flags |= B.BSPL_COEFS_DEVICE
    if cell == "box":
        box = (1.2, 0.9, 1.1)
        A = np.diag(box)
        h = B.spline_table_create(*dims, n, src, "f32", box, flags)
    else:
        A = HEX
        h = B.spline_table_create_lattice(*dims, n, src, A, "f32", flags)
    try:
        if where == "device":  # the caller's values are left untouched
            assert np.array_equal(src.cpu().numpy(), values)
        g = np.meshgrid(*[np.arange(d) / d for d in dims], indexing="ij")
        frac = np.stack([x.ravel() for x in g])
        grid_pos = np.ascontiguousarray(A.T @ frac)
        out, _ = run_gpu(B, h, "v", grid_pos, n)
        err = np.abs(out["v"] - values.reshape(-1, n)).max() / np.abs(values).max()
        assert err <= FIT_TOL, err
        coef = oracle.fit_interpolating(values.astype(np.float64))
        pos = np.ascontiguousarray(A.T @ (synth.positions(150, stream=105) * 3 - 1))
        for kind in ("vgl", "vgh"):
            gpu, _ = run_gpu(B, h, kind, pos, n)
            ref = oracle.evaluate_lattice(kind, coef, pos, A)
            assert_close(kind, gpu, ref, label=f"{where} {cell} {kind}")
    finally:
        B.spline_table_destroy(h)


def test_fit_paper_scale_sampled_columns():
    """48^3 x 2048 values drawn on the device; 8 spline columns of the GPU
    fit checked against the oracle's fit of those columns, and a table made
    from the same values reproduces them at 256 sampled grid points."""
    dims, n = (48, 48, 48), 2048
    dev = torch.device("cuda")
    vals = synth.coef_table_torch(torch, *dims, n, device=dev, stream=106)
    coefs = torch.empty_like(vals)
    B.spline_fit_interpolating(*dims, n, vals, coefs)
    cols = np.array([0, 1, 63, 64, 777, 1500, 2046, 2047])
    got = coefs[..., torch.from_numpy(cols).to(dev)].cpu().numpy()
    del coefs
    host_cols = synth.coef_table(*dims, n, stream=106, splines=cols)
    ref = oracle.fit_interpolating(host_cols.astype(np.float64))
    assert _rel_err(got, ref) <= FIT_TOL
    h = B.spline_table_create(*dims, n, vals, "f32", None,
                              B.BSPL_COEFS_DEVICE | B.BSPL_COEFS_GRID_VALUES)
    try:
        rng = np.random.default_rng(107)
        pts = np.stack([rng.integers(0, d, 256) for d in dims])
        out, _ = run_gpu(B, h, "v", np.ascontiguousarray(pts / np.array(dims)[:, None]), n,
                         canary=False)
        ti = [torch.from_numpy(x).to(dev) for x in pts]
        want = vals[ti[0], ti[1], ti[2]].cpu().numpy()
        assert np.abs(out["v"] - want).max() / np.abs(want).max() <= FIT_TOL
    finally:
        B.spline_table_destroy(h)


def test_fit_argument_errors():
    t = torch.zeros(2, 2, 2, 3, device="cuda")
    for args in [(0, 2, 2, 3, t, t), (2, 2, 2, 0, t, t), (2, 2, 2, 3, None, t),
                 (2, 2, 2, 3, t, None)]:
        with pytest.raises(B.BsplineError) as e:
            B.spline_fit_interpolating(*args)
        assert e.value.status == B.BSPL_EINVAL
