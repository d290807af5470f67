"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

Every check here compares the oracle with something other than itself:
exact rationals of the cubic B-spline basis, partition of unity, exact
polynomial reproduction (Marsden's identity), periodicity, finite
differences, C2 continuity and a brute-force sum over all grid points and
periodic images.  ``test_planted_mistakes_fail_a_pin`` plants plausible
mistakes in a copy of the oracle source and checks that a pin catches each.
"""

import os
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_basis():
    rows = []
    with open(os.path.join(GOLDEN, "cubic_bspline_basis.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t, kind, *vals = line.split()
            rows.append((Fraction(t), kind, [Fraction(v) for v in vals]))
    return rows


# ----------------------------------------------------------------- checks
# Each check takes an oracle object (the real one, or a planted mutant) and
# raises AssertionError when the pin does not hold.

def check_basis_golden(orc):
    for t, kind, vals in _golden_basis():
        w, dw, d2w = orc.weights(float(t), 1.0)
        got = {"w": w, "dw": dw, "d2w": d2w}[kind]
        np.testing.assert_allclose(got, [float(v) for v in vals], rtol=0, atol=1e-15)


def check_basis_identities(orc):
    rng = np.random.default_rng(1)
    for t in np.concatenate([[0.0, 0.5, 1 - 2**-40], rng.random(50)]):
        for delta in (1.0, 0.37):
            w, dw, d2w = orc.weights(t, delta)
            assert abs(w.sum() - 1) < 1e-15
            assert abs(dw.sum()) < 1e-13 / delta
            assert abs(d2w.sum()) < 1e-12 / delta**2
            assert np.all(w >= 0)
            assert 0.46 < (w * w).sum() <= 0.5 + 1e-15
            # mirror symmetry: w_m(t) = w_{3-m}(1-t), dw odd, d2w even
            w2, dw2, d2w2 = orc.weights(1 - t, delta)
            np.testing.assert_allclose(w, w2[::-1], atol=1e-14)
            np.testing.assert_allclose(dw, -dw2[::-1], atol=1e-13 / delta)
            np.testing.assert_allclose(d2w, d2w2[::-1], atol=1e-12 / delta**2)
            # first moments: sum_m (m-1) w_m = t (linear reproduction)
            assert abs(((np.arange(4) - 1) * w).sum() - t) < 1e-14


def _padded_poly_table(nx, ny, nz):
    """Padded table whose 64 columns hold products of Marsden polynomials.

    Column (ax, ay, az) holds f_ax(px-1) f_ay(py-1) f_az(pz-1) at padded index
    (px, py, pz) with f_0 = 1, f_1(m) = m, f_2(m) = m^2 - 1/3,
    f_3(m) = m^3 - m, so that the spline reproduces u^ax v^ay w^az exactly.
    """
    def f(deg, m):
        return [np.ones_like(m), m, m * m - 1.0 / 3.0, m**3 - m][deg]

    mx = np.arange(nx + 3, dtype=np.float64) - 1
    my = np.arange(ny + 3, dtype=np.float64) - 1
    mz = np.arange(nz + 3, dtype=np.float64) - 1
    cols = []
    degs = [(a, b, c) for a in range(4) for b in range(4) for c in range(4)]
    for a, b, c in degs:
        cols.append(f(a, mx)[:, None, None] * f(b, my)[None, :, None] * f(c, mz)[None, None, :])
    return np.stack(cols, axis=-1), degs


def check_polynomial_reproduction(orc):
    nx, ny, nz = 5, 6, 7
    box = (1.3, 0.7, 2.1)
    tab, degs = _padded_poly_table(nx, ny, nz)
    rng = np.random.default_rng(2)
    pos = rng.random((3, 40)) * np.array(box)[:, None]
    out = orc.evaluate("vgh", tab, pos, box=box, padded=True)
    outl = orc.evaluate("vgl", tab, pos, box=box, padded=True)
    d = [box[0] / nx, box[1] / ny, box[2] / nz]
    u = pos / np.array(d)[:, None]

    def p(deg, x, der):
        if der > deg:
            return np.zeros_like(x)
        c = 1.0
        for k in range(der):
            c *= deg - k
        return c * x ** (deg - der)

    for col, (a, b, c) in enumerate(degs):
        def comp(dx, dy, dz):
            return (p(a, u[0], dx) * p(b, u[1], dy) * p(c, u[2], dz)
                    / (d[0] ** dx * d[1] ** dy * d[2] ** dz))
        ref_v = comp(0, 0, 0)
        ref_g = [comp(1, 0, 0), comp(0, 1, 0), comp(0, 0, 1)]
        ref_h = [comp(2, 0, 0), comp(1, 1, 0), comp(1, 0, 1), comp(0, 2, 0), comp(0, 1, 1),
                 comp(0, 0, 2)]
        scale = 1e-11 * max(1.0, np.abs(ref_v).max())
        np.testing.assert_allclose(out["v"][:, col], ref_v, rtol=1e-12, atol=scale)
        for k in range(3):
            np.testing.assert_allclose(out["g"][:, k, col], ref_g[k], rtol=1e-11,
                                       atol=scale / min(d))
        for k in range(6):
            np.testing.assert_allclose(out["h"][:, k, col], ref_h[k], rtol=1e-10,
                                       atol=scale / min(d) ** 2)
        np.testing.assert_allclose(outl["l"][:, col], ref_h[0] + ref_h[3] + ref_h[5],
                                   rtol=1e-10, atol=3 * scale / min(d) ** 2)


def check_constant_coefficients(orc):
    nx, ny, nz, n = 4, 5, 3, 3
    consts = np.array([1.0, -2.5, 0.125])
    tab = np.broadcast_to(consts, (nx, ny, nz, n)).copy()
    rng = np.random.default_rng(3)
    pos = (rng.random((3, 30)) - 0.3) * 3.0
    out = orc.evaluate("vgh", tab, pos)
    np.testing.assert_allclose(out["v"], np.broadcast_to(consts, (30, n)), atol=1e-14)
    assert np.abs(out["g"]).max() < 1e-12
    assert np.abs(out["h"]).max() < 1e-10
    outl = orc.evaluate("vgl", tab, pos)
    assert np.abs(outl["l"]).max() < 1e-10


def check_bruteforce(orc):
    rng = np.random.default_rng(4)
    shapes = [(1, 1, 1, 1), (2, 2, 2, 2), (3, 4, 5, 3), (6, 2, 1, 2), (4, 4, 4, 1),
              (5, 3, 6, 2)]
    for (nx, ny, nz, n) in shapes:
        tab = rng.uniform(-1, 1, (nx, ny, nz, n))
        box = (1.0, 1.7, 0.6)
        pos = (rng.random((3, 12)) * 5.0 - 2.0) * np.array(box)[:, None]
        bf = orc.evaluate_bruteforce(tab, pos, box=box)
        vgh = orc.evaluate("vgh", tab, pos, box=box)
        vgl = orc.evaluate("vgl", tab, pos, box=box)
        dm = min(box[0] / nx, box[1] / ny, box[2] / nz)
        np.testing.assert_allclose(vgh["v"], bf["v"], atol=1e-13)
        np.testing.assert_allclose(vgh["g"], bf["g"], atol=1e-12 / dm)
        np.testing.assert_allclose(vgh["h"], bf["h"], atol=1e-11 / dm**2)
        np.testing.assert_allclose(vgl["l"], bf["l"], atol=3e-11 / dm**2)
        np.testing.assert_allclose(vgl["g"], bf["g"], atol=1e-12 / dm)


def check_periodic_images(orc):
    nx, ny, nz, n = 6, 5, 7, 4
    box = (1.0, 1.0, 1.0)
    tab = synth.coef_table(nx, ny, nz, n, stream=7).astype(np.float64)
    pos = synth.positions(20, stream=9)
    base = orc.evaluate("vgh", tab, pos, box=box)
    gscale = max(nx, ny, nz)
    for k, tol in (((1, -2, 3), 1e-12), ((-7, 0, 11), 1e-12),
                   ((10**6, -10**6, 10**6), 2e-6)):
        shifted = pos + np.array(k, dtype=np.float64)[:, None] * np.array(box)[:, None]
        o = orc.evaluate("vgh", tab, shifted, box=box)
        np.testing.assert_allclose(o["v"], base["v"], atol=tol)
        np.testing.assert_allclose(o["g"], base["g"], atol=tol * gscale * 4)
        np.testing.assert_allclose(o["h"], base["h"], atol=tol * gscale**2 * 8)


def _interior_positions(rng, npos, dims, box, margin=0.05):
    cells = np.stack([rng.integers(0, d, npos) for d in dims])
    frac = margin + (1 - 2 * margin) * rng.random((3, npos))
    return (cells + frac) * (np.array(box) / np.array(dims))[:, None]


def check_finite_differences(orc):
    dims = (5, 6, 4)
    box = (1.0, 0.8, 1.4)
    rng = np.random.default_rng(5)
    tab = rng.uniform(-1, 1, dims + (3,))
    pos = _interior_positions(rng, 16, dims, box)
    base = orc.evaluate("vgh", tab, pos, box=box)
    deltas = np.array(box) / np.array(dims)
    hidx = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
    for d in range(3):
        h = 1e-4 * deltas[d]
        pp, pm = pos.copy(), pos.copy()
        pp[d] += h
        pm[d] -= h
        op = orc.evaluate("vgh", tab, pp, box=box)
        om = orc.evaluate("vgh", tab, pm, box=box)
        fd_g = (op["v"] - om["v"]) / (2 * h)
        gs = np.abs(base["g"][:, d]).max()
        np.testing.assert_allclose(fd_g, base["g"][:, d], atol=1e-6 * gs)
        for e in range(3):
            fd_h = (op["g"][:, e] - om["g"][:, e]) / (2 * h)
            k = hidx[tuple(sorted((d, e)))]
            hs = np.abs(base["h"][:, k]).max()
            np.testing.assert_allclose(fd_h, base["h"][:, k], atol=1e-6 * hs)


def check_c2_continuity(orc):
    dims = (4, 5, 6)
    rng = np.random.default_rng(6)
    tab = rng.uniform(-1, 1, dims + (2,))
    deltas = 1.0 / np.array(dims)
    for d in range(3):
        pos = rng.random((3, 10))
        face = rng.integers(0, dims[d], 10)
        pos[d] = face * deltas[d]
        eps = 1e-9 * deltas[d]
        lo, hi = pos.copy(), pos.copy()
        lo[d] -= eps
        hi[d] += eps
        a = orc.evaluate("vgh", tab, lo)
        b = orc.evaluate("vgh", tab, hi)
        c = orc.evaluate("vgh", tab, pos)
        for key, sc in (("v", 1.0), ("g", 1 / deltas.min()), ("h", 1 / deltas.min() ** 2)):
            np.testing.assert_allclose(a[key], b[key], atol=1e-6 * sc)
            np.testing.assert_allclose(a[key], c[key], atol=1e-6 * sc)


def check_cross_kind(orc):
    dims = (7, 3, 5)
    rng = np.random.default_rng(7)
    tab = rng.uniform(-1, 1, dims + (5,))
    pos = rng.random((3, 25)) * 2 - 0.5
    ov = orc.evaluate("v", tab, pos)
    ol = orc.evaluate("vgl", tab, pos)
    oh = orc.evaluate("vgh", tab, pos)
    np.testing.assert_allclose(ov["v"], oh["v"], atol=1e-15)
    np.testing.assert_allclose(ol["v"], oh["v"], atol=1e-15)
    np.testing.assert_allclose(ol["g"], oh["g"], atol=1e-12)
    tr = oh["h"][:, 0] + oh["h"][:, 3] + oh["h"][:, 5]
    np.testing.assert_allclose(ol["l"], tr, atol=1e-9)


def check_wrap_edges(orc):
    """Positions a hair below a lattice translation, or a tiny negative
    number, are images of the origin: results must equal those at 0."""
    dims = (3, 5, 7)
    box = (1.1, 0.9, 1.3)
    rng = np.random.default_rng(8)
    tab = rng.uniform(-1, 1, dims + (2,))
    xs = [[-1e-300, -1e-17]]
    for j in range(1, 40):
        xs.append([np.nextafter(j * b, -np.inf) for b in box])
        xs.append([np.nextafter(-j * b, -np.inf) for b in box])
    cols = []
    for d in range(3):
        row = []
        for item in xs:
            row.extend(item if len(item) == 2 else [item[d]])
        cols.append(row)
    pos = np.array(cols, dtype=np.float64)
    zero = orc.evaluate("vgh", tab, np.zeros((3, 1)), box=box)
    out = orc.evaluate("vgh", tab, pos, box=box)
    dm = min(b / n for b, n in zip(box, dims))
    np.testing.assert_allclose(out["v"], np.broadcast_to(zero["v"], out["v"].shape), atol=1e-12)
    np.testing.assert_allclose(out["g"], np.broadcast_to(zero["g"], out["g"].shape),
                               atol=1e-11 / dm)
    np.testing.assert_allclose(out["h"], np.broadcast_to(zero["h"], out["h"].shape),
                               atol=1e-10 / dm**2)


ALL_CHECKS = [check_wrap_edges, check_basis_golden, check_basis_identities, check_polynomial_reproduction,
              check_constant_coefficients, check_bruteforce, check_periodic_images,
              check_finite_differences, check_c2_continuity, check_cross_kind]


@pytest.fixture(scope="module")
def orc():
    oracle.build(force=False)
    return oracle.Oracle()


@pytest.mark.parametrize("check", list(ALL_CHECKS), ids=[c.__name__ for c in ALL_CHECKS])
def test_oracle_pin(orc, check):
    check(orc)


def test_non_finite_position_gives_nan(orc):
    tab = np.ones((3, 3, 3, 2))
    pos = np.array([[0.1, np.nan, 0.3], [0.2, 0.2, np.inf], [0.3, 0.3, 0.3]])
    out = orc.evaluate("vgh", tab, pos)
    assert np.all(np.isfinite(out["v"][0]))
    assert np.all(np.isnan(out["v"][1])) and np.all(np.isnan(out["h"][2]))


def test_locate_wrap_edges():
    # a tiny negative u wraps to n - tiny, which rounds to n: the image of 0
    i0, t = oracle.locate(-1e-300, 1.0, 48)
    assert i0 == 0 and t == 0.0
    i0, t = oracle.locate(-0.5 / 48, 1.0, 48)
    assert i0 == 47 and abs(t - 0.5) < 1e-12
    i0, t = oracle.locate(1.0, 1.0, 48)
    assert i0 == 0 and t == 0.0
    with pytest.raises(ValueError):
        oracle.locate(1e300, 1.0, 48)


# ------------------------------------------------------- planted mistakes
# (pattern, replacement) applied to a copy of the oracle source; each models
# a plausible slip and must make at least one pin fail.
MUTANTS = [
    ("oracle_basis(t + 1.0 - m,", "oracle_basis(t + 1.0 + m - 3.0,"),  # reversed m (symmetric!)
    ("*db = sg * (-2.0 * a + 1.5 * a * a);", "*db = sg * (2.0 * a - 1.5 * a * a);"),  # sign
    ("*d2b = r;", "*d2b = -r;"),  # sign of the outer second derivative
    ("dw[m] = db / delta;", "dw[m] = db * delta;"),  # wrong chain rule
    ("d2w[m] = d2b / (delta * delta);", "d2w[m] = d2b / delta;"),
    ("wrap_index(i0[0] - 1 + a, nx)", "wrap_index(i0[0] + a, nx)"),  # off-by-one
    ("wrap_index(i0[1] - 1 + b, ny)", "wrap_index(i0[1] - 1 + b, nx)"),  # wrong dim
    ("const double whxy = dw[0][a] * dw[1][b] * w[2][c];",
     "const double whxy = dw[0][a] * w[1][b] * dw[2][c];"),  # transposed component
    ("const double wgz = w[0][a] * w[1][b] * dw[2][c];",
     "const double wgz = w[0][a] * dw[1][b] * w[2][c];"),
    ("l[p * ldo + n] += (whxx + whyy + whzz) * cf;", "l[p * ldo + n] += (whxx + whyy) * cf;"),
    ("oracle_locate(x, L[d], dims[d],", "oracle_locate(x, L[d], dims[0],"),  # wrong dim
    ("i = 0;\n        u = 0.0;", "i = n - 1;\n        u = n - 1;"),  # wrong image of n
    ("*b = 2.0 / 3.0 - a * a + 0.5 * a * a * a;", "*b = 2.0 / 3.0 - a * a + 0.5 * a * a;"),
    ("int ix = padded ? i0[0] + a :", "int ix = padded ? i0[0] + a - 1 :"),
    ("double delta = box_len / n;", "double delta = box_len / (n + 1);"),
]


def _mutant_fails(src_text, pat, rep, tmpdir):
    assert src_text.count(pat) == 1, f"mutation pattern not unique: {pat}"
    mutated = src_text.replace(pat, rep)
    cpath = os.path.join(tmpdir, "mutant.c")
    with open(cpath, "w") as f:
        f.write(mutated)
    so = os.path.join(tmpdir, f"mutant_{abs(hash(pat))}.so")
    oracle.compile_source(cpath, so)
    orc = oracle.Oracle(so)
    for check in ALL_CHECKS:
        try:
            check(orc)
        except (AssertionError, ValueError):
            return check.__name__
    return None


def test_planted_mistakes_fail_a_pin():
    src_path = os.path.join(os.path.dirname(oracle.__file__), "bspline_oracle.c")
    text = open(src_path).read()
    with tempfile.TemporaryDirectory() as tmp:
        survivors = []
        for pat, rep in MUTANTS:
            caught = _mutant_fails(text, pat, rep, tmp)
            if caught is None:
                survivors.append(pat)
        assert not survivors, f"planted mistakes no pin caught: {survivors}"


# ---------------------------------------------------------- determinant ratios
def _bf_matrix(orc, coef, pos, box):
    """A[n][e] = phi_n(r_e) and derivatives from the brute-force evaluator."""
    return orc.evaluate_bruteforce(coef, pos, box=box)


def check_ratio_is_determinant_ratio(orc):
    """The ratio sum equals det(A')/det(A) for A[n][e] = phi_n(r_e), A' with
    column e replaced by phi(r'), ainv row = (A^-1)[e, :]; its gradient,
    Laplacian and Hessian match finite differences of that determinant
    ratio (all built from the brute-force evaluator)."""
    rng = np.random.default_rng(11)
    dims, nel = (4, 3, 5), 6
    box = (1.0, 0.9, 1.2)
    coef = rng.uniform(-1, 1, dims + (nel,))
    r = rng.random((3, nel)) * np.array(box)[:, None]
    A = _bf_matrix(orc, coef, r, box)["v"].T            # A[n][e]
    Ainv = np.linalg.inv(A)
    detA = np.linalg.det(A)
    e = 2
    rnew = (rng.random(3) * np.array(box))[:, None]

    def R(x):
        phi = _bf_matrix(orc, coef, x[:, None], box)["v"][0]
        A2 = A.copy()
        A2[:, e] = phi
        return np.linalg.det(A2) / detA

    got = orc.evaluate_ratio("vgh", coef, rnew, Ainv[e][None, :], box=box)[0]
    gotl = orc.evaluate_ratio("vgl", coef, rnew, Ainv[e][None, :], box=box)[0]
    gotv = orc.evaluate_ratio("v", coef, rnew, Ainv[e][None, :], box=box)[0]
    x0 = rnew[:, 0]
    assert abs(got[0] - R(x0)) < 1e-10 * max(1, abs(R(x0)))
    assert abs(gotv[0] - got[0]) < 1e-14 and abs(gotl[0] - got[0]) < 1e-14
    hstep = 1e-4 * min(b / n for b, n in zip(box, dims))
    grad = np.zeros(3)
    hess = np.zeros((3, 3))
    for a in range(3):
        da = np.zeros(3)
        da[a] = hstep
        grad[a] = (R(x0 + da) - R(x0 - da)) / (2 * hstep)
        for b in range(3):
            db = np.zeros(3)
            db[b] = hstep
            hess[a, b] = (R(x0 + da + db) - R(x0 + da - db) - R(x0 - da + db)
                          + R(x0 - da - db)) / (4 * hstep * hstep)
    scale_g = np.abs(grad).max()
    np.testing.assert_allclose(got[1:4], grad, atol=1e-5 * scale_g)
    np.testing.assert_allclose(gotl[1:4], grad, atol=1e-5 * scale_g)
    hidx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    scale_h = np.abs(hess).max()
    np.testing.assert_allclose(got[4:], [hess[i, j] for i, j in hidx], atol=1e-4 * scale_h)
    assert abs(gotl[4] - np.trace(hess)) < 1e-4 * scale_h


def test_ratio_pin(orc):
    check_ratio_is_determinant_ratio(orc)


ALL_CHECKS.append(check_ratio_is_determinant_ratio)
MUTANTS += [
    ("else if (c <= 3) x = g + (p * 3 + (c - 1)) * ncoef;",
     "else if (c <= 3) x = g + (p * 3 + (3 - c)) * ncoef;"),  # gradient components reversed
    ("for (int64_t n = 0; n < ncoef; ++n) sum += x[n] * a[n];",
     "for (int64_t n = 0; n < ncoef; ++n) sum += x[n] * a[ncoef - 1 - n];"),  # ainv reversed
]


# ------------------------------------------------------------ general cells
HEX = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3) / 2, 0.0], [0.0, 0.0, 1.6]])
TRICLINIC = np.array([[1.1, 0.1, -0.2], [0.3, 0.9, 0.15], [-0.25, 0.2, 1.3]])


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def check_lattice_diagonal_is_box(orc):
    rng = np.random.default_rng(21)
    tab = rng.uniform(-1, 1, (5, 4, 6, 3))
    box = (1.3, 0.7, 2.1)
    pos = (rng.random((3, 30)) * 3 - 1) * np.array(box)[:, None]
    a = orc.evaluate_lattice("vgh", tab, pos, np.diag(box))
    b = orc.evaluate("vgh", tab, pos, box=box)
    for k in ("v", "g", "h"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-10 * np.abs(b[k]).max())
    al = orc.evaluate_lattice("vgl", tab, pos, np.diag(box))
    bl = orc.evaluate("vgl", tab, pos, box=box)
    np.testing.assert_allclose(al["l"], bl["l"], rtol=1e-12, atol=1e-10 * np.abs(bl["l"]).max())


def check_lattice_rotation_covariance(orc):
    """Rotating the cell and the positions together leaves V unchanged and
    rotates G (g' = g R) and H (H' = R^T H R), row-vector convention."""
    rng = np.random.default_rng(22)
    tab = rng.uniform(-1, 1, (4, 5, 3, 2))
    R = _rotation(rng)
    pos = rng.random((3, 25)) * 2 - 0.5
    a = orc.evaluate_lattice("vgh", tab, pos, TRICLINIC)
    b = orc.evaluate_lattice("vgh", tab, (pos.T @ R).T, TRICLINIC @ R)
    np.testing.assert_allclose(b["v"], a["v"], atol=1e-12)
    gr = np.einsum("pan,ab->pbn", a["g"], R)
    np.testing.assert_allclose(b["g"], gr, atol=1e-10 * np.abs(gr).max())
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    H = np.zeros(a["h"].shape[:1] + (3, 3) + a["h"].shape[2:])
    for k, (i, j) in enumerate(idx):
        H[:, i, j] = a["h"][:, k]
        H[:, j, i] = a["h"][:, k]
    Hr = np.einsum("ai,pabn,bj->pijn", R, H, R)
    want = np.stack([Hr[:, i, j] for i, j in idx], axis=1)
    np.testing.assert_allclose(b["h"], want, atol=1e-9 * np.abs(want).max())
    lb = orc.evaluate_lattice("vgl", tab, (pos.T @ R).T, TRICLINIC @ R)["l"]
    np.testing.assert_allclose(lb, Hr[:, 0, 0] + Hr[:, 1, 1] + Hr[:, 2, 2],
                               atol=1e-9 * np.abs(want).max())


def check_lattice_polynomials(orc):
    """Padded tables holding f(p-1) reproduce u_d and u_d^2 - 1/3 -> u_d^2
    exactly in grid coordinates u = n (r A^-1): G = M[d] and G = 2 u_d M[d],
    H = 0 and H = 2 M[d]^T M[d], for every cell axis d."""
    dims = (5, 6, 4)
    ntot = [n + 3 for n in dims]
    cols = []
    for d in range(3):
        m = np.arange(ntot[d], dtype=np.float64) - 1
        for f in (m, m * m - 1.0 / 3.0):
            shape = [1, 1, 1]
            shape[d] = ntot[d]
            cols.append(np.broadcast_to(f.reshape(shape), ntot))
    tab = np.stack(cols, axis=-1)
    A = HEX
    M = np.array(dims)[:, None] * np.linalg.inv(A).T      # M[d][a] = n_d inv(A)[a][d]
    rng = np.random.default_rng(23)
    s = rng.random((25, 3)) * 0.999
    pos = (s @ A).T                                        # inside the cell
    out = orc.evaluate_lattice("vgh", tab, pos, A, padded=True)
    u = (M @ pos)                                          # [3][npos]
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for d in range(3):
        lin, quad = 2 * d, 2 * d + 1
        np.testing.assert_allclose(out["v"][:, lin], u[d], atol=1e-11)
        np.testing.assert_allclose(out["v"][:, quad], u[d] ** 2, atol=1e-10)
        for a in range(3):
            np.testing.assert_allclose(out["g"][:, a, lin], M[d, a], atol=1e-11)
            np.testing.assert_allclose(out["g"][:, a, quad], 2 * u[d] * M[d, a], atol=1e-9)
        for k, (a, b) in enumerate(idx):
            np.testing.assert_allclose(out["h"][:, k, lin], 0.0, atol=1e-9)
            np.testing.assert_allclose(out["h"][:, k, quad], 2 * M[d, a] * M[d, b], atol=1e-8)


def check_lattice_fd_and_periodicity(orc):
    rng = np.random.default_rng(24)
    dims = (4, 5, 6)
    tab = rng.uniform(-1, 1, dims + (3,))
    A = TRICLINIC
    M = np.array(dims)[:, None] * np.linalg.inv(A).T
    # interior points of random cells (away from faces in grid coordinates)
    cells = np.stack([rng.integers(0, n, 12) for n in dims])
    u = cells + 0.1 + 0.8 * rng.random((3, 12))
    pos = np.linalg.solve(M, u)
    base = orc.evaluate_lattice("vgh", tab, pos, A)
    hstep = 1e-5
    idx = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
    for a in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[a] += hstep
        pm[a] -= hstep
        op = orc.evaluate_lattice("vgh", tab, pp, A)
        om = orc.evaluate_lattice("vgh", tab, pm, A)
        gs = np.abs(base["g"]).max()
        np.testing.assert_allclose((op["v"] - om["v"]) / (2 * hstep), base["g"][:, a],
                                   atol=1e-6 * gs)
        for b in range(3):
            hs = np.abs(base["h"]).max()
            np.testing.assert_allclose((op["g"][:, b] - om["g"][:, b]) / (2 * hstep),
                                       base["h"][:, idx[tuple(sorted((a, b)))]], atol=1e-6 * hs)
    for k in ((1, 0, 0), (0, -2, 0), (3, 1, -1)):
        shifted = pos + (np.array(k) @ A)[:, None]
        o = orc.evaluate_lattice("vgh", tab, shifted, A)
        for key in ("v", "g", "h"):
            np.testing.assert_allclose(o[key], base[key], atol=1e-9 * np.abs(base[key]).max())


LATTICE_CHECKS = [check_lattice_diagonal_is_box, check_lattice_rotation_covariance,
                  check_lattice_polynomials, check_lattice_fd_and_periodicity]


@pytest.mark.parametrize("check", LATTICE_CHECKS, ids=[c.__name__ for c in LATTICE_CHECKS])
def test_lattice_pin(orc, check):
    check(orc)


ALL_CHECKS.extend(LATTICE_CHECKS)
MUTANTS += [
    ("for (int a = 0; a < 3; ++a) M[d][a] = dims[d] * ainv[3 * a + d];",
     "for (int a = 0; a < 3; ++a) M[d][a] = dims[d] * ainv[3 * d + a];"),  # transposed inverse
    ("for (int d = 0; d < 3; ++d) s += M[d][a] * G[d];",
     "for (int d = 0; d < 3; ++d) s += M[a][d] * G[d];"),  # gradient transform transposed
    ("for (int e = 0; e < 3; ++e) s += M[d][a] * M[e][b] * H[d][e];",
     "for (int e = 0; e < 3; ++e) s += M[d][a] * M[e][a] * H[d][e];"),  # wrong Hessian index
]


# ----------------------------------------------- interpolating coefficients
def _grid_positions(dims, box):
    axes = [np.arange(n) * (L / n) for n, L in zip(dims, box)]
    g = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.ravel() for a in g])


def check_fit_interpolates(orc):
    """The fitted spline takes the given value at every grid point, also on
    axes of 1, 2 and 3 points."""
    rng = np.random.default_rng(31)
    for dims in ((5, 4, 6), (1, 3, 2), (2, 7, 1)):
        f = rng.uniform(-1, 1, dims + (3,))
        box = (1.3, 0.7, 2.1)
        c = orc.fit_interpolating(f)
        v = orc.evaluate("v", c, _grid_positions(dims, box), box=box)["v"]
        np.testing.assert_allclose(v, f.reshape(-1, 3), atol=1e-12)


def check_fit_fourier_modes(orc):
    """A periodic Fourier mode is an eigenvector of every axis system: values
    prod_d cos(2 pi k_d i_d / n_d + phi_d) give coefficients equal to the
    values times prod_d 3 / (2 + cos(2 pi k_d / n_d))."""
    dims = (6, 5, 8)
    idx = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    modes = [((0, 0, 0), (0.0, 0.0, 0.0)), ((1, 2, 3), (0.3, -1.1, 0.0)),
             ((3, 1, 4), (0.0, 0.5, 2.0)), ((2, 0, 1), (1.0, 0.0, -0.7))]
    f = np.zeros(dims + (len(modes),))
    want = np.zeros_like(f)
    for m, (k, ph) in enumerate(modes):
        val, fac = np.ones(dims), 1.0
        for d in range(3):
            th = 2 * np.pi * k[d] / dims[d]
            val = val * np.cos(th * idx[d] + ph[d])
            fac *= 3.0 / (2.0 + np.cos(th))
        f[..., m] = val
        want[..., m] = val * fac
    np.testing.assert_allclose(orc.fit_interpolating(f), want, atol=1e-12)


def check_fit_recovers_coefficients(orc):
    """Sampling a known spline at its grid points (brute force, no cell
    logic) and fitting returns its coefficients."""
    rng = np.random.default_rng(32)
    dims = (4, 3, 5)
    c0 = rng.uniform(-1, 1, dims + (2,))
    box = (1.0, 1.0, 1.0)
    f = orc.evaluate_bruteforce(c0, _grid_positions(dims, box), box=box)["v"]
    c = orc.fit_interpolating(f.reshape(dims + (2,)))
    np.testing.assert_allclose(c, c0, atol=1e-11)


FIT_CHECKS = [check_fit_interpolates, check_fit_fourier_modes, check_fit_recovers_coefficients]


@pytest.mark.parametrize("check", FIT_CHECKS, ids=[c.__name__ for c in FIT_CHECKS])
def test_fit_pin(orc, check):
    check(orc)


ALL_CHECKS.extend(FIT_CHECKS)
MUTANTS += [
    ("A[i * n + (i - 1 + n) % n] += 1.0 / 6.0;", "A[i * n + (i - 2 + n) % n] += 1.0 / 6.0;"),
    ("A[i * n + i] += 4.0 / 6.0;", "A[i * n + i] += 4.0;"),  # unnormalised diagonal
    ("A[i * n + (i + 1) % n] += 1.0 / 6.0;",
     "if (i + 1 < n) A[i * n + i + 1] += 1.0 / 6.0;"),  # no periodic wrap
    ("const int n = dims[d];\n        double* A", "const int n = dims[2 - d];\n        double* A"),
]
