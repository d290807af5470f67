"""Randomised property checks of the oracle (hypothesis), on the CPU.

Each draws shapes, cells and positions at random and checks the oracle
against facts that do not depend on its own formulation:
  - the cell-indexed evaluator equals brute-force summation of B over every
    grid point and periodic image (no cell index, no wrap);
  - a general cell evaluates like its own rotation (covariance) and is
    periodic under the cell vectors;
  - the interpolating fit reproduces its data at the grid points.
"""

import numpy as np
import pytest

import oracle

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True)

dims = st.tuples(st.integers(1, 5), st.integers(1, 5), st.integers(1, 5))
lengths = st.tuples(*[st.floats(0.3, 3.0) for _ in range(3)])
seeds = st.integers(0, 2**31 - 1)


@SETTINGS
@given(d=dims, n=st.integers(1, 3), box=lengths, seed=seeds)
def test_cell_indexed_equals_bruteforce(d, n, box, seed):
    rng = np.random.default_rng(seed)
    tab = rng.uniform(-1, 1, d + (n,))
    pos = (rng.random((3, 6)) * 4.0 - 1.5) * np.array(box)[:, None]
    bf = oracle.evaluate_bruteforce(tab, pos, box=box)
    got = oracle.evaluate("vgh", tab, pos, box=box)
    dm = min(L / k for L, k in zip(box, d))
    np.testing.assert_allclose(got["v"], bf["v"], atol=1e-12)
    np.testing.assert_allclose(got["g"], bf["g"], atol=1e-11 / dm)
    np.testing.assert_allclose(got["h"], bf["h"], atol=1e-10 / dm ** 2)


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _cell(rng):
    while True:
        a = np.eye(3) + 0.4 * rng.standard_normal((3, 3))
        if abs(np.linalg.det(a)) > 0.3:
            return a


@SETTINGS
@given(d=dims, seed=seeds)
def test_general_cell_covariance_and_periodicity(d, seed):
    rng = np.random.default_rng(seed)
    tab = rng.uniform(-1, 1, d + (2,))
    A = _cell(rng)
    R = _rotation(rng)
    pos = A.T @ (rng.random((3, 5)) * 2 - 0.5)
    a = oracle.evaluate_lattice("vgh", tab, pos, A)
    b = oracle.evaluate_lattice("vgh", tab, (pos.T @ R).T, A @ R)
    np.testing.assert_allclose(b["v"], a["v"], atol=1e-11)
    gr = np.einsum("pan,ab->pbn", a["g"], R)
    np.testing.assert_allclose(b["g"], gr, atol=1e-9 * (1 + np.abs(gr).max()))
    shift = np.array([rng.integers(-3, 4) for _ in range(3)]) @ A
    c = oracle.evaluate_lattice("vgh", tab, pos + shift[:, None], A)
    for k in ("v", "g", "h"):
        np.testing.assert_allclose(c[k], a[k], atol=1e-9 * (1 + np.abs(a[k]).max()))


@SETTINGS
@given(d=dims, n=st.integers(1, 3), seed=seeds)
def test_fit_reproduces_grid_values(d, n, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1, 1, d + (n,))
    c = oracle.fit_interpolating(f)
    g = np.meshgrid(*[np.arange(k) / k for k in d], indexing="ij")
    pos = np.stack([x.ravel() for x in g])
    v = oracle.evaluate("v", c, pos)["v"]
    np.testing.assert_allclose(v, f.reshape(-1, n), atol=1e-11 * (1 + np.abs(c).max()))
