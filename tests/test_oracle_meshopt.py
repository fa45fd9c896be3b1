"""Pins of the near-wall mesh optimisation oracle (Appendix B).

* g_analytic: the overflow-free form against the direct sinh quotient where
  the latter is finite, the wall values, and the differential equation
  g'' = k* g by sixth-order central differences on a fine uniform grid.
* g_numeric: on a resolved layer (k* = 4) the seven-point compact solution
  matches the analytic one to the scheme's accuracy (a sign slip in k*
  turns sinh into sin: an O(1) error); as k* grows without bound the rows
  reduce to A2 g = 0, whose Dirichlet solution is computed separately
  (swapping the roles of A2 and B2 fails this).
* the descent: every accepted step lowers L, the mesh stays strictly
  increasing and exactly symmetric, the walls and the nodes beyond the m
  free ones stay put, a dominant penalty leaves the reference mesh as it is,
  and on tanh meshes with an unresolved layer a few steps lower
  ||g - g_ana|| while A2's condition number stays within the bound (ten
  times the reference mesh's).
* cond1: the banded-to-dense 1-norm condition number against the textbook
  value of a matrix with a known inverse.
"""
import math

import numpy as np
import pytest

import synth
from oracle import compact, meshopt


def test_analytic_closed_form():
    y = np.linspace(-1.0, 1.0, 41)
    for ks in (0.25, 9.0, 400.0):
        q = math.sqrt(ks)
        direct = np.array([math.sinh(q * (1.0 - v)) / math.sinh(2.0 * q) for v in y])
        np.testing.assert_allclose(meshopt.g_analytic(y, ks), direct, rtol=1e-13, atol=1e-300)
    for ks in (1.0, 1e6, 1e12):
        g = meshopt.g_analytic(np.array([-1.0, 1.0]), ks)
        assert g[0] == pytest.approx(1.0, abs=1e-15) and g[1] == 0.0


def test_analytic_solves_the_equation():
    ks = 30.0
    h = 1e-3
    y = np.arange(-1.0 + 3 * h, 1.0 - 3 * h, h)
    g = lambda v: meshopt.g_analytic(v, ks)
    # sixth-order central second difference
    c = (2 / 180, -27 / 180, 270 / 180, -490 / 180, 270 / 180, -27 / 180, 2 / 180)
    d2 = sum(ci * g(y + (k - 3) * h) for k, ci in enumerate(c)) / h ** 2
    np.testing.assert_allclose(d2, ks * g(y), rtol=1e-7, atol=1e-9)


def test_numeric_resolved_layer():
    y = synth.mesh_tanh(65)
    e = meshopt.homogeneous_error(y, 4.0)
    assert e < 1e-9, e


def test_numeric_unresolved_limit_is_A2_nullspace():
    y = synth.mesh_tanh(33)
    A, B = compact.operators(y, 2)
    n = len(y)
    M = compact.band_to_dense(A)
    M[0] = 0.0
    M[0, 0] = 1.0
    M[-1] = 0.0
    M[-1, -1] = 1.0
    r = np.zeros(n)
    r[0] = 1.0
    g_inf = np.linalg.solve(M, r)
    g = meshopt.g_numeric(A, B, 1e15)
    np.testing.assert_allclose(g, g_inf, atol=1e-7)
    # the first interior value is far from the analytic ~0: the error the descent attacks
    assert abs(g[1]) > 1e-2


def _assert_admissible(y, y_ref):
    """cond_1 of A2 and of A1 within COND_GROWTH of the reference mesh's, spacing ratios in [1/2, 2]."""
    for p in (2, 1):
        A_opt, _ = compact.operators(y, p)
        A_ref, _ = compact.operators(y_ref, p)
        assert meshopt.cond1(A_opt) <= meshopt.COND_GROWTH * meshopt.cond1(A_ref), p
    h = np.diff(y)
    r = h[1:] / h[:-1]
    assert r.max() <= 2.0 and r.min() >= 0.5, (r.min(), r.max())


def test_spacing_ratio_bound():
    y = np.cumsum([0.0, 1.0, 2.0, 4.0, 2.0, 1.0])
    assert meshopt.spacing_ratio_ok(y)          # ratios 2, 2, 1/2, 1/2: on the bound
    assert not meshopt.spacing_ratio_ok(np.cumsum([0.0, 1.0, 2.5, 2.5]))
    assert not meshopt.spacing_ratio_ok(np.cumsum([0.0, 1.0, 1.0, 0.3]))


def test_descent_lowers_the_error():
    n2, m = 33, 6
    y_ref = synth.mesh_tanh(n2)
    hist = []
    y, e0, e1, it = meshopt.optimise_mesh(y_ref, m=m, kstar=1e10, max_iter=5, history=hist)
    assert it == 5 and len(hist) == 5
    assert all(b < a for a, b in zip(hist, hist[1:]))
    assert e1 < 0.8 * e0, (e0, e1)
    _assert_admissible(y, y_ref)
    assert np.all(np.diff(y) > 0)
    np.testing.assert_array_equal(y, -y[::-1])
    assert y[0] == -1.0 and y[-1] == 1.0
    np.testing.assert_array_equal(y[m + 1:n2 - 1 - m], y_ref[m + 1:n2 - 1 - m])
    assert np.any(y[1:m + 1] != y_ref[1:m + 1])
    # the reported error is that of the returned mesh
    assert e1 == pytest.approx(meshopt.homogeneous_error(y, 1e10), rel=1e-12)
    assert e0 == pytest.approx(meshopt.homogeneous_error(y_ref, 1e10), rel=1e-12)


def test_dominant_penalty_keeps_the_mesh():
    y_ref = synth.mesh_tanh(33)
    y, e0, e1, it = meshopt.optimise_mesh(y_ref, m=4, kstar=1e10, penalty=1e6, max_iter=3)
    assert it == 0
    np.testing.assert_array_equal(y, y_ref)
    assert e1 == e0


def test_cond1_closed_form():
    # bidiagonal I + a S (S the sub-diagonal shift): the inverse has entries
    # (-a)^(i-j), so ||M||_1 = 1 + |a| and ||M^-1||_1 = sum_{k<n} |a|^k
    n, a = 12, 0.5
    band = np.zeros((n, compact.NB))
    band[:, compact.HALF] = 1.0
    band[1:, compact.HALF - 1] = a
    expect = (1 + a) * sum(a ** k for k in range(n))
    assert meshopt.cond1(band) == pytest.approx(expect, rel=1e-13)


def test_guard_bounds_the_stretching():
    # 65 nodes, 20 free per wall, the 64 x 65 x 64 workload's critical k*:
    # unguarded, this descent drives A2 to numerical singularity
    y_ref = synth.mesh_tanh(65)
    y, e0, e1, it = meshopt.optimise_mesh(y_ref, m=20, kstar=3364805.0, max_iter=2)
    assert it == 2 and e1 < e0
    _assert_admissible(y, y_ref)
