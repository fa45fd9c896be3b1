"""Near-wall mesh optimisation for the homogeneous Helmholtz solutions (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Appendix B: the implicit step's homogeneous problem (B2 - k* A2) g = 0 with
g = 1 at the lower wall and g = 0 at the upper wall has the analytic solution
g_ana(y) = sinh(q (1 - y)) / sinh(2 q), q = sqrt(k*).  On a given mesh the
compact-difference solution g departs from it near the wall when the
boundary layer 1/q is thinner than the first cells.  The paper moves the
first near-wall nodes to minimise

    L(mu) = ||g - g_ana|| + C ||mu - mu_ref||

by steepest descent, mu being the positions of the near-wall nodes, with
C about 1e-3.

Readings (where the paper is silent):
- mu = y_1 .. y_m (the wall node y_0 = -1 stays; the paper's 21 nodes are
  the wall node and m = 20 free ones).  The upper wall is the mirror image,
  y_{n-1-j} = -y_j, so the mesh stays symmetric.
- Both norms are Euclidean: over all n2 nodes for g, over the m free
  positions for mu.
- Rows 1 .. n2-2 hold (B2 - k* A2) g = 0; rows 0 and n2-1 are the Dirichlet
  values (the same A-form as the implicit steps).
- Steepest descent in the spacing-scaled coordinates xi_j = y_j / s_j
  (s_j = y_ref[j+1] - y_ref[j]), i.e. the step in y_j is -t s_j^2 dL/dy_j;
  the gradient by central differences with step 1e-6 s_j; the step length
  by halving from twice the last accepted one (t starts at 1, so the first
  trial is 2) until the mesh
  is strictly increasing, L strictly decreases and the Armijo condition
  L(new) <= L + 1e-4 t (grad . d) holds (strict decrease rejects a step that
  rounds to no move at all); the descent stops after max_iter iterations,
  or when t falls below 1e-30.
- A trial mesh must also keep the compact operators well posed: its A2 and
  its A1 may each have a 1-norm condition number at most 10 times that of
  the reference mesh's.  The paper's functional only sees B2 - k* A2, and
  without this guard the descent can reach meshes on which A2 itself is
  singular (the maximum-order stencils degenerate for some local
  stretchings) while the homogeneous error keeps falling; A1 (the first
  derivative of the velocity recovery and of the non-linear forcing) is
  bounded the same way.
- The paper moves the nodes without changing much the individual grid
  spacings; read as: every ratio of adjacent spacings of a trial mesh lies
  in [1/2, 2].  (The displacement penalty, measured in absolute y, is far
  too small against the error to enforce this by itself.)

The compact rows come from ``compact.row_coefficients`` (exact rationals);
only the rows whose stencils contain a moved node are recomputed.
"""
from __future__ import annotations

import numpy as np

from . import compact

FD_REL = 1e-6       # central-difference step, relative to the local spacing
ARMIJO = 1e-4
T_MIN = 1e-30
COND_GROWTH = 10.0  # allowed growth of cond_1(A2) and cond_1(A1) over the reference mesh
SPACING_RATIO = 2.0  # adjacent spacings of a trial mesh within a factor 2 of each other


def cond1(A):
    """1-norm condition number of the banded matrix A (dense inverse)."""
    M = compact.band_to_dense(A)
    return float(np.linalg.norm(M, 1) * np.linalg.norm(np.linalg.inv(M), 1))


def g_analytic(y, kstar):
    """sinh(q (1 - y)) / sinh(2 q), q = sqrt(k*), written without overflow."""
    q = np.sqrt(kstar)
    y = np.asarray(y, dtype=np.float64)
    return np.exp(-q * (1.0 + y)) * (-np.expm1(-2.0 * q * (1.0 - y))) / (-np.expm1(-4.0 * q))


def spacing_ratio_ok(y):
    """Every ratio of adjacent spacings of mesh y within [1/SPACING_RATIO, SPACING_RATIO]."""
    h = np.diff(y)
    r = h[1:] / h[:-1]
    return bool(np.all(r <= SPACING_RATIO) and np.all(r >= 1.0 / SPACING_RATIO))


def _rows(y, rows, A, B, p=2):
    """Recompute the compact rows ``rows`` of the order-p pair (A, B) in place."""
    for i in rows:
        S, a, b = compact.row_coefficients(y, i, p)
        A[i] = 0.0
        B[i] = 0.0
        for j, aj, bj in zip(S, a, b):
            A[i, compact.HALF + j - i] = float(aj)
            B[i, compact.HALF + j - i] = float(bj)


def g_numeric(A, B, kstar):
    """Solve (B - k* A) g = 0 in rows 1..n-2, g_0 = 1, g_{n-1} = 0 (dense solve)."""
    n = A.shape[0]
    M = compact.band_to_dense(B) - kstar * compact.band_to_dense(A)
    M[0] = 0.0
    M[0, 0] = 1.0
    M[-1] = 0.0
    M[-1, -1] = 1.0
    r = np.zeros(n)
    r[0] = 1.0
    return np.linalg.solve(M, r)


def homogeneous_error(y, kstar, A=None, B=None):
    """||g - g_ana||_2 over all nodes of mesh y."""
    if A is None:
        A, B = compact.operators(y, 2)
    return float(np.linalg.norm(g_numeric(A, B, kstar) - g_analytic(y, kstar)))


class _Problem:
    def __init__(self, y_ref, m, kstar, penalty):
        y_ref = np.asarray(y_ref, dtype=np.float64)
        n = len(y_ref)
        if m < 1 or 2 * m + 2 > n:
            raise ValueError("need 1 <= m and 2 m + 2 <= n2")
        self.n, self.m, self.kstar, self.C = n, m, kstar, penalty
        self.y_ref = y_ref
        self.x_ref = y_ref[1:m + 1].copy()
        self.s = y_ref[2:m + 2] - y_ref[1:m + 1]
        A, B = compact.operators(y_ref, 2)
        self.A0, self.B0 = A.copy(), B.copy()
        self.cond_max = COND_GROWTH * cond1(A)
        A1, B1 = compact.operators(y_ref, 1)
        self.A10, self.B10 = A1, B1
        self.cond1_max = COND_GROWTH * cond1(A1)

    def mesh(self, x):
        y = self.y_ref.copy()
        y[1:self.m + 1] = x
        y[self.n - 1 - self.m:self.n - 1] = -x[::-1]
        return y

    def _touched(self):
        n, m = self.n, self.m
        return [i for i in range(n) if i <= m + compact.HALF or i >= n - 1 - m - compact.HALF]

    def operators(self, y):
        """(A2, B2) of mesh y: the rows whose stencils hold a moved node recomputed."""
        A, B = self.A0.copy(), self.B0.copy()
        _rows(y, self._touched(), A, B)
        return A, B

    def a1(self, y):
        """A1 of mesh y (rows recomputed as for A2)."""
        A, B = self.A10.copy(), self.B10.copy()
        _rows(y, self._touched(), A, B, p=1)
        return A

    def admissible(self, y, A2):
        """The trial-mesh conditions besides the descent: spacing ratios and conditioning."""
        return (spacing_ratio_ok(y) and cond1(A2) <= self.cond_max
                and cond1(self.a1(y)) <= self.cond1_max)

    def L_from(self, x, y, A, B):
        e = homogeneous_error(y, self.kstar, A, B)
        return e + self.C * float(np.linalg.norm(x - self.x_ref)), e

    def L(self, x):
        y = self.mesh(x)
        return self.L_from(x, y, *self.operators(y))[0]

    def L_moved(self, x, A, B, j, h):
        """L with node j+1 (and its mirror) moved by h; A, B are the operators at x."""
        n = self.n
        xm = x.copy()
        xm[j] += h
        y = self.mesh(xm)
        i0 = j + 1
        rows = [i for i in range(i0 - compact.HALF, i0 + compact.HALF + 1) if 0 <= i < n]
        rows += [n - 1 - i for i in rows]
        A, B = A.copy(), B.copy()
        _rows(y, sorted(set(rows)), A, B)
        return self.L_from(xm, y, A, B)[0]


def optimise_mesh(y_ref, m=20, kstar=1e10, penalty=1e-3, max_iter=60, history=None):
    """Steepest descent on L; returns (y_opt, err_ref, err_opt, iterations).

    ``history``, if a list, receives L after every accepted step.
    """
    P = _Problem(y_ref, m, kstar, penalty)
    x = P.x_ref.copy()
    y = P.mesh(x)
    A, B = P.operators(y)
    f, err_ref = P.L_from(x, y, A, B)
    t = 1.0
    it = 0
    while it < max_iter:
        grad = np.empty(m)
        for j in range(m):
            h = FD_REL * P.s[j]
            grad[j] = (P.L_moved(x, A, B, j, h) - P.L_moved(x, A, B, j, -h)) / (2.0 * h)
        d = -(P.s ** 2) * grad
        slope = float(np.dot(grad, d))
        t *= 2.0
        accepted = False
        while t >= T_MIN:
            xn = x + t * d
            yn = P.mesh(xn)
            if np.all(np.diff(yn) > 0):
                An, Bn = P.operators(yn)
                fn = P.L_from(xn, yn, An, Bn)[0]
                if fn < f and fn <= f + ARMIJO * t * slope and P.admissible(yn, An):
                    accepted = True
                    break
            t *= 0.5
        if not accepted:
            break
        x, f, A, B = xn, fn, An, Bn
        it += 1
        if history is not None:
            history.append(f)
    y = P.mesh(x)
    return y, err_ref, homogeneous_error(y, kstar, A, B), it
