"""Orr-Sommerfeld eigenvalues of plane Poiseuille flow by Chebyshev collocation (oracle pin).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

An independent check on the time stepper: a small-amplitude two-dimensional
eigenmode evolved by the RK3 solver must grow at the rate alpha * c_i of the
linear stability problem

  (U - c)(v'' - alpha^2 v) - U'' v = (v'''' - 2 alpha^2 v'' + alpha^4 v) / (i alpha Re),
  v = v' = 0 at y = +-1,   U = 1 - y^2 (centre-line units).

Clamped conditions are built in by writing v = (1 - y^2) phi with phi = 0 at
the ends.  Reference value for the pin: Orszag (1971), Re = 10^4, alpha = 1,
c = 0.23752649 + 0.00373967 i.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as C


def cheb(n):
    """Chebyshev points x_j = cos(pi j/n) and the differentiation matrix (Trefethen's construction)."""
    x = np.cos(np.pi * np.arange(n + 1) / n)
    c = np.r_[2.0, np.ones(n - 1), 2.0] * (-1.0) ** np.arange(n + 1)
    X = np.tile(x, (n + 1, 1)).T
    dX = X - X.T
    D = np.outer(c, 1 / c) / (dX + np.eye(n + 1))
    D = D - np.diag(D.sum(axis=1))
    return D, x


def least_stable(re, alpha, n=128):
    """(c, v) of the least stable mode; v sampled at the Chebyshev points (ends included)."""
    D, x = cheb(n)
    D2 = D @ D
    D3 = D2 @ D
    D4 = D3 @ D
    I = np.eye(n + 1)
    X = np.diag(x)
    W = np.diag(1 - x ** 2)
    # exact derivatives of v = (1 - y^2) p(y), p the interpolant of phi
    V0 = W
    V2 = -2 * I - 4 * X @ D + W @ D2
    V4 = -12 * D2 - 8 * X @ D3 + W @ D4
    U = 1 - x ** 2
    Upp = -2.0 * np.ones(n + 1)
    L2 = V2 - alpha ** 2 * V0
    L4 = V4 - 2 * alpha ** 2 * V2 + alpha ** 4 * V0
    A = np.diag(U) @ L2 - np.diag(Upp) @ V0 - L4 / (1j * alpha * re)
    B = L2
    inner = slice(1, n)
    A, B = A[inner, inner], B[inner, inner]
    import scipy.linalg as sl
    w, V = sl.eig(A, B)
    # discard the spurious eigenvalues of the collocated pencil (infinite or far
    # outside the physical range 0 < c_r < 1 of the base flow)
    ok = np.isfinite(w) & (np.abs(w) < 2.0)
    w, V = w[ok], V[:, ok]
    k = np.argmax(w.imag)
    phi = np.zeros(n + 1, dtype=complex)
    phi[inner] = V[:, k]
    v = (1 - x ** 2) * phi
    v = v / v[np.argmax(np.abs(v))]
    return w[k], x, v


def eigenfunction_on(y, re, alpha, n=128):
    """Least-stable eigenvalue and its v(y) interpolated (exactly, degree n) onto mesh y."""
    c, x, v = least_stable(re, alpha, n)
    coef_r = C.chebfit(x, v.real, n)
    coef_i = C.chebfit(x, v.imag, n)
    return c, C.chebval(y, coef_r) + 1j * C.chebval(y, coef_i)
