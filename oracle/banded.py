"""Seven-banded matrix products and solves (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Band storage: ``band[i, 3 + o]`` = M[i, i + o], o = -3..3.  A band may carry
trailing batch axes (``band[i, c, ...]``), one matrix per batch entry; the
right-hand side is ``rhs[i, ...]`` with matching batch axes.  The solve is
plain Gaussian elimination without pivoting restricted to the band, batched
over independent systems; it is pinned against numpy's dense LU solve in the
tests.
"""
from __future__ import annotations

import numpy as np

HALF = 3


def matvec(band, x):
    """y = M x along axis 0 (x: [n, ...])."""
    n = x.shape[0]
    y = np.zeros((n,) + np.broadcast_shapes(band.shape[2:], x.shape[1:]),
                 dtype=np.result_type(band, x))
    for o in range(-HALF, HALF + 1):
        lo, hi = max(0, -o), min(n, n - o)
        y[lo:hi] += _expand(band[lo:hi, HALF + o], x.ndim) * x[lo + o:hi + o]
    return y


def _expand(c, ndim):
    """Append unit axes so a per-row coefficient broadcasts over x's trailing axes."""
    return c.reshape(c.shape + (1,) * (ndim - c.ndim))


def solve(band, rhs):
    """x with M x = rhs, Gaussian elimination restricted to the band, no pivoting."""
    n = rhs.shape[0]
    dt = np.result_type(band, rhs)
    bshape = np.broadcast_shapes(band.shape[2:], rhs.shape[1:])
    U = np.zeros((n, HALF + 1) + band.shape[2:], dtype=band.dtype)
    yv = np.zeros((n,) + bshape, dtype=dt)
    for i in range(n):
        row = np.array(band[i], dtype=band.dtype, copy=True)  # entries at cols i-3..i+3
        r = np.array(rhs[i], dtype=dt, copy=True) * np.ones(bshape, dtype=dt)
        for c in range(max(0, i - HALF), i):
            o = c - i
            l = row[HALF + o] / U[c, 0]
            for t in range(1, HALF + 1):
                row[HALF + o + t] = row[HALF + o + t] - l * U[c, t]
            r = r - l * yv[c]
        U[i] = row[HALF:]
        yv[i] = r
    x = np.zeros_like(yv)
    for i in range(n - 1, -1, -1):
        s = yv[i].copy()
        for t in range(1, HALF + 1):
            if i + t < n:
                s = s - U[i, t] * x[i + t]
        x[i] = s / U[i, 0]
    return x


def dirichlet_rows(band):
    """Copy of band with rows 0 and n-1 replaced by identity rows."""
    b = np.array(band, copy=True)
    b[0] = 0
    b[-1] = 0
    b[0, HALF] = 1
    b[-1, HALF] = 1
    return b
