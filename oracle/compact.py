"""Compact finite differences on the non-uniform wall-normal mesh (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Appendix B: a derivative is the solution of a banded problem A d = B f, with
A and B seven-banded.  Row i's coefficients solve one small linear system that
makes the scheme exact for the monomials (y - y_i)^k; at the rows nearest
each wall the stencil is truncated to the nodes that exist, keeping maximum
order.  The paper's equation for this system is garbled; the reading used
here is:

  stencil S_i = {max(0, i-3) .. min(n-1, i+3)}, w = |S_i| nodes,
  unknowns B_ij, A_ij (j in S_i), 2w of them,
  for k = 0 .. 2w-2:   sum_j B_ij d_j^k = D_k sum_j A_ij d_j^(k-p),
      d_j = y_j - y_i,  p = derivative order,
      D_k = k(k-1) (second derivative) or k (first derivative), 0 if k < p,
  normalisation A_ii = 1.

The system is solved in exact rational arithmetic from the float64 mesh
values (``fractions.Fraction``), so each coefficient is the correctly rounded
float64 of the exact solution; the paper's row premultiplication (a
conditioning device for a floating-point solve) has no effect on an exact
solve and is therefore not needed here.

Band storage: ``band[i][3 + o]`` holds M[i, i + o] for o = -3..3.
"""
from __future__ import annotations

import functools
from fractions import Fraction

import numpy as np

HALF = 3
NB = 2 * HALF + 1


def _solve_exact(M, r):
    """Gaussian elimination with exact rationals (first nonzero pivot)."""
    n = len(M)
    M = [row[:] + [r[i]] for i, row in enumerate(M)]
    for c in range(n):
        p = next(k for k in range(c, n) if M[k][c] != 0)
        M[c], M[p] = M[p], M[c]
        inv = 1 / M[c][c]
        for k in range(c + 1, n):
            f = M[k][c]
            if f:
                f = f * inv
                rk, rc = M[k], M[c]
                for j in range(c, n + 1):
                    rk[j] -= f * rc[j]
    x = [Fraction(0)] * n
    for c in range(n - 1, -1, -1):
        s = M[c][n]
        for j in range(c + 1, n):
            s -= M[c][j] * x[j]
        x[c] = s / M[c][c]
    return x


def row_coefficients(y, i, p, half=HALF):
    """Exact compact-scheme coefficients of row i for derivative order p (1 or 2).

    ``half`` is the stencil half-width (3 for the seven-point scheme of the
    paper; narrower widths reproduce the classical tri/penta-diagonal schemes).
    Returns (S, A_row, B_row) with Fractions, S the stencil indices.
    """
    n = len(y)
    S = list(range(max(0, i - half), min(n - 1, i + half) + 1))
    w = len(S)
    yi = Fraction(float(y[i]))
    d = [Fraction(float(y[j])) - yi for j in S]
    M, r = [], []
    for k in range(2 * w - 1):
        row = [dj ** k for dj in d]
        if k >= p:
            fac = k * (k - 1) if p == 2 else k
            row += [-fac * dj ** (k - p) for dj in d]
        else:
            row += [Fraction(0)] * w
        M.append(row)
        r.append(Fraction(0))
    norm = [Fraction(0)] * (2 * w)
    norm[w + S.index(i)] = Fraction(1)
    M.append(norm)
    r.append(Fraction(1))
    sol = _solve_exact(M, r)
    return S, sol[w:], sol[:w]


@functools.lru_cache(maxsize=16)
def _operators_cached(ykey: bytes, p: int):
    y = np.frombuffer(ykey, dtype=np.float64)
    n = len(y)
    A = np.zeros((n, NB))
    B = np.zeros((n, NB))
    for i in range(n):
        S, a, b = row_coefficients(y, i, p)
        for j, aj, bj in zip(S, a, b):
            A[i, HALF + j - i] = float(aj)
            B[i, HALF + j - i] = float(bj)
    A.setflags(write=False)
    B.setflags(write=False)
    return A, B


def operators(y, p):
    """Banded (A, B) of the compact p-th derivative on mesh y: A f^(p) = B f."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    return _operators_cached(y.tobytes(), p)


def band_to_dense(band):
    n = band.shape[0]
    M = np.zeros((n, n))
    for i in range(n):
        for o in range(-HALF, HALF + 1):
            j = i + o
            if 0 <= j < n:
                M[i, j] = band[i, HALF + o]
    return M


@functools.lru_cache(maxsize=16)
def _quad_cached(ykey: bytes):
    y = [Fraction(float(v)) for v in np.frombuffer(ykey, dtype=np.float64)]
    n = len(y)
    w = [Fraction(0)] * n
    for j in range(n - 1):
        # degree-5 Lagrange interpolant through 6 nodes around [y_j, y_{j+1}]
        lo = min(max(j - 2, 0), n - 6) if n >= 6 else 0
        nodes = list(range(lo, min(lo + 6, n)))
        a, b = y[j], y[j + 1]
        for m in nodes:
            # integral over [a, b] of the Lagrange basis polynomial of node m
            coeffs = [Fraction(1)]  # polynomial in t, ascending powers
            den = Fraction(1)
            for q in nodes:
                if q == m:
                    continue
                coeffs = [Fraction(0)] + coeffs  # multiply by t
                for c in range(len(coeffs) - 1):
                    coeffs[c] -= y[q] * coeffs[c + 1]
                den *= (y[m] - y[q])
            integ = sum(c * (b ** (e + 1) - a ** (e + 1)) / (e + 1) for e, c in enumerate(coeffs))
            w[m] += integ / den
    return np.array([float(v) for v in w])


def quadrature_weights(y):
    """Weights w with w.f = integral of f over [-1, 1], exact for degree <= 5.

    Each interval [y_j, y_j+1] integrates the degree-5 Lagrange interpolant
    through nodes j-2 .. j+3, the window shifted to stay inside the mesh.
    """
    y = np.ascontiguousarray(y, dtype=np.float64)
    return _quad_cached(y.tobytes())
