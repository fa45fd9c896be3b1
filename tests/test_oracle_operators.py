"""Pins of the oracle's wall-normal operators, banded solver and Fourier transforms.

Each check is against something other than the oracle's own formula: the
classical compact schemes of Lele (1992) that the construction must reduce to
for narrower stencils, polynomial exactness, convergence order, the analytic
solution of the homogeneous Helmholtz problem (Appendix B), numpy's dense LU,
brute-force DFT sums and Parseval's identity.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import synth
from oracle import banded, brute, compact, fourier, kmm


# ---------------------------------------------------------------- compact FD
@pytest.mark.parametrize("half,p,A,B", [
    # Lele (1992): tridiagonal fourth-order schemes
    (1, 1, [F(1, 4), 1, F(1, 4)], [F(-3, 4), 0, F(3, 4)]),
    (1, 2, [F(1, 10), 1, F(1, 10)], [F(6, 5), F(-12, 5), F(6, 5)]),
    # Lele (1992): pentadiagonal eighth-order schemes (alpha=4/9, beta=1/36,
    # a=40/27, b=25/54 for f'; alpha=344/1179, beta=23/2358, a=320/393,
    # b=310/393 for f'')
    (2, 1, [F(1, 36), F(4, 9), 1, F(4, 9), F(1, 36)],
     [F(-25, 216), F(-20, 27), 0, F(20, 27), F(25, 216)]),
    (2, 2, [F(23, 2358), F(344, 1179), 1, F(344, 1179), F(23, 2358)],
     [F(155, 786), F(320, 393), F(-265, 131), F(320, 393), F(155, 786)]),
])
def test_compact_reduces_to_classical_schemes(half, p, A, B):
    y = np.arange(-6, 7) * 1.0  # unit spacing
    S, a, b = compact.row_coefficients(y, 6, p, half)
    assert [F(v) for v in A] == a
    assert [F(v) for v in B] == b


@pytest.mark.parametrize("p", [1, 2])
def test_compact_polynomial_exactness(p):
    """Each row is exact for polynomials up to its order (12 inside, lower at the walls)."""
    y = synth.mesh_tanh(33)
    A, B = compact.operators(y, p)
    Ad, Bd = compact.band_to_dense(A), compact.band_to_dense(B)
    for i in range(len(y)):
        w = min(len(y) - 1, i + 3) - max(0, i - 3) + 1
        for k in range(0, 2 * w - 1):
            d = y - y[i]
            f = d ** k  # monomials centred on the row (well scaled)
            if k < p:
                df = 0 * y
            elif p == 1:
                df = k * d ** (k - 1)
            else:
                df = k * (k - 1) * d ** (k - 2)
            lhs = Bd[i] @ f
            rhs = Ad[i] @ df
            scale = np.abs(Bd[i]).max() * np.abs(f).max() + np.abs(Ad[i]).max() * np.abs(df).max()
            assert abs(lhs - rhs) <= 1e-13 * scale, (i, k)


@pytest.mark.parametrize("p", [1, 2])
def test_compact_twelfth_order_truncation(p):
    """Interior local truncation error of the seven-point schemes falls like h^12 (uniform grid)."""
    errs = {}
    k = 6.0
    for n in (17, 33):
        y = np.linspace(-1, 1, n)
        A, B = compact.operators(y, p)
        f = np.sin(k * y + 0.3)
        df = k * np.cos(k * y + 0.3) if p == 1 else -k * k * f
        r = compact.band_to_dense(B) @ f - compact.band_to_dense(A) @ df
        errs[n] = np.abs(r[n // 2 - 1:n // 2 + 2]).max()
    order = np.log2(errs[17] / errs[33])
    assert 11.3 < order < 13.0, errs


def test_compact_derivatives_accurate_on_mesh():
    y = synth.mesh_tanh(65)
    S = kmm.Setup(n1=4, n2=65, n3=4, lx=2 * np.pi, lz=np.pi, nu=1e-3, dt=1e-3, mass_flux=2, y=y)
    f = np.sin(3 * y + 0.2)
    assert np.abs(kmm.d1(S, f) - 3 * np.cos(3 * y + 0.2)).max() < 1e-9
    assert np.abs(kmm.d2(S, f) + 9 * f).max() < 1e-6


def test_quadrature_exact_to_degree_five():
    y = synth.mesh_tanh(33)
    w = compact.quadrature_weights(y)
    for k in range(6):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(w @ y ** k - exact) < 1e-14


# ---------------------------------------------------------------- banded solver
def _random_band(rng, n, dominant):
    band = rng.standard_normal((n, 7))
    if dominant:
        band[:, 3] = 8 + np.abs(rng.standard_normal(n))
    else:
        band[:, 3] += 2.5
    for i in range(n):
        for o in range(-3, 4):
            if not 0 <= i + o < n:
                band[i, 3 + o] = 0
    return band


@pytest.mark.parametrize("dominant", [True, False])
def test_banded_solve_matches_dense_lu(dominant):
    rng = np.random.default_rng(5)
    n = 23
    band = _random_band(rng, n, dominant)
    M = compact.band_to_dense(band)
    rhs = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
    x = banded.solve(band, rhs)
    ref = np.linalg.solve(M, rhs)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(banded.matvec(band, rhs) - M @ rhs).max() < 1e-12


def test_banded_solve_batched_matrices():
    rng = np.random.default_rng(6)
    n, m = 17, 5
    bands = np.stack([_random_band(rng, n, True) for _ in range(m)], axis=-1)  # [n][7][m]
    rhs = rng.standard_normal((n, m))
    x = banded.solve(bands, rhs)
    for j in range(m):
        ref = np.linalg.solve(compact.band_to_dense(bands[..., j]), rhs[:, j])
        assert np.abs(x[:, j] - ref).max() < 1e-12


@pytest.mark.parametrize("kstar", [1.0, 50.0, 2000.0])
def test_homogeneous_helmholtz_matches_sinh(kstar):
    """(B - k* A) g = 0, g(-1) = 1, g(1) = 0 approximates sinh(sqrt(k*)(1-y))/sinh(2 sqrt(k*))."""
    y = synth.mesh_tanh(97)
    S = kmm.Setup(n1=4, n2=97, n3=4, lx=2 * np.pi, lz=np.pi, nu=1e-3, dt=1e-3, mass_flux=2, y=y)
    c = 1.0 / kstar  # (1 - c D2) g = 0  <=>  (B - A/c) g = 0
    g = kmm.helmholtz(S, np.zeros(97), c, 0.0, lo=1.0, hi=0.0)
    s = np.sqrt(kstar)
    exact = np.sinh(s * (1 - y)) / np.sinh(2 * s)
    assert g[0] == 1.0 and g[-1] == 0.0
    assert np.abs(g - exact).max() < 2e-6


# ---------------------------------------------------------------- transforms
def _random_plane(rng, n1, n3):
    uh = rng.standard_normal((n1 // 2, n3)) + 1j * rng.standard_normal((n1 // 2, n3))
    uh[:, n3 // 2] = 0
    for kz in range(1, n3 // 2):
        uh[0, n3 - kz] = np.conj(uh[0, kz])
    uh[0, 0] = uh[0, 0].real
    return uh


def test_inverse_transform_brute_force():
    rng = np.random.default_rng(1)
    n1, n3, lx, lz = 8, 6, 2 * np.pi, np.pi
    uh = _random_plane(rng, n1, n3)
    p1, p3 = fourier.padded_size(n1), fourier.padded_size(n3)
    f = fourier.to_physical(uh, p1, p3)
    x = np.arange(p1) * lx / p1
    z = np.arange(p3) * lz / p3
    ref = brute.synth_points(brute.full_modes(uh), lx, lz, x[None, :], z[:, None])
    assert np.abs(f - ref).max() < 1e-13


def test_forward_transform_brute_force():
    rng = np.random.default_rng(2)
    n1, n3, lx, lz = 8, 8, 2 * np.pi, np.pi
    p1, p3 = fourier.padded_size(n1), fourier.padded_size(n3)
    f = rng.standard_normal((p3, p1))
    uh = fourier.to_spectral(f, n1, n3)
    for kx in range(n1 // 2):
        for s in range(n3):
            kz = s if s < n3 // 2 else s - n3
            ref = 0 if s == n3 // 2 else brute.dft_plane(f, lx, lz, kx, kz)
            assert abs(uh[kx, s] - ref) < 1e-14


def test_parseval_and_round_trip():
    rng = np.random.default_rng(3)
    n1, n3 = 48, 32
    uh = _random_plane(rng, n1, n3)
    p1, p3 = fourier.padded_size(n1), fourier.padded_size(n3)
    f = fourier.to_physical(uh, p1, p3)
    wts = np.where(np.arange(n1 // 2)[:, None] == 0, 1.0, 2.0)
    assert abs(np.mean(f ** 2) - np.sum(wts * np.abs(uh) ** 2)) < 1e-12 * np.mean(f ** 2)
    assert np.abs(fourier.to_spectral(f, n1, n3) - uh).max() < 1e-14


def test_dealiased_product_cosines():
    """cos(m x) cos(n x) keeps exactly 1/2 cos((m+n) x) + 1/2 cos((m-n) x); nothing aliases back."""
    n1, n3 = 16, 4
    p1, p3 = fourier.padded_size(n1), fourier.padded_size(n3)
    for m in range(1, n1 // 2):
        for n in range(1, n1 // 2):
            a = np.zeros((n1 // 2, n3), complex)
            b = np.zeros((n1 // 2, n3), complex)
            a[m, 0] = 0.5  # cos(m x) = (e^{imx} + e^{-imx})/2
            b[n, 0] = 0.5
            prod = fourier.to_physical(a, p1, p3) * fourier.to_physical(b, p1, p3)
            h = fourier.to_spectral(prod, n1, n3)
            ref = np.zeros_like(h)
            for k, c in ((m + n, 0.25), (abs(m - n), 0.25 if m != n else 0.5)):
                if k < n1 // 2:
                    ref[k, 0] += c
            assert np.abs(h - ref).max() < 1e-15, (m, n)
