"""Brute-force Fourier sums on tiny grids (oracle pins).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Direct O(N^2) evaluations with no FFT, used to pin the transform conventions,
the dealiased products and the filtered-stress stage: a direct DFT of a plane,
the exact convolution of two band-limited fields over the Hermitian-complete
mode set, and direct Fourier synthesis at arbitrary points.
"""
from __future__ import annotations

import numpy as np


def full_modes(uh):
    """Hermitian-complete dict {(kx, kz): coefficient} of a stored plane uh[kx, kz]."""
    n1h, n3 = uh.shape
    out = {}
    for kx in range(n1h):
        for s in range(n3):
            if s == n3 // 2:
                continue
            kz = s if s < n3 // 2 else s - n3
            c = uh[kx, s]
            if c == 0:
                continue
            if kx == 0:
                # the kx = 0 line of a real field contributes its Hermitian part
                out[(0, kz)] = out.get((0, kz), 0) + 0.5 * c
                out[(0, -kz)] = out.get((0, -kz), 0) + 0.5 * np.conj(c)
            else:
                out[(kx, kz)] = out.get((kx, kz), 0) + c
                out[(-kx, -kz)] = out.get((-kx, -kz), 0) + np.conj(c)
    return out


def synth_points(modes, lx, lz, x, z):
    """u(x, z) = sum_k c_k exp(i(a x + b z)) evaluated directly (real part)."""
    u = np.zeros(np.broadcast_shapes(np.shape(x), np.shape(z)), dtype=np.complex128)
    for (kx, kz), c in modes.items():
        u += c * np.exp(1j * (2 * np.pi * kx / lx * x + 2 * np.pi * kz / lz * z))
    return u.real


def dft_plane(f, lx, lz, kx, kz):
    """(1/(P1 P3)) sum_{p,q} f[q, p] exp(-i(a x_p + b z_q)) for one mode."""
    p3, p1 = f.shape
    x = np.arange(p1) * lx / p1
    z = np.arange(p3) * lz / p3
    ph = np.exp(-1j * (2 * np.pi * kx / lx * x[None, :] + 2 * np.pi * kz / lz * z[:, None]))
    return np.sum(f * ph) / (p1 * p3)


def product_modes(ma, mb):
    """Exact convolution: coefficients of the product of two band-limited fields."""
    out = {}
    for (ax, az), ca in ma.items():
        for (bx, bz), cb in mb.items():
            k = (ax + bx, az + bz)
            out[k] = out.get(k, 0) + ca * cb
    return out
