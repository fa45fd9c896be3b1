"""Fourier projection in the periodic directions with 3/2-rule padding (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 2.1 / Appendix A: fields are expanded on N1/2 x N3/2 Fourier modes per
wall-parallel plane; products are formed on a grid padded to 3N1/2 x 3N3/2
collocation points (zero padding to 3N/4 modes per direction) and truncated
back.  Conventions (readings of the paper, which does not state them):

* spectral plane ``uh[kx, kz]``: kx = 0..n1/2-1, kz in FFT slot order over n3
  slots, slot n3/2 (Nyquist) always zero; the field is real, so the kx < 0 half
  is the complex conjugate and is not stored.
* inverse (synthesis) is unscaled: u(x_p, z_q) = sum over the Hermitian-complete
  mode set of uh e^{i(a x_p + b z_q)}, x_p = p L1/P1, z_q = q L3/P3.
* forward (analysis) is scaled by 1/(P1 P3) and keeps |kz| < n3/2, kx < n1/2.

scipy's FFTs (pocketfft) are the library steps; the tests pin them to
brute-force DFT sums.  ``WORKERS`` threads split a batch of planes (1 unless
a caller, such as the benchmark's all-cores CPU baseline, raises it; the
results do not depend on it).  Physical planes are ``f[z, x]`` (P3 rows of
P1 points).
"""
from __future__ import annotations

import numpy as np
import scipy.fft

WORKERS = 1


def padded_size(n):
    return 3 * n // 2


def _zslots(n3, p3):
    """Map stored kz slots (non-Nyquist) to slots of a length-p3 FFT."""
    src = np.array([k for k in range(n3) if k != n3 // 2])
    kz = np.where(src < n3 // 2, src, src - n3)
    dst = np.where(kz >= 0, kz, p3 + kz)
    return src, dst


def to_physical(uh, p1, p3):
    """uh[..., kx, kz] -> real f[..., z, x] on the p3 x p1 grid."""
    n1h, n3 = uh.shape[-2], uh.shape[-1]
    src, dst = _zslots(n3, p3)
    F = np.zeros(uh.shape[:-2] + (p3, p1 // 2 + 1), dtype=np.complex128)
    F[..., dst, :n1h] = np.swapaxes(uh, -1, -2)[..., src, :]
    # kx = 0 column: the real-signal synthesis uses its Hermitian part only
    return scipy.fft.irfft2(F, s=(p3, p1), workers=WORKERS) * (p1 * p3)


def to_spectral(f, n1, n3):
    """Real f[..., z, x] -> uh[..., kx, kz] (kx < n1/2, |kz| < n3/2), scaled 1/(P1 P3)."""
    p3, p1 = f.shape[-2], f.shape[-1]
    F = scipy.fft.rfft2(f, workers=WORKERS) / (p1 * p3)
    src, dst = _zslots(n3, p3)
    out = np.zeros(f.shape[:-2] + (n1 // 2, n3), dtype=np.complex128)
    out[..., :, src] = np.swapaxes(F[..., dst, : n1 // 2], -1, -2)
    return out
