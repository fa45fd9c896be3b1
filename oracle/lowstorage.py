"""Low-storage database stage: sharp cut-off filter, filtered stresses, SGS tensor,
filtered enstrophy (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 3.1 of the paper: the velocities are truncated in Fourier space in the
two wall-parallel directions only (no filtering in y); the database also keeps
the truncated products u_i u_j, from which the sub-grid stress
tau_ij = F(u_i u_j) - F(u_i) F(u_j) follows.  Readings:

* the retained set is K_c = {0 <= kx <= kcx, |kz| <= kcz} in index units (the
  printed filter has garbled arguments and uses strict "<" without absolute
  values; the inclusive form is used here),
* the products u_i u_j of the full fields are formed on the 3/2 padded grid,
  which represents every retained product mode exactly,
* tau_ij is evaluated pointwise on a (q3, q1) grid of the periodic plane,
  from the zero-padded inverse transforms of F(u_i) and F(u_i u_j),
* the SGS definition's typo (a repeated index j) is read as tau_ij = F(u_i u_j) - F(u_i) F(u_j),
* tau_ij is unchanged when a plane-constant field c_i(y) is added to u_i (F
  keeps the (0,0) mode, so the c_i c_j and c_i F(u_j) terms cancel exactly);
  tau is therefore evaluated from the fluctuations u_i - <u_i>, which avoids
  cancelling the large U_i U_j terms in rounding.  F(u_i u_j) itself is
  formed from the full fields.

The tenth variable of the database is the filtered enstrophy
F(omega_i omega_i): the sum of the squared vorticity components, formed from
the full vorticity (mean shear included) on the 3/2 padded grid like the
products u_i u_j, then cut off to K_c.

Output layouts: retained modes ``[n2][kcx+1][2kcz+1]`` with kz in FFT slot
order (0..kcz, then -kcz..-1); tau ``[6][n2][q3][q1]`` for the pairs
(11, 12, 13, 22, 23, 33).
"""
from __future__ import annotations

import numpy as np

from . import compact, fourier

PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def kc_slots(n3, kcz):
    """Stored kz slots (over n3) of the retained kz values, in output order."""
    kz = list(range(0, kcz + 1)) + list(range(-kcz, 0))
    return np.array([k if k >= 0 else n3 + k for k in kz])


def truncate(uh, kcx, kcz):
    """F(u) on K_c from a full field uh[n2][n1/2][n3]."""
    n3 = uh.shape[-1]
    return uh[..., : kcx + 1, :][..., kc_slots(n3, kcz)]


def synth_plane(ch, q1, q3):
    """Real field on the (q3, q1) grid from retained coefficients ch[..., kcx+1, 2kcz+1]."""
    kcx1, nz = ch.shape[-2], ch.shape[-1]
    kcz = (nz - 1) // 2
    F = np.zeros(ch.shape[:-2] + (q3, q1 // 2 + 1), dtype=np.complex128)
    kz = np.array(list(range(0, kcz + 1)) + list(range(-kcz, 0)))
    F[..., kz % q3, :kcx1] = np.swapaxes(ch, -1, -2)
    return np.fft.irfft2(F, s=(q3, q1)) * (q1 * q3)


def filter_and_stress(u1, u2, u3, kcx, kcz, q1, q3):
    """Returns (ubar[3], uubar[6], tau[6]) as described in the module docstring."""
    n2, n1h, n3 = u1.shape
    n1 = 2 * n1h
    p1, p3 = fourier.padded_size(n1), fourier.padded_size(n3)
    ub = np.stack([truncate(u, kcx, kcz) for u in (u1, u2, u3)])

    def filtered_products(fields):
        phys = [fourier.to_physical(u, p1, p3) for u in fields]
        return np.stack([truncate(fourier.to_spectral(phys[i] * phys[j], n1, n3), kcx, kcz) for i, j in PAIRS])

    uu = filtered_products((u1, u2, u3))
    # tau from the fluctuations (plane means removed, see the module docstring)
    fl = []
    for u in (u1, u2, u3):
        f = np.array(u, copy=True)
        f[:, 0, 0] = 0.0
        fl.append(f)
    ubq = synth_plane(np.stack([truncate(f, kcx, kcz) for f in fl]), q1, q3)
    uuq = synth_plane(filtered_products(fl), q1, q3)
    tau = np.stack([uuq[p] - ubq[i] * ubq[j] for p, (i, j) in enumerate(PAIRS)])
    return ub, uu, tau


def filtered_enstrophy(om1, om2, om3, kcx, kcz):
    """F(omega_i omega_i) on K_c from the full vorticity fields om*[n2][n1/2][n3] (Section 3.1)."""
    n2, n1h, n3 = om1.shape
    n1 = 2 * n1h
    p1, p3 = fourier.padded_size(n1), fourier.padded_size(n3)
    e = np.zeros((n2, p3, p1))
    for w in (om1, om2, om3):
        e += fourier.to_physical(w, p1, p3) ** 2
    return truncate(fourier.to_spectral(e, n1, n3), kcx, kcz)


def spectra(u1, u2, u3):
    """Two-dimensional spectra |u_i(kx, y, kz)|^2 of one sample (the paper's E_ii
    before the ensemble average), on the stored half-plane of modes, with the
    mean mode (0,0) set to zero (fluctuations only): [3][n2][n1/2][n3]."""
    E = np.stack([np.abs(u) ** 2 for u in (u1, u2, u3)])
    E[:, :, 0, 0] = 0.0
    return E


def rms_profiles(E):
    """Plane-mean squared fluctuations <u'_i u'_i>(y) from spectra E[3][n2][n1/2][n3]
    (Parseval: a stored kx > 0 mode stands for +kx and -kx)."""
    w = np.full(E.shape[-2], 2.0)
    w[0] = 1.0
    return np.einsum("iykz,k->iy", E, w)


def filtered_pressure(S, uu, ub, kcx, kcz):
    """Filtered pressure on K_c from F(u_i u_j) uu[6][n2][kcx+1][2kcz+1] (pairs 11, 12,
    13, 22, 23, 33) and F(u_i) ub[3][...] (Section 3.1: d_kk p = -d_i d_j F(u_i u_j)).

    Readings (the paper states the Poisson equation only):
    * per retained mode (kx, kz) != (0, 0) the interior rows take the A-form of
      the implicit steps, (B2 - k^2 A2) p = A2 r with r = -d_i d_j F(u_i u_j),
      d_x -> i a, d_z -> i b, d_y -> the compact D1 (D2 for the 22 term);
    * the wall rows are the wall-normal filtered momentum equation at a wall,
      where the velocity and hence F(u_2 u_j) and its wall-parallel derivatives
      vanish: D1 p = nu D2 F(v), with the full compact rows of D1 and D2;
    * mode (0, 0): the mean wall-normal momentum balance, P = -F(u_2 u_2)(0, 0)
      (the additive constant chosen so that P = 0 at the walls).
    Dense linear algebra, one mode at a time.  Returns p[n2][kcx+1][2kcz+1]."""
    A1, B1 = compact.band_to_dense(S.A1), compact.band_to_dense(S.B1)
    A2, B2 = compact.band_to_dense(S.A2), compact.band_to_dense(S.B2)
    D1 = np.linalg.solve(A1, B1)
    D2 = np.linalg.solve(A2, B2)
    kzs = list(range(0, kcz + 1)) + list(range(-kcz, 0))
    p = np.zeros(uu.shape[1:], dtype=np.complex128)
    for ix in range(kcx + 1):
        for iz, kz in enumerate(kzs):
            u11, u12, u13, u22, u23, u33 = (uu[q][:, ix, iz] for q in range(6))
            if ix == 0 and kz == 0:
                p[:, 0, 0] = -u22.real
                continue
            a, b = 2 * np.pi * ix / S.lx, 2 * np.pi * kz / S.lz
            r = -((1j * a) ** 2 * u11 + 2 * (1j * a) * (D1 @ u12) + 2 * (1j * a) * (1j * b) * u13
                  + D2 @ u22 + 2 * (1j * b) * (D1 @ u23) + (1j * b) ** 2 * u33)
            M = B2 - (a * a + b * b) * A2
            M[0], M[-1] = D1[0], D1[-1]
            rhs = A2 @ r
            g = S.nu * (D2 @ ub[1][:, ix, iz])
            rhs[0], rhs[-1] = g[0], g[-1]
            p[:, ix, iz] = np.linalg.solve(M, rhs)
    return p
