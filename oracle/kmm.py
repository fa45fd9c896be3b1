"""One RK3 step of the velocity-vorticity channel solver, float64 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Appendix A of the paper (equations for chi = lap(u2) and omega2, their
non-linear forcings, the semi-implicit three-stage RK3 with the particular +
homogeneous treatment of the fourth-order u2 problem), Appendix B (compact
wall-normal operators and the discrete Helmholtz problem (B - k* A) g = 0 with
Dirichlet end values) and Section 2.1 (constant mass flux through a
time-varying mean pressure gradient; free spanwise mean).

State per Fourier mode (kx, kz): v = u2, chi, omega2 on the n2 wall-normal
nodes; mean profiles U1, U3.  Readings of points the paper leaves open are
listed in the module docstrings and in the design notes.
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction

import numpy as np

from . import banded, compact, fourier

# Spalart, Moser & Rogers (1991) low-storage semi-implicit RK3 coefficients
# (the paper cites the scheme without printing the values).
RK3_ALPHA = (Fraction(29, 96), Fraction(-3, 40), Fraction(1, 6))
RK3_BETA = (Fraction(37, 160), Fraction(5, 24), Fraction(1, 6))
RK3_GAMMA = (Fraction(8, 15), Fraction(5, 12), Fraction(3, 4))
RK3_ZETA = (Fraction(0), Fraction(-17, 60), Fraction(-5, 12))


def rk3_update(x, n_now, n_old, s, dt, lap, implicit):
    """One sub-step of the semi-implicit RK3 (Appendix A, eqs. for chi and omega2).

    x_new solves (1 - dt beta_s L) x_new = x + dt (alpha_s L x + gamma_s N + zeta_s N_old),
    where ``lap(x)`` applies L and ``implicit(r, c)`` solves (1 - c L) x = r.
    """
    al, be, ga, ze = (float(c[s]) for c in (RK3_ALPHA, RK3_BETA, RK3_GAMMA, RK3_ZETA))
    r = x + dt * (al * lap(x) + ga * n_now + ze * n_old)
    return implicit(r, dt * be)


@dataclasses.dataclass
class Setup:
    n1: int
    n2: int
    n3: int
    lx: float
    lz: float
    nu: float
    dt: float
    mass_flux: float
    y: np.ndarray

    def __post_init__(self):
        self.p1 = fourier.padded_size(self.n1)
        self.p3 = fourier.padded_size(self.n3)
        kx = np.arange(self.n1 // 2)
        kz = np.fft.fftfreq(self.n3, 1.0 / self.n3)
        kz[self.n3 // 2] = 0
        self.a = (2 * np.pi / self.lx) * kx[:, None] * np.ones((1, self.n3))
        self.b = (2 * np.pi / self.lz) * kz[None, :] * np.ones((self.n1 // 2, 1))
        self.k2 = self.a ** 2 + self.b ** 2
        # modes evolved by the v/omega2 equations: all but (0,0) and the Nyquist slot
        self.live = np.ones((self.n1 // 2, self.n3), bool)
        self.live[0, 0] = False
        self.live[:, self.n3 // 2] = False
        self.A1, self.B1 = compact.operators(self.y, 1)
        self.A2, self.B2 = compact.operators(self.y, 2)
        self.w = compact.quadrature_weights(self.y)


def d1(S, f):
    """Compact first derivative along axis 0: A1 f' = B1 f."""
    return banded.solve(S.A1, banded.matvec(S.B1, f))


def d2(S, f):
    """Compact second derivative along axis 0: A2 f'' = B2 f."""
    return banded.solve(S.A2, banded.matvec(S.B2, f))


def _bc(n2, lo, hi, shape):
    """Right-hand side carrying Dirichlet values in rows 0 and n2-1."""
    r = np.zeros((n2,) + shape)
    r[0], r[-1] = lo, hi
    return r


def helmholtz(S, r, c, k2, lo=0.0, hi=0.0):
    """Solve (1 - c (D2 - k2)) x = r in interior rows, x = lo/hi at the walls.

    A-form of Appendix B: ((1 + c k2) A2 - c B2) x = A2 r in rows 1..n2-2.
    ``k2`` broadcasts over the trailing axes of r.
    """
    k2 = np.asarray(k2, dtype=float)
    band = (1 + c * k2)[None, None] * S.A2[(...,) + (None,) * k2.ndim] \
        - c * S.B2[(...,) + (None,) * k2.ndim]
    band = banded.dirichlet_rows(band)
    rhs = banded.matvec(S.A2, r)
    rhs[0], rhs[-1] = lo, hi
    return banded.solve(band, rhs)


def poisson(S, chi, k2):
    """Solve (D2 - k2) v = chi in interior rows, v = 0 at the walls (A-form)."""
    k2 = np.asarray(k2, dtype=float)
    band = S.B2[(...,) + (None,) * k2.ndim] - k2[None, None] * S.A2[(...,) + (None,) * k2.ndim]
    band = banded.dirichlet_rows(band)
    rhs = banded.matvec(S.A2, chi)
    rhs[0] = 0
    rhs[-1] = 0
    return banded.solve(band, rhs)


def chi_from_v(S, v):
    """chi = lap(v) = D2 v - k^2 v."""
    return d2(S, v) - S.k2[None] * v


@dataclasses.dataclass
class State:
    v: np.ndarray
    chi: np.ndarray
    om2: np.ndarray
    U1: np.ndarray
    U3: np.ndarray

    def copy(self):
        return State(*(np.array(getattr(self, f.name), copy=True) for f in dataclasses.fields(self)))


def make_state(S, v, om2, U1, U3):
    v = np.where(S.live[None], v, 0)
    om2 = np.where(S.live[None], om2, 0)
    return State(v=v.astype(np.complex128), chi=chi_from_v(S, v), om2=om2.astype(np.complex128),
                 U1=np.array(U1, float), U3=np.array(U3, float))


def velocities(S, st):
    """u1, u3 in Fourier space from continuity (Appendix C, first steps of the sub-step).

    From i a u1 + dv/dy + i b u3 = 0 and omega2 = i b u1 - i a u3:
      u1 = i(a dv - b omega2)/k^2,  u3 = i(b dv + a omega2)/k^2;
    mode (0,0): u1 = U1, u3 = U3.
    """
    k2 = np.where(S.live, S.k2, 1.0)[None]
    dv = d1(S, st.v)
    u1 = np.where(S.live[None], 1j * (S.a * dv - S.b * st.om2) / k2, 0)
    u3 = np.where(S.live[None], 1j * (S.b * dv + S.a * st.om2) / k2, 0)
    del dv
    u1[:, 0, 0] = st.U1
    u3[:, 0, 0] = st.U3
    return u1, u3


def recover(S, st):
    """Velocities and vorticities in Fourier space (Appendix C, first steps of the sub-step).

    u1, u3 as in ``velocities``; omega1 = du3/dy - i b v, omega3 = i a v - du1/dy,
    with v = omega2 = 0 in mode (0,0).
    """
    u1, u3 = velocities(S, st)
    du1 = d1(S, u1)
    du3 = d1(S, u3)
    om1 = du3 - 1j * S.b * st.v
    om3 = 1j * S.a * st.v - du1
    return u1, st.v.copy(), u3, om1, st.om2.copy(), om3


def nonlinear(S, fields):
    """H = u x omega formed on the padded grid plane by plane, returned in Fourier space."""
    u1, u2, u3, o1, o2, o3 = (fourier.to_physical(f, S.p1, S.p3) for f in fields)
    h1 = u2 * o3 - u3 * o2
    h2 = u3 * o1 - u1 * o3
    h3 = u1 * o2 - u2 * o1
    return tuple(fourier.to_spectral(h, S.n1, S.n3) for h in (h1, h2, h3))


def physical_velocity(S, st):
    u1, u2, u3, *_ = recover(S, st)
    return tuple(fourier.to_physical(f, S.p1, S.p3) for f in (u1, u2, u3))


def cfl(S, st, dt):
    """dt * max over the padded grid of |u1|/dx + |u2|/dy_j + |u3|/dz."""
    u1, u2, u3 = physical_velocity(S, st)
    dx, dz = S.lx / S.n1, S.lz / S.n3
    gaps = np.diff(S.y)
    dy = np.minimum(np.r_[gaps[0], gaps], np.r_[gaps, gaps[-1]])
    c = np.abs(u1) / dx + np.abs(u2) / dy[:, None, None] + np.abs(u3) / dz
    return dt * c.max()


@dataclasses.dataclass
class History:
    n_chi: np.ndarray
    n_om: np.ndarray
    n_u: np.ndarray
    n_w: np.ndarray


def zero_history(S):
    z = np.zeros((S.n2, S.n1 // 2, S.n3), complex)
    return History(z, z.copy(), np.zeros(S.n2), np.zeros(S.n2))


def substep(S, st, hist, s, diag=None):
    """Sub-step s (0, 1, 2) of the RK3 step; returns (new state, new history)."""
    nu, dt = S.nu, S.dt
    al, be = float(RK3_ALPHA[s]), float(RK3_BETA[s])
    live = S.live[None]
    k2 = S.k2

    # non-linear terms (Appendix A)
    H1, H2, H3 = nonlinear(S, recover(S, st))
    n_om = np.where(live, 1j * S.b * H1 - 1j * S.a * H3, 0)
    G = 1j * (S.a * H1 + S.b * H3)
    n_chi = np.where(live, -d1(S, G) - k2 * H2, 0)
    n_u = H1[:, 0, 0].real.copy()
    n_w = H3[:, 0, 0].real.copy()

    lap = lambda f: d2(S, f) - k2[None] * f  # noqa: E731

    # omega2 with omega2 = 0 at the walls
    om2 = rk3_update(st.om2, n_om, hist.n_om, s, dt, lambda f: nu * lap(f),
                     lambda r, c: helmholtz(S, r, c * nu, k2))
    # particular chi and v
    chi_p = rk3_update(st.chi, n_chi, hist.n_chi, s, dt, lambda f: nu * lap(f),
                       lambda r, c: helmholtz(S, r, c * nu, k2))
    v_p = poisson(S, chi_p, k2)
    # homogeneous solutions: chi_h = 1 at one wall, 0 at the other (Appendix B)
    cb = dt * be * nu
    zero = np.zeros((S.n2,) + k2.shape)
    chi_lo = helmholtz(S, zero, cb, k2, lo=1.0, hi=0.0).real
    chi_hi = helmholtz(S, zero, cb, k2, lo=0.0, hi=1.0).real
    v_lo = poisson(S, chi_lo, k2)
    v_hi = poisson(S, chi_hi, k2)
    # enforce dv/dy = 0 at both walls (full compact D1 at the wall rows)
    dvp, dlo, dhi = d1(S, v_p), d1(S, v_lo), d1(S, v_hi)
    m00, m01, m10, m11 = dlo[0], dhi[0], dlo[-1], dhi[-1]
    det = np.where(live[0], m00 * m11 - m01 * m10, 1.0)
    c_lo = (-dvp[0] * m11 + dvp[-1] * m01) / det
    c_hi = (-dvp[-1] * m00 + dvp[0] * m10) / det
    v = np.where(live, v_p + c_lo * v_lo + c_hi * v_hi, 0)
    chi = np.where(live, chi_p + c_lo * chi_lo + c_hi * chi_hi, 0)
    om2 = np.where(live, om2, 0)
    if diag is not None:
        diag.append(dict(dv_wall=d1(S, v)[[0, -1]], v_wall=v[[0, -1]]))

    # mean profiles: U1 with constant mass flux, U3 free (Section 2.1)
    lap0 = lambda f: nu * d2(S, f)  # noqa: E731
    imp0 = lambda r, c: helmholtz(S, r, c * nu, 0.0).real  # noqa: E731
    U_p = rk3_update(st.U1, n_u, hist.n_u, s, dt, lap0, imp0)
    U_h = helmholtz(S, np.ones(S.n2), cb, 0.0).real
    phi = (S.mass_flux - S.w @ U_p) / (S.w @ U_h)
    U1 = U_p + phi * U_h
    f_mean = phi / (dt * (al + be))
    U3 = rk3_update(st.U3, n_w, hist.n_w, s, dt, lap0, imp0)

    new = State(v=v, chi=chi, om2=om2, U1=U1, U3=U3)
    return new, History(n_chi=n_chi, n_om=n_om, n_u=n_u, n_w=n_w), f_mean


def step(S, st, nsteps=1, diag=None):
    """nsteps full RK3 steps; returns (state, last mean pressure gradient)."""
    f = 0.0
    for _ in range(nsteps):
        hist = zero_history(S)
        for s in range(3):
            st, hist, f = substep(S, st, hist, s, diag)
    return st, f
