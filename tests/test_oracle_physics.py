"""Pins of the oracle's RK3 channel step against closed forms and invariants.

* RK3 coefficients: the explicit part reproduces the Taylor polynomial of
  exp(z) to third order and the implicit part to second order (Spalart, Moser
  & Rogers 1991), checked in exact arithmetic.
* Laminar Poiseuille flow is a steady state with pressure gradient 3 nu.
* A small Orr-Sommerfeld eigenmode grows at the rate of the linear stability
  problem (Orszag 1971: c = 0.23752649 + 0.00373967 i at Re_c = 1e4, alpha = 1).
* A wall-normal vorticity mode with no flow decays at exp(-nu (a^2 + (pi/2)^2) t).
* Every sub-step leaves v = dv/dy = 0 at the walls, the mass flux at its
  target, the field divergence-free and a z-reflection symmetry intact.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import synth
from oracle import kmm, orr_sommerfeld


def _poly_mul(p, q):
    out = [F(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _poly_add(p, q):
    n = max(len(p), len(q))
    return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]


def test_rk3_explicit_part_is_third_order_taylor():
    """x' = lam x treated explicitly: one step multiplies x by 1 + z + z^2/2 + z^3/6 exactly."""
    x_prev, x = [F(1)], [F(1)]  # polynomials in z = h lam
    for s in range(3):
        ga, ze = kmm.RK3_GAMMA[s], kmm.RK3_ZETA[s]
        nxt = _poly_add(x, _poly_add([0] + [ga * c for c in x], [0] + [ze * c for c in x_prev]))
        x_prev, x = x, nxt
    assert x == [F(1), F(1), F(1, 2), F(1, 6)]


def test_rk3_implicit_part_is_second_order():
    """x' = lam x treated with the alpha/beta split: product of (1+a z)/(1-b z) = exp(z) + O(z^3)."""
    num, den = [F(1)], [F(1)]
    for s in range(3):
        num = _poly_mul(num, [F(1), kmm.RK3_ALPHA[s]])
        den = _poly_mul(den, [F(1), -kmm.RK3_BETA[s]])
    # series of num/den to second order
    inv = [F(1), -den[1], den[1] ** 2 - den[2]]
    ser = _poly_mul(num, inv)[:3]
    assert ser == [F(1), F(1), F(1, 2)]
    # consistency of the two splits in every sub-step
    for s in range(3):
        assert kmm.RK3_ALPHA[s] + kmm.RK3_BETA[s] == kmm.RK3_GAMMA[s] + kmm.RK3_ZETA[s]


def test_rk3_update_scalar_recursion():
    """rk3_update on a scalar ODE equals the recursion with the cited coefficients."""
    lam_i, lam_e, h = -3.0, 0.7, 0.1
    x, xold = 1.0, 0.0
    ref = 1.0
    rprev = 0.0
    for s in range(3):
        n_now = lam_e * x
        x_new = kmm.rk3_update(x, n_now, lam_e * xold, s, h, lambda f: lam_i * f,
                               lambda r, c: r / (1 - c * lam_i))
        a, b, g, z = (float(c[s]) for c in (kmm.RK3_ALPHA, kmm.RK3_BETA, kmm.RK3_GAMMA, kmm.RK3_ZETA))
        ref_new = (ref * (1 + a * h * lam_i) + h * (g * lam_e * ref + z * lam_e * rprev)) / (1 - b * h * lam_i)
        xold, x = x, x_new
        rprev, ref = ref, ref_new
        assert abs(x - ref) < 1e-15
    assert abs(x - np.exp((lam_i + lam_e) * h)) < 1e-3


def _setup(n1, n2, n3, re_b, dt, q=2.0, lz=np.pi):
    y = synth.mesh_tanh(n2)
    return kmm.Setup(n1=n1, n2=n2, n3=n3, lx=2 * np.pi, lz=lz, nu=1 / re_b, dt=dt, mass_flux=q, y=y)


def test_poiseuille_is_steady():
    S = _setup(8, 65, 8, 2800.0, 0.005)
    z = np.zeros((65, 4, 8), complex)
    st = kmm.make_state(S, z, z, synth.poiseuille(S.y), np.zeros(65))
    st2, f = kmm.step(S, st, 10)
    assert np.abs(st2.U1 - st.U1).max() < 1e-13
    assert abs(f / (3 * S.nu) - 1) < 1e-9  # f is a small difference of O(1) integrals
    assert np.abs(st2.v).max() == 0 and np.abs(st2.om2).max() == 0


def test_orr_sommerfeld_solver_matches_orszag():
    c, _, _ = orr_sommerfeld.least_stable(10000.0, 1.0, 128)
    assert abs(c - (0.23752649 + 0.00373967j)) < 2e-8


@pytest.mark.slow
def test_orr_sommerfeld_growth_rate():
    """The RK3 solver grows a small OS eigenmode at 2 alpha c_i (bulk units: x 1.5)."""
    n2 = 129
    S = _setup(4, n2, 2, 10000.0 / 1.5, 0.02)
    c, vy = orr_sommerfeld.eigenfunction_on(S.y, 10000.0, 1.0)
    V = np.zeros((n2, 2, 2), complex)
    V[:, 1, 0] = 1e-6 * vy
    st = kmm.make_state(S, V, np.zeros_like(V), synth.poiseuille(S.y), np.zeros(n2))

    def energy(st):
        u1, u2, u3, *_ = kmm.recover(S, st)
        return S.w @ (np.abs(u1[:, 1, 0]) ** 2 + np.abs(u2[:, 1, 0]) ** 2 + np.abs(u3[:, 1, 0]) ** 2)

    st, _ = kmm.step(S, st, 15)
    e0 = energy(st)
    st, _ = kmm.step(S, st, 30)
    rate = np.log(energy(st) / e0) / (2 * 30 * S.dt)
    expected = 1.5 * c.imag
    assert abs(rate / expected - 1) < 1e-3, (rate, expected)


def test_viscous_decay_of_wall_normal_vorticity():
    n2 = 65
    S = _setup(4, n2, 4, 500.0, 0.01, q=0.0)
    om = np.zeros((n2, 2, 4), complex)
    om[:, 1, 0] = 1e-6 * np.sin(np.pi * (S.y + 1) / 2)
    st = kmm.make_state(S, np.zeros_like(om), om, np.zeros(n2), np.zeros(n2))
    st2, f = kmm.step(S, st, 10)
    lam = -S.nu * (1.0 + np.pi ** 2 / 4)
    ratio = st2.om2[n2 // 2, 1, 0] / st.om2[n2 // 2, 1, 0]
    assert abs(ratio - np.exp(lam * 10 * S.dt)) < 1e-8
    assert abs(f) < 1e-12


@pytest.fixture(scope="module")
def c1_small():
    """A reduced C1-like case (32 x 33 x 32) with broadband perturbations."""
    case = synth.Case(n1=32, n2=33, n3=32, lx=2 * np.pi, lz=np.pi, re_b=2800.0, dt=0.005,
                      amp=0.1, kmax=6, cfg=11)
    v, om, U1, U3, y = synth.turbulent_field(case)
    S = kmm.Setup(n1=32, n2=33, n3=32, lx=case.lx, lz=case.lz, nu=1 / case.re_b, dt=case.dt,
                  mass_flux=2.0, y=y)
    return S, kmm.make_state(S, v, om, U1, U3)


def test_substep_invariants(c1_small):
    S, st = c1_small
    diag = []
    hist = kmm.zero_history(S)
    for s in range(3):
        st, hist, f = kmm.substep(S, st, hist, s, diag)
        vscale = np.abs(st.v).max()
        assert np.abs(diag[-1]["v_wall"]).max() == 0
        assert np.abs(diag[-1]["dv_wall"]).max() < 1e-11 * vscale / (S.y[1] - S.y[0])
        assert abs(S.w @ st.U1 - 2.0) < 1e-14
        u1, u2, u3, *_ = kmm.recover(S, st)
        div = 1j * S.a * u1 + kmm.d1(S, u2) + 1j * S.b * u3
        div[:, 0, 0] = 0
        assert np.abs(div).max() < 1e-13 * np.abs(u1[:, :, 1:]).max()


def test_z_reflection_symmetry_preserved():
    """u3 odd and u1, u2 even in z stays so: v(kz) = v(-kz), omega2(kz) = -omega2(-kz)."""
    case = synth.Case(n1=16, n2=33, n3=16, lx=2 * np.pi, lz=np.pi, re_b=2800.0, dt=0.005,
                      amp=0.1, kmax=4, cfg=12)
    v, om, U1, U3, y = synth.turbulent_field(case)
    n3 = 16
    for kz in range(1, n3 // 2):
        v[:, :, n3 - kz] = v[:, :, kz]
        om[:, :, n3 - kz] = -om[:, :, kz]
    om[:, :, 0] = 0
    v[:, 0, :] = v[:, 0, :].real  # kx = 0 Hermitian and even => real
    om[:, 0, :] = 1j * om[:, 0, :].imag
    S = kmm.Setup(n1=16, n2=33, n3=16, lx=case.lx, lz=case.lz, nu=1 / 2800, dt=0.005, mass_flux=2.0, y=y)
    st, _ = kmm.step(S, kmm.make_state(S, v, om, U1, U3), 2)
    sl = slice(1, n3 // 2)
    mir = [n3 - k for k in range(1, n3 // 2)]
    rel = lambda d, ref: np.linalg.norm(d) / np.linalg.norm(ref)  # noqa: E731
    assert rel(st.v[:, :, sl] - st.v[:, :, mir], st.v) < 1e-12
    assert rel(st.om2[:, :, sl] + st.om2[:, :, mir], st.om2) < 1e-12
    assert rel(st.om2[:, :, 0], st.om2) < 1e-12
    assert np.abs(st.U3).max() < 1e-14


@pytest.mark.slow
def test_chi_wall_rows_amplify_rounding():
    """The conditioning that sets the element-wise parity bounds of chi.

    chi's wall values are the influence-matrix coefficients c = -D1 v_p / D1 v_h
    at the walls, a quotient of two small numbers (the homogeneous layers are
    far thinner than the first cell), so they amplify rounding.  The oracle's
    own 10-step run of the 64 x 65 x 64 workload, restarted from a state
    perturbed by one ulp, moves chi by 1e-11 (L2) and ~1e-10 of max|chi| at the
    wall rows, ~1e-11 inside, while v and omega2 stay at 1e-15."""
    case = synth.CASES["c1"]
    v, om, U1, U3, y = synth.turbulent_field(case)
    S = kmm.Setup(n1=case.n1, n2=case.n2, n3=case.n3, lx=case.lx, lz=case.lz, nu=1 / case.re_b, dt=case.dt,
                  mass_flux=2.0, y=y)
    a, _ = kmm.step(S, kmm.make_state(S, v, om, U1, U3), 10)
    g = np.random.default_rng(1)
    vp = v * (1 + 2.2e-16 * g.standard_normal(v.shape))
    op = om * (1 + 2.2e-16 * g.standard_normal(om.shape))
    b, _ = kmm.step(S, kmm.make_state(S, vp, op, U1, U3), 10)
    d = np.abs(a.chi - b.chi)
    scale = np.abs(a.chi).max()
    wall, inner = d[[0, -1]].max() / scale, d[1:-1].max() / scale
    l2 = np.linalg.norm(a.chi - b.chi) / np.linalg.norm(a.chi)
    print(f"chi: L2 {l2:.2e}, wall rows {wall:.2e}, interior {inner:.2e}")
    assert 3e-11 < wall < 1e-9 and inner < 5e-11 and l2 < 3e-11
    for f in ("v", "om2"):
        x, z = getattr(a, f), getattr(b, f)
        assert np.abs(x - z).max() < 1e-14 * np.abs(x).max(), f
