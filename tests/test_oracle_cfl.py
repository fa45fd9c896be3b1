"""Pins of the oracle's CFL number (the time-step criterion of Section 2.1's runs).

CFL = dt max over the 3n1/2 x 3n3/2 grid of every plane of
|u1|/dx + |u2|/dy_j + |u3|/dz, with dx = lx/n1, dz = lz/n3 and dy_j the smaller
of the two gaps next to node j.  Each term is exercised on a field whose
physical velocity is known in closed form, evaluated here directly from the
mesh (no transform, no compact operator):

* a mean profile U1(y) alone gives dt max_j |U1(y_j)| / dx, and U3 alone
  dt max_j |U3(y_j)| / dz;
* one Fourier mode of v, v(kx=1) = e^{i phi} f(y) / 2 with
  f = (1 - y^2)^2 (1 + y) and omega2 = 0, gives u2 = f cos(a x + phi) and, by
  continuity, u1 = -f'(y) sin(a x + phi) / a (the compact D1 is exact on this
  quintic at every row, walls included); the same on kz = 1 gives
  u3 = -f'(y) sin(b z + phi) / b;
* all of them together.

The closed forms are also evaluated with the plausible mistakes (unpadded
grid, one-sided gaps, a missing term) to show that each would fail the pin.
"""
import numpy as np
import pytest

import synth
from oracle import kmm


# phase of the Fourier mode: the peaks of cos and sin then fall between the
# nodes of both the padded and the unpadded grid, which sample them differently
PHASE = 0.3


def _f(y, s=1):
    """Wall-normal profile of the mode (twice v): vanishes with its slope at
    both walls and peaks off the centre (at y = 0.2 s), where the two gaps
    next to a node differ (s = -1: the mirror image)."""
    y = s * y
    return (1 - y ** 2) ** 2 * (1 + y)


def _df(y, s=1):
    y = s * y
    return s * (1 - y ** 2) * (1 - 4 * y - 5 * y ** 2)


def _setup(n1=8, n2=33, n3=8, lx=2 * np.pi, lz=np.pi):
    y = synth.mesh_tanh(n2, 1.5)
    return kmm.Setup(n1=n1, n2=n2, n3=n3, lx=lx, lz=lz, nu=1e-3, dt=1.0, mass_flux=2.0, y=y)


def _state(S, vmodes=(), U1=None, U3=None, s=1):
    v = np.zeros((S.n2, S.n1 // 2, S.n3), complex)
    for kx, kz in vmodes:
        prof = _f(S.y, s) / 2 * np.exp(1j * PHASE)
        v[:, kx, kz % S.n3] += prof
        if kx == 0:
            v[:, 0, (-kz) % S.n3] += np.conj(prof)  # Hermitian partner
    om = np.zeros_like(v)
    U1 = np.zeros(S.n2) if U1 is None else U1
    U3 = np.zeros(S.n2) if U3 is None else U3
    return kmm.make_state(S, v, om, U1, U3)


def _gaps(y, kind="min"):
    g = np.diff(y)
    left, right = np.r_[g[0], g], np.r_[g, g[-1]]
    return {"min": np.minimum(left, right), "left": left, "right": right, "mean": (left + right) / 2}[kind]


def _closed(S, dt, kx_mode=False, kz_mode=False, U1=None, U3=None, grid="padded", gaps="min", drop=None,
            s=1):
    """dt max over the grid of |u1|/dx + |u2|/dy + |u3|/dz from the closed-form velocities."""
    n1, n3 = S.n1, S.n3
    P1, P3 = (3 * n1 // 2, 3 * n3 // 2) if grid == "padded" else (n1, n3)
    y = S.y[:, None, None]
    x = (np.arange(P1) * S.lx / P1)[None, None, :]
    z = (np.arange(P3) * S.lz / P3)[None, :, None]
    a, b = 2 * np.pi / S.lx, 2 * np.pi / S.lz
    u1 = np.zeros((S.n2, P3, P1)) + (0 if U1 is None else U1[:, None, None])
    u3 = np.zeros_like(u1) + (0 if U3 is None else U3[:, None, None])
    u2 = np.zeros_like(u1)
    if kx_mode:
        u2 = u2 + _f(y, s) * np.cos(a * x + PHASE)
        u1 = u1 - _df(y, s) * np.sin(a * x + PHASE) / a
    if kz_mode:
        u2 = u2 + _f(y, s) * np.cos(b * z + PHASE)
        u3 = u3 - _df(y, s) * np.sin(b * z + PHASE) / b
    dx, dz = S.lx / n1, S.lz / n3
    dy = _gaps(S.y, gaps)[:, None, None]
    terms = {"u1": np.abs(u1) / dx, "u2": np.abs(u2) / dy, "u3": np.abs(u3) / dz}
    if drop:
        terms.pop(drop)
    return dt * sum(terms.values()).max()


def test_cfl_of_streamwise_mean_alone():
    S = _setup()
    U1 = 1.5 * (1 - S.y ** 2) + 0.3 * S.y
    got = kmm.cfl(S, _state(S, U1=U1), 0.01)
    assert got == pytest.approx(0.01 * np.abs(U1).max() * S.n1 / S.lx, rel=1e-14)
    assert got == pytest.approx(_closed(S, 0.01, U1=U1), rel=1e-14)


def test_cfl_of_spanwise_mean_alone():
    S = _setup(lz=np.pi / 2)
    U3 = 0.2 - 0.7 * S.y ** 3
    got = kmm.cfl(S, _state(S, U3=U3), 0.02)
    assert got == pytest.approx(0.02 * np.abs(U3).max() * S.n3 / S.lz, rel=1e-14)


@pytest.mark.parametrize("s", [1, -1])
@pytest.mark.parametrize("mode", ["kx", "kz"])
def test_cfl_of_one_fourier_mode(mode, s):
    S = _setup()
    st = _state(S, vmodes=[(1, 0)] if mode == "kx" else [(0, 1)], s=s)
    kw = dict(kx_mode=mode == "kx", kz_mode=mode == "kz", s=s)
    got = kmm.cfl(S, st, 0.003)
    ref = _closed(S, 0.003, **kw)
    assert got == pytest.approx(ref, rel=1e-13)
    # the pin separates the plausible mistakes (the one-sided gap that is the
    # smaller one at the peak agrees with the pin; the mirror case has the other)
    one_sided = dict(gaps="left") if s == 1 else dict(gaps="right")
    for wrong in (dict(grid="unpadded"), one_sided, dict(gaps="mean"), dict(drop="u2"),
                  dict(drop="u1" if mode == "kx" else "u3")):
        assert abs(_closed(S, 0.003, **kw, **wrong) / ref - 1) > 1e-3, wrong


def test_cfl_of_everything_together():
    S = _setup(n1=12, n2=41, n3=16)
    U1 = 1.5 * (1 - S.y ** 2)
    U3 = 0.1 * S.y
    st = _state(S, vmodes=[(1, 0), (0, 1)], U1=U1, U3=U3)
    got = kmm.cfl(S, st, 0.005)
    assert got == pytest.approx(_closed(S, 0.005, kx_mode=True, kz_mode=True, U1=U1, U3=U3), rel=1e-13)
