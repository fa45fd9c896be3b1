"""Pins of the oracle's filtered pressure (Section 3.1: d_kk p = -d_i d_j F(u_i u_j)).

Each term of the right-hand side and the wall condition is checked against
the continuous solution of the same problem, on a 97-point wall-refined mesh:

* with p = cos(pi y) (dp/dy = 0 at both walls), r = p'' - k^2 p is produced
  by F(u_1 u_1), F(u_1 u_2), F(u_1 u_3), F(u_2 u_2), F(u_2 u_3) or F(u_3 u_3)
  alone (each term inverted by hand: factors i a, i b, 2 and signs), and the
  solver must return cos(pi y);
* with no stresses and F(v) = (1 - y^2)^2 the wall condition dp/dy = nu v''
  = 8 nu gives p = 8 nu sinh(k y) / (k cosh k);
* mode (0, 0) returns -F(u_2 u_2).
"""
import numpy as np
import pytest

from oracle import kmm, lowstorage

N2 = 97
LX, LZ = 2 * np.pi, np.pi
NU = 1e-3


def _setup():
    s = -1 + 2 * np.arange(N2) / (N2 - 1)
    y = np.tanh(2.0 * s) / np.tanh(2.0)
    return kmm.Setup(n1=8, n2=N2, n3=8, lx=LX, lz=LZ, nu=NU, dt=1e-3, mass_flux=2.0, y=y)


S = _setup()
Y = S.y
A, B = 2 * np.pi / LX * 1, 2 * np.pi / LZ * 1   # mode (kx, kz) = (1, 1): slots ix = 1, iz = 1
K2 = A * A + B * B
R = -(np.pi ** 2 + K2) * np.cos(np.pi * Y)       # r for p = cos(pi y)


def _run(term=None, values=None, vbar=None):
    uu = np.zeros((6, N2, 2, 3), complex)
    ub = np.zeros((3, N2, 2, 3), complex)
    if term is not None:
        uu[term][:, 1, 1] = values
    if vbar is not None:
        ub[1][:, 1, 1] = vbar
    return lowstorage.filtered_pressure(S, uu, ub, 1, 1)[:, 1, 1]


@pytest.mark.parametrize("term,values", [
    (0, R / A ** 2),                                                # r = a^2 F(u1u1)
    (1, (np.pi ** 2 + K2) / (2j * A) * np.sin(np.pi * Y) / np.pi),  # r = -2 i a D1 F(u1u2)
    (2, R / (2 * A * B)),                                           # r = 2 a b F(u1u3)
    (3, -(np.pi ** 2 + K2) / np.pi ** 2 * np.cos(np.pi * Y)),       # r = -D2 F(u2u2)
    (4, (np.pi ** 2 + K2) / (2j * B) * np.sin(np.pi * Y) / np.pi),  # r = -2 i b D1 F(u2u3)
    (5, R / B ** 2),                                                # r = b^2 F(u3u3)
])
def test_each_term_against_the_continuous_solution(term, values):
    p = _run(term, values)
    err = np.abs(p - np.cos(np.pi * Y)).max()
    assert err < 1e-9, (term, err)


def test_wall_condition_against_the_continuous_solution():
    k = np.sqrt(K2)
    p = _run(vbar=(1 - Y ** 2) ** 2)
    ref = 8 * NU * np.sinh(k * Y) / (k * np.cosh(k))
    assert np.abs(p - ref).max() < 1e-11, np.abs(p - ref).max()


def test_mean_mode():
    uu = np.zeros((6, N2, 2, 3), complex)
    uu[3][:, 0, 0] = (1 - Y ** 2) * 0.3
    p = lowstorage.filtered_pressure(S, uu, np.zeros((3, N2, 2, 3), complex), 1, 1)
    assert np.array_equal(p[:, 0, 0], -uu[3][:, 0, 0].real)
