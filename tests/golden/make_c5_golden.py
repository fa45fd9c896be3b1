"""Oracle reference for the low-storage stage on the 1536 x 385 x 1152 field.

Runs only the oracle (float64, CPU): the seeded Re_tau ~ 950 field, u1, u2, u3
by continuity and omega1, omega2, omega3 (computed in blocks of kx columns,
keeping only the sampled planes), then the cut-off filter, stresses and
filtered enstrophy on those wall-normal planes (the stage is plane-local).
Stores, per sampled plane, seeded samples of F(u_i), F(u_i u_j), tau_ij and
F(omega_i omega_i) in tests/golden/c5_filter.npz.  kc = (N1/16, N3/16) =
(96, 72), q = (432, 324).
Run: python tests/golden/make_c5_golden.py   (about 15 min, ~20 GB RAM)
"""
import copy
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import kmm, lowstorage  # noqa: E402

PLANES = (3, 96, 192)
KCX, KCZ, Q1, Q3 = 96, 72, 432, 324
NS = 4096


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_filter.npz")):
    t0 = time.time()
    c = synth.CASES["c5"]
    v, om, U1, U3, y = synth.turbulent_field(c)
    print(f"field {time.time() - t0:.0f}s", flush=True)
    S = kmm.Setup(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, nu=1 / c.re_b, dt=1e-3, mass_flux=c.mass_flux, y=y)
    v *= S.live[None]
    om *= S.live[None]
    pl = list(PLANES)
    u = np.zeros((3, len(pl), c.n1 // 2, c.n3), complex)
    w = np.zeros((3, len(pl), c.n1 // 2, c.n3), complex)
    u[1] = v[pl]
    w[1] = om[pl]
    # kmm.recover on blocks of kx columns; a block starting at k0 > 0 also
    # takes column k0 - 1, whose first slot velocities() reserves for the mean
    step = 48
    for k0 in range(0, c.n1 // 2, step):
        lo = max(k0 - 1, 0)
        hi = min(k0 + step, c.n1 // 2)
        Sb = copy.copy(S)
        for name in ("a", "b", "k2", "live"):
            setattr(Sb, name, getattr(S, name)[lo:hi])
        stb = kmm.State(v=v[:, lo:hi], chi=None, om2=om[:, lo:hi], U1=U1, U3=U3)
        b1, _, b3, o1, _, o3 = kmm.recover(Sb, stb)
        u[0][:, k0:hi] = b1[pl, k0 - lo:]
        u[2][:, k0:hi] = b3[pl, k0 - lo:]
        w[0][:, k0:hi] = o1[pl, k0 - lo:]
        w[2][:, k0:hi] = o3[pl, k0 - lo:]
        del b1, b3, o1, o3
    del v, om
    print(f"velocities and vorticities {time.time() - t0:.0f}s", flush=True)
    g = np.random.default_rng(5050)
    ge = np.random.default_rng(5051)  # enstrophy samples (a generator of their own)
    res = {"planes": np.array(PLANES), "kc": np.array([KCX, KCZ, Q1, Q3])}
    for n, p in enumerate(PLANES):
        ub, uu, tau = lowstorage.filter_and_stress(u[0][n:n + 1], u[1][n:n + 1], u[2][n:n + 1], KCX, KCZ, Q1, Q3)
        ik, iz = g.integers(0, KCX + 1, NS), g.integers(0, 2 * KCZ + 1, NS)
        tz, tx = g.integers(0, Q3, NS), g.integers(0, Q1, NS)
        res[f"y{p}_ik"], res[f"y{p}_iz"], res[f"y{p}_tz"], res[f"y{p}_tx"] = ik, iz, tz, tx
        res[f"y{p}_ubar"] = ub[:, 0, ik, iz]
        res[f"y{p}_uubar"] = uu[:, 0, ik, iz]
        res[f"y{p}_tau"] = tau[:, 0, tz, tx]
        res[f"y{p}_tau_norm"] = np.sqrt((tau[:, 0] ** 2).mean(axis=(1, 2)))
        ens = lowstorage.filtered_enstrophy(w[0][n:n + 1], w[1][n:n + 1], w[2][n:n + 1], KCX, KCZ)
        ek, ez = ge.integers(0, KCX + 1, NS), ge.integers(0, 2 * KCZ + 1, NS)
        res[f"y{p}_ek"], res[f"y{p}_ez"] = ek, ez
        res[f"y{p}_ens"] = ens[0, ek, ez]
        res[f"y{p}_ens00"] = ens[0, 0, 0]
        print(f"plane {p} {time.time() - t0:.0f}s", flush=True)
    np.savez_compressed(out, **res)
    print("wrote", out)


if __name__ == "__main__":
    main()
