"""Oracle reference for the low-storage stage on the 1536 x 385 x 1152 field.

Runs only the oracle (float64, CPU): the seeded Re_tau ~ 950 field, u1, u2, u3
by continuity (full field), then the cut-off filter and stresses on a few
sampled wall-normal planes (the stage is plane-local).  Stores, per sampled
plane, seeded samples of F(u_i), F(u_i u_j) and tau_ij in
tests/golden/c5_filter.npz.  kc = (N1/16, N3/16) = (96, 72), q = (432, 324).
Run: python tests/golden/make_c5_golden.py   (about 10 min, ~40 GB RAM)
"""
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
    live = S.live[None]
    st = kmm.State(v=np.where(live, v, 0), chi=None, om2=np.where(live, om, 0), U1=U1, U3=U3)
    del v, om
    u1, u3 = kmm.velocities(S, st)
    u2 = st.v
    print(f"velocities {time.time() - t0:.0f}s", flush=True)
    g = np.random.default_rng(5050)
    res = {"planes": np.array(PLANES), "kc": np.array([KCX, KCZ, Q1, Q3])}
    for p in PLANES:
        ub, uu, tau = lowstorage.filter_and_stress(u1[p:p + 1], u2[p:p + 1], u3[p:p + 1], KCX, KCZ, Q1, Q3)
        ik, iz = g.integers(0, KCX + 1, NS), g.integers(0, 2 * KCZ + 1, NS)
        tz, tx = g.integers(0, Q3, NS), g.integers(0, Q1, NS)
        res[f"y{p}_ik"], res[f"y{p}_iz"], res[f"y{p}_tz"], res[f"y{p}_tx"] = ik, iz, tz, tx
        res[f"y{p}_ubar"] = ub[:, 0, ik, iz]
        res[f"y{p}_uubar"] = uu[:, 0, ik, iz]
        res[f"y{p}_tau"] = tau[:, 0, tz, tx]
        res[f"y{p}_tau_norm"] = np.sqrt((tau[:, 0] ** 2).mean(axis=(1, 2)))
        print(f"plane {p} {time.time() - t0:.0f}s", flush=True)
    np.savez_compressed(out, **res)
    print("wrote", out)


if __name__ == "__main__":
    main()
