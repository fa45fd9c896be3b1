"""Time step of the 384 x 193 x 384 workload: CFL 0.5 at t = 0.

Computes, with the oracle only, CFL = dt * max over the padded grid of
|u1|/dx + |u2|/dy_j + |u3|/dz for the seeded initial field, and prints
dt = 0.5 / CFL(dt=1).  The value is stored as ``synth.CASES['c2'].dt``.
Run: python tests/golden/make_dt.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import synth  # noqa: E402
from oracle import kmm  # noqa: E402


def main(name="c2", target=0.5):
    c = synth.CASES[name]
    v, om, U1, U3, y = synth.turbulent_field(c)
    S = kmm.Setup(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, nu=1 / c.re_b, dt=1.0,
                  mass_flux=c.mass_flux, y=y)
    st = kmm.make_state(S, v, om, U1, U3)
    cfl1 = kmm.cfl(S, st, 1.0)
    dt = target / cfl1
    print(json.dumps({"case": name, "cfl_per_unit_dt": cfl1, "dt": dt}))
    return dt


if __name__ == "__main__":
    main(*(sys.argv[1:2] or ["c2"]))
