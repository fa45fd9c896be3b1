"""Oracle reference for the 384 x 193 x 384 workload after 20 RK3 steps.

Runs only the oracle (float64, CPU) from the seeded initial field and stores,
for a seeded sample of 8192 mode-points, the values of v, omega2, chi, u1, u3,
omega1, omega3, plus the full mean profiles U1, U3 and the mean pressure
gradient of the last sub-step, in tests/golden/c2_20steps.npz.
Run: python tests/golden/make_c2_golden.py   (about 30 min, ~10 GB RAM)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import kmm  # noqa: E402

NSTEPS = 20
NSAMPLE = 8192


def sample_index(n2, n1h, n3, seed=2020):
    g = np.random.default_rng(seed)
    return (g.integers(0, n2, NSAMPLE), g.integers(0, n1h, NSAMPLE), g.integers(0, n3, NSAMPLE))


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_20steps.npz")):
    c = synth.CASES["c2"]
    v, om, U1, U3, y = synth.turbulent_field(c)
    S = kmm.Setup(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, nu=1 / c.re_b, dt=c.dt, mass_flux=c.mass_flux, y=y)
    st = kmm.make_state(S, v, om, U1, U3)
    t0 = time.time()
    f = 0.0
    for k in range(NSTEPS):
        st, f = kmm.step(S, st, 1)
        print(f"step {k + 1}/{NSTEPS} {time.time() - t0:.0f}s", flush=True)
    u1, u2, u3, o1, o2, o3 = kmm.recover(S, st)
    idx = sample_index(c.n2, c.n1 // 2, c.n3)
    np.savez_compressed(out, iy=idx[0], ikx=idx[1], ikz=idx[2], nsteps=NSTEPS, dt=c.dt,
                        v=st.v[idx], omega2=st.om2[idx], chi=st.chi[idx], u1=u1[idx], u3=u3[idx],
                        omega1=o1[idx], omega3=o3[idx], U1=st.U1, U3=st.U3, f=f)
    print("wrote", out)


if __name__ == "__main__":
    main()
