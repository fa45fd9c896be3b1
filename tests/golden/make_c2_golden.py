"""Oracle reference for the 384 x 193 x 384 workload after 20 RK3 steps.

Runs only the oracle (float64, CPU) from the seeded initial field and stores,
in tests/golden/c2_20steps.npz:
  - for a seeded sample of 8192 mode-points, the values of v, omega2, chi, u1,
    u3, omega1, omega3;
  - whole wall-normal pencils (all 193 nodes) of the same fields for a fixed
    list of modes from the lowest to the highest retained wavenumbers
    (``PENCIL_MODES``), so that errors confined to a band of modes or to the
    near-wall rows show up per mode;
  - the full mean profiles U1, U3 and the mean pressure gradient of the last
    sub-step;
  - the step diagnostics the library reports: the CFL number of the velocities
    entering the last sub-step (dt max |u1|/dx + |u2|/dy_j + |u3|/dz on the
    padded grid) and u_tau = sqrt(nu |dU1/dy|) at both walls after the run.
Run: python tests/golden/make_c2_golden.py   (about 45 min, ~10 GB RAM)
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
# (kx, kz) of the stored pencils: the (0,0) line is excluded (it carries the
# mean profiles, stored whole), the rest spans the retained set of 192 x 383
PENCIL_MODES = [(0, 1), (0, -1), (0, 7), (0, 150), (1, 0), (1, 1), (1, -1), (2, 5), (3, -40),
                (5, 0), (8, 8), (13, -13), (20, 100), (40, -3), (64, 64), (90, -170), (120, 0),
                (150, 191), (170, -191), (191, 1), (191, -100), (191, 191), (100, -191), (60, 120)]


def sample_index(n2, n1h, n3, seed=2020):
    g = np.random.default_rng(seed)
    return (g.integers(0, n2, NSAMPLE), g.integers(0, n1h, NSAMPLE), g.integers(0, n3, NSAMPLE))


def pencil_slots(n3):
    kx = np.array([m[0] for m in PENCIL_MODES])
    kz = np.array([m[1] % n3 for m in PENCIL_MODES])
    return kx, kz


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_20steps.npz")):
    c = synth.CASES["c2"]
    v, om, U1, U3, y = synth.turbulent_field(c)
    S = kmm.Setup(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, nu=1 / c.re_b, dt=c.dt, mass_flux=c.mass_flux, y=y)
    st = kmm.make_state(S, v, om, U1, U3)
    t0 = time.time()
    f = 0.0
    cfl_last = None
    for k in range(NSTEPS):
        hist = kmm.zero_history(S)
        for s in range(3):
            if k == NSTEPS - 1 and s == 2:
                cfl_last = kmm.cfl(S, st, c.dt)
            st, hist, f = kmm.substep(S, st, hist, s)
        print(f"step {k + 1}/{NSTEPS} {time.time() - t0:.0f}s", flush=True)
    u1, u2, u3, o1, o2, o3 = kmm.recover(S, st)
    dU = kmm.d1(S, st.U1)
    idx = sample_index(c.n2, c.n1 // 2, c.n3)
    pkx, pkz = pencil_slots(c.n3)
    fields = dict(v=st.v, omega2=st.om2, chi=st.chi, u1=u1, u3=u3, omega1=o1, omega3=o3)
    extra = {f"pen_{k}": a[:, pkx, pkz] for k, a in fields.items()}
    np.savez_compressed(out, iy=idx[0], ikx=idx[1], ikz=idx[2], nsteps=NSTEPS, dt=c.dt,
                        **{k: a[idx] for k, a in fields.items()}, U1=st.U1, U3=st.U3, f=f,
                        pen_kx=pkx, pen_kz=pkz, cfl_last=cfl_last,
                        utau_lo=np.sqrt(S.nu * abs(dU[0])), utau_hi=np.sqrt(S.nu * abs(dU[-1])), **extra)
    print("wrote", out)


if __name__ == "__main__":
    main()
