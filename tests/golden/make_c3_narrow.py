"""Oracle reference for a narrow channel on the Re_tau 5300 share's wall-normal mesh.

The pencil share of the Re_tau 5300 workload (1537 wall-normal nodes) is too
large for the oracle, so its 1537-point wall-normal operators, banded solves
and influence matrix are checked on a narrow channel with the same nodes,
Reynolds number and time-step criterion: 16 x 1537 x 16 (8 x 16 Fourier
modes), box 2 pi x 2 x pi, Re_b from Dean's correlation at Re_tau 5300, the
turbulent-field recipe of the inputs (Reichardt mean plus a k^(-5/3)
perturbation of RMS 0.1), dt from CFL 0.5 at t = 0 (oracle CFL), three RK3
steps, on two meshes:
  - the tanh mesh of the workload (g = 2);
  - that mesh after the oracle's near-wall optimisation (Appendix B) at
    k* = 1e10 with 20 free nodes per wall, 60 descent steps.
Stored (tests/golden/c3_narrow.npz): both meshes; per mesh dt, whole pencils
(all 1537 nodes) of v, omega2, chi, u1, u3 for the modes of PENCIL_MODES,
4096 seeded mode-point samples of those fields and of omega1, omega3, U1, U3, the
mean pressure gradient of the last sub-step, the CFL number entering the
last sub-step, u_tau at both walls, and per field the oracle's own
sensitivity to rounding (the relative change of the samples when the
initial v and omega2 change by one ulp), which sets the parity bound of
the fields whose near-wall derivatives amplify rounding on this mesh.
Run: python tests/golden/make_c3_narrow.py   (about 20 min; the optimisation
with dense 1537-point solves dominates)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import kmm, meshopt  # noqa: E402

NSTEPS = 3
NSAMPLE = 4096
PENCIL_MODES = [(0, 1), (1, 0), (1, -1), (2, 5), (3, -7), (5, -3), (6, 7), (7, -7)]
PENCIL_FIELDS = ("v", "omega2", "chi", "u1", "u3")


def case():
    return synth.Case(n1=16, n2=1537, n3=16, lx=2 * np.pi, lz=np.pi, re_b=synth.dean_re_b(5300.0), dt=0.0,
                      amp=0.1, kmax=None, mean="reichardt", re_tau=5300.0, cfg=7)


def run(y, tag, out):
    c = case()
    v, om, U1, U3, y = synth.turbulent_field(c, y=y)
    S = kmm.Setup(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, nu=1 / c.re_b, dt=1.0, mass_flux=c.mass_flux, y=y)
    st = kmm.make_state(S, v, om, U1, U3)
    S.dt = 0.5 / kmm.cfl(S, st, 1.0)
    f, cfl_last = 0.0, None
    for k in range(NSTEPS):
        hist = kmm.zero_history(S)
        for s in range(3):
            if k == NSTEPS - 1 and s == 2:
                cfl_last = kmm.cfl(S, st, S.dt)
            st, hist, f = kmm.substep(S, st, hist, s)
    u1, _, u3, o1, _, o3 = kmm.recover(S, st)
    dU = kmm.d1(S, st.U1)
    # the oracle's own sensitivity to rounding: the same run from a state
    # perturbed by one ulp (relative 2.2e-16 normal noise on v and omega2)
    r = np.random.default_rng(1537)
    vp = v * (1 + 2.2e-16 * r.standard_normal(v.shape))
    op = om * (1 + 2.2e-16 * r.standard_normal(om.shape))
    sp = kmm.make_state(S, vp, op, U1, U3)
    for k in range(NSTEPS):
        sp, _ = kmm.step(S, sp, 1)
    pu1, _, pu3, po1, _, po3 = kmm.recover(S, sp)
    g = np.random.default_rng(5300)
    idx = (g.integers(0, c.n2, NSAMPLE), g.integers(0, c.n1 // 2, NSAMPLE), g.integers(0, c.n3, NSAMPLE))
    pkx = np.array([m[0] for m in PENCIL_MODES])
    pkz = np.array([m[1] % c.n3 for m in PENCIL_MODES])
    fields = dict(v=st.v, omega2=st.om2, chi=st.chi, u1=u1, u3=u3, omega1=o1, omega3=o3)
    perturbed = dict(v=sp.v, omega2=sp.om2, chi=sp.chi, u1=pu1, u3=pu3, omega1=po1, omega3=po3)
    for k, a in fields.items():
        out[f"{tag}_{k}"] = a[idx]
        out[f"{tag}_sens_{k}"] = np.linalg.norm(perturbed[k][idx] - a[idx]) / np.linalg.norm(a[idx])
        if k in PENCIL_FIELDS:
            out[f"{tag}_pen_{k}"] = a[:, pkx, pkz]
    out.update({f"{tag}_y": y, f"{tag}_dt": S.dt, f"{tag}_U1": st.U1, f"{tag}_U3": st.U3, f"{tag}_f": f,
                f"{tag}_cfl_last": cfl_last, f"{tag}_utau_lo": np.sqrt(S.nu * abs(dU[0])),
                f"{tag}_utau_hi": np.sqrt(S.nu * abs(dU[-1]))})
    out.update(iy=idx[0], ikx=idx[1], ikz=idx[2], pen_kx=pkx, pen_kz=pkz, nsteps=NSTEPS)


def main(path=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_narrow.npz")):
    t0 = time.time()
    y_tanh = synth.mesh_tanh(1537)
    y_opt, e0, e1, it = meshopt.optimise_mesh(y_tanh, m=20, kstar=1e10, penalty=1e-3, max_iter=60)
    print(f"optimised mesh: {e0:.4e} -> {e1:.4e} in {it} steps, {time.time() - t0:.0f}s", flush=True)
    out = dict(opt_err_ref=e0, opt_err=e1, opt_iterations=it)
    for y, tag in ((y_tanh, "tanh"), (y_opt, "opt")):
        run(y, tag, out)
        print(f"{tag}: dt {out[tag + '_dt']:.4e}, {time.time() - t0:.0f}s", flush=True)
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()
