"""One GPU's share of the Re_tau = 5300 channel (8192 x 1537 x 6144), at its real shapes.

Plane slab: 48 x-z planes of 8192 x 6144 modes (12288 x 9216 padded) through
chn_plane_products on a planes_only context (mixed precision).  The oracle
(tests/golden/make_c3_golden.py) computed the products of two of the planes
from the same seeded float32 spectra; 4096 sampled coefficients of H1, H2, H3
per plane must agree to 1e-5 relative (e(X) over the samples).

Pencil share: 196608 Fourier modes on 1537 wall-normal nodes (a 512 x 1537 x
768 channel) advanced one RK3 step in mixed precision.  The oracle cannot run
this size, so the checks are properties that hold at any size: finite
fields, v = 0 and no slip (u1 = u3 = 0) at both walls, and the mass flux
held at its target.
"""
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_planes.npz")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.gpu
def test_c3_plane_slab_against_oracle_samples():
    from paper_1808_06461_amd import Channel
    g = np.load(GOLDEN)
    c = synth.C3_PLANES
    n1, n3, P = c["n1"], c["n3"], c["nplanes"]
    planes = [int(p) for p in g["planes"]]
    print(f"[c3] plane slab {P} x {n1} x {n3}, sampled planes {planes}", flush=True)
    ch = Channel(n1, P, n3, c["lx"], c["lz"], synth.dean_re_b(c["re_tau"]), precision="mixed",
                 planes_only=True, plane_chunk=8)
    try:
        fields = [torch.empty((P, n1 // 2, n3), dtype=torch.complex64, device="cuda") for _ in range(6)]
        synth.c3_fill_slab(fields, planes_from_numpy=planes, cfg=c["cfg"])
        H = ch.plane_products(fields)
        del fields
        torch.cuda.synchronize()
        for p in planes:
            ik, iz = torch.from_numpy(g[f"p{p}_ik"]).cuda(), torch.from_numpy(g[f"p{p}_iz"]).cuda()
            for f in range(3):
                got = H[f][p][ik, iz].cpu().numpy().astype(np.complex128)
                e = rel(got, g[f"p{p}_H"][f])
                print(f"[c3] plane {p} H{f + 1}: {e:.2e}", flush=True)
                assert e < 1e-5, (p, f, e)
    finally:
        ch.close()


@pytest.mark.gpu
@pytest.mark.parametrize("mesh", ["tanh", "optimised"])
def test_c3_pencil_share_invariants(mesh):
    """One mixed RK3 step of the 1537-node pencil share: finite, walls and mass
    flux exact; on the tanh mesh and on that mesh after the near-wall
    optimisation (k* = 1e10, 20 nodes per wall), the mesh the optimisation is
    meant to make safe for this Reynolds number."""
    from paper_1808_06461_amd import Channel, chn
    case = synth.c3_pencil_case()
    print(f"[c3] pencil share {case.n1 // 2 * case.n3} modes x {case.n2}, {mesh} mesh", flush=True)
    y = synth.mesh_tanh(case.n2)
    if mesh == "optimised":
        y, e0, e1, it = chn.optimise_mesh(y, m=20, kstar=1e10, max_iter=60)
        print(f"[c3] optimised mesh: {e0:.3e} -> {e1:.3e} in {it} steps", flush=True)
        assert e1 < e0
    v, om, U1, U3, y = synth.turbulent_field(case, y=y)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, mass_flux=case.mass_flux,
                 precision="mixed", y=y)
    try:
        state = [torch.from_numpy(a) for a in (v, om, U1, U3)]
        del v, om
        ch.set_state(*state)
        probe = ch.step(1e-6, 1, info=True)  # CFL per unit time step at t = 0
        dt = 0.5 * 1e-6 / probe["cfl_max"]
        ch.set_state(*state)
        info = ch.step(dt, 1, info=True)
        print(f"[c3] dt {dt:.3e} info {info}", flush=True)
        assert abs(info["mass_flux"] - case.mass_flux) < 1e-10 * case.mass_flux
        f = ch.get_fields("v", "u1", "u3", "omega2")
        for k, t in f.items():
            assert bool(torch.isfinite(torch.view_as_real(t)).all()), k
        for k in ("v", "u1", "u3"):
            t = f[k]
            wall = max(float(t[0].abs().max()), float(t[-1].abs().max()))
            scale = float(t.abs().max())
            print(f"[c3] {k}: wall {wall:.2e} max {scale:.2e}", flush=True)
            assert wall <= 1e-9 * scale, (k, wall, scale)
    finally:
        ch.close()
