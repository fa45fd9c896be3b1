"""Parity at full size: the low-storage stage on the 1536 x 385 x 1152 field (Re_tau ~ 950).

Cut-off kc = (N1/16, N3/16) = (96, 72), stresses on the 432 x 324 grid.  The
stored oracle values (tests/golden/make_c5_golden.py, oracle only) are seeded
samples of F(u_i), F(u_i u_j) and tau_ij on the planes y_3, y_96 and y_192;
the GPU computes every plane with the launch configuration of the full stage
and is compared there: e(X) = ||X_gpu[s] - X_oracle[s]|| / ||X_oracle[s]||
per component.  Bounds: float64 as for the small cases (F(u_i) 1e-13,
F(u_i u_j) 1e-12, tau 1e-10); mixed (float32 coefficients and inverse
transforms, float64 products and forward sums) 1e-5 on F(u_i u_j) and tau.
The filtered enstrophy F(omega_i omega_i) is compared on its own seeded
samples and its (0,0) mode: 1e-12 (float64), 1e-5 (mixed).
"""
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_filter.npz")
TOL = {"fp64": (1e-13, 1e-12, 1e-10), "mixed": (1e-5, 1e-5, 1e-5)}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def field():
    c = synth.CASES["c5"]
    return c, synth.turbulent_field(c)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_c5_filter_against_oracle_samples(field, precision):
    from paper_1808_06461_amd import Channel
    g = np.load(GOLDEN)
    kcx, kcz, q1, q3 = (int(v) for v in g["kc"])
    c, (v, om, U1, U3, y) = field
    print(f"[c5] {precision}: {c.n1}x{c.n2}x{c.n3}, kc=({kcx},{kcz}), q=({q1},{q3})", flush=True)
    ch = Channel(c.n1, c.n2, c.n3, c.lx, c.lz, c.re_b, mass_flux=c.mass_flux, precision=precision, y=y)
    try:
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        ub, uu, tau = ch.filter_and_stress(kcx, kcz, q1, q3)
        t_ub, t_uu, t_tau = TOL[precision]
        for p in (int(p) for p in g["planes"]):
            ik, iz = torch.from_numpy(g[f"y{p}_ik"]), torch.from_numpy(g[f"y{p}_iz"])
            tz, tx = torch.from_numpy(g[f"y{p}_tz"]), torch.from_numpy(g[f"y{p}_tx"])
            gub = ub[:, p].cpu()[:, ik, iz].numpy()
            guu = uu[:, p].cpu()[:, ik, iz].numpy()
            gtau = tau[:, p].cpu()[:, tz, tx].numpy()
            e_ub = [rel(gub[i], g[f"y{p}_ubar"][i]) for i in range(3)]
            e_uu = [rel(guu[k], g[f"y{p}_uubar"][k]) for k in range(6)]
            e_tau = [rel(gtau[k], g[f"y{p}_tau"][k]) for k in range(6)]
            print(f"[c5] {precision} y{p}: ubar {max(e_ub):.2e} uubar {max(e_uu):.2e} tau {max(e_tau):.2e}",
                  flush=True)
            assert max(e_ub) <= t_ub, (p, e_ub)
            assert max(e_uu) <= t_uu, (p, e_uu)
            assert max(e_tau) <= t_tau, (p, e_tau)
        ens = ch.filtered_enstrophy(kcx, kcz)
        for p in (int(p) for p in g["planes"]):
            ek, ez = torch.from_numpy(g[f"y{p}_ek"]), torch.from_numpy(g[f"y{p}_ez"])
            got = ens[p].cpu()[ek, ez].numpy()
            e_ens = rel(got, g[f"y{p}_ens"])
            e_00 = abs(complex(ens[p, 0, 0].item()) - complex(g[f"y{p}_ens00"])) / abs(complex(g[f"y{p}_ens00"]))
            print(f"[c5] {precision} y{p}: enstrophy {e_ens:.2e}, mode (0,0) {e_00:.2e}", flush=True)
            t_ens = 1e-12 if precision == "fp64" else 1e-5
            assert e_ens <= t_ens and e_00 <= t_ens, (p, e_ens, e_00)
    finally:
        ch.close()
