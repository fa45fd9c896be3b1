"""Parity at full size: the 384 x 193 x 384 channel (Re_tau ~ 550) after 20 RK3 steps.

The oracle takes about 45 minutes for this run, so its result is stored:
tests/golden/make_c2_golden.py runs only the oracle and keeps 8192 seeded
mode-point samples of v, omega2, chi, u1, u3, omega1, omega3 plus the full
mean profiles.  Here the GPU path runs the same 20 steps, in the launch
configuration the benchmark times, and is compared on those samples:
e(X) = ||X_gpu[s] - X_oracle[s]|| / ||X_oracle[s]||.
"""
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_20steps.npz")
FIELDS = ("v", "omega2", "chi", "u1", "u3", "omega1", "omega3")

# float64: 1e-11 per field, chi (wall values from the influence-matrix
# cancellation) 1e-10.  Mixed: 1e-5 on the velocities; the vorticities and
# chi, one derivative further from the products, get 1e-4.
TOL64 = dict(v=1e-11, omega2=1e-11, chi=1e-10, u1=1e-11, u3=1e-11, omega1=1e-11, omega3=1e-11,
             U1=1e-11, U3=1e-11)
TOLMX = dict(v=1e-5, omega2=1e-4, chi=1e-4, u1=1e-5, u3=1e-5, omega1=1e-4, omega3=1e-4, U1=1e-5, U3=1e-5)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _run(precision, g):
    from paper_1808_06461_amd import Channel
    c = synth.CASES["c2"]
    v, om, U1, U3, y = synth.turbulent_field(c)
    ch = Channel(c.n1, c.n2, c.n3, c.lx, c.lz, c.re_b, mass_flux=c.mass_flux, precision=precision, y=y)
    try:
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        info = ch.step(float(g["dt"]), int(g["nsteps"]), info=True)
        f = ch.get_fields(*FIELDS, "u1mean", "u3mean")
        idx = (torch.from_numpy(g["iy"]), torch.from_numpy(g["ikx"]), torch.from_numpy(g["ikz"]))
        out = {k: f[k].cpu()[idx].numpy() if f[k].dim() == 3 else f[k].cpu().numpy() for k in f}
        out["U1"], out["U3"] = out.pop("u1mean"), out.pop("u3mean")
        return out, info
    finally:
        ch.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_twenty_steps_against_oracle_samples(precision):
    g = np.load(GOLDEN)
    out, info = _run(precision, g)
    tol = TOL64 if precision == "fp64" else TOLMX
    errs = {k: rel(out[k], g[k]) for k in tol}
    print(precision, {k: f"{e:.2e}" for k, e in errs.items()}, "f", info["f_mean"], float(g["f"]))
    for k, e in errs.items():
        assert e <= tol[k], (k, e)
    assert abs(info["f_mean"] - float(g["f"])) <= (1e-9 if precision == "fp64" else 1e-4) * abs(float(g["f"]))
