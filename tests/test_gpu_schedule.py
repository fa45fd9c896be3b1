"""Plane-phase schedules (chn_set_plan / chn_autotune) against the oracle.

Every schedule must give the oracle's non-linear term to the same bounds as
the default one (float64 1e-13, mixed 2e-6 relative per component): the
x pass with 8, 4, 2 or one row per workgroup, z-pass workgroups of one line up to the
largest that fits, planes in chunks, and the runtime or compile-time radix
schedule (576-point lines).  The autotuner must pick a schedule that fits and leave
results within those bounds.
"""
import numpy as np
import pytest

import synth
from oracle import kmm

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu

CASES = {
    "small": synth.Case(n1=16, n2=33, n3=16, lx=2 * np.pi, lz=np.pi, re_b=2800.0, dt=0.005, amp=0.1, kmax=5,
                        cfg=21),
    "ragged": synth.Case(n1=24, n2=25, n3=12, lx=2 * np.pi, lz=np.pi / 2, re_b=1500.0, dt=0.004, amp=0.1,
                         kmax=None, cfg=22),
    "wide": synth.Case(n1=96, n2=17, n3=48, lx=2 * np.pi, lz=np.pi, re_b=3000.0, dt=0.002, amp=0.1, kmax=None,
                       cfg=23),
    # 576-point lines in x and z: the compile-time radix schedule applies
    "p576": synth.Case(n1=384, n2=9, n3=384, lx=2 * np.pi, lz=np.pi, re_b=10000.0, dt=0.002, amp=0.1,
                       kmax=None, cfg=24),
}
TOL = {"fp64": 1e-13, "mixed": 2e-6}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle(case):
    v, om, U1, U3, y = synth.turbulent_field(case)
    S = kmm.Setup(n1=case.n1, n2=case.n2, n3=case.n3, lx=case.lx, lz=case.lz, nu=1 / case.re_b, dt=case.dt,
                  mass_flux=case.mass_flux, y=y)
    fields = kmm.recover(S, kmm.make_state(S, v, om, U1, U3))
    return y, fields, kmm.nonlinear(S, fields)


def _check(ch, fields, ref, tol, what):
    got = [h.cpu().numpy() for h in ch.nonlinear([torch.from_numpy(f) for f in fields])]
    for g, r, name in zip(got, ref, ("H1", "H2", "H3")):
        e = rel(g, r)
        print(f"{what} {name}: {e:.2e}")
        assert e < tol, (what, name, e)


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_every_schedule_matches_oracle(name, precision):
    from paper_1808_06461_amd import Channel, ChnError
    case = CASES[name]
    y, fields, ref = _oracle(case)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
    try:
        default = ch.plan()
        assert default["x_rows"] == 2
        kmax = 0
        for k in range(1, case.n1 // 2 + 1):  # largest z_lines the context accepts
            try:
                ch.set_plan(2, k)
                kmax = k
            except ChnError:
                break
        assert kmax >= 1
        tried = set()
        for pipe in (0, 1):
            for fixed in (0, 1):
                for x_rows in (8, 4, 2, 1):
                    for k in sorted({1, 2, 3, kmax}):
                        if k > kmax:
                            continue
                        try:
                            ch.set_plan(x_rows, k, None, fixed, pipe)
                        except ChnError:  # more rows than the staging registers or LDS hold
                            assert x_rows > 2, (x_rows, k)
                            continue
                        tried.add(x_rows)
                        _check(ch, fields, ref, TOL[precision],
                               f"{precision} rows={x_rows} lines={k} fixed={fixed} pipeline={pipe}")
        assert {1, 2} <= tried
        ch.set_plan(2, 1, max(1, case.n2 // 3))  # planes in chunks
        _check(ch, fields, ref, TOL[precision], f"{precision} chunked planes")
        with pytest.raises(ChnError):
            ch.set_plan(3, 1)
        with pytest.raises(ChnError):
            ch.set_plan(1, 0)
    finally:
        ch.close()


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_picks_a_fitting_schedule(precision):
    from paper_1808_06461_amd import Channel
    case = CASES["wide"]
    y, fields, ref = _oracle(case)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
    try:
        v, om, U1, U3, _ = synth.turbulent_field(case)
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        before = {k: t.cpu().numpy() for k, t in ch.get_fields("v", "omega2", "chi").items()}
        p = ch.autotune(reps=2)
        print(precision, "autotune ->", p)
        assert p == ch.plan() and p["x_rows"] in (1, 2) and p["z_lines"] >= 1
        after = {k: t.cpu().numpy() for k, t in ch.get_fields("v", "omega2", "chi").items()}
        for k in before:  # the state is untouched
            assert np.array_equal(before[k], after[k]), k
        _check(ch, fields, ref, TOL[precision], f"{precision} autotuned")
    finally:
        ch.close()
