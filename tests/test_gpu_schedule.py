"""Plane-phase schedules (chn_set_plan / chn_autotune) against the oracle.

Every schedule must give the oracle's non-linear term to the same bounds as
the default one (float64 1e-13, mixed 2e-6 relative per component): the
x pass with 8, 4, 2 or one row per workgroup, z-pass workgroups of one line up to the
largest that fits, planes in chunks, the runtime or compile-time radix
schedule (576-point lines), and the radix sets of the x and z transforms
(passes of radix 8, 4, 2, 3, or the fewest passes with the composite
radices 6, 9, 12, 16).  The
autotuner must pick a schedule that fits and leave results within those
bounds; its cache file must be written, and a cached schedule reused
without timing.
"""
import json
import os

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
        for radix in (0, 1, 2, 3):
            for pipe in (0, 1):
                for fixed in (0, 1):
                    for x_rows in (8, 4, 2, 1):
                        for k in sorted({1, 2, 3, kmax}):
                            if k > kmax:
                                continue
                            try:
                                ch.set_plan(x_rows, k, None, fixed, pipe, radix)
                            except ChnError:  # more rows or lines than the staging registers or LDS hold
                                assert x_rows > 2 or radix > 0, (x_rows, k, radix)
                                continue
                            tried.add((radix, x_rows))
                            _check(ch, fields, ref, TOL[precision],
                                   f"{precision} radix set {radix} rows={x_rows} lines={k} fixed={fixed} "
                                   f"pipeline={pipe}")
        assert {(0, 1), (0, 2), (1, 2), (2, 2), (3, 2)} <= tried, tried
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
def test_autotune_picks_a_fitting_schedule(precision, tmp_path, monkeypatch):
    from paper_1808_06461_amd import Channel
    monkeypatch.setenv("CHN_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    case = CASES["wide"]
    y, fields, ref = _oracle(case)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
    try:
        v, om, U1, U3, _ = synth.turbulent_field(case)
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        before = {k: t.cpu().numpy() for k, t in ch.get_fields("v", "omega2", "chi").items()}
        p = ch.autotune(reps=2)
        print(precision, "autotune ->", p)
        assert p == ch.plan() and p["x_rows"] in (1, 2, 4, 8) and p["z_lines"] >= 1
        after = {k: t.cpu().numpy() for k, t in ch.get_fields("v", "omega2", "chi").items()}
        for k in before:  # the state is untouched
            assert np.array_equal(before[k], after[k]), k
        _check(ch, fields, ref, TOL[precision], f"{precision} autotuned")
    finally:
        ch.close()


@gpu
def test_autotune_cache_is_reused(tmp_path, monkeypatch):
    """A cached schedule for the context's key is applied without timing (the
    last entry of a key wins), still matches the oracle, and an empty
    CHN_TUNE_CACHE writes no file."""
    from paper_1808_06461_amd import Channel
    case = CASES["wide"]
    y, fields, ref = _oracle(case)
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("CHN_TUNE_CACHE", str(path))
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision="mixed", y=y)
    try:
        p = ch.autotune(reps=1)
    finally:
        ch.close()
    rows = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(rows) == 1 and rows[0]["plan"] == [p[k] for k in ("x_rows", "z_lines", "y_chunk", "fixed_radix",
                                                                 "z_pipeline", "radix_set")]
    key = rows[0]["key"]
    assert "/96x17x48/mixed/" in key, key
    # a different schedule under the same key, appended: the later entry wins
    other = [1, 1, case.n2, 0, 0, 3 - p["radix_set"]]
    with open(path, "a") as f:
        f.write(json.dumps({"key": key, "plan": other}) + "\n")
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision="mixed", y=y)
    try:
        q = ch.autotune(reps=1)
        assert [q[k] for k in ("x_rows", "z_lines", "y_chunk", "fixed_radix", "z_pipeline", "radix_set")] == other
        assert ch.plan() == q
        _check(ch, fields, ref, TOL["mixed"], "cached schedule")
    finally:
        ch.close()
    assert len(path.read_text().splitlines()) == 2  # reused, nothing appended
    off = tmp_path / "off"
    monkeypatch.setenv("CHN_TUNE_CACHE", "")
    monkeypatch.setenv("HOME", str(off))
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision="mixed", y=y)
    try:
        ch.autotune(reps=1)
    finally:
        ch.close()
    assert not off.exists()
