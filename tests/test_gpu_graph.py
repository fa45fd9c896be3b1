"""Graph-replayed RK3 steps (chn_step_rk3 with the step graph, the default)
against steps whose kernels are launched one by one: the same bits for the
state and the step record, across a change of time step (a new capture),
a chn_get_fields call that reuses the per-dt tables' scratch (an eager step
first), and on both precisions; the instability guard still stops a
replayed step."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu

CASE = synth.Case(n1=24, n2=33, n3=16, lx=2 * np.pi, lz=np.pi, re_b=2800.0, dt=0.004, amp=0.1, kmax=5, cfg=71)


def _pair(precision):
    from paper_1808_06461_amd import Channel
    v, om, U1, U3, y = synth.turbulent_field(CASE)
    chs = []
    for graph in (False, True):
        ch = Channel(CASE.n1, CASE.n2, CASE.n3, CASE.lx, CASE.lz, CASE.re_b, precision=precision, y=y)
        ch.step_graph(graph)
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        chs.append(ch)
    return chs


def _same(chs, what):
    a, b = (ch.get_fields("v", "omega2", "chi", "u1mean", "u3mean") for ch in chs)
    for k in a:
        assert torch.equal(a[k], b[k]), (what, k)


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_steps_match_launched_steps(precision):
    chs = _pair(precision)
    try:
        for ch in chs:
            ch.step(CASE.dt, 5)
        _same(chs, "5 steps")
        for ch in chs:  # a new time step: eager first step, then a new capture
            ch.step(0.7 * CASE.dt, 4)
        _same(chs, "new dt")
        for ch in chs:
            ch.get_fields("u1", "omega3")  # reuses the scratch of the per-dt tables
            ch.step(0.7 * CASE.dt, 3)
        _same(chs, "after get_fields")
        infos = [ch.step(0.7 * CASE.dt, 3, info=True) for ch in chs]
        _same(chs, "with a step record")
        for k in ("cfl_max", "mass_flux", "utau_lo", "utau_hi", "f_mean", "max_abs_div", "fail_step"):
            assert infos[0][k] == infos[1][k], k
    finally:
        for ch in chs:
            ch.close()


@gpu
def test_guard_stops_a_replayed_step():
    """Steps 1.. of a call are replayed; a time step whose CFL crosses the
    limit during them is still refused with the state of that sub-step."""
    from paper_1808_06461_amd import ChnError
    chs = _pair("fp64")
    try:
        probe = [ch.step(1e-6, 1, info=True) for ch in chs][0]
        dt = 1.95 / (probe["cfl_max"] / 1e-6)
        out = []
        for ch in chs:
            try:
                ch.step(dt, 8)
                out.append("ok")
            except ChnError as e:
                out.append(str(e))
        assert out[0] == out[1], out
        _same(chs, "guard")
    finally:
        for ch in chs:
            ch.close()
