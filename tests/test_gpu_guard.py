"""The boundary's safety checks, through the C ABI.

* Instability guard: a sub-step whose CFL number is above CHN_CFL_LIMIT or
  not finite is not applied, whether or not a step record is requested; the
  call returns CHN_EUNSTABLE naming the step and sub-step, and the state is
  as at the start of that sub-step (for sub-step 0: the start of the step).
* Step record: divergence of the transformed velocities at rounding level,
  per-phase times of the last step, no failure reported on a good step.
* Mesh checks at chn_create: the default mesh (y = NULL) has well-conditioned
  compact operators for every size (checked against the oracle's operators
  on the mesh the library reports), and a mesh on which the maximum-order
  stencils degenerate is refused with CHN_EINVAL.
"""
import numpy as np
import pytest

import synth
from oracle import compact, meshopt

torch = pytest.importorskip("torch")

gpu = pytest.mark.gpu
CASE = synth.Case(n1=16, n2=33, n3=16, lx=2 * np.pi, lz=np.pi, re_b=2800.0, dt=0.005, amp=0.1, kmax=5, cfg=61)


def _channel(precision="fp64", y=None, case=CASE):
    from paper_1808_06461_amd import Channel
    return Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)


def _state(ch):
    return {k: t.cpu().numpy().copy() for k, t in ch.get_fields("v", "omega2", "chi", "u1mean", "u3mean").items()}


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_huge_time_step_is_refused_without_a_step_record(precision):
    from paper_1808_06461_amd import ChnError
    v, om, U1, U3, y = synth.turbulent_field(CASE)
    ch = _channel(precision, y)
    try:
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        before = _state(ch)
        with pytest.raises(ChnError, match="CHN_EUNSTABLE.*step 0, sub-step 0"):
            ch.step(10.0, 3)                  # CFL of the initial field ~ 1e3
        after = _state(ch)
        for k in before:                      # not one bit of the state changed
            assert np.array_equal(before[k], after[k]), k
        st, rec, msg = ch.step_status(10.0, 1)
        assert st == "CHN_EUNSTABLE" and rec["fail_step"] == 0 and rec["fail_substep"] == 0
        assert rec["cfl_max"] > 2.0, rec
        info = ch.step(CASE.dt, 2, info=True)  # the context goes on with a stable step
        assert info["fail_step"] == -1 and 0 < info["cfl_max"] < 2.0
    finally:
        ch.close()


@gpu
def test_nan_is_refused_without_a_step_record():
    from paper_1808_06461_amd import ChnError
    v, om, U1, U3, y = synth.turbulent_field(CASE)
    v = v.copy()
    v[CASE.n2 // 2, 2, 3] = np.nan
    ch = _channel("mixed", y)
    try:
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        with pytest.raises(ChnError, match="CHN_EUNSTABLE.*not finite"):
            ch.step(CASE.dt, 1)
    finally:
        ch.close()


@gpu
def test_instability_in_a_later_sub_step_stops_there():
    """A CFL limit crossed between two steps: the record names the step, the
    state stays finite (later sub-steps skipped)."""
    v, om, U1, U3, y = synth.turbulent_field(CASE)
    ch = _channel("fp64", y)
    try:
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        probe = ch.step(1e-6, 1, info=True)
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        dt = 1.9 / (probe["cfl_max"] / 1e-6)  # CFL 1.9 at t = 0: over 2 after some growth, or stays below
        st, rec, msg = ch.step_status(dt, 6)
        f = _state(ch)
        assert all(np.isfinite(a).all() for a in f.values())
        if st == "CHN_EUNSTABLE":
            assert 0 <= rec["fail_step"] < 6 and 0 <= rec["fail_substep"] < 3 and rec["cfl_max"] > 2.0
        else:
            assert st == "CHN_OK" and rec["fail_step"] == -1 and rec["cfl_max"] <= 2.0
    finally:
        ch.close()


@gpu
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("mixed", 1e-6)])
def test_step_record(precision, tol):
    v, om, U1, U3, y = synth.turbulent_field(CASE)
    ch = _channel(precision, y)
    try:
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        info = ch.step(CASE.dt, 2, info=True)
        u = ch.get_fields("u1", "u3")
        umax = max(float(t.abs().max()) for t in u.values())
        print(precision, info)
        assert info["fail_step"] == -1 and info["fail_substep"] == -1
        assert 0 <= info["max_abs_div"] < tol * umax, (info["max_abs_div"], umax)
        assert all(t > 0 for t in info["ms_phase"][:4]), info["ms_phase"]
    finally:
        ch.close()


def _cond_dirichlet_a2(y):
    A2, _ = compact.operators(y, 2)
    A2 = A2.copy()
    A2[0] = 0.0
    A2[0, compact.HALF] = 1.0
    A2[-1] = 0.0
    A2[-1, compact.HALF] = 1.0
    return meshopt.cond1(A2)


@gpu
@pytest.mark.parametrize("n2", [33, 49, 65, 97])
def test_default_mesh_is_well_conditioned(n2):
    from paper_1808_06461_amd import Channel
    ch = Channel(8, n2, 8, 2 * np.pi, np.pi, 1000.0)
    try:
        y = ch.mesh()
    finally:
        ch.close()
    assert y[0] == -1.0 and y[-1] == 1.0 and np.all(np.diff(y) > 0)
    np.testing.assert_array_equal(y, -y[::-1])
    c2 = _cond_dirichlet_a2(y)
    c1 = meshopt.cond1(compact.operators(y, 1)[0])
    print(n2, f"cond1(A2 Dirichlet) {c2:.3e}, cond1(A1) {c1:.3e}")
    assert c2 < 1e4 and c1 < 1e5


@gpu
@pytest.mark.parametrize("n2", [49, 65])
def test_degenerate_mesh_is_refused(n2):
    from paper_1808_06461_amd import ChnError
    y = synth.mesh_tanh(n2, 2.0)
    assert _cond_dirichlet_a2(y) > 1e9  # the oracle's operators: near singular
    with pytest.raises(ChnError, match="CHN_EINVAL.*ill-conditioned"):
        _channel("fp64", y, synth.Case(n1=8, n2=n2, n3=8, lx=2 * np.pi, lz=np.pi, re_b=1000.0, dt=0.01))
