"""Error behaviour of the C ABI (include/chn.h).

CPU part: chn_workspace_bytes rejects every invalid configuration (it returns
0 before any device call), and accepts the workloads' sizes.  GPU part: calls
in the wrong order or with bad arguments return the documented status and
leave the context usable.
"""
import ctypes as C
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def _lib():
    from paper_1808_06461_amd import chn
    if not os.path.exists(chn.LIB_PATH):
        pytest.skip("libchn.so not built")
    return chn, chn.lib()


def _bytes(n1, n2, n3, precision=1, lx=2 * np.pi, lz=np.pi, re_b=1000.0, planes_only=0, chunk=0, y=None):
    chn, L = _lib()
    yp = C.POINTER(C.c_double)()
    keep = None
    if y is not None:
        keep = (C.c_double * len(y))(*y)
        yp = C.cast(keep, C.POINTER(C.c_double))
    cfg = chn.Config(n1, n2, n3, lx, lz, re_b, 2.0, precision, yp, None, planes_only, chunk)
    return L.chn_workspace_bytes(C.byref(cfg))


@pytest.mark.parametrize("args", [
    dict(n1=7, n2=33, n3=16),          # n1 odd
    dict(n1=16, n2=33, n3=14),         # n3 not a multiple of 4
    dict(n1=20, n2=33, n3=16),         # 3 n1 / 2 = 30 has a factor 5
    dict(n1=16, n2=33, n3=40),         # 3 n3 / 2 = 60 has a factor 5
    dict(n1=16, n2=8, n3=16),          # n2 < 9
    dict(n1=16, n2=4096, n3=16),       # n2 > 2048
    dict(n1=16, n2=33, n3=16, lx=0.0),
    dict(n1=16, n2=33, n3=16, re_b=-1.0),
    dict(n1=16, n2=33, n3=16, precision=2),
    dict(n1=16, n2=33, n3=16, chunk=40),        # plane_chunk > n2
    dict(n1=16, n2=33, n3=16, planes_only=1),   # planes_only needs plane_chunk
    dict(n1=16384, n2=33, n3=16, precision=0),  # float64 rows of 24576 points: no x pass holds them
    dict(n1=16, n2=9, n3=16, y=[-1, -0.5, -0.2, 0.0, 0.1, 0.3, 0.5, 0.9, 0.99]),  # y[-1] != 1
    dict(n1=16, n2=9, n3=16, y=[-1, -0.5, -0.2, 0.0, 0.0, 0.3, 0.5, 0.9, 1.0]),   # not ascending
])
def test_invalid_configurations_are_rejected(args):
    assert _bytes(**args) == 0


@pytest.mark.parametrize("name", ["c1", "c2", "c5"])
@pytest.mark.parametrize("precision", [0, 1])
def test_workload_configurations_are_accepted(name, precision):
    c = synth.CASES[name]
    assert _bytes(c.n1, c.n2, c.n3, precision, c.lx, c.lz, c.re_b) > 0


def test_share_configurations_are_accepted():
    c = synth.C3_PLANES
    assert _bytes(c["n1"], c["nplanes"], c["n3"], 1, planes_only=1, chunk=8) > 0
    p = synth.c3_pencil_case()
    assert _bytes(p.n1, p.n2, p.n3, 1) > 0


@pytest.mark.gpu
def test_misuse_returns_errors_and_leaves_context_usable():
    from paper_1808_06461_amd import Channel, ChnError
    case = synth.Case(n1=16, n2=33, n3=16, lx=2 * np.pi, lz=np.pi, re_b=2000.0, dt=0.005, amp=0.1, cfg=41)
    v, om, U1, U3, y = synth.turbulent_field(case)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, y=y)
    try:
        with pytest.raises(ChnError, match="CHN_ESTATE"):
            ch.step(case.dt, 1)
        with pytest.raises(ChnError, match="CHN_ESTATE"):
            ch.get_fields("v")
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        with pytest.raises(ChnError, match="CHN_EINVAL"):
            ch.step(-1.0, 1)
        with pytest.raises(ChnError, match="CHN_EINVAL"):
            ch.filter_and_stress(8, 2, 16, 12)      # kcx >= n1 / 2
        with pytest.raises(ChnError, match="CHN_EINVAL"):
            ch.filter_and_stress(3, 2, 6, 12)       # q1 <= 2 kcx
        with pytest.raises(ChnError, match="CHN_EINVAL"):
            ch.set_plan(2, 1, 0)                    # no planes per launch
        info = ch.step(case.dt, 1, info=True)       # still usable
        assert np.isfinite(info["cfl_max"]) and abs(info["mass_flux"] - 2.0) < 1e-12
    finally:
        ch.close()


@pytest.mark.gpu
def test_planes_only_context_refuses_state_calls():
    from paper_1808_06461_amd import Channel, ChnError
    ch = Channel(16, 12, 16, 2 * np.pi, np.pi, 1000.0, precision="mixed", planes_only=True, plane_chunk=4)
    try:
        z = torch.zeros((12, 8, 16), dtype=torch.complex128)
        with pytest.raises(ChnError, match="CHN_EUNSUPPORTED"):
            ch.set_state(z, z, torch.zeros(12, dtype=torch.float64), torch.zeros(12, dtype=torch.float64))
        with pytest.raises(ChnError, match="CHN_EUNSUPPORTED"):
            ch.autotune(1)
        with pytest.raises(ChnError, match="CHN_EINVAL"):
            ch.set_plan(2, 1, 5)                    # more planes than the workspace holds
        f = [torch.zeros((12, 8, 16), dtype=torch.complex64, device="cuda") for _ in range(6)]
        H = ch.plane_products(f)                    # zero fields give zero products
        assert all(float(h.abs().max()) == 0.0 for h in H)
    finally:
        ch.close()
