"""Parity of the low-storage stage (chn_filter_and_stress, chn_filtered_enstrophy) with the oracle.

Float64 path: 1e-12 relative per output component.  Mixed path (the float32
velocity and vorticity coefficients of the time step, float32 inverse
transforms, float64 products, forward transforms and sums): 1e-7 on F(u_i)
(the float32 rounding of the data) and 1e-5 relative on F(u_i u_j), tau_ij
and the filtered enstrophy, the bound the workload states; float64 1e-12 on
the enstrophy.  Filter calls share pencil scratch and the phase fields with
the time step, so time stepping after them must match uninterrupted
stepping bit for bit.  The
filtered pressure (float64 on both paths): from the oracle's own F(u_i u_j),
F(u_i) (the solve alone) 1e-11; from the library's filter outputs 1e-11
(float64) and 1e-5 (mixed, whose stresses carry float32 data).
"""
import numpy as np
import pytest

import synth
from oracle import kmm, lowstorage

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = {
    "small": (synth.Case(n1=32, n2=17, n3=24, lx=2 * np.pi, lz=np.pi, re_b=2000.0, dt=0.0, amp=0.1,
                         mean="reichardt", re_tau=180.0, cfg=31), 3, 2, 16, 12),
    "ragged": (synth.Case(n1=48, n2=13, n3=36, lx=2 * np.pi, lz=np.pi, re_b=2000.0, dt=0.0, amp=0.1,
                          mean="reichardt", re_tau=180.0, cfg=32), 5, 4, 24, 18),
    "mid": (synth.Case(n1=192, n2=25, n3=144, lx=2 * np.pi, lz=np.pi, re_b=18863.0, dt=0.0, amp=0.1,
                       mean="reichardt", re_tau=950.0, spectrum=-8.0 / 3.0, cfg=33), 12, 9, 54, 48),
}


def _run(name, precision):
    from paper_1808_06461_amd import Channel
    case, kcx, kcz, q1, q3 = CASES[name]
    v, om, U1, U3, y = synth.turbulent_field(case)
    S = kmm.Setup(n1=case.n1, n2=case.n2, n3=case.n3, lx=case.lx, lz=case.lz, nu=1 / case.re_b, dt=1e-3,
                  mass_flux=2.0, y=y)
    st = kmm.make_state(S, v, om, U1, U3)
    u1, u2, u3, *_ = kmm.recover(S, st)
    ub, uu, tau = lowstorage.filter_and_stress(u1, u2, u3, kcx, kcz, q1, q3)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
    ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
    gub, guu, gtau = (t.cpu().numpy() for t in ch.filter_and_stress(kcx, kcz, q1, q3))
    ch.close()
    return (ub, uu, tau), (gub, guu, gtau)


@gpu
@pytest.mark.parametrize("name", ["small", "ragged", "mid"])
def test_filter_and_stress_fp64(name):
    (ub, uu, tau), (gub, guu, gtau) = _run(name, "fp64")
    for i in range(3):
        assert rel(gub[i], ub[i]) < 1e-13, ("ubar", i, rel(gub[i], ub[i]))
    for p in range(6):
        e_uu, e_tau = rel(guu[p], uu[p]), rel(gtau[p], tau[p])
        print(f"fp64 {name} pair {p}: uu {e_uu:.2e} tau {e_tau:.2e}")
        assert e_uu < 1e-12 and e_tau < 1e-10, (p, e_uu, e_tau)


@gpu
@pytest.mark.parametrize("name", ["small", "ragged", "mid"])
def test_filter_and_stress_mixed(name):
    (ub, uu, tau), (gub, guu, gtau) = _run(name, "mixed")
    for i in range(3):  # the mixed path stores the velocity coefficients in float32
        assert rel(gub[i], ub[i]) < 1e-7, ("ubar", i, rel(gub[i], ub[i]))
    for p in range(6):
        e_uu, e_tau = rel(guu[p], uu[p]), rel(gtau[p], tau[p])
        print(f"mixed {name} pair {p}: uu {e_uu:.2e} tau {e_tau:.2e}")
        assert e_uu < 1e-5 and e_tau < 1e-5, (p, e_uu, e_tau)


@gpu
def test_device_limits_report():
    import torch as T
    p = T.cuda.get_device_properties(0)
    print("device:", p.name, "LDS/block:", getattr(p, "shared_memory_per_block", None),
          "LDS/block optin:", getattr(p, "shared_memory_per_block_optin", None),
          "multiprocessors:", p.multi_processor_count)


def _ens_case(name, kc=None):
    case, kcx, kcz, _, _ = CASES[name]
    if kc is not None:
        kcx, kcz = kc
    v, om, U1, U3, y = synth.turbulent_field(case)
    S = kmm.Setup(n1=case.n1, n2=case.n2, n3=case.n3, lx=case.lx, lz=case.lz, nu=1 / case.re_b, dt=1e-3,
                  mass_flux=2.0, y=y)
    *_, o1, o2, o3 = kmm.recover(S, kmm.make_state(S, v, om, U1, U3))
    return case, (v, om, U1, U3, y), kcx, kcz, lowstorage.filtered_enstrophy(o1, o2, o3, kcx, kcz)


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["small", "ragged", "mid"])
def test_filtered_enstrophy(name, precision):
    from paper_1808_06461_amd import Channel
    case, (v, om, U1, U3, y), kcx, kcz, ref = _ens_case(name)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
    try:
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        got = ch.filtered_enstrophy(kcx, kcz).cpu().numpy()
        e = rel(got, ref)
        e0 = float(np.abs(got[:, 0, 0] - ref[:, 0, 0]).max() / np.abs(ref[:, 0, 0]).max())
        print(f"{precision} {name}: enstrophy {e:.2e}, mode (0,0) {e0:.2e}")
        tol = 1e-12 if precision == "fp64" else 1e-5
        assert e < tol and e0 < tol, (e, e0)
    finally:
        ch.close()


@gpu
@pytest.mark.parametrize("kc", [(0, 0), (7, 11), (15, 11)])
def test_filtered_enstrophy_extreme_cutoffs(kc):
    """Only the (0,0) mode, half the kx, and every stored mode of the 32 x 24
    context; the full cut-off of filter_and_stress, whose six products on
    the retained set exceed the context's workspace, is CHN_EUNSUPPORTED."""
    from paper_1808_06461_amd import Channel, ChnError
    case, (v, om, U1, U3, y), kcx, kcz, ref = _ens_case("small", kc)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision="fp64", y=y)
    try:
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        e = rel(ch.filtered_enstrophy(kcx, kcz).cpu().numpy(), ref)
        print(f"kc={kc}: {e:.2e}")
        assert e < 1e-12, e
        with pytest.raises(ChnError, match="CHN_EUNSUPPORTED"):
            ch.filter_and_stress(case.n1 // 2 - 1, case.n3 // 2 - 1, 32, 24)
    finally:
        ch.close()


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_filter_calls_leave_time_stepping_intact(precision):
    from paper_1808_06461_amd import Channel, ChnError
    case, kcx, kcz, q1, q3 = CASES["small"]
    v, om, U1, U3, y = synth.turbulent_field(case)
    dt = 0.004
    out = []
    for interrupt in (False, True):
        ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
        try:
            ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
            ch.step(dt, 1)
            if interrupt:
                ch.filter_and_stress(kcx, kcz, q1, q3)
                ch.filtered_enstrophy(kcx, kcz)
                ch.get_fields("u1", "omega3")
                with pytest.raises(ChnError, match="CHN_EINVAL"):
                    ch.filtered_enstrophy(case.n1 // 2, kcz)
            ch.step(dt, 2)
            out.append({k: t.cpu().numpy() for k, t in ch.get_fields("v", "omega2", "chi").items()})
        finally:
            ch.close()
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["small", "ragged", "mid"])
def test_filtered_pressure(name, precision):
    from paper_1808_06461_amd import Channel, ChnError
    case, kcx, kcz, q1, q3 = CASES[name]
    v, om, U1, U3, y = synth.turbulent_field(case)
    S = kmm.Setup(n1=case.n1, n2=case.n2, n3=case.n3, lx=case.lx, lz=case.lz, nu=1 / case.re_b, dt=1e-3,
                  mass_flux=2.0, y=y)
    u1, u2, u3, *_ = kmm.recover(S, kmm.make_state(S, v, om, U1, U3))
    ub, uu, _ = lowstorage.filter_and_stress(u1, u2, u3, kcx, kcz, q1, q3)
    ref = lowstorage.filtered_pressure(S, uu, ub, kcx, kcz)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
    try:
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
        e1 = rel(ch.filtered_pressure(kcx, kcz, dev(uu), dev(ub)).cpu().numpy(), ref)
        gub, guu, _ = ch.filter_and_stress(kcx, kcz, q1, q3, with_tau=False)
        e2 = rel(ch.filtered_pressure(kcx, kcz, guu, gub).cpu().numpy(), ref)
        print(f"{precision} {name}: pressure from oracle stresses {e1:.2e}, from library stresses {e2:.2e}")
        assert e1 < 1e-11, e1
        assert e2 < (1e-11 if precision == "fp64" else 1e-5), e2
        # only the mean mode retained
        ub0, uu0, _ = lowstorage.filter_and_stress(u1, u2, u3, 0, 0, 2, 2)
        p0 = ch.filtered_pressure(0, 0, dev(uu0), dev(ub0)).cpu().numpy()
        assert np.array_equal(p0[:, 0, 0], -uu0[3][:, 0, 0].real + 0j)
        with pytest.raises(ChnError, match="CHN_EINVAL"):
            ch._check(ch.L.chn_filtered_pressure(ch.ctx, kcx, kcz, None, None, None), "chn_filtered_pressure")
    finally:
        ch.close()


@gpu
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_filter_after_a_step_reads_the_current_fields(precision, tol):
    """After a step the stage reads the velocity and vorticity coefficients the
    step left for its next transforms; they must be those of the state it
    reached: the same outputs as a new context set to that state."""
    from paper_1808_06461_amd import Channel
    case, kcx, kcz, q1, q3 = CASES["small"]
    v, om, U1, U3, y = synth.turbulent_field(case)
    outs = []
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
    try:
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        ch.step(0.004, 2)
        outs.append([t.cpu().numpy() for t in ch.filter_and_stress(kcx, kcz, q1, q3)] +
                    [ch.filtered_enstrophy(kcx, kcz).cpu().numpy()])
        st = ch.get_fields("v", "omega2", "u1mean", "u3mean")
    finally:
        ch.close()
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, precision=precision, y=y)
    try:
        ch.set_state(st["v"], st["omega2"], st["u1mean"], st["u3mean"])
        outs.append([t.cpu().numpy() for t in ch.filter_and_stress(kcx, kcz, q1, q3)] +
                    [ch.filtered_enstrophy(kcx, kcz).cpu().numpy()])
    finally:
        ch.close()
    for name, a, b in zip(("ubar", "uubar", "tau", "enstrophy"), *outs):
        e = rel(a, b)
        print(f"{precision} {name}: {e:.2e}")
        assert e < tol, (name, e)
