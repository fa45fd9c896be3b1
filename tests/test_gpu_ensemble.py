"""Ensemble path (batched launches over uneven channels, HIP graph) against
single-context runs and, for one channel, the oracle."""
import numpy as np
import pytest

import synth
from oracle import kmm

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu

SPECS = [
    synth.Case(n1=16, n2=33, n3=16, lx=2 * np.pi, lz=np.pi, re_b=2800.0, dt=0.004, amp=0.1, kmax=5, cfg=41),
    synth.Case(n1=24, n2=25, n3=12, lx=np.pi, lz=np.pi / 2, re_b=1500.0, dt=0.003, amp=0.1, cfg=42),
    synth.Case(n1=32, n2=17, n3=24, lx=np.pi, lz=np.pi / 2, re_b=2000.0, dt=0.002, amp=0.1, cfg=43),
    synth.Case(n1=16, n2=49, n3=32, lx=np.pi, lz=np.pi / 2, re_b=3000.0, dt=0.003, amp=0.1, cfg=44),
    synth.Case(n1=48, n2=25, n3=16, lx=2 * np.pi, lz=np.pi, re_b=2500.0, dt=0.004, amp=0.1, cfg=45),
]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _spec(c, y):
    return dict(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, re_b=c.re_b, mass_flux=c.mass_flux, y=y)


def _same_radix(single, channel):
    """The single context takes the radix sets the ensemble gave the channel."""
    p, q = single.plan(), channel.plan()
    single.set_plan(p["x_rows"], p["z_lines"], p["y_chunk"], p["fixed_radix"], p["z_pipeline"], q["radix_set"])


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ensemble_matches_single_contexts(precision):
    from paper_1808_06461_amd import Channel
    from paper_1808_06461_amd.chn import Ensemble
    fields = [synth.turbulent_field(c) for c in SPECS]
    ens = Ensemble([_spec(c, f[4]) for c, f in zip(SPECS, fields)], precision=precision)
    for ch, (v, om, U1, U3, y) in zip(ens.channels, fields):
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
    ens.step([c.dt for c in SPECS], 2)
    for k, (c, (v, om, U1, U3, y)) in enumerate(zip(SPECS, fields)):
        got = {n: t.cpu().numpy() for n, t in ens.channels[k].get_fields("v", "omega2", "chi", "u1mean").items()}
        single = Channel(c.n1, c.n2, c.n3, c.lx, c.lz, c.re_b, precision=precision, y=y)
        _same_radix(single, ens.channels[k])
        single.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        single.step(c.dt, 2)
        ref = {n: t.cpu().numpy() for n, t in single.get_fields("v", "omega2", "chi", "u1mean").items()}
        single.close()
        for n in ref:
            e = rel(got[n], ref[n])
            print(f"{precision} channel {k} {n}: {e:.2e}")
            assert e < 1e-14, (k, n, e)
    ens.close()


@gpu
def test_ensemble_one_wall_normal_size_matches_single_contexts():
    """Channels of one n2 run on two graph branches with the second group one
    plane phase behind; every channel still steps exactly as alone."""
    from paper_1808_06461_amd import Channel
    from paper_1808_06461_amd.chn import Ensemble
    specs = [synth.Case(n1=16, n2=33, n3=16, lx=2 * np.pi, lz=np.pi, re_b=2800.0, dt=0.004, amp=0.1, kmax=5, cfg=51),
             synth.Case(n1=24, n2=33, n3=12, lx=np.pi, lz=np.pi / 2, re_b=1500.0, dt=0.003, amp=0.1, cfg=52),
             synth.Case(n1=32, n2=33, n3=24, lx=np.pi, lz=np.pi / 2, re_b=2000.0, dt=0.002, amp=0.1, cfg=53)]
    fields = [synth.turbulent_field(c) for c in specs]
    ens = Ensemble([_spec(c, f[4]) for c, f in zip(specs, fields)], precision="mixed")
    for ch, (v, om, U1, U3, y) in zip(ens.channels, fields):
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
    ens.step([c.dt for c in specs], 3)
    for k, (c, (v, om, U1, U3, y)) in enumerate(zip(specs, fields)):
        got = {n: t.cpu().numpy() for n, t in ens.channels[k].get_fields("v", "omega2", "chi", "u1mean").items()}
        single = Channel(c.n1, c.n2, c.n3, c.lx, c.lz, c.re_b, precision="mixed", y=y)
        _same_radix(single, ens.channels[k])
        single.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        single.step(c.dt, 3)
        ref = {n: t.cpu().numpy() for n, t in single.get_fields("v", "omega2", "chi", "u1mean").items()}
        single.close()
        for n in ref:
            e = rel(got[n], ref[n])
            print(f"one-n2 channel {k} {n}: {e:.2e}")
            assert e < 1e-14, (k, n, e)
    ens.close()


@gpu
def test_ensemble_of_one_channel_matches_single_context():
    """One channel: a graph of one branch."""
    from paper_1808_06461_amd import Channel
    from paper_1808_06461_amd.chn import Ensemble
    c = SPECS[0]
    v, om, U1, U3, y = synth.turbulent_field(c)
    ens = Ensemble([_spec(c, y)], precision="mixed")
    ens.channels[0].set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
    ens.step([c.dt], 2)
    got = {n: t.cpu().numpy() for n, t in ens.channels[0].get_fields("v", "omega2", "chi", "u1mean").items()}
    single = Channel(c.n1, c.n2, c.n3, c.lx, c.lz, c.re_b, precision="mixed", y=y)
    _same_radix(single, ens.channels[0])
    single.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
    single.step(c.dt, 2)
    ref = {n: t.cpu().numpy() for n, t in single.get_fields("v", "omega2", "chi", "u1mean").items()}
    single.close()
    ens.close()
    for n in ref:
        e = rel(got[n], ref[n])
        print(f"one channel {n}: {e:.2e}")
        assert e < 1e-14, (n, e)


@gpu
def test_ensemble_channel_matches_oracle():
    from paper_1808_06461_amd.chn import Ensemble
    fields = [synth.turbulent_field(c) for c in SPECS]
    ens = Ensemble([_spec(c, f[4]) for c, f in zip(SPECS, fields)])
    for ch, (v, om, U1, U3, y) in zip(ens.channels, fields):
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
    ens.step([c.dt for c in SPECS], 1)
    k = 3
    c = SPECS[k]
    v, om, U1, U3, y = fields[k]
    S = kmm.Setup(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, nu=1 / c.re_b, dt=c.dt, mass_flux=c.mass_flux, y=y)
    ref, _ = kmm.step(S, kmm.make_state(S, v, om, U1, U3), 1)
    got = {n: t.cpu().numpy() for n, t in ens.channels[k].get_fields("v", "omega2", "u1mean").items()}
    for n, r in (("v", ref.v), ("omega2", ref.om2), ("u1mean", ref.U1)):
        e = rel(got[n], r)
        print(f"oracle channel {k} {n}: {e:.2e}")
        assert e < 1e-11, (n, e)
    ens.close()


def c4_ensemble(precision="fp64", n=96):
    """The 96-channel workload (sizes, Re_tau and seeds from synth.ensemble_cases),
    each channel's dt from CFL 0.5 at t = 0 measured by a probe step."""
    from paper_1808_06461_amd.chn import Ensemble
    cases = synth.ensemble_cases(n)
    fields = [synth.turbulent_field(c) for c in cases]
    ens = Ensemble([_spec(c, f[4]) for c, f in zip(cases, fields)], precision=precision)
    dts = []
    for ch, (v, om, U1, U3, y) in zip(ens.channels, fields):
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        info = ch.step(1e-6, 1, info=True)
        dts.append(0.5 * 1e-6 / info["cfl_max"])
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
    return ens, cases, fields, dts


@gpu
def test_c4_ensemble_fifty_steps():
    """96 uneven minimal channels, 50 RK3 steps in the graph: finite, walls, mass flux,
    and two channels bitwise equal to single-context runs."""
    from oracle import compact
    from paper_1808_06461_amd import Channel
    ens, cases, fields, dts = c4_ensemble()
    ens.step(dts, 50)
    for k, (c, ch) in enumerate(zip(cases, ens.channels)):
        got = {n: t.cpu().numpy() for n, t in ch.get_fields("v", "omega2", "u1mean").items()}
        assert all(np.isfinite(a).all() for a in got.values()), k
        assert np.abs(got["v"][[0, -1]]).max() == 0.0
        w = compact.quadrature_weights(fields[k][4])
        assert abs(w @ got["u1mean"] - 2.0) < 1e-12, (k, w @ got["u1mean"])
    for k in (0, len(cases) - 1):
        c = cases[k]
        v, om, U1, U3, y = fields[k]
        single = Channel(c.n1, c.n2, c.n3, c.lx, c.lz, c.re_b, y=y)
        _same_radix(single, ens.channels[k])
        single.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        single.step(dts[k], 50)
        ref = single.get_fields("v", "omega2")
        got = ens.channels[k].get_fields("v", "omega2")
        for n in ref:
            assert torch.equal(got[n], ref[n]), (k, n)
        single.close()
    ens.close()


@gpu
def test_ens_set_state_index_checked():
    """chn_ens_set_state sets channel i like chn_set_state on its context and
    rejects an index outside the ensemble without touching any channel."""
    from paper_1808_06461_amd import chn
    from paper_1808_06461_amd.chn import Ensemble
    c = SPECS[0]
    v, om, U1, U3, y = synth.turbulent_field(c)
    ens = Ensemble([_spec(c, y)], precision="fp64")
    try:
        ch = ens.channels[0]
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        got = ch.get_fields("v")["v"].cpu().numpy()
        assert rel(got, v) < 1e-15
        keep = [t.to("cuda") for t in (torch.from_numpy(v), torch.from_numpy(om),
                                       torch.from_numpy(U1), torch.from_numpy(U3))]
        ptrs = [chn._ptr(t) for t in keep]
        for bad in (-1, 1):
            assert ens.L.chn_ens_set_state(ens.ens, bad, *ptrs) == 1  # CHN_EINVAL
        assert b"out of range" in ens.L.chn_ens_last_error(ens.ens)
    finally:
        ens.close()


@gpu
def test_ensemble_channels_keep_their_radix_sets():
    """chn_ens_create gives a channel the composite radices where they take
    fewer passes (48 = 8 x 6, 72 = 9 x 8, 96 = 12 x 8); the batched tables are
    built with them, so another radix set on a channel is refused
    (CHN_EUNSUPPORTED) and the autotuner keeps the channel's set."""
    from paper_1808_06461_amd import ChnError
    from paper_1808_06461_amd.chn import Ensemble
    c = SPECS[4]  # 48 x 25 x 16: x lines of 72 points, z lines of 24
    v, om, U1, U3, y = synth.turbulent_field(c)
    ens = Ensemble([_spec(c, y)], precision="mixed")
    try:
        ch = ens.channels[0]
        ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
        p = ch.plan()
        assert p["radix_set"] & 1, p  # 72 = 9 x 8 (two passes) against 8, 3, 3
        with pytest.raises(ChnError, match="CHN_EUNSUPPORTED"):
            ch.set_plan(p["x_rows"], p["z_lines"], p["y_chunk"], p["fixed_radix"], p["z_pipeline"], 0)
        assert ch.plan() == p
        assert ch.autotune(reps=1)["radix_set"] == p["radix_set"]
        ens.step([c.dt], 2)
        f = ch.get_fields("v")["v"].cpu().numpy()
        assert np.isfinite(f).all()
    finally:
        ens.close()
