"""On-the-fly statistics (chn_accumulate_statistics) against the oracle.

The running sums of the two-dimensional spectra |u_i|^2 (mean mode
excluded) and of the mean profiles, for a new state (velocities recovered
by the library) and after one RK3 step (velocities from the fused recovery
of the pencil kernel), on the 64 x 65 x 64 channel.  Bounds: float64 1e-13
for the new state, 1e-10 after the step (the one-step trajectory parity);
mixed 5e-7 (the fields are float32 on that path).  Mean profiles: exact for
the new state; after the step 1e-12 (float64) and 1e-9 (mixed, whose mean
forcing comes from float32 products).
"""
import numpy as np
import pytest

import synth
from oracle import kmm, lowstorage

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_statistics_against_oracle(precision):
    from paper_1808_06461_amd import Channel, ChnError
    c = synth.CASES["c1"]
    v, om, U1, U3, y = synth.turbulent_field(c)
    S = kmm.Setup(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, nu=1 / c.re_b, dt=c.dt, mass_flux=c.mass_flux, y=y)
    st = kmm.make_state(S, v, om, U1, U3)
    u1, u2, u3, *_ = kmm.recover(S, st)
    E0 = lowstorage.spectra(u1, u2, u3)
    M0 = np.stack([st.U1, st.U3])
    st, _ = kmm.step(S, st, 1)
    u1, u2, u3, *_ = kmm.recover(S, st)
    E1 = lowstorage.spectra(u1, u2, u3)
    M1 = np.stack([st.U1, st.U3])
    tol0, tol1, tolm = (1e-13, 1e-10, 1e-12) if precision == "fp64" else (5e-7, 5e-7, 1e-9)
    ch = Channel(c.n1, c.n2, c.n3, c.lx, c.lz, c.re_b, mass_flux=c.mass_flux, precision=precision, y=y)
    try:
        ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
        spec, mean = ch.accumulate_statistics()
        ch.accumulate_statistics(spec, mean)
        e_s, e_m = rel(spec.cpu().numpy(), 2 * E0), rel(mean.cpu().numpy(), 2 * M0)
        print(f"{precision} new state: spectra {e_s:.2e} means {e_m:.2e}")
        assert e_s < tol0 and e_m < 1e-15, (e_s, e_m)
        ch.step(c.dt, 1)
        spec.zero_()
        mean.zero_()
        ch.accumulate_statistics(spec, mean)
        got = spec.cpu().numpy()
        e_s, e_m = rel(got, E1), rel(mean.cpu().numpy(), M1)
        m_rms = lowstorage.rms_profiles(got)
        e_rms = rel(m_rms, lowstorage.rms_profiles(E1))
        print(f"{precision} after a step: spectra {e_s:.2e} means {e_m:.2e} rms {e_rms:.2e}")
        assert e_s < tol1 and e_rms < tol1 and e_m < tolm, (e_s, e_m, e_rms)
        assert np.all(got[:, :, 0, 0] == 0)
        with pytest.raises(ChnError, match="CHN_EINVAL"):
            ch.L.chn_accumulate_statistics and ch._check(ch.L.chn_accumulate_statistics(ch.ctx, None, None),
                                                        "chn_accumulate_statistics")
    finally:
        ch.close()
