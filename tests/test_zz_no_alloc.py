"""chn_plane_products_static, the entry point for callers that cannot
allocate, against chn_plane_products on the same inputs: two calls in a row,
the second on a smaller context; the first context's intermediate needs
several chunks of the static array; a plane larger than the array is refused.
The two entry points run the same kernels plane by plane, so the products
agree bit for bit."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def _fields(n1, n2, n3, precision, seed):
    """Six seeded spectral fields [n2][n1/2][n3], Hermitian kx = 0 lines, zero Nyquist slot."""
    dt = torch.complex64 if precision == "mixed" else torch.complex128
    out = []
    for f in range(6):
        a = synth.random_spectral((n2, n1 // 2, n3), 990, 10 * seed + f) * 0.1
        a[:, :, n3 // 2] = 0
        for kz in range(1, n3 // 2):
            a[:, 0, n3 - kz] = np.conj(a[:, 0, kz])
        a[:, 0, 0] = a[:, 0, 0].real
        out.append(torch.from_numpy(a).to("cuda", dt).contiguous())
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_scratch_products_match_the_workspace_ones(precision):
    from paper_1808_06461_amd import Channel
    for k, (n1, n2, n3) in enumerate(((384, 40, 384), (24, 9, 24))):
        print(f"[no-alloc] {precision} {n1} x {n2} x {n3}", flush=True)
        ch = Channel(n1, n2, n3, 2 * np.pi, np.pi, 1000.0, precision=precision, planes_only=True, plane_chunk=n2)
        try:
            fields = _fields(n1, n2, n3, precision, k)
            ref = ch.plane_products(fields)
            out = [torch.full_like(r, float("nan")) for r in ref]  # allocated before the call
            ch.plane_products_static(fields, out)
            torch.cuda.synchronize()
            for f in range(3):
                assert torch.equal(out[f], ref[f]), (precision, n1, n2, n3, f)
                scale = float(ref[f].abs().max())
                assert scale > 0 and bool(torch.isfinite(torch.view_as_real(out[f])).all())
        finally:
            ch.close()


@pytest.mark.gpu
def test_static_scratch_refuses_a_plane_larger_than_the_array():
    from paper_1808_06461_amd import Channel, ChnError
    n1 = n3 = 2048  # one plane of the float32 intermediate: 6 x 3072 x 1024 x 8 B = 151 MB
    n2 = 9
    ch = Channel(n1, n2, n3, 2 * np.pi, np.pi, 1000.0, precision="mixed", planes_only=True, plane_chunk=1)
    try:
        f = [torch.zeros((n2, n1 // 2, n3), dtype=torch.complex64, device="cuda") for _ in range(6)]
        out = [torch.zeros_like(f[0]) for _ in range(3)]
        with pytest.raises(ChnError, match="CHN_EUNSUPPORTED.*static scratch"):
            ch.plane_products_static(f, out)
    finally:
        ch.close()
