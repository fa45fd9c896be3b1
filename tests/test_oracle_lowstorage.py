"""Pins of the oracle's low-storage stage (Section 3.1: cut-off filter, F(u_i u_j), tau_ij).

* brute force: the filtered products equal the exact convolution of the
  Hermitian-complete mode sets, and tau at every Q-grid point equals the direct
  Fourier sums, with no FFT anywhere;
* a field band-limited to kc/2 has tau == 0 (the filter acts as the identity on
  its products);
* a single mode u1 = A cos(k x) with k > kc has tau_11 = A^2/2;
* tau is invariant to adding a plane-constant c(y) to the velocity;
* tau equals the Germano decomposition -(1-G)(ub_i ub_j) + G(ub_i u''_j +
  u''_i ub_j + u''_i u''_j), u'' = u - ub;
* the filtered enstrophy F(omega_i omega_i) equals the exact self-convolution
  of the three vorticity mode sets (no FFT), its (0,0) mode equals the plane
  mean sum_i sum_k |omega_i(k)|^2 (Parseval, a direct sum), and a pure mean
  shear W(y) gives W^2 in mode (0,0) and nothing else;
* the spectra summed with the Hermitian weights give the plane mean of the
  squared fluctuation computed pointwise from a direct synthesis (no FFT);
* the filter equals the physical-space convolution with the sharp cut-off
  kernel (inclusive cut-off, no FFT), and it commutes with the compact
  wall-normal D1 and D2 (it acts on x and z only);
* the retained modes of a product are exact on any grid with f > 2 h + kc
  per direction (h the highest stored wavenumber), the reading behind the
  smaller product grid of the library, and not on f = 2 h + kc.
"""
import numpy as np
import pytest

from oracle import brute, fourier, lowstorage

N1, N2, N3 = 16, 5, 12
LX, LZ = 2 * np.pi, np.pi


def _field(rng, n1=N1, n3=N3, kmax=None):
    uh = rng.standard_normal((N2, n1 // 2, n3)) + 1j * rng.standard_normal((N2, n1 // 2, n3))
    uh[:, :, n3 // 2] = 0
    for kz in range(1, n3 // 2):
        uh[:, 0, n3 - kz] = np.conj(uh[:, 0, kz])
    uh[:, 0, 0] = uh[:, 0, 0].real
    if kmax is not None:
        kx = np.arange(n1 // 2)[:, None]
        kz = np.abs(np.fft.fftfreq(n3, 1 / n3))[None, :]
        uh = uh * ((kx <= kmax) & (kz <= kmax))[None]
    return uh


@pytest.mark.parametrize("kcx,kcz", [(2, 2), (3, 2), (2, 3)])
def test_filtered_stress_brute_force(kcx, kcz):
    rng = np.random.default_rng(7)
    u = [_field(rng) for _ in range(3)]
    q1, q3 = 4 * kcx + 2, 4 * kcz + 2
    ub, uu, tau = lowstorage.filter_and_stress(*u, kcx, kcz, q1, q3)
    xq = np.arange(q1) * LX / q1
    zq = np.arange(q3) * LZ / q3
    slots = lowstorage.kc_slots(N3, kcz)
    kzs = [s if s < N3 // 2 else s - N3 for s in slots]
    for y in range(N2):
        modes = [brute.full_modes(ui[y]) for ui in u]
        for p, (i, j) in enumerate(lowstorage.PAIRS):
            prod = brute.product_modes(modes[i], modes[j])
            for kx in range(kcx + 1):
                for c, kz in enumerate(kzs):
                    ref = prod.get((kx, kz), 0)
                    assert abs(uu[p, y, kx, c] - ref) < 1e-13 * (1 + abs(ref)), (p, y, kx, kz)
        # tau by direct Fourier sums on the Q grid
        fm = [{k: v for k, v in m.items() if abs(k[0]) <= kcx and abs(k[1]) <= kcz} for m in modes]
        ubq = [brute.synth_points(m, LX, LZ, xq[None, :], zq[:, None]) for m in fm]
        for p, (i, j) in enumerate(lowstorage.PAIRS):
            prod = brute.product_modes(modes[i], modes[j])
            fp = {k: v for k, v in prod.items() if abs(k[0]) <= kcx and abs(k[1]) <= kcz}
            uuq = brute.synth_points(fp, LX, LZ, xq[None, :], zq[:, None])
            ref = uuq - ubq[i] * ubq[j]
            assert np.abs(tau[p, y] - ref).max() < 1e-13 * np.abs(uuq).max()


def test_band_limited_field_has_zero_stress():
    rng = np.random.default_rng(8)
    u = [_field(rng, kmax=1) for _ in range(3)]
    ub, _, tau = lowstorage.filter_and_stress(*u, 2, 2, 10, 10)
    scale = np.abs(lowstorage.synth_plane(ub, 10, 10)).max() ** 2
    assert np.abs(tau).max() < 1e-14 * scale


def test_single_subfilter_mode():
    """u1 = A cos(k x), k > kc: ub = 0, F(u1 u1) = A^2/2, tau_11 = A^2/2."""
    A, k = 0.7, 5
    u1 = np.zeros((N2, N1 // 2, N3), complex)
    u1[:, k, 0] = A / 2  # stored kx > 0 coefficient; the -kx conjugate is implicit
    z = np.zeros_like(u1)
    ub, uu, tau = lowstorage.filter_and_stress(u1, z, z, 2, 2, 10, 10)
    assert np.abs(ub).max() == 0
    assert np.abs(tau[0] - A * A / 2).max() < 1e-14
    assert np.abs(tau[1:]).max() < 1e-14


def test_plane_constant_invariance():
    rng = np.random.default_rng(9)
    u = [_field(rng) for _ in range(3)]
    _, _, tau = lowstorage.filter_and_stress(*u, 3, 2, 14, 10)
    shifted = [x.copy() for x in u]
    for i, c in enumerate((1.3, -0.4, 0.25)):
        shifted[i][:, 0, 0] += c * (1 + np.arange(N2))
    _, _, tau2 = lowstorage.filter_and_stress(*shifted, 3, 2, 14, 10)
    assert np.abs(tau2 - tau).max() < 1e-12 * np.abs(tau).max() * 10


def test_germano_decomposition():
    rng = np.random.default_rng(10)
    u = [_field(rng) for _ in range(3)]
    kcx, kcz, q1, q3 = 3, 2, 14, 10
    ub, uu, tau = lowstorage.filter_and_stress(*u, kcx, kcz, q1, q3)
    p1, p3 = fourier.padded_size(N1), fourier.padded_size(N3)
    full = [fourier.to_physical(x, p1, p3) for x in u]
    # ub padded back to the full mode set, and the sub-filter part
    ubf = []
    for x in u:
        y = np.zeros_like(x)
        y[:, : kcx + 1][..., lowstorage.kc_slots(N3, kcz)] = lowstorage.truncate(x, kcx, kcz)
        ubf.append(fourier.to_physical(y, p1, p3))
    upp = [f - g for f, g in zip(full, ubf)]

    def G(f):
        return lowstorage.synth_plane(lowstorage.truncate(fourier.to_spectral(f, N1, N3), kcx, kcz), q1, q3)

    ubq = lowstorage.synth_plane(ub, q1, q3)
    for p, (i, j) in enumerate(lowstorage.PAIRS):
        bb = ubf[i] * ubf[j]
        germ = -(ubq[i] * ubq[j] - G(bb)) + G(ubf[i] * upp[j] + upp[i] * ubf[j] + upp[i] * upp[j])
        assert np.abs(germ - tau[p]).max() < 1e-13 * np.abs(ubq[i] * ubq[j]).max()


@pytest.mark.parametrize("kcx,kcz", [(2, 2), (3, 4)])
def test_filtered_enstrophy_brute_force(kcx, kcz):
    rng = np.random.default_rng(11)
    w = [_field(rng) for _ in range(3)]
    ens = lowstorage.filtered_enstrophy(*w, kcx, kcz)
    slots = lowstorage.kc_slots(N3, kcz)
    kzs = [s if s < N3 // 2 else s - N3 for s in slots]
    for y in range(N2):
        modes = [brute.full_modes(wi[y]) for wi in w]
        prods = [brute.product_modes(m, m) for m in modes]
        for kx in range(kcx + 1):
            for c, kz in enumerate(kzs):
                ref = sum(p.get((kx, kz), 0) for p in prods)
                assert abs(ens[y, kx, c] - ref) < 1e-13 * (1 + abs(ref)), (y, kx, kz)


def test_filtered_enstrophy_parseval():
    rng = np.random.default_rng(12)
    w = [_field(rng) for _ in range(3)]
    ens = lowstorage.filtered_enstrophy(*w, 1, 1)
    for y in range(N2):
        ref = sum(sum(abs(c) ** 2 for c in brute.full_modes(wi[y]).values()) for wi in w)
        assert abs(ens[y, 0, 0] - ref) < 1e-13 * ref
        assert abs(ens[y, 0, 0].imag) < 1e-13 * ref


def test_filtered_enstrophy_of_a_mean_shear():
    W = 0.5 + np.arange(N2)
    z = np.zeros((N2, N1 // 2, N3), complex)
    w3 = z.copy()
    w3[:, 0, 0] = W
    ens = lowstorage.filtered_enstrophy(z, z, w3, 2, 2)
    assert np.abs(ens[:, 0, 0] - W ** 2).max() < 1e-13 * W.max() ** 2
    rest = ens.copy()
    rest[:, 0, 0] = 0
    assert np.abs(rest).max() < 1e-13 * W.max() ** 2


def test_spectra_parseval_against_direct_synthesis():
    rng = np.random.default_rng(13)
    u = [_field(rng) for _ in range(3)]
    E = lowstorage.spectra(*u)
    msq = lowstorage.rms_profiles(E)
    x = np.arange(N1)[None, :] * LX / N1
    z = np.arange(N3)[:, None] * LZ / N3
    for y in range(N2):
        for i in range(3):
            modes = {k: c for k, c in brute.full_modes(u[i][y]).items() if k != (0, 0)}
            f = brute.synth_points(modes, LX, LZ, x, z)
            ref = float(np.mean(f ** 2))
            assert abs(msq[i, y] - ref) < 1e-13 * ref, (i, y)
    assert np.all(E[:, :, 0, 0] == 0)


def test_filter_is_the_sharp_kernel_convolution():
    """Section 3.1's cut-off filter as a physical-space convolution, no FFT:
    F u(x_p, z_q) = (1/(N1 N3)) sum_{j,l} u(x_j, z_l) D_kcx(x_p - x_j) D_kcz(z_q - z_l)
    with D_K(t) = 1 + 2 sum_{k=1..K} cos(k t) (in units of the box wavenumber),
    against the oracle's truncation synthesised on the same grid."""
    rng = np.random.default_rng(71)
    uh = _field(rng)[2]
    kcx, kcz = 3, 2
    x = np.arange(N1) * LX / N1
    z = np.arange(N3) * LZ / N3
    X, Z = np.meshgrid(x, z)
    u = brute.synth_points(brute.full_modes(uh), LX, LZ, X, Z)          # [N3][N1]
    tx = 2 * np.pi / LX * (x[:, None] - x[None, :])
    tz = 2 * np.pi / LZ * (z[:, None] - z[None, :])
    Dx = 1 + 2 * sum(np.cos(k * tx) for k in range(1, kcx + 1))
    Dz = 1 + 2 * sum(np.cos(k * tz) for k in range(1, kcz + 1))
    Fu = Dz @ u @ Dx.T / (N1 * N3)
    got = lowstorage.synth_plane(lowstorage.truncate(uh[None], kcx, kcz), N1, N3)[0]
    np.testing.assert_allclose(got, Fu, rtol=0, atol=1e-13 * np.abs(Fu).max())


def test_filter_commutes_with_the_wall_normal_derivative():
    """The filter acts on x and z only, so it commutes with the compact D1 and
    D2 of the wall-normal direction (the property the a-posteriori filtered
    pressure rests on): F(D u) = D F(u) mode by mode."""
    import synth
    from oracle import kmm
    n2 = 17
    y = synth.mesh_tanh(n2)
    S = kmm.Setup(n1=N1, n2=n2, n3=N3, lx=LX, lz=LZ, nu=1e-3, dt=1e-3, mass_flux=0.0, y=y)
    rng = np.random.default_rng(72)
    uh = rng.standard_normal((n2, N1 // 2, N3)) + 1j * rng.standard_normal((n2, N1 // 2, N3))
    for d in (kmm.d1, kmm.d2):
        lhs = lowstorage.truncate(d(S, uh), 3, 2)
        rhs = d(S, lowstorage.truncate(uh, 3, 2))
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13 * np.abs(lhs).max())


@pytest.mark.parametrize("kcx,kcz", [(2, 2), (5, 3)])
def test_retained_product_modes_exact_above_2h_plus_kc(kcx, kcz):
    """Products formed on an f1 x f3 grid with the oracle's transforms (no
    padding rule): equal to the brute-force convolution on the retained set
    when f1 > 2 h1 + kcx and f3 > 2 h3 + kcz, aliased one point below."""
    rng = np.random.default_rng(11)
    a, b = _field(rng), _field(rng)
    h1, h3 = N1 // 2 - 1, N3 // 2 - 1
    slots = lowstorage.kc_slots(N3, kcz)
    kzs = [s if s < N3 // 2 else s - N3 for s in slots]

    def retained(f1, f3):
        fa, fb = fourier.to_physical(a, f1, f3), fourier.to_physical(b, f1, f3)
        # forward transform onto the full stored set of the f1 x f3 grid
        F = np.fft.rfft2(fa * fb) / (f1 * f3)
        return np.array([[[F[y, kz % f3, kx] for kz in kzs] for kx in range(kcx + 1)] for y in range(N2)])

    ref = np.zeros((N2, kcx + 1, len(kzs)), complex)
    for y in range(N2):
        prod = brute.product_modes(brute.full_modes(a[y]), brute.full_modes(b[y]))
        for kx in range(kcx + 1):
            for c, kz in enumerate(kzs):
                ref[y, kx, c] = prod.get((kx, kz), 0)
    scale = np.abs(ref).max()
    f1, f3 = 2 * h1 + kcx + 1, 2 * h3 + kcz + 1
    assert np.abs(retained(f1, f3) - ref).max() < 1e-13 * scale
    assert np.abs(retained(f1 + 3, f3 + 2) - ref).max() < 1e-13 * scale
    assert np.abs(retained(f1 - 1, f3) - ref).max() > 1e-3 * scale
    assert np.abs(retained(f1, f3 - 1) - ref).max() > 1e-3 * scale
