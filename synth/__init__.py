"""Seeded synthetic inputs for the channel RK3 path and for its FP64 oracle.

This module is the only code shared by the GPU path's tests/bench and the
oracle.  It generates *inputs* (a wall-normal mesh, spectral initial fields,
mean profiles, run parameters) and holds none of the method's arithmetic: no
compact finite differences, no Fourier transforms of the method, no time
stepping.  Wall-normal derivatives needed to size the perturbation energy are
taken analytically on the Chebyshev series the fields are built from.

Layout of every spectral field: complex128 array ``[n2][n1//2][n3]`` (y, kx,
kz), kx = 0..n1/2-1, kz in FFT slot order (slot n3/2 is the Nyquist slot and is
always zero).  Physical wavenumbers are a = 2*pi*kx/lx, b = 2*pi*kz/lz.

Random numbers come from ``numpy.random.Generator(PCG64(SeedSequence([180806461,
cfg, i])))``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from numpy.polynomial import chebyshev as C
from numpy.polynomial import legendre as L

SEED_ROOT = 180806461

# tanh stretching per wall-normal size.  The maximum-order seven-point compact
# scheme becomes singular for some local stretching ratios (its left-hand
# matrix loses rank, e.g. n2=65 with gamma=2, n2=33 with gamma=1.5); these
# values keep the Dirichlet-row Helmholtz matrices and A1 well conditioned
# (2-norm condition numbers of a few hundred and ~1e4) for each size used.
_GAMMA = {9: 0.75, 13: 0.75, 17: 0.75, 25: 0.75, 33: 1.0, 49: 1.25, 65: 1.5,
          97: 2.0, 129: 2.0, 193: 2.0, 385: 1.5, 1537: 2.0}


def rng(cfg: int, i: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg, i])))


def mesh_gamma(n2: int) -> float:
    return _GAMMA.get(n2, 2.0)


def mesh_tanh(n2: int, gamma: float | None = None) -> np.ndarray:
    """Wall-normal nodes y_j = tanh(g s_j)/tanh(g), s_j uniform on [-1, 1]."""
    g = mesh_gamma(n2) if gamma is None else gamma
    s = -1.0 + 2.0 * np.arange(n2) / (n2 - 1)
    y = np.tanh(g * s) / math.tanh(g)
    y[0], y[-1] = -1.0, 1.0
    # exact mirror symmetry
    y[n2 // 2:] = -y[: (n2 + 1) // 2][::-1]
    if n2 % 2 == 1:
        y[n2 // 2] = 0.0
    return y


def reichardt(y: np.ndarray, re_tau: float) -> np.ndarray:
    """Reichardt's mean profile in outer units, rescaled to bulk velocity 1."""
    kap = 0.41

    def uplus(yp):
        return np.log1p(kap * yp) / kap + 7.8 * (1 - np.exp(-yp / 11) - (yp / 11) * np.exp(-yp / 3))

    x, w = L.leggauss(256)
    d = (x + 1) / 2  # wall distance on [0, 1]
    ub = np.sum(w * uplus(d * re_tau)) / 2
    return uplus((1 - np.abs(y)) * re_tau) / ub


def poiseuille(y: np.ndarray) -> np.ndarray:
    return 1.5 * (1 - y * y)


def dean_re_b(re_tau: float) -> float:
    """Dean (1978) correlation Re_tau = 0.09 Re_b^0.88, inverted (Re_b on the half height)."""
    return 0.5 * (re_tau / 0.09) ** (1 / 0.88)


@dataclasses.dataclass
class Case:
    n1: int
    n2: int
    n3: int
    lx: float
    lz: float
    re_b: float
    dt: float
    mass_flux: float = 2.0
    amp: float = 0.1
    kmax: int | None = None       # |kx|,|kz| <= kmax (index units) carry the perturbation
    mean: str = "poiseuille"      # 'poiseuille' | 'reichardt' | 'zero'
    re_tau: float = 180.0
    spectrum: float = -8.0 / 3.0  # modal energy ~ k_h**spectrum
    cfg: int = 0


def wavenumbers(n1, n3, lx, lz):
    kx = np.arange(n1 // 2)
    kz = np.fft.fftfreq(n3, 1.0 / n3).astype(np.int64)
    kz[n3 // 2] = 0
    return kx, kz, 2 * np.pi * kx / lx, 2 * np.pi * kz / lz


def _leg(n=96):
    x, w = L.leggauss(n)
    return x, w


def turbulent_field(case: Case, seed_i: int = 0, y: np.ndarray | None = None):
    """Divergence-free random perturbation + mean profile.

    Per retained mode m != (0,0):
      v_m(y)  = (1-y^2)^2 * sum_{n<5} a_mn T_n(y)
      w2_m(y) = (1-y^2)   * sum_{n<5} b_mn T_n(y)
    with a, b complex standard normal, rescaled so each mode's kinetic energy
    is proportional to k_h**spectrum, then globally so that the volume RMS of
    |u'| equals ``case.amp``.  kx=0 modes are made Hermitian in kz.
    Returns (v, omega2, U1, U3, y) with v/omega2 complex [n2][n1/2][n3].
    ``y`` (n2 nodes) replaces the default tanh mesh; the profiles are the
    same functions of y, so only the sampling changes.
    """
    n1, n2, n3 = case.n1, case.n2, case.n3
    y = mesh_tanh(n2) if y is None else np.asarray(y, dtype=np.float64)
    assert y.shape == (n2,)
    kxi, kzi, a, b = wavenumbers(n1, n3, case.lx, case.lz)
    g = rng(case.cfg, seed_i)
    nk = n1 // 2
    A = g.standard_normal((nk, n3, 5)) + 1j * g.standard_normal((nk, n3, 5))
    B = g.standard_normal((nk, n3, 5)) + 1j * g.standard_normal((nk, n3, 5))
    # mask of carrying modes
    mask = np.ones((nk, n3), bool)
    mask[:, n3 // 2] = False
    mask[0, 0] = False
    if case.kmax is not None:
        mask &= (kxi[:, None] <= case.kmax) & (np.abs(kzi)[None, :] <= case.kmax)
    # kx = 0: keep kz > 0 only and mirror afterwards
    mask[0, n3 // 2:] = False
    # Chebyshev evaluation (analytic derivative for energy)
    T = np.stack([C.chebval(y, np.eye(5)[n]) for n in range(5)], 0)          # [5][n2]
    xq, wq = _leg(96)
    Tq = np.stack([C.chebval(xq, np.eye(5)[n]) for n in range(5)], 0)
    dTq = np.stack([C.chebval(xq, C.chebder(np.eye(5)[n])) for n in range(5)], 0)
    fv, dfv, fw = (1 - xq**2) ** 2, -4 * xq * (1 - xq**2), (1 - xq**2)
    k2 = a[:, None] ** 2 + b[None, :] ** 2
    kh = np.sqrt(np.where(mask, k2, 1.0))
    # energy of each mode (integral over y of |u|^2 summed over components, Hermitian weight)
    pv = np.einsum('ijn,nq->ijq', A, Tq)
    dpv = np.einsum('ijn,nq->ijq', A, dTq)
    vq = fv * pv
    dvq = dfv * pv + fv * dpv
    wqv = fw * np.einsum('ijn,nq->ijq', B, Tq)
    k2s = np.where(mask, k2, 1.0)[..., None]
    e = (np.abs(vq) ** 2 + (np.abs(dvq) ** 2 + np.abs(wqv) ** 2) / k2s) @ wq
    # every carrying mode stands for itself and its conjugate partner (kx=0: the
    # mirrored kz slot filled below; kx>0: the implicit -kx half)
    wt = 2.0
    target = kh ** case.spectrum
    scale = np.where(mask, np.sqrt(target / np.maximum(e, 1e-300)), 0.0)
    tot = np.sum(np.where(mask, target * wt, 0.0))  # sum over the Hermitian-complete set of int |u|^2 dy
    # volume mean square = tot / 2 (y-length 2)
    g_scale = case.amp / math.sqrt(tot / 2.0) if tot > 0 else 0.0
    scale = scale * g_scale
    v = np.einsum('ijn,ny->yij', A * scale[..., None], T) * ((1 - y**2) ** 2)[:, None, None]
    w2 = np.einsum('ijn,ny->yij', B * scale[..., None], T) * (1 - y**2)[:, None, None]
    # Hermitian completion of kx = 0
    for kz in range(1, n3 // 2):
        v[:, 0, n3 - kz] = np.conj(v[:, 0, kz])
        w2[:, 0, n3 - kz] = np.conj(w2[:, 0, kz])
    v[:, :, n3 // 2] = 0
    w2[:, :, n3 // 2] = 0
    v[:, 0, 0] = 0
    w2[:, 0, 0] = 0
    if case.mean == "poiseuille":
        U1 = poiseuille(y)
    elif case.mean == "reichardt":
        U1 = reichardt(y, case.re_tau)
    else:
        U1 = np.zeros(n2)
    U3 = np.zeros(n2)
    return v.astype(np.complex128), w2.astype(np.complex128), U1, U3, y


def random_spectral(shape, cfg: int, i: int, dtype=np.complex128):
    """Plain complex-Gaussian array (used for unit-level parity cases)."""
    g = rng(cfg, i)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(dtype)


# Workloads.  The time step of the 384x193x384 case corresponds to CFL 0.5 at
# t = 0 for its seeded field (padded-grid CFL max(|u1|/dx + |u2|/dy_j + |u3|/dz)).
CASES = {
    # small channel, Re_tau ~ 180, 10 RK3 steps at dt = 0.005
    "c1": Case(n1=64, n2=65, n3=64, lx=2 * np.pi, lz=np.pi, re_b=2800.0, dt=0.005,
               amp=0.1, kmax=8, mean="poiseuille", cfg=1),
    # Re_tau ~ 550, k^-5/3 spectrum, turbulent mean
    # dt = CFL 0.5 at t = 0, written by tests/golden/make_dt.py (oracle CFL)
    "c2": Case(n1=384, n2=193, n3=384, lx=2 * np.pi, lz=np.pi, re_b=10000.0, dt=0.004810960127275536,
               amp=0.1, kmax=None, mean="reichardt", re_tau=550.0, cfg=2),
    # low-storage stage input, Re_tau ~ 950
    "c5": Case(n1=1536, n2=385, n3=1152, lx=2 * np.pi, lz=np.pi, re_b=18863.0, dt=0.0,
               amp=0.1, kmax=None, mean="reichardt", re_tau=950.0, cfg=5),
}


def ensemble_cases(n=96, cfg=4):
    """Uneven minimal channels: n1 in {32,48,64}, n2 in {49,65,97}, n3 in {32,48},
    Re_tau ~ U[180, 400] (Re_b from Dean's correlation), box pi x 2 x pi/2,
    Reichardt mean + 0.1 RMS perturbations, each channel with its own seed."""
    g = rng(cfg, 0)
    out = []
    for i in range(n):
        n1 = int(g.choice([32, 48, 64]))
        n2 = int(g.choice([49, 65, 97]))
        n3 = int(g.choice([32, 48]))
        rt = float(g.uniform(180.0, 400.0))
        out.append(Case(n1=n1, n2=n2, n3=n3, lx=np.pi, lz=np.pi / 2, re_b=dean_re_b(rt), dt=0.0, amp=0.1,
                        mean="reichardt", re_tau=rt, cfg=1000 + i))
    return out


# One GPU's share of the Re_tau = 5300 channel (box 2pi x 2 x pi, 8192 x 1537 x 6144):
# a slab of 48 x-z planes for the transforms and products, and 1/128 of the
# (kx, kz) modes as full 1537-point wall-normal lines for the pencil phase.
C3_PLANES = dict(n1=8192, n3=6144, nplanes=48, lx=2 * np.pi, lz=np.pi, re_tau=5300.0, cfg=3)


def c3_amplitude(n1: int = 8192, n3: int = 6144) -> np.ndarray:
    """k_h^(-4/3) over [n1/2][n3] (index units, 1 at (0,0)), zero Nyquist slot; float32."""
    kx = np.arange(n1 // 2, dtype=np.float32)[:, None]
    s = np.arange(n3)
    kz = np.where(s < n3 // 2, s, s - n3).astype(np.float32)[None, :]
    kh = np.sqrt(kx * kx + kz * kz)
    kh[0, 0] = 1.0
    amp = kh ** np.float32(-4.0 / 3.0)
    amp[:, n3 // 2] = 0.0
    return amp


def c3_plane_fields(plane: int, n1: int = 8192, n3: int = 6144, cfg: int = 3):
    """Six spectral fields (u1, u2, u3, omega1, omega2, omega3) of one x-z plane,
    complex64 [n1/2][n3]: complex Gaussian coefficients times k_h^(-4/3)
    (k_h in index units, k_h = 1 for the (0,0) mode), Hermitian kx = 0 line,
    zero Nyquist slot, each field scaled to a physical RMS of 0.1."""
    n1h = n1 // 2
    amp = c3_amplitude(n1, n3)
    out = []
    for f in range(6):
        g = rng(cfg, 100000 + plane * 8 + f)
        c = g.standard_normal((n1h, n3), dtype=np.float32) + 1j * g.standard_normal((n1h, n3), dtype=np.float32)
        c = (c * amp).astype(np.complex64)
        # Hermitian kx = 0 line: c(0, -kz) = conj c(0, kz), c(0, 0) real
        pos = np.arange(1, n3 // 2)
        c[0, n3 - pos] = np.conj(c[0, pos])
        c[0, 0] = c[0, 0].real
        # physical mean square = |c00|^2 + 2 sum_{kx>0}|c|^2 + sum_{kx=0, kz!=0}|c|^2
        ms = float(np.sum(np.abs(c[1:]) ** 2) * 2 + np.sum(np.abs(c[0]) ** 2))
        out.append((c * np.float32(0.1 / math.sqrt(ms))).astype(np.complex64))
    return out


def c3_pencil_case() -> Case:
    """The pencil share as a channel of the same wall-normal size: 256 x 768 =
    196608 Fourier modes (1/128 of the 4096 x 6144 modes) on 1537 nodes."""
    rt = C3_PLANES["re_tau"]
    return Case(n1=512, n2=1537, n3=768, lx=2 * np.pi, lz=np.pi, re_b=dean_re_b(rt), dt=0.0, amp=0.1,
                kmax=None, mean="reichardt", re_tau=rt, cfg=6)


def c3_fill_slab(fields, planes_from_numpy=(), cfg: int = 3, device="cuda"):
    """Fills six device tensors [nplanes][n1/2][n3] (complex64) with the slab's
    spectra: planes listed in planes_from_numpy come from c3_plane_fields (the
    oracle's inputs); the others are drawn on the device from a seeded torch
    generator with the same amplitude law (each field scaled to RMS 0.1)."""
    import torch
    P, n1h, n3 = fields[0].shape
    amp = torch.from_numpy(c3_amplitude(2 * n1h, n3)).to(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_ROOT + cfg)
    pos = torch.arange(1, n3 // 2, device=device)
    for p in range(P):
        if p in planes_from_numpy:
            for f, c in enumerate(c3_plane_fields(p, 2 * n1h, n3, cfg)):
                fields[f][p].copy_(torch.from_numpy(c))
            continue
        for f in range(6):
            c = torch.complex(torch.randn(n1h, n3, generator=gen, device=device),
                              torch.randn(n1h, n3, generator=gen, device=device)) * amp
            c[0, n3 - pos] = torch.conj(c[0, pos])
            c[0, 0] = complex(float(c[0, 0].real))
            ms = float((c[1:].abs() ** 2).sum() * 2 + (c[0].abs() ** 2).sum())
            fields[f][p].copy_(c * (0.1 / math.sqrt(ms)))
