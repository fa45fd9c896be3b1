"""Python binding of the C ABI in include/chn.h (argument marshalling only).

Device memory and the HIP stream come from PyTorch; every computation runs in
the library's HIP kernels.  The library must be built (``build.py``); there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchn.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "chn.h")

FP64, MIXED = 0, 1
F_V, F_OMEGA2, F_CHI, F_U1, F_U3, F_OMEGA1, F_OMEGA3, F_U1MEAN, F_U3MEAN = (1 << k for k in range(9))
FIELD_BITS = {"v": F_V, "omega2": F_OMEGA2, "chi": F_CHI, "u1": F_U1, "u3": F_U3,
              "omega1": F_OMEGA1, "omega3": F_OMEGA3, "u1mean": F_U1MEAN, "u3mean": F_U3MEAN}
STATUS = {0: "CHN_OK", 1: "CHN_EINVAL", 2: "CHN_ENOMEM", 3: "CHN_EDEVICE", 4: "CHN_ESTATE",
          5: "CHN_EUNSTABLE", 6: "CHN_EUNSUPPORTED"}


class Config(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32), ("lx", C.c_double),
                ("lz", C.c_double), ("re_b", C.c_double), ("mass_flux", C.c_double),
                ("precision", C.c_int32), ("y", C.POINTER(C.c_double)), ("stream", C.c_void_p),
                ("planes_only", C.c_int32), ("plane_chunk", C.c_int32)]


class Plan(C.Structure):
    _fields_ = [("x_rows", C.c_int32), ("z_lines", C.c_int32), ("y_chunk", C.c_int32),
                ("fixed_radix", C.c_int32), ("z_pipeline", C.c_int32), ("radix_set", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepInfo(C.Structure):
    _fields_ = [("f_mean", C.c_double), ("mass_flux", C.c_double), ("cfl_max", C.c_double),
                ("utau_lo", C.c_double), ("utau_hi", C.c_double), ("max_abs_div", C.c_double),
                ("ms_phase", C.c_float * 5), ("fail_step", C.c_int32), ("fail_substep", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["ms_phase"] = list(self.ms_phase)
        return d


_lib = None


def lib():
    """Loads libchn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1808_06461_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.chn_workspace_bytes.argtypes = [C.POINTER(Config)]
        L.chn_workspace_bytes.restype = C.c_size_t
        L.chn_create.argtypes = [C.POINTER(Config), P, C.c_size_t, C.POINTER(P)]
        L.chn_destroy.argtypes = [P]
        L.chn_set_state.argtypes = [P, P, P, P, P]
        L.chn_step_rk3.argtypes = [P, C.c_double, C.c_int32, C.POINTER(StepInfo)]
        L.chn_step_graph_enable.argtypes = [P, C.c_int32]
        L.chn_get_fields.argtypes = [P, C.c_uint32, C.POINTER(P)]
        L.chn_nonlinear.argtypes = [P, C.POINTER(P), C.POINTER(P)]
        L.chn_filter_and_stress.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P]
        L.chn_filtered_enstrophy.argtypes = [P, C.c_int32, C.c_int32, P]
        L.chn_accumulate_statistics.argtypes = [P, P, P]
        L.chn_filtered_pressure.argtypes = [P, C.c_int32, C.c_int32, P, P, P]
        L.chn_get_operators.argtypes = [P, P, P, P, P, P]
        L.chn_get_mesh.argtypes = [P, P]
        L.chn_get_plan.argtypes = [P, C.POINTER(Plan)]
        L.chn_plane_products.argtypes = [P, C.POINTER(P), C.POINTER(P)]
        L.chn_plane_products_static.argtypes = [P, C.POINTER(P), C.POINTER(P)]
        L.chn_set_plan.argtypes = [P, C.POINTER(Plan)]
        L.chn_autotune.argtypes = [P, C.c_int32, C.POINTER(Plan)]
        L.chn_timing_enable.argtypes = [P, C.c_int32]
        L.chn_timing_read.argtypes = [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.chn_ens_workspace_bytes.argtypes = [C.c_int32, C.POINTER(Config)]
        L.chn_ens_workspace_bytes.restype = C.c_size_t
        L.chn_ens_create.argtypes = [C.c_int32, C.POINTER(Config), P, C.c_size_t, C.POINTER(P)]
        L.chn_ens_destroy.argtypes = [P]
        L.chn_ens_context.argtypes = [P, C.c_int32]
        L.chn_ens_context.restype = P
        L.chn_ens_step.argtypes = [P, C.POINTER(C.c_double), C.c_int32]
        L.chn_ens_set_state.argtypes = [P, C.c_int32, P, P, P, P]
        L.chn_ens_last_error.argtypes = [P]
        L.chn_ens_last_error.restype = C.c_char_p
        L.chn_last_error.argtypes = [P]
        L.chn_last_error.restype = C.c_char_p
        D = C.POINTER(C.c_double)
        L.chn_optimise_mesh.argtypes = [D, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, D, D, D,
                                        C.POINTER(C.c_int)]
        for name in ("chn_create", "chn_destroy", "chn_set_state", "chn_step_rk3", "chn_get_fields",
                     "chn_nonlinear", "chn_filter_and_stress", "chn_filtered_enstrophy", "chn_accumulate_statistics",
                     "chn_filtered_pressure",
                     "chn_get_operators", "chn_get_mesh",
                     "chn_timing_enable", "chn_timing_read", "chn_ens_create", "chn_ens_destroy", "chn_ens_step",
                     "chn_get_plan", "chn_set_plan", "chn_autotune", "chn_plane_products",
                     "chn_plane_products_static",
                     "chn_optimise_mesh", "chn_ens_set_state"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def header_symbols():
    """Names of the functions declared in include/chn.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(chn_\w+)\s*\(", text, re.M)))


def optimise_mesh(y_ref, m=20, kstar=1e10, penalty=1e-3, max_iter=60):
    """Near-wall mesh optimisation (``chn_optimise_mesh``, a host routine).

    Returns (y_opt, err_ref, err_opt, iterations); raises ChnError on a
    non-OK status."""
    import numpy as np
    y_ref = np.ascontiguousarray(y_ref, dtype=np.float64)
    n2 = len(y_ref)
    y_out = np.empty(n2)
    e0, e1, it = C.c_double(), C.c_double(), C.c_int()
    D = C.POINTER(C.c_double)
    st = lib().chn_optimise_mesh(y_ref.ctypes.data_as(D), n2, int(m), float(kstar), float(penalty),
                                 int(max_iter), y_out.ctypes.data_as(D), C.byref(e0), C.byref(e1),
                                 C.byref(it))
    if st != 0:
        raise ChnError(f"chn_optimise_mesh: {STATUS.get(st, st)}")
    return y_out, e0.value, e1.value, it.value


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class ChnError(RuntimeError):
    pass


class Channel:
    """One channel context on one GPU stream (see include/chn.h)."""

    def __init__(self, n1, n2, n3, lx, lz, re_b, mass_flux=2.0, precision="fp64", y=None,
                 device="cuda:0", planes_only=False, plane_chunk=0):
        self.L = lib()
        self.device = torch.device(device)
        self.n1, self.n2, self.n3 = n1, n2, n3
        self.n1h = n1 // 2
        self.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        self._y = None
        yp = C.POINTER(C.c_double)()
        if y is not None:
            self._y = (C.c_double * n2)(*[float(v) for v in y])
            yp = C.cast(self._y, C.POINTER(C.c_double))
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        self.cfg = Config(n1, n2, n3, lx, lz, re_b, mass_flux, self.precision, yp,
                          C.c_void_p(self.stream.cuda_stream), int(bool(planes_only)), int(plane_chunk))
        nbytes = self.L.chn_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise ChnError("invalid channel configuration")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.ctx = C.c_void_p()
        s = self.L.chn_create(C.byref(self.cfg), C.c_void_p(base + off), nbytes, C.byref(self.ctx))
        if s != 0:
            raise ChnError(f"chn_create: {STATUS.get(s, s)}: {self.L.chn_last_error(None).decode()}")

    # -- helpers
    def _check(self, s, what):
        if s != 0:
            raise ChnError(f"{what}: {STATUS.get(s, s)}: {self.L.chn_last_error(self.ctx).decode()}")

    def spectral_empty(self):
        return torch.empty((self.n2, self.n1h, self.n3), dtype=torch.complex128, device=self.device)

    def _dev(self, t, dtype):
        t = torch.as_tensor(t).to(device=self.device, dtype=dtype)
        return t.contiguous()

    # -- C ABI
    def set_state(self, v, omega2, u1mean, u3mean):
        self._keep = [self._dev(v, torch.complex128), self._dev(omega2, torch.complex128),
                      self._dev(u1mean, torch.float64), self._dev(u3mean, torch.float64)]
        self._check(self.L.chn_set_state(self.ctx, *[_ptr(t) for t in self._keep]), "chn_set_state")

    def step_graph(self, enable=True):
        """Replay steady steps from a captured graph (default) or launch every kernel."""
        self._check(self.L.chn_step_graph_enable(self.ctx, 1 if enable else 0), "chn_step_graph_enable")

    def step(self, dt, nsteps=1, info=False):
        si = StepInfo()
        self._check(self.L.chn_step_rk3(self.ctx, float(dt), int(nsteps), C.byref(si) if info else None),
                    "chn_step_rk3")
        if info:
            return si.as_dict()
        return None

    def step_status(self, dt, nsteps=1):
        """chn_step_rk3 with a step record; returns (status name, record, message) without raising."""
        si = StepInfo()
        s = self.L.chn_step_rk3(self.ctx, float(dt), int(nsteps), C.byref(si))
        msg = self.L.chn_last_error(self.ctx).decode() if s else ""
        return STATUS.get(s, s), si.as_dict(), msg

    def get_fields(self, *names):
        mask = 0
        for n in names:
            mask |= FIELD_BITS[n]
        outs = {}
        ptrs = []
        for n, bit in FIELD_BITS.items():
            if mask & bit:
                t = (torch.empty(self.n2, dtype=torch.float64, device=self.device) if n.endswith("mean")
                     else self.spectral_empty())
                outs[n] = t
                ptrs.append(t.data_ptr())
        arr = (C.c_void_p * max(1, len(ptrs)))(*ptrs)
        self._check(self.L.chn_get_fields(self.ctx, mask, arr), "chn_get_fields")
        return outs

    def nonlinear(self, fields):
        ins = [self._dev(f, torch.complex128) for f in fields]
        outs = [self.spectral_empty() for _ in range(3)]
        a = (C.c_void_p * 6)(*[t.data_ptr() for t in ins])
        b = (C.c_void_p * 3)(*[t.data_ptr() for t in outs])
        self._check(self.L.chn_nonlinear(self.ctx, a, b), "chn_nonlinear")
        return outs

    def plane_products(self, fields, out=None):
        """H1, H2, H3 from (u1, u2, u3, omega1, omega2 or None, omega3), device tensors in the
        transform precision (complex64 for mixed, complex128 for fp64), [n2][n1/2][n3]."""
        dt = torch.complex64 if self.precision == MIXED else torch.complex128
        for f in fields:
            if f is not None and (f.dtype != dt or not f.is_contiguous() or f.device != self.device
                                  or tuple(f.shape) != (self.n2, self.n1h, self.n3)):
                raise ChnError(f"plane_products needs contiguous {dt} [{self.n2}, {self.n1h}, {self.n3}] on {self.device}")
        if out is None:
            out = [torch.empty((self.n2, self.n1h, self.n3), dtype=dt, device=self.device) for _ in range(3)]
        a = (C.c_void_p * 6)(*[None if f is None else f.data_ptr() for f in fields])
        b = (C.c_void_p * 3)(*[t.data_ptr() for t in out])
        self._check(self.L.chn_plane_products(self.ctx, a, b), "chn_plane_products")
        return out

    def plane_products_static(self, fields, out):
        """chn_plane_products_static: as plane_products, with the transform
        intermediate in the library's static device array; `out` must be given
        (three tensors as plane_products returns), so that nothing is allocated."""
        dt = torch.complex64 if self.precision == MIXED else torch.complex128
        for f in list(fields) + list(out):
            if f is not None and (f.dtype != dt or not f.is_contiguous() or f.device != self.device
                                  or tuple(f.shape) != (self.n2, self.n1h, self.n3)):
                raise ChnError(f"plane_products_static needs contiguous {dt} [{self.n2}, {self.n1h}, {self.n3}] "
                               f"on {self.device}")
        a = (C.c_void_p * 6)(*[None if f is None else f.data_ptr() for f in fields])
        b = (C.c_void_p * 3)(*[t.data_ptr() for t in out])
        self._check(self.L.chn_plane_products_static(self.ctx, a, b), "chn_plane_products_static")
        return out

    def filter_and_stress(self, kcx, kcz, q1, q3, with_tau=True):
        nk = (self.n2, kcx + 1, 2 * kcz + 1)
        ub = torch.empty((3,) + nk, dtype=torch.complex128, device=self.device)
        uu = torch.empty((6,) + nk, dtype=torch.complex128, device=self.device)
        tau = torch.empty((6, self.n2, q3, q1), dtype=torch.float64, device=self.device) if with_tau else None
        self._check(self.L.chn_filter_and_stress(self.ctx, kcx, kcz, q1, q3, _ptr(ub), _ptr(uu), _ptr(tau)),
                    "chn_filter_and_stress")
        return ub, uu, tau

    def filtered_enstrophy(self, kcx, kcz):
        """F(omega_i omega_i) on 0 <= kx <= kcx, |kz| <= kcz: complex128 [n2][kcx+1][2kcz+1]."""
        out = torch.empty((self.n2, kcx + 1, 2 * kcz + 1), dtype=torch.complex128, device=self.device)
        self._check(self.L.chn_filtered_enstrophy(self.ctx, kcx, kcz, _ptr(out)), "chn_filtered_enstrophy")
        return out

    def filtered_pressure(self, kcx, kcz, uubar, ubar):
        """Filtered pressure [n2][kcx+1][2kcz+1] (complex128) from the outputs of filter_and_stress."""
        nk = (self.n2, kcx + 1, 2 * kcz + 1)
        for t, lead in ((uubar, 6), (ubar, 3)):
            if (t.dtype != torch.complex128 or tuple(t.shape) != (lead,) + nk or not t.is_contiguous()
                    or t.device != self.device):
                raise ValueError("uubar / ubar must be contiguous complex128 device tensors from filter_and_stress")
        out = torch.empty(nk, dtype=torch.complex128, device=self.device)
        self._check(self.L.chn_filtered_pressure(self.ctx, kcx, kcz, _ptr(uubar), _ptr(ubar), _ptr(out)),
                    "chn_filtered_pressure")
        return out

    def accumulate_statistics(self, spec=None, mean=None):
        """Adds |u_i|^2 per mode (mean mode excluded) to spec [3][n2][n1/2][n3] and U1, U3
        to mean [2][n2] (float64 device tensors, zeroed here when not given)."""
        if spec is None:
            spec = torch.zeros((3, self.n2, self.n1h, self.n3), dtype=torch.float64, device=self.device)
        if mean is None:
            mean = torch.zeros((2, self.n2), dtype=torch.float64, device=self.device)
        self._check(self.L.chn_accumulate_statistics(self.ctx, _ptr(spec), _ptr(mean)), "chn_accumulate_statistics")
        return spec, mean

    def plan(self):
        p = Plan()
        self._check(self.L.chn_get_plan(self.ctx, C.byref(p)), "chn_get_plan")
        return p.as_dict()

    def set_plan(self, x_rows, z_lines, y_chunk=None, fixed_radix=0, z_pipeline=0, radix_set=0):
        p = Plan(int(x_rows), int(z_lines), int(self.n2 if y_chunk is None else y_chunk), int(fixed_radix),
                 int(z_pipeline), int(radix_set))
        self._check(self.L.chn_set_plan(self.ctx, C.byref(p)), "chn_set_plan")

    def autotune(self, reps=3):
        p = Plan()
        self._check(self.L.chn_autotune(self.ctx, int(reps), C.byref(p)), "chn_autotune")
        return p.as_dict()

    def operators(self):
        import numpy as np
        arrs = [np.zeros((self.n2, 7)) for _ in range(4)] + [np.zeros(self.n2)]
        self._check(self.L.chn_get_operators(self.ctx, *[C.c_void_p(a.ctypes.data) for a in arrs]),
                    "chn_get_operators")
        return arrs

    def mesh(self):
        """The context's wall-normal nodes (numpy float64[n2])."""
        import numpy as np
        y = np.zeros(self.n2)
        self._check(self.L.chn_get_mesh(self.ctx, C.c_void_p(y.ctypes.data)), "chn_get_mesh")
        return y

    KERNELS = ("recover", "zinv", "xpass", "zfwd", "advance", "filter")

    def timing(self, enable=True):
        self._check(self.L.chn_timing_enable(self.ctx, 1 if enable else 0), "chn_timing_enable")

    def timing_read(self):
        """{kernel kind: (total ms, launches)} since timing() was enabled."""
        out = {}
        for k, name in enumerate(self.KERNELS):
            ms, n = C.c_double(), C.c_int32()
            self._check(self.L.chn_timing_read(self.ctx, k, C.byref(ms), C.byref(n)), "chn_timing_read")
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if getattr(self, "ctx", None):
            self.L.chn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _EnsChannel(Channel):
    """A channel context owned by an Ensemble (same methods as Channel)."""

    def __init__(self, ens, i, cfg):
        self.L = ens.L
        self.device = ens.device
        self.n1, self.n2, self.n3 = cfg.n1, cfg.n2, cfg.n3
        self.n1h = cfg.n1 // 2
        self.ctx = C.c_void_p(self.L.chn_ens_context(ens.ens, i))
        self._owner = ens
        self._i = i

    def set_state(self, v, omega2, u1mean, u3mean):
        self._keep = [self._dev(v, torch.complex128), self._dev(omega2, torch.complex128),
                      self._dev(u1mean, torch.float64), self._dev(u3mean, torch.float64)]
        s = self.L.chn_ens_set_state(self._owner.ens, self._i, *[_ptr(t) for t in self._keep])
        if s != 0:
            raise ChnError(f"chn_ens_set_state: {STATUS.get(s, s)}: "
                           f"{self.L.chn_ens_last_error(self._owner.ens).decode()}")

    def close(self):
        self.ctx = None


class Ensemble:
    """Uneven channels advanced together by batched launches in a HIP graph."""

    def __init__(self, specs, precision="fp64", device="cuda:0"):
        """specs: list of dicts with n1, n2, n3, lx, lz, re_b, mass_flux, y."""
        self.L = lib()
        self.device = torch.device(device)
        prec = {"fp64": FP64, "mixed": MIXED}[precision]
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
        self._ys = []
        cfgs = (Config * len(specs))()
        for k, sp in enumerate(specs):
            yarr = (C.c_double * sp["n2"])(*[float(v) for v in sp["y"]])
            self._ys.append(yarr)
            cfgs[k] = Config(sp["n1"], sp["n2"], sp["n3"], sp["lx"], sp["lz"], sp["re_b"], sp.get("mass_flux", 2.0),
                             prec, C.cast(yarr, C.POINTER(C.c_double)), C.c_void_p(stream.cuda_stream))
        self.cfgs = cfgs
        self.n = len(specs)
        nbytes = self.L.chn_ens_workspace_bytes(self.n, cfgs)
        if nbytes == 0:
            raise ChnError("invalid ensemble configuration")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.ens = C.c_void_p()
        s = self.L.chn_ens_create(self.n, cfgs, C.c_void_p(base + off), nbytes, C.byref(self.ens))
        if s != 0:
            raise ChnError(f"chn_ens_create: {STATUS.get(s, s)}: {self.L.chn_ens_last_error(None).decode()}")
        self.channels = [_EnsChannel(self, i, cfgs[i]) for i in range(self.n)]

    def step(self, dts, nsteps=1):
        arr = (C.c_double * self.n)(*[float(d) for d in dts])
        s = self.L.chn_ens_step(self.ens, arr, int(nsteps))
        if s != 0:
            raise ChnError(f"chn_ens_step: {STATUS.get(s, s)}: {self.L.chn_ens_last_error(self.ens).decode()}")

    def close(self):
        if getattr(self, "ens", None):
            for c in self.channels:
                c.close()
            self.L.chn_ens_destroy(self.ens)
            self.ens = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
