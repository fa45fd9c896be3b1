"""Throughput of the channel RK3 step on one MI355X: grid points x RK3 steps per second.

Workload: the 384 x 193 x 384 channel at Re_tau ~ 550 (Re_b = 10000, box
2pi x 2 x pi, dt from CFL 0.5 at t = 0), seeded k^-5/3 divergence-free
perturbations on a turbulent mean profile.  Both precisions run from the same
initial state: the mixed path (FP32 transforms and products, FP64 solves,
mean modes and mass flux) gives `value`; the FP64 path and the relative
difference between the two after warmup + steps are reported beside it.

Prints one JSON line (rank 0).  Only single-GPU runs are supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-points x RK3 steps/sec, mixed-prec vs FP64 GPU at stated rel. error"
UNIT = "grid-points*RK3-steps/s"
HBM_PEAK_GBS = 8000.0
FIXED_PLAN = None  # (x_rows, z_lines, y_chunk[, fixed_radix[, z_pipeline[, radix_set]]]) from --plan; None: autotune


def algorithmic_bytes(kind, n1, n2, n3, elem):
    """Bytes one launch of a kernel kind must move (inputs read once, outputs written once)."""
    n1h, p3 = n1 // 2, 3 * n3 // 2
    NP = n2 * n1h * n3          # mode-points per spectral field
    IP = n2 * p3 * n1h          # points per field of the z-padded intermediate
    return {
        "recover": (32 + 5 * elem) * NP,          # v, omega2 (fp64) -> u1 u2 u3 o1 o3
        "zinv": 5 * elem * NP + 6 * elem * IP,    # 5 spectral fields -> 6 padded lines
        "xpass": 6 * elem * IP + 3 * elem * IP,   # 6 fields in, H1 H2 H3 out
        "zfwd": 3 * elem * IP + 3 * elem * NP,    # 3 padded fields -> 3 spectral
        # the pencil phase's compulsory bytes: H in, chi, omega2 and two
        # histories in and out (float64 state), the next sub-step's five
        # velocity/vorticity fields out (192 B per mode-point mixed, 256 float64)
        "advance": (3 * elem + 64 + 64 + 5 * elem) * NP,
    }[kind]


# float64 store of v, which the state keeps besides chi and omega2 (it is
# recomputable from chi, so it is not in the compulsory count above)
V_STORE_BYTES = 16

# Nominal floating-point operations per sub-step (for the FLOP/s figure):
# 2.5 n log2 n per real two-dimensional transform of n points (six inverse,
# three forward per plane), 20 per padded point for the products, the CFL
# terms and the plane sums, and 560 per mode-point for the pencil sweeps (the
# compact derivatives, the right-hand sides, the factorisations and the
# substitutions of the six sweeps, counted without the lane pair's duplicate
# factorisation).
PENCIL_FLOPS_PER_MODE_POINT = 560


def nominal_flops_per_substep(n1, n2, n3):
    import math
    p1, p3 = 3 * n1 // 2, 3 * n3 // 2
    n = p1 * p3
    fft = 9 * n2 * 2.5 * n * math.log2(n)
    return fft + 20 * n2 * n + PENCIL_FLOPS_PER_MODE_POINT * n2 * (n1 // 2) * n3


# Source files that make up each kernel kind; the HBM traffic measured with
# rocprofv3 counters (profiles/traffic_<kind>_channel_384x193x384.md) is used
# only while these files are unchanged since the measurement.
KERNEL_SOURCES = {
    "advance": ["pencil.hip", "kernels.hpp", "common.hpp", "host.hpp"],
    "zinv": ["plane.hpp", "plane_zinv_f.hip", "fft.hpp", "kernels.hpp", "common.hpp", "host.hpp"],
    "xpass": ["plane.hpp", "plane_xpass_f.hip", "fft.hpp", "kernels.hpp", "common.hpp", "host.hpp"],
    "zfwd": ["plane.hpp", "plane_zfwd_f.hip", "fft.hpp", "kernels.hpp", "common.hpp", "host.hpp"],
}


def kernel_source_hash(kind):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kind, []):
        with open(os.path.join(ROOT, "paper_1808_06461_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kind, precision="mixed"):
    """HBM bytes per launch from the committed counter summary, or None if the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kind}_channel_384x193x384.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash(kind) or vals.get("precision") != precision:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_path(case, v, om, U1, U3, y, precision, steps, warmup):
    import torch

    from paper_1808_06461_amd import Channel
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, mass_flux=case.mass_flux,
                 precision=precision, y=y)
    ch.set_state(torch.from_numpy(v), torch.from_numpy(om), torch.from_numpy(U1), torch.from_numpy(U3))
    if FIXED_PLAN:
        ch.set_plan(*FIXED_PLAN)
        plan = ch.plan()
    else:
        plan = ch.autotune(reps=3)  # plane-phase schedule, chosen before the timed steps
    print(f"[bench] {precision}: plane schedule {plan}", file=sys.stderr, flush=True)
    if warmup:
        ch.step(case.dt, warmup)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the timed steps run exactly as a user's would: no per-kernel events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ch.step(case.dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    fields = {k: t.cpu().numpy() for k, t in ch.get_fields("v", "omega2", "u1", "u3", "u1mean").items()}
    # then the same number of steps with every kernel bracketed by HIP events
    # on the context's stream: the per-kernel durations and the roofline
    ch.timing(True)
    e0.record(stream)
    ch.step(case.dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    kern = ch.timing_read()
    ch.timing(False)
    kern["_instrumented_ms"] = e0.elapsed_time(e1)
    ch.close()
    kern["_plan"] = plan
    return ms, wall, kern, fields


def ensemble_run(steps=50, precision="mixed"):
    """The 96-channel ensemble (uneven sizes) advanced `steps` RK3 steps in the graph."""
    import torch

    import synth
    from paper_1808_06461_amd.chn import Ensemble
    cases = synth.ensemble_cases(96)
    fields = [synth.turbulent_field(c) for c in cases]
    specs = [dict(n1=c.n1, n2=c.n2, n3=c.n3, lx=c.lx, lz=c.lz, re_b=c.re_b, mass_flux=c.mass_flux, y=f[4])
             for c, f in zip(cases, fields)]
    ens = Ensemble(specs, precision=precision)
    dts = []
    for ch, (v, om, U1, U3, y) in zip(ens.channels, fields):
        args = [torch.from_numpy(a) for a in (v, om, U1, U3)]
        ch.set_state(*args)
        info = ch.step(1e-6, 1, info=True)   # probe: CFL per unit dt at t = 0
        dts.append(0.5 * 1e-6 / info["cfl_max"])
        ch.set_state(*args)
    ens.step(dts, 1)  # warm-up: graph capture and instantiation
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    ens.step(dts, steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    G = sum(c.n1 * c.n2 * c.n3 for c in cases)
    ens.close()
    return {"workload": "96 minimal channels, n1 in {32,48,64}, n2 in {49,65,97}, n3 in {32,48}, "
                        "Re_tau in [180,400], one HIP graph per RK3 step of the whole ensemble",
            "precision": precision, "steps": steps, "grid_points": G, "ms_per_step": ms / steps,
            "value": G * steps / (ms / 1e3), "unit": UNIT}


def c3_run(reps=3):
    """One GPU's share of the Re_tau = 5300 channel, timed per phase (mixed precision):
    the 48-plane slab of 8192 x 6144 modes through the three plane kernels, and
    196608 modes x 1537 wall-normal nodes through the pencil kernel."""
    import torch

    import synth
    from paper_1808_06461_amd import Channel
    c = synth.C3_PLANES
    n1, n3, P = c["n1"], c["n3"], c["nplanes"]
    ch = Channel(n1, P, n3, c["lx"], c["lz"], synth.dean_re_b(c["re_tau"]), precision="mixed",
                 planes_only=True, plane_chunk=8)
    fields = [torch.empty((P, n1 // 2, n3), dtype=torch.complex64, device="cuda") for _ in range(6)]
    synth.c3_fill_slab(fields, (), cfg=c["cfg"])
    fields[4] = None  # omega2 formed in the z pass, as in the RK3 sub-step
    out = [torch.empty((P, n1 // 2, n3), dtype=torch.complex64, device="cuda") for _ in range(3)]
    # the slab's schedule: the default one under each radix set (a planes_only
    # context has no buffers of its own for chn_autotune), the fastest kept
    base = ch.plan()
    by_set = {}
    for rs in range(4):
        ch.set_plan(base["x_rows"], base["z_lines"], base["y_chunk"], base["fixed_radix"], base["z_pipeline"], rs)
        ch.plane_products(fields, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.plane_products(fields, out)
        torch.cuda.synchronize()
        by_set[rs] = round((time.perf_counter() - t0) * 1e3, 2)
    best = min(by_set, key=by_set.get)
    ch.set_plan(base["x_rows"], base["z_lines"], base["y_chunk"], base["fixed_radix"], base["z_pipeline"], best)
    ch.plane_products(fields, out)
    ch.timing(True)
    for _ in range(reps):
        ch.plane_products(fields, out)
    kern = ch.timing_read()
    ch.timing(False)
    planes = {"shape": f"{P} planes x {n1} x {n3} modes ({3 * n1 // 2} x {3 * n3 // 2} padded)",
              "plan": ch.plan(), "ms_by_radix_set": by_set}
    tot = 0.0
    for k in ("zinv", "xpass", "zfwd"):
        t, n = kern[k]
        b = algorithmic_bytes(k, n1, P, n3, 8)
        planes[k] = {"ms": round(t / reps, 3), "alg_GBps": round(b / (t / reps / 1e3) / 1e9, 1)}
        tot += t / reps
    planes["ms_total"] = round(tot, 3)
    ch.close()
    del fields, out
    torch.cuda.empty_cache()
    case = synth.c3_pencil_case()
    v, om, U1, U3, y = synth.turbulent_field(case)
    ch = Channel(case.n1, case.n2, case.n3, case.lx, case.lz, case.re_b, mass_flux=case.mass_flux,
                 precision="mixed", y=y)
    state = [torch.from_numpy(a) for a in (v, om, U1, U3)]
    del v, om
    ch.set_state(*state)
    probe = ch.step(1e-6, 1, info=True)
    dt = 0.5 * 1e-6 / probe["cfl_max"]
    ch.set_state(*state)
    ch.step(dt, 1)
    ch.timing(True)
    ch.step(dt, 1)
    kern = ch.timing_read()
    ch.timing(False)
    t, n = kern["advance"]
    b = algorithmic_bytes("advance", case.n1, case.n2, case.n3, 8)
    pencils = {"shape": f"{case.n1 // 2 * case.n3} modes x {case.n2} nodes", "ms_per_substep": round(t / n, 3),
               "alg_GBps": round(b / (t / n / 1e3) / 1e9, 1), "dt": dt}
    ch.close()
    torch.cuda.empty_cache()
    return {"workload": "one GPU's share of Re_tau 5300 (8192 x 1537 x 6144): 48-plane slab and 1/128 of the "
                        "modes as 1537-point pencils, mixed precision, seeded spectra", "planes": planes,
            "pencils": pencils}


def meshopt_run():
    """Near-wall mesh optimisation (a host routine, run once before a simulation):
    the 193-node mesh of the 384 x 193 x 384 workload at its critical modified
    wavenumber k^2_max + 1/(beta_min nu dt), and the 1537-node mesh of the
    Re_tau 5300 channel at k* = 1e10 (the unresolved-layer regime, where the
    homogeneous error has saturated); 20 free nodes per wall, C = 1e-3, at
    most 60 descent steps; wall time of the call on the host."""
    import math

    import synth
    from paper_1808_06461_amd import chn
    c = synth.CASES["c2"]
    kx = 2 * math.pi / c.lx * (c.n1 // 2 - 1)
    kz = 2 * math.pi / c.lz * (c.n3 // 2 - 1)
    out = {}
    for name, n2, ks in (("mesh_193", c.n2, kx * kx + kz * kz + 6.0 * c.re_b / c.dt), ("mesh_1537", 1537, 1e10)):
        y = synth.mesh_tanh(n2)
        t0 = time.perf_counter()
        yo, e0, e1, it = chn.optimise_mesh(y, m=20, kstar=ks, penalty=1e-3, max_iter=60)
        ms = (time.perf_counter() - t0) * 1e3
        s = np.diff(y)[1:21]
        out[name] = {"kstar": ks, "err_ref": e0, "err_opt": e1, "reduction": e0 / e1, "steps": it,
                     "max_shift_in_spacings": float((np.abs(yo - y)[1:21] / s).max()), "host_ms": round(ms, 1)}
    return out


def c5_run(reps=5, precision="mixed"):
    """The low-storage stage on the 1536 x 385 x 1152 field (Re_tau ~ 950): cut-off
    kc = (96, 72), filtered products and tau_ij on the 432 x 324 grid, the
    filtered enstrophy and the filtered pressure at the same cut-off; medians of reps."""
    import torch

    import synth
    from paper_1808_06461_amd import Channel
    c = synth.CASES["c5"]
    v, om, U1, U3, y = synth.turbulent_field(c)
    ch = Channel(c.n1, c.n2, c.n3, c.lx, c.lz, c.re_b, mass_flux=c.mass_flux, precision=precision, y=y)
    ch.set_state(*(torch.from_numpy(a) for a in (v, om, U1, U3)))
    del v, om
    kcx, kcz, q1, q3 = c.n1 // 16, c.n3 // 16, 432, 324
    ub, uu, tau = ch.filter_and_stress(kcx, kcz, q1, q3)  # warm-up, allocates the outputs
    ens = ch.filtered_enstrophy(kcx, kcz)

    def timed(fn):
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        times.sort()
        return times[len(times) // 2], times[0]

    ms, ms_min = timed(lambda: ch.filter_and_stress(kcx, kcz, q1, q3))
    ms_e, ms_e_min = timed(lambda: ch.filtered_enstrophy(kcx, kcz))
    pr = ch.filtered_pressure(kcx, kcz, uu, ub)
    ms_p, ms_p_min = timed(lambda: ch.filtered_pressure(kcx, kcz, uu, ub))
    ch.close()
    del ub, uu, tau, ens, pr
    torch.cuda.empty_cache()
    G = c.n1 * c.n2 * c.n3
    # algorithmic bytes: the three velocity coefficient fields in (float32
    # complex on the mixed path), F(u_i) and F(u_i u_j) out (complex128 on the
    # retained set), tau_ij out (float64 on the q grid); nominal flops: the
    # inverse transforms of u_i and the forward transforms of the six
    # products (2.5 n log2 n each) on the grid the stage uses, the smallest
    # 2,3-smooth f > 2 h + kc per direction (h the highest stored
    # wavenumber), the tau grid's transforms ignored
    NP = c.n2 * (c.n1 // 2) * c.n3
    R = (kcx + 1) * (2 * kcz + 1)
    alg = 3 * NP * (8 if precision == "mixed" else 16) + 9 * c.n2 * R * 16 + 6 * c.n2 * q1 * q3 * 8
    import math

    def grid(h, kc):
        n = 2 * h + kc + 1
        while True:
            m = n
            for p in (2, 3):
                while m % p == 0:
                    m //= p
            if m == 1:
                return n
            n += 1
    f1, f3 = grid(c.n1 // 2 - 1, kcx), grid(c.n3 // 2 - 1, kcz)
    n = f1 * f3
    fl = 9 * c.n2 * 2.5 * n * math.log2(n)
    roof = {"bound": "hbm", "achieved": round(alg / (ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes": alg,
            "nominal_flop": fl, "TFLOPs": round(fl / (ms / 1e3) / 1e12, 2), "product_grid": [f1, f3]}
    return {"workload": f"low-storage stage, {c.n1}x{c.n2}x{c.n3}, kc=({kcx},{kcz}), q=({q1},{q3})",
            "precision": precision, "ms_median": round(ms, 3), "ms_min": round(ms_min, 3),
            "roofline": roof,
            "grid_points_per_s": G / (ms / 1e3),
            "enstrophy": {"ms_median": round(ms_e, 3), "ms_min": round(ms_e_min, 3),
                          "grid_points_per_s": G / (ms_e / 1e3)},
            "pressure": {"ms_median": round(ms_p, 3), "ms_min": round(ms_p_min, 3)}}


def host_cpu():
    """Model name of the host CPU and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count(), usable


def cpu_baseline(case, v, om, U1, U3, y):
    """The oracle on the host: one RK3 sub-step of the same workload, scaled to a
    step, once on one thread and once with the FFTs on every usable core (the
    banded solves are numpy array sweeps over all modes, one thread either way)."""
    from oracle import fourier, kmm
    S = kmm.Setup(n1=case.n1, n2=case.n2, n3=case.n3, lx=case.lx, lz=case.lz, nu=1 / case.re_b,
                  dt=case.dt, mass_flux=case.mass_flux, y=y)
    st = kmm.make_state(S, v, om, U1, U3)
    G = case.n1 * case.n2 * case.n3
    model, ncpu, usable = host_cpu()
    runs = {}
    for workers in (1, usable):
        fourier.WORKERS = workers
        t0 = time.perf_counter()
        kmm.substep(S, st, kmm.zero_history(S), 0)
        runs[workers] = time.perf_counter() - t0
    fourier.WORKERS = 1
    t1, tn = runs[1], runs[usable]
    sample = (f"one RK3 sub-step (of 3) of the {case.n1}x{case.n2}x{case.n3} workload, scaled x3 to a step; "
              f"host: {model}, os.cpu_count() = {ncpu}, {usable} usable")
    return {"value": G / (3 * tn), "unit": UNIT, "cores": usable, "kind": "oracle",
            "sample": f"{sample}; {tn:.1f} s with the FFTs on {usable} threads",
            "cpu_model": model, "cpu_count": ncpu,
            "single_thread": {"value": G / (3 * t1), "cores": 1, "seconds_per_substep": round(t1, 2)},
            "all_cores": {"value": G / (3 * tn), "cores": usable, "seconds_per_substep": round(tn, 2)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the per-phase timing of the Re_tau 5300 share")
    ap.add_argument("--no-c5", action="store_true", help="skip the timing of the low-storage stage")
    ap.add_argument("--no-meshopt", action="store_true", help="skip the near-wall mesh optimisation leg")
    ap.add_argument("--plan", default=None, metavar="XROWS,ZLINES,YCHUNK[,FIXED[,ZPIPE[,RADIXSET]]]",
                    help="fixed plane-phase schedule instead of the autotuner (for profiling one schedule)")
    ap.add_argument("--source-hash", default=None, metavar="KIND",
                    help="print the source hash a traffic summary of this kernel kind must carry, then exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="also run five plain device copies of BYTES bytes (calibrates HBM byte counters)")
    ap.add_argument("--only", choices=("fp64", "mixed"), default=None,
                    help="run one precision only (for profiling; the JSON then lacks the comparison)")
    ap.add_argument("--leg", choices=("ensemble", "c3", "c5", "meshopt"), default=None,
                    help="run one of the other workloads only (for profiling) and print its JSON object")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash(args.source_hash))
        return
    if args.plan:
        global FIXED_PLAN
        FIXED_PLAN = tuple(int(v) for v in args.plan.split(","))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: 5 copies of {args.copy_probe} bytes", file=sys.stderr, flush=True)
        del src, dst

    if args.leg:
        leg = {"ensemble": ensemble_run, "c3": c3_run, "c5": c5_run, "meshopt": meshopt_run}[args.leg]
        print(json.dumps({args.leg: leg()}))
        return

    import synth
    case = synth.CASES["c2"]
    v, om, U1, U3, y = synth.turbulent_field(case)
    G = case.n1 * case.n2 * case.n3

    res = {}
    if args.only:
        print(f"[bench] {args.only} only: {args.warmup} warmup + {args.steps} timed RK3 steps", file=sys.stderr)
        ms, _, kern, _ = run_path(case, v, om, U1, U3, y, args.only, args.steps, args.warmup)
        plan = kern.pop("_plan")
        kern.pop("_instrumented_ms")
        print(json.dumps({"precision": args.only, "ms_per_step": ms / args.steps, "plane_schedule": plan,
                          "value": G * args.steps / (ms / 1e3), "kernels_ms": {k: t / max(n, 1) for k, (t, n) in kern.items()}}))
        return
    for prec in ("fp64", "mixed"):
        print(f"[bench] {prec}: {args.warmup} warmup + {args.steps} timed RK3 steps", file=sys.stderr, flush=True)
        res[prec] = run_path(case, v, om, U1, U3, y, prec, args.steps, args.warmup)
    ms_mixed, _, kern, fm = res["mixed"]
    ms_fp64, _, kern64, f64 = res["fp64"]
    step_ms = ms_mixed / args.steps
    value = G * args.steps / (ms_mixed / 1e3)
    errs = {k: float(np.linalg.norm(fm[k] - f64[k]) / np.linalg.norm(f64[k])) for k in fm}

    plan_mixed, plan64 = kern.pop("_plan"), kern64.pop("_plan")
    inst_ms, inst_ms64 = kern.pop("_instrumented_ms"), kern64.pop("_instrumented_ms")
    nsub = 3 * args.steps  # sub-steps in the timed region; a kernel kind may launch once per plane chunk
    # roofline of the dominant kernel of the mixed path
    dom = max(kern, key=lambda k: kern[k][0])
    tot, cnt = kern[dom]
    elem = 8
    alg = algorithmic_bytes(dom, case.n1, case.n2, case.n3, elem)  # per sub-step (all planes / modes)
    avg_s = tot / nsub / 1e3
    achieved = alg / avg_s / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
            "algorithmic_bytes_per_launch": alg * nsub // cnt, "avg_launch_ms": round(tot / cnt, 4)}
    if dom == "advance":
        NP = case.n2 * (case.n1 // 2) * case.n3
        withv = (alg + V_STORE_BYTES * NP) / avg_s / 1e9
        roof["frac_with_v_store"] = round(withv / HBM_PEAK_GBS, 4)
    fl = nominal_flops_per_substep(case.n1, case.n2, case.n3) * 3  # per RK3 step
    flops = {"nominal_flop_per_step": fl,
             "mixed": {"TFLOPs": round(fl / step_ms / 1e9, 2), "peak_fp32_vector": 157.3,
                       "frac": round(fl / step_ms / 1e9 / 157.3, 4)},
             "fp64": {"TFLOPs": round(fl / (ms_fp64 / args.steps) / 1e9, 2), "peak_fp64_vector": 78.6,
                      "frac": round(fl / (ms_fp64 / args.steps) / 1e9 / 78.6, 4)}}

    def table(kk, e):
        out = {}
        for k, (t, n) in kk.items():
            if n:
                b = algorithmic_bytes(k, case.n1, case.n2, case.n3, e) * (n if k == "recover" else nsub)
                out[k] = {"avg_ms": round(t / n, 4), "launches": n, "alg_GBps": round(b / (t / 1e3) / 1e9, 1)}
        return out
    per_kernel, per_kernel64 = table(kern, elem), table(kern64, 16)

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 transforms/products + f64 solves", "data": "synthetic",
        "config": {"workload": "channel 384x193x384 (Re_tau~550, Re_b=10000, box 2pi x 2 x pi), "
                               "k^-5/3 perturbations on a Reichardt mean, dt at CFL 0.5, mixed precision",
                   "grid_points": G, "dt": case.dt},
        "fp64": {"value": G * args.steps / (ms_fp64 / 1e3), "ms_per_step": ms_fp64 / args.steps,
                 "kernels": per_kernel64, "instrumented_ms_per_step": inst_ms64 / args.steps},
        "instrumented_ms_per_step": inst_ms / args.steps,
        "flops": flops,
        "plane_schedule": {"mixed": plan_mixed, "fp64": plan64},
        "mixed_vs_fp64_rel_err": errs,
        "speedup_mixed_over_fp64": ms_fp64 / ms_mixed,
        "kernels": per_kernel,
        "roofline": roof,
    }
    if not args.no_ensemble:
        print("[bench] ensemble of 96 channels, 50 steps", file=sys.stderr, flush=True)
        out["ensemble"] = ensemble_run()
    if not args.no_c3:
        print("[bench] Re_tau 5300 share: plane slab and pencil share", file=sys.stderr, flush=True)
        out["c3_share"] = c3_run()
    if not args.no_c5:
        print("[bench] low-storage stage, 1536x385x1152", file=sys.stderr, flush=True)
        out["c5_filter"] = c5_run()
    if not args.no_meshopt:
        print("[bench] near-wall mesh optimisation (host)", file=sys.stderr, flush=True)
        out["mesh_opt"] = meshopt_run()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, one sub-step)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, v, om, U1, U3, y)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
