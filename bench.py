"""Benchmark of the D2Q37 step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the Rayleigh-Taylor lattice of the paper's Table 1, 1920 x 2048
sites (Sec. 5), FP64, tau 0.7, g = 1e-4 along -y, walls at T = 1.5 / 0.5.  A
step is one pass of the whole hot path: periodic halo, propagate, bc and
collide, run as the fused kernel (one launch per step).  Inputs are resident
in HBM before timing starts.  Printed: one JSON line with the headline FP64
MLUPS, the roofline of the fused kernel, the split kernels, the adjoint, the
FP32 storage forms on this lattice and on the 4096 x 4096 precision lattice
(each against the FP64 GPU run after 2000 steps), the 8192 x 4096 production
lattice, a small graph-captured lattice, and the CPU oracle timed on a bounded
sample on this host.  Other modes: --workloads, --ablations, --variants,
--forms, --rt-run.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "D2Q37 MLUPS FP64 vs FP32-shifted at stated error; % HBM/FP64 roofline"
HBM_PEAK_GBS = 8000.0
Q = 37


def bytes_per_site(precision: str = "fp64") -> int:
    """Algorithmic HBM bytes of one site update: read and write 37 populations
    (8 or 4 bytes each); the local-reference FP32 forms ("fp32c", "fp32l")
    also read and write their site's packed reference (4 bytes)."""
    if precision == "fp64":
        return 2 * Q * 8
    return 2 * (Q + 1) * 4 if precision in ("fp32c", "fp32l") else 2 * Q * 4


def mlups(sites: int, seconds: float) -> float:
    return sites / seconds / 1e6


PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_SUMMARY = os.path.join(PROFILES, "k_fused_fp64_rt1920x2048_hbm_traffic.md")
VALU_SUMMARY = os.path.join(PROFILES, "k_fused_forms_rt1920x2048_valu.md")
FP32_VALU_SUMMARY = VALU_SUMMARY
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
KERNEL_SOURCES = ["paper_1703_00186_amd/csrc/d2q37_kernels.hip",
                  "paper_1703_00186_amd/csrc/d2q37_device.h",
                  "paper_1703_00186_amd/csrc/d2q37_constants.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def summary_values(path: str) -> dict:
    """The '- key: value' lines of a committed profile summary, if the kernel
    sources still hash to the value recorded with its counters."""
    try:
        vals = {}
        for line in open(path):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip()
    except OSError:
        return {}
    return vals if vals.get("source_sha256_16") == kernel_source_hash() else {}


def measured_traffic(lx: int, ly: int):
    """HBM bytes per fused launch from the committed counter summary, or None
    when the summary is missing, is for another lattice, or the kernel
    sources changed since the counters were taken."""
    vals = summary_values(TRAFFIC_SUMMARY)
    try:
        if vals.get("lattice") != "%dx%d" % (lx, ly):
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def counted_flop_per_site():
    """FP64 flop per site counted by the VALU counters (None if stale)."""
    try:
        return float(summary_values(VALU_SUMMARY)["flop_per_site"])
    except (KeyError, ValueError):
        return None


def counted_fp32_mode_flops(prec: str):
    """(FP64, FP32) flop per site of the FP32-storage step `prec` from the
    committed VALU counter summary, or None if missing or stale."""
    vals = summary_values(FP32_VALU_SUMMARY)
    try:
        return float(vals[prec + "_flop64_per_site"]), float(vals[prec + "_flop32_per_site"])
    except (KeyError, ValueError):
        return None


def copy_calibration(torch, nbytes: int = 1 << 30, reps: int = 3) -> None:
    """A plain device copy of known size (nbytes read + nbytes written per
    launch), run so that a counter profile of this process can be scaled."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def field_errors(m, ref) -> dict:
    """Relative errors per field of (rho, ux, uy, T): rho and T as max|d| over
    max|ref|; u as max|du| over max|u| (the vector error over the largest
    speed).  u_thermal: the same velocity error over the thermal speed
    sqrt(min T), for reference only."""
    import numpy as np
    m = [np.asarray(a, dtype=np.float64) for a in m]
    r = [np.asarray(a, dtype=np.float64) for a in ref]
    du = np.hypot(m[1] - r[1], m[2] - r[2])
    return {"rho": float(np.abs(m[0] - r[0]).max() / np.abs(r[0]).max()),
            "u": float(du.max() / max(float(np.hypot(r[1], r[2]).max()), 1e-300)),
            "T": float(np.abs(m[3] - r[3]).max() / np.abs(r[3]).max()),
            "u_thermal": float(du.max() / float(np.sqrt(r[3].min())))}


def host_moments(lb, torch):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in lb.moments()]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def time_steps(lb, steps: int, torch) -> float:
    """Seconds for `steps` steps, HIP events on the stream the kernels use."""
    s = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    lb.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def time_adjoint(lb, steps: int, torch) -> dict:
    """The adjoint on the headline lattice with a full tape: `steps` steps
    recorded (fused step + 4-moment tape, 624 B/site), then `steps` transposed
    steps in one lb_adjoint_run (gather form, k_adjoint_mu: 624 B/site) and,
    for comparison, as single lb_adjoint_step calls (scatter form, k_adjoint);
    HIP events on the kernels' stream.  The lattice advances by `steps`."""
    sites = lb.lx * lb.ly
    tape = lb.new_tape(steps)
    lam, spare = lb.new_lambda(), lb.new_lambda()
    lb.step_record(2, tape)  # warm-up of the kernels
    lb.adjoint_step(tape[0], lam.zero_(), spare)
    lb.adjoint_run(tape, lam, 2)
    s = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record(s)
    lb.step_record(steps, tape)
    ev[1].record(s)
    _, lam = lb.loss_ke(with_lambda=True)
    lam1 = lam.clone()
    ev[2].record(s)
    lb.adjoint_run(tape, lam, steps)
    ev[3].record(s)
    ev[4].record(s)
    for j in range(steps - 1, -1, -1):
        lb.adjoint_step(tape[j], lam1, spare)
        lam1, spare = spare, lam1
    ev[5].record(s)
    torch.cuda.synchronize()
    same = bool(torch.equal(lam, lam1))
    t_rec = ev[0].elapsed_time(ev[1]) / 1e3 / steps
    t_run = ev[2].elapsed_time(ev[3]) / 1e3 / steps
    t_one = ev[4].elapsed_time(ev[5]) / 1e3 / steps
    gbs = lambda t: round(624 * sites / t / 1e9, 1)  # noqa: E731
    return {"steps": steps, "record_ms_per_step": round(t_rec * 1e3, 5),
            "record_GB/s": gbs(t_rec),
            "adjoint_ms_per_step": round(t_run * 1e3, 5), "adjoint_GB/s": gbs(t_run),
            "adjoint_frac": round(624 * sites / t_run / 1e9 / HBM_PEAK_GBS, 4),
            "single_step_ms_per_step": round(t_one * 1e3, 5), "single_step_GB/s": gbs(t_one),
            "run_equals_single_steps": same,
            "note": "lambda in 296 + tape 32 + lambda out 296 B/site; adjoint_*: lb_adjoint_run "
                    "(gather form), single_step_*: lb_adjoint_step (scatter form)"}


def time_split_kernels(lb, steps: int, torch) -> dict:
    """Per-kernel seconds of the split path (halo, propagate, bc, collide)."""
    s = torch.cuda.current_stream()
    names = ["halo", "propagate", "bc", "collide"]
    calls = [lb.halo, lb.propagate, lb.bc, lb.collide]
    tot = {n: 0.0 for n in names}
    torch.cuda.synchronize()
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(s)
        for i, c in enumerate(calls):
            c()
            ev[i + 1].record(s)
        torch.cuda.synchronize()
        for i, n in enumerate(names):
            tot[n] += ev[i].elapsed_time(ev[i + 1]) / 1e3
    return {n: tot[n] / steps for n in names}


# FP32 forms timed beside the FP64 headline: (key, precision, what it is)
FP32_FORMS = (
    ("fp32_local", "fp32l",
     "FP32 storage of each population's deviation from the rest Maxwellian of the site that "
     "collided it (+ that site's FP16 density and temperature), FP64 collision"),
    ("fp32_local_fp32_collide", "fp32c",
     "the same storage with an FP32 collision (FP32 Hermite sums of the deviation; FP64 for "
     "the collision invariants, the equilibrium coefficients and a conservation correction)"),
    ("fp32_shifted", "fp32s", "FP32 storage of f - w rho_ref (rho_ref = 1), FP64 collision"),
    ("fp32_shifted_f32sum", "fp32s_f32sum",
     "ablation: FP32 storage of f - w rho_ref, the FP64 collision's Hermite sums in FP32"),
)
FP32_WARMUP, FP32_TIMED, FP32_ERROR_STEPS = 20, 200, 2000


def fp32_legs(lx: int, ly: int, fields, layout: str, fp64_mlups: float, torch) -> dict:
    """Each FP32 form on the headline lattice: FP32_TIMED steps timed after
    FP32_WARMUP warm-up steps (independent of --steps), then run on to
    FP32_ERROR_STEPS steps and compared per field with the FP64 GPU run of as
    many steps."""
    from paper_1703_00186_amd.lb import LB

    sites = lx * ly
    lb = LB(lx, ly, *fields, layout=layout)
    lb.step(FP32_ERROR_STEPS)
    m64 = host_moments(lb, torch)
    del lb
    torch.cuda.empty_cache()
    out = {}
    for key, prec, what in FP32_FORMS:
        lb32 = LB(lx, ly, *fields, precision=prec, layout=layout, kernel="fused")
        lb32.step(FP32_WARMUP)
        t32 = time_steps(lb32, FP32_TIMED, torch)
        lb32.step(FP32_ERROR_STEPS - FP32_WARMUP - FP32_TIMED)
        errs = field_errors(host_moments(lb32, torch), m64)
        v32 = mlups(sites * FP32_TIMED, t32)
        gbs = bytes_per_site(prec) * sites / (t32 / FP32_TIMED) / 1e9
        out[key] = {
            "form": what, "precision": prec,
            "MLUPS": round(v32, 2), "ms_per_step": round(t32 / FP32_TIMED * 1e3, 5),
            "steps_timed": FP32_TIMED, "warmup": FP32_WARMUP,
            "ratio_vs_fp64": round(v32 / fp64_mlups, 3),
            "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "error_vs_fp64_gpu": {k: float("%.3g" % v) for k, v in errs.items()},
            "error_after_steps": FP32_ERROR_STEPS}
        vals = summary_values(TRAFFIC_SUMMARY)
        if vals.get("lattice") == "%dx%d" % (lx, ly) and (prec + "_hbm_bytes_per_launch") in vals:
            out[key]["traffic"] = float(vals[prec + "_hbm_bytes_per_launch"])
            out[key]["traffic_unit"] = "bytes per launch"
        fl = counted_fp32_mode_flops(prec)
        if fl is not None:
            rate = sites / (t32 / FP32_TIMED) / 1e12
            out[key]["compute"] = {
                "fp64_flop_per_site_counted": fl[0], "fp32_flop_per_site_counted": fl[1],
                "fp64_TFLOPs": round(fl[0] * rate, 2),
                "fp64_frac": round(fl[0] * rate / FP64_VECTOR_PEAK_TFLOPS, 4),
                "fp32_TFLOPs": round(fl[1] * rate, 2),
                "fp32_frac": round(fl[1] * rate / FP32_VECTOR_PEAK_TFLOPS, 4)}
        log("bench: fused %s %.1f MLUPS (x%.2f), errors after %d steps %s" % (
            prec, v32, v32 / fp64_mlups, FP32_ERROR_STEPS, errs))
        del lb32
        torch.cuda.empty_cache()
    return out


def precision_leg(torch, layout: str = "column") -> dict:
    """The precision workload's lattice, 4096 x 4096 (sinusoidal RT): the FP64
    step and each FP32 form timed over FP32_TIMED steps after FP32_WARMUP
    (the FP32 MLUPS over the FP64 MLUPS of this lattice), every run carried
    on to FP32_ERROR_STEPS steps and the FP32 fields compared with the FP64
    GPU run's."""
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    lx, ly = 4096, 4096
    sites = lx * ly
    fields = workload.rt_fields(lx, ly, seed=workload.config_seed(3))[:4]
    rec = {"lattice": [lx, ly], "steps_timed": FP32_TIMED, "warmup": FP32_WARMUP,
           "error_after_steps": FP32_ERROR_STEPS}
    m64 = None
    for prec in ("fp64", "fp32c", "fp32l", "fp32s"):
        torch.cuda.empty_cache()
        lb = LB(lx, ly, *fields, precision=prec, layout=layout)
        lb.step(FP32_WARMUP)
        t = time_steps(lb, FP32_TIMED, torch)
        lb.step(FP32_ERROR_STEPS - FP32_WARMUP - FP32_TIMED)
        v = mlups(sites * FP32_TIMED, t)
        gbs = bytes_per_site(prec) * sites / (t / FP32_TIMED) / 1e9
        rec[prec] = {"MLUPS": round(v, 1), "ms_per_step": round(t / FP32_TIMED * 1e3, 4),
                     "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        if prec == "fp64":
            m64 = host_moments(lb, torch)
        else:
            errs = field_errors(host_moments(lb, torch), m64)
            rec[prec]["ratio_vs_fp64"] = round(v / rec["fp64"]["MLUPS"], 3)
            rec[prec]["error_vs_fp64_gpu"] = {k: float("%.3g" % e) for k, e in errs.items()}
        log("bench: 4096x4096 %s %s" % (prec, rec[prec]))
        del lb
    torch.cuda.empty_cache()
    return rec


def production_leg(torch, steps: int = 200, warmup: int = 10, n_adj: int = 100,
                   k: int = 20) -> dict:
    """The production lattice, 8192 x 4096 (multimode RT): FP64 and FP32 step
    speed and workspace, then the adjoint of the last n_adj FP64 steps with
    checkpoints every k steps (backward cost over the plain forward run of the
    same steps)."""
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    lx, ly = 8192, 4096
    sites = lx * ly
    fields = workload.rt_fields(lx, ly, seed=workload.config_seed(5), mode="multimode")[:4]
    rec = {"lattice": [lx, ly], "steps_timed": steps, "warmup": warmup}
    for prec in ("fp32c", "fp32l", "fp32s", "fp64"):
        torch.cuda.empty_cache()
        lb = LB(lx, ly, *fields, precision=prec)
        ws = int(lb.workspace.numel())
        lb.step(warmup)
        t = time_steps(lb, steps, torch)
        v = mlups(sites * steps, t)
        gbs = bytes_per_site(prec) * sites / (t / steps) / 1e9
        rec[prec] = {"MLUPS": round(v, 1), "ms_per_step": round(t / steps * 1e3, 4),
                     "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "workspace_bytes": ws}
        log("bench: 8192x4096 %s %.1f MLUPS (%.1f GB/s)" % (prec, v, gbs))
        if prec != "fp64":
            del lb
    # adjoint of the last n_adj steps (the schedule of adjoint.kinetic_energy:
    # checkpoints at the start of every segment but the last, whose tape the
    # forward pass records)
    base = device_bytes_in_use(torch)
    ckpts = []
    tape = lb.new_tape(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(0, n_adj - k, k):
        ckpts.append(lb.get_state())
        lb.step(k)
    lb.step_record(k, tape)
    _, lam = lb.loss_ke(with_lambda=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lb.adjoint_run(tape, lam, k)
    for ck in reversed(ckpts):
        lb.set_state(ck)
        lb.step_record(k, tape)
        lb.adjoint_run(tape, lam, k)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    t_plain = n_adj * rec["fp64"]["ms_per_step"] / 1e3
    rec["fp64"]["adjoint_last_steps"] = {
        "steps": n_adj, "checkpoint_every": k,
        "forward_with_checkpoints_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
        "backward_over_forward": round((t2 - t1) / t_plain, 3),
        "checkpoints_tape_lambda_bytes": int(device_bytes_in_use(torch) - base),
        "finite": bool(torch.isfinite(lam).all())}
    rec["peak_device_bytes"] = int(torch.cuda.max_memory_allocated())
    log("bench: 8192x4096 adjoint %s" % rec["fp64"]["adjoint_last_steps"])
    del lb, ckpts, tape, lam
    torch.cuda.empty_cache()
    return rec


# Host threads of the CPU legs: every core this process may run on, capped at
# 16, the host-core share of one GPU on the MI355X nodes this runs on (their
# affinity mask can show more cores than that share).
CPU_THREAD_CAP = 16


def cpu_threads() -> int:
    return min(CPU_THREAD_CAP, len(os.sched_getaffinity(0)))


def cpu_baseline(lx: int, ly: int, fields, steps: int) -> dict:
    import oracle

    threads = cpu_threads()
    oracle.set_threads(threads)
    P = oracle.Params(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5)
    f = oracle.init_feq(*fields)
    f = oracle.run(f, P, 1)  # warm-up step
    t0 = time.perf_counter()
    oracle.run(f, P, steps)
    dt = time.perf_counter() - t0
    return {"value": round(mlups(lx * ly * steps, dt), 4), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d steps of the %dx%d FP64 RT lattice after 1 warm-up step (%.1f s), %s, "
                      "%d threads (all affine cores, at most %d: one GPU's host-core share)"
                      % (steps, lx, ly, dt, cpu_model(), threads, CPU_THREAD_CAP)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def device_bytes_in_use(torch) -> int:
    torch.cuda.synchronize()
    return int(torch.cuda.memory_allocated())


def run_workloads(args, torch) -> list:
    """One JSON record per workload: parity (256 x 128), FP32 precision
    (4096 x 4096), adjoint (512 x 512) and production (8192 x 4096); the
    1920 x 2048 speed workload is the headline line."""
    import oracle

    out = []
    P = oracle.Params(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5)
    todo = set(args.workloads or ["parity", "fp32", "adjoint", "production"])
    if "parity" in todo:
        out.append(_parity_workload(P, torch))
    if "fp32" in todo:
        out.append(_fp32_workload(args, P, torch))
    if "adjoint" in todo:
        out.append(_adjoint_workload(torch))
    if "production" in todo:
        out.append(_production_workload(args, torch))
    return out


def _parity_workload(P, torch) -> dict:
    import oracle
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    lx, ly, n = 256, 128, 50
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(1))[:4]
    lb = LB(lx, ly, *f)
    lb.step(n)
    m = host_moments(lb, torch)
    f0 = oracle.init_feq(*f)
    t0 = time.perf_counter()
    ref = oracle.moments(oracle.run(f0, P, n))
    t_or = time.perf_counter() - t0
    ext = oracle.run_moments_extended(f0, P, n)
    rec = {"workload": "parity 256x128", "lattice": [lx, ly], "steps": n, "precision": "fp64",
           "error_vs_extended_oracle": field_errors(m, ext),
           "error_vs_oracle": field_errors(m, ref),
           "oracle_fp64_vs_extended": field_errors(ref, ext),
           "oracle": {"MLUPS": round(mlups(lx * ly * n, t_or), 2), "seconds": round(t_or, 3),
                      "threads": oracle.get_threads()}}
    log("workloads: %s" % rec)
    return rec


def _fp32_workload(args, P, torch) -> dict:
    """4096 x 4096, the FP32 forms vs FP64 on the GPU, plus each FP32 form vs
    the oracle on 256 x 256."""
    import oracle
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    lx, ly, n = 4096, 4096, args.fp32_steps
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(3))[:4]
    rec = {"workload": "FP32 precision 4096x4096", "lattice": [lx, ly], "steps": n}
    ms = {}
    for prec in ("fp64", "fp32c", "fp32l", "fp32s", "fp32s_f32sum"):
        lb = LB(lx, ly, *f, precision=prec)
        t = time_steps(lb, n, torch)
        ms[prec] = host_moments(lb, torch)
        rec[prec] = {"MLUPS": round(mlups(lx * ly * n, t), 1)}
        del lb
        torch.cuda.empty_cache()
    for prec in ("fp32c", "fp32l", "fp32s", "fp32s_f32sum"):
        rec[prec]["error_vs_fp64_gpu"] = field_errors(ms[prec], ms["fp64"])
        rec[prec]["ratio_vs_fp64"] = round(rec[prec]["MLUPS"] / rec["fp64"]["MLUPS"], 3)
    lxs = 256
    fs = workload.rt_fields(lxs, lxs, seed=workload.config_seed(3))[:4]
    t0 = time.perf_counter()
    ref = oracle.moments(oracle.run(oracle.init_feq(*fs), P, n))
    t_or = time.perf_counter() - t0
    for prec in ("fp32c", "fp32l", "fp32s", "fp32s_f32sum"):
        lb = LB(lxs, lxs, *fs, precision=prec)
        lb.step(n)
        rec[prec]["error_vs_oracle_256x256"] = field_errors(host_moments(lb, torch), ref)
        del lb
    rec["oracle_256x256"] = {"MLUPS": round(mlups(lxs * lxs * n, t_or), 2),
                             "seconds": round(t_or, 2), "threads": oracle.get_threads()}
    torch.cuda.empty_cache()
    log("workloads: %s" % rec)
    return rec


def _adjoint_workload(torch) -> dict:
    """512 x 512, 200 steps: gradient of the final kinetic energy w.r.t. the 16
    interface amplitudes (adjoint, checkpoints every 20) against central
    finite differences, and its cost relative to the forward run; then the
    same gradient from a full tape (no recomputation)."""
    import numpy as np

    from paper_1703_00186_amd import adjoint, workload
    from paper_1703_00186_amd.lb import LB

    lx, ly, n, k = 512, 512, 200, 20
    seed = workload.config_seed(4)
    rho, ux, uy, T, info = workload.rt_fields(lx, ly, seed=seed, mode="multimode")
    lb = LB(lx, ly, rho, ux, uy, T)
    fields = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (rho, ux, uy, T)]
    adjoint.kinetic_energy(lb, *fields, nsteps=40, checkpoint_every=k).backward()  # warm-up
    fields = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (rho, ux, uy, T)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ke = adjoint.kinetic_energy(lb, *fields, nsteps=n, checkpoint_every=k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ke.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = workload.amplitude_gradient(lx, ly, fields[0].grad.cpu().numpy(),
                                    fields[3].grad.cpu().numpy(), seed=seed)
    lb.reinit(rho, ux, uy, T)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    lb.step(n)
    lb.loss_ke(with_lambda=False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t3

    def ke_of(amp):
        ff = workload.rt_fields(lx, ly, seed=seed, mode="multimode", amplitudes=amp)[:4]
        lb.reinit(*ff)
        lb.step(n)
        return float(lb.loss_ke(with_lambda=False)[0].cpu()[0])

    # rounding noise of KE: nine points of a line through the amplitudes
    # (|t| <= 4e-9) minus their least-squares quadratic; a central
    # difference at h carries sigma / (sqrt(2) h) per component
    d = np.random.default_rng(7).standard_normal(16)
    d /= np.linalg.norm(d)
    ts = np.arange(-4, 5) * 1e-9
    kes = np.array([ke_of(info["amplitudes"] + t * d) for t in ts])
    dke = kes - kes[4]
    resid = dke - np.polyval(np.polyfit(ts / 1e-9, dke, 2), ts / 1e-9)
    sigma = float(np.sqrt(np.sum(resid ** 2) / (len(ts) - 3)))
    fd = {}
    for h in (1e-6, 1e-5):
        gfd = np.zeros(16)
        for j in range(16):
            e = np.zeros(16)
            e[j] = h
            gfd[j] = (ke_of(info["amplitudes"] + e) - ke_of(info["amplitudes"] - e)) / (2 * h)
        fd["%g" % h] = float(np.abs(g - gfd).max() / np.abs(gfd).max())
    # full tape: the forward run records the moments of all n steps, the
    # backward run only applies the transposed steps
    fields = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (rho, ux, uy, T)]
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    ke_t = adjoint.kinetic_energy(lb, *fields, nsteps=n, checkpoint_every=0)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    ke_t.backward()
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    g_t = workload.amplitude_gradient(lx, ly, fields[0].grad.cpu().numpy(),
                                      fields[3].grad.cpu().numpy(), seed=seed)
    rec = {"workload": "adjoint 512x512", "lattice": [lx, ly], "steps": n, "checkpoint_every": k,
           "KE": float(ke.detach().cpu()), "max_abs_grad": float(np.abs(g).max()),
           "adjoint_vs_central_fd": fd,
           # measured rounding noise of KE and of a central difference at h,
           # relative to max |dKE/da|: at h = 1e-6 it is the size of the
           # difference itself (h = 1e-5 is below both noise and truncation)
           "ke_rounding_noise": sigma,
           "fd_noise_per_component": {"%g" % h: float(sigma / (np.sqrt(2) * h) / np.abs(g).max())
                                      for h in (1e-6, 1e-5)},
           "forward_s": round(t_plain, 5),
           "forward_with_checkpoints_s": round(t1 - t0, 5), "backward_s": round(t2 - t1, 5),
           "backward_over_forward": round((t2 - t1) / t_plain, 3),
           "full_tape": {"tape_GB": round(n * 4 * lx * ly * 8 / 1e9, 3),
                         "forward_recording_s": round(t5 - t4, 5),
                         "backward_s": round(t6 - t5, 5),
                         "backward_over_forward": round((t6 - t5) / t_plain, 3),
                         "gradient_vs_checkpointed": float(np.abs(g_t - g).max() /
                                                           np.abs(g).max())}}
    log("workloads: %s" % rec)
    del lb, fields
    torch.cuda.empty_cache()
    return rec


def _production_workload(args, torch) -> dict:
    """8192 x 4096: FP64 and FP32 shifted speed and footprint, then the
    adjoint of the last 100 FP64 steps, with checkpoints every 20 steps and
    with a full tape."""
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    lx, ly, n, n_adj = 8192, 4096, args.production_steps, 100
    sites = lx * ly
    seed = workload.config_seed(5)
    rho, ux, uy, T, info = workload.rt_fields(lx, ly, seed=seed, mode="multimode")
    rec = {"workload": "production 8192x4096", "lattice": [lx, ly], "steps": n}
    for prec in ("fp32c", "fp32s", "fp64"):
        base = device_bytes_in_use(torch)
        lb = LB(lx, ly, rho, ux, uy, T, precision=prec)
        foot = device_bytes_in_use(torch) - base
        t = time_steps(lb, n - (n_adj if prec == "fp64" else 0), torch)
        steps_done = n - (n_adj if prec == "fp64" else 0)
        v = mlups(sites * steps_done, t)
        bps = bytes_per_site(prec)
        rec[prec] = {"MLUPS": round(v, 1), "GB/s": round(bps * v * 1e6 / 1e9, 1),
                     "hbm_frac": round(bps * v * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
                     "workspace_GB": round(foot / 1e9, 3), "steps_timed": steps_done}
        if prec != "fp64":
            del lb
            torch.cuda.empty_cache()
    # adjoint of the last n_adj steps: d KE(final) / d (state at step n - n_adj)
    # (the schedule of adjoint.kinetic_energy: checkpoints at the start of
    # every segment but the last, whose tape the forward pass records)
    k = 20
    base = device_bytes_in_use(torch)
    ckpts = []
    tape = lb.new_tape(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s0 in range(0, n_adj - k, k):
        ckpts.append(lb.get_state())
        lb.step(k)
    lb.step_record(k, tape)
    ke, lam = lb.loss_ke(with_lambda=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lb.adjoint_run(tape, lam, k)
    for ck in reversed(ckpts):
        lb.set_state(ck)
        lb.step_record(k, tape)
        lb.adjoint_run(tape, lam, k)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    extra = device_bytes_in_use(torch) - base
    rec["fp64"]["adjoint_last_steps"] = {
        "steps": n_adj, "checkpoint_every": k, "forward_s": round(t1 - t0, 4),
        "backward_s": round(t2 - t1, 4), "backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
        "checkpoints_tape_lambda_GB": round(extra / 1e9, 3),
        "lambda_norm": float(lam.norm().cpu())}
    # the same gradient from a full tape of the n_adj steps (32 B per site and
    # step) instead of checkpoints and recomputation
    ck0, lam_ckpt = ckpts[0], lam  # the state n_adj steps before the end
    del ckpts, tape
    torch.cuda.empty_cache()
    base = device_bytes_in_use(torch)
    lb.set_state(ck0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tape = lb.new_tape(n_adj)
    lb.step_record(n_adj, tape)
    ke, lam = lb.loss_ke(with_lambda=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lb.adjoint_run(tape, lam, n_adj)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    extra = device_bytes_in_use(torch) - base
    rec["fp64"]["adjoint_last_steps_full_tape"] = {
        "steps": n_adj, "forward_recording_s": round(t1 - t0, 4),
        "backward_s": round(t2 - t1, 4),
        "backward_over_forward": round((t2 - t1) / rec["fp64"]["adjoint_last_steps"]["forward_s"],
                                       3),
        "tape_lambda_GB": round(extra / 1e9, 3),
        "lambda_vs_checkpointed": float((lam - lam_ckpt).norm().cpu() / lam_ckpt.norm().cpu())}
    rec["peak_device_GB"] = round(torch.cuda.max_memory_allocated() / 1e9, 2)
    del lb, ck0, tape, lam, lam_ckpt
    torch.cuda.empty_cache()
    log("workloads: %s" % rec)
    return rec


def run_rt(args, torch) -> dict:
    """A long Rayleigh-Taylor run on the headline lattice with the in-situ
    observables recorded on the device (lb_run_observed) every `every`
    steps: total mass, kinetic energy, sum rho T and the mixing-layer width,
    plus a finiteness scan (check_finite) at the same interval."""
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    lx, ly, n, every = args.lx, args.ly, args.rt_steps, args.rt_every
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(2))[:4]
    lb = LB(lx, ly, *f, check_finite=every)
    prof0, sc0 = lb.observables()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    series = lb.run_observed(n, every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s = series.cpu().numpy()
    sc0 = sc0.cpu().numpy()
    rec = {"run": "Rayleigh-Taylor %dx%d, %d steps, observables every %d" % (lx, ly, n, every),
           "MLUPS_with_observables": round(mlups(lx * ly * n, dt), 1),
           "initial": {"mass": float(sc0[0]), "KE": float(sc0[1]), "width": float(sc0[3])},
           "series": {"step": [every * (i + 1) for i in range(len(s))],
                      "mass_rel_change": [float(v / sc0[0] - 1) for v in s[:, 0]],
                      "KE": [float(v) for v in s[:, 1]],
                      "width": [float(v) for v in s[:, 3]]}}
    log("rt run: %.1f MLUPS, final width %.2f, KE %.3e" % (
        rec["MLUPS_with_observables"], s[-1, 3], s[-1, 1]))
    return rec


def run_ablations(args, torch) -> list:
    """Variants of the step: memory layout, plain BGK vs Hermite-regularized
    collision (speed, and the smallest tau that stays finite), and the FP32
    shift density."""
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB, LBError

    out = []
    lx, ly = args.lx, args.ly
    sites = lx * ly
    f = workload.rt_fields(lx, ly, seed=workload.config_seed(2))[:4]
    speed = {}
    for layout in ("soa", "column"):
        for prec in ("fp64", "fp32c", "fp32l", "fp32s"):
            for reg in (1, 0):
                lb = LB(lx, ly, *f, precision=prec, layout=layout, regularize=reg)
                lb.step(20)
                t = time_steps(lb, 200, torch)
                speed["%s/%s/%s" % (layout, prec, "regularized" if reg else "bgk")] = round(
                    mlups(sites * 200, t), 1)
                del lb
                torch.cuda.empty_cache()
    out.append({"ablation": "layout x precision x collision, fused step MLUPS",
                "lattice": [lx, ly], "MLUPS": speed})
    log("ablations: %s" % out[-1])

    # stability: first step (to within 100) at which the RT run stops being
    # finite, for each tau, with and without the Hermite projection
    sl, n = 512, args.stability_steps
    fs = workload.rt_fields(sl, sl, seed=workload.config_seed(2))[:4]
    stab = {}
    for reg in (1, 0):
        for tau in (0.6, 0.62, 0.64, 0.66, 0.68, 0.7):
            lb = LB(sl, sl, *fs, tau=tau, regularize=reg, check_finite=100)
            status = "finite after %d" % n
            for done in range(0, n, 100):
                try:
                    lb.step(100)
                except LBError as e:
                    if e.code != -5:
                        raise
                    status = "non-finite by step %d" % (done + 100)
                    break
            stab["%s tau=%g" % ("regularized" if reg else "bgk", tau)] = status
            del lb
    out.append({"ablation": "stability of the RT run (rho<=0, T<=0 or NaN, checked every 100 "
                            "steps)", "lattice": [sl, sl], "steps": n, "result": stab})
    log("ablations: %s" % out[-1])

    # FP32 shift density rho_ref: error after 2000 steps vs FP64
    al, n = 1024, 2000
    fa = workload.rt_fields(al, al, seed=workload.config_seed(3))[:4]
    lb = LB(al, al, *fa)
    lb.step(n)
    m64 = host_moments(lb, torch)
    del lb
    shift = {}
    for prec in ("fp32s", "fp32s_f32sum"):
        for rho_ref in (0.0, 1.0):
            lb = LB(al, al, *fa, precision=prec, rho_ref=rho_ref)
            lb.step(n)
            shift["%s rho_ref=%g" % (prec, rho_ref)] = field_errors(host_moments(lb, torch), m64)
            del lb
    out.append({"ablation": "FP32 storage: shift density and sum precision, error vs FP64 "
                            "after %d steps" % n, "lattice": [al, al], "errors": shift})
    log("ablations: %s" % out[-1])
    return out


def run_variants(args, torch) -> list:
    """The split stages with each alternative kernel on the headline lattice:
    propagate direct / staged through LDS / with 16-byte accesses (FP64 and
    shifted FP32), collide on the vector units / on the FP64 matrix cores.
    --warmup untimed split steps, then --steps timed ones per kernel set
    (HIP events around every stage on the kernels' stream); one record per
    set.  For the design comparison and its kernel trace."""
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    lx, ly = args.lx, args.ly
    sites = lx * ly
    fields = workload.rt_fields(lx, ly, seed=workload.config_seed(2))[:4]
    out = []
    for prec in ("fp64", "fp32s"):
        for kernel in ("split", "split_lds", "split_wide", "split_mfma"):
            if kernel == "split_mfma" and prec != "fp64":
                continue
            lb = LB(lx, ly, *fields, precision=prec, layout=args.layout, kernel=kernel)
            time_split_kernels(lb, args.warmup, torch)
            sp = time_split_kernels(lb, args.steps, torch)
            bps = bytes_per_site(prec)
            rec = {"kernel": kernel, "precision": prec, "lattice": [lx, ly],
                   "steps": args.steps, "layout": args.layout}
            for stage in ("propagate", "collide"):
                rec[stage + "_ms"] = round(sp[stage] * 1e3, 5)
                rec[stage + "_GB/s"] = round(bps * sites / sp[stage] / 1e9, 1)
            rec["step_MLUPS"] = round(mlups(sites, sum(sp.values())), 1)
            out.append(rec)
            log("variants: %s" % rec)
            del lb
            torch.cuda.empty_cache()
    return out


def run_forms(args, torch) -> list:
    """Only the fused step of each named storage form on the headline lattice:
    --warmup untimed steps, then --steps timed ones (HIP events on the
    kernels' stream); one record per form.  For counter and trace profiles."""
    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    lx, ly = args.lx, args.ly
    fields = workload.rt_fields(lx, ly, seed=workload.config_seed(2))[:4]
    out = []
    for prec in args.forms:
        lb = LB(lx, ly, *fields, precision=prec, layout=args.layout)
        lb.step(args.warmup)
        t = time_steps(lb, args.steps, torch)
        gbs = bytes_per_site(prec) * lx * ly / (t / args.steps) / 1e9
        out.append({"form": prec, "lattice": [lx, ly], "steps": args.steps,
                    "ms_per_step": round(t / args.steps * 1e3, 5),
                    "MLUPS": round(mlups(lx * ly * args.steps, t), 1), "GB/s": round(gbs, 1),
                    "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
        log("forms: %s" % out[-1])
        del lb
        torch.cuda.empty_cache()
    return out


def cpu_optimised(lx: int, ly: int, fields, steps: int = 40) -> dict:
    """The vectorised multicore CPU implementation of the same step (a
    stronger CPU comparison than the oracle), on this host's cores."""
    import cpu_step
    import oracle

    threads = cpu_threads()
    cpu_step.set_threads(threads)
    lat = cpu_step.CpuLattice(lx, ly, oracle.init_feq(*fields))
    lat.step(2)
    t0 = time.perf_counter()
    lat.step(steps)
    dt = time.perf_counter() - t0
    return {"value": round(mlups(lx * ly * steps, dt), 2), "unit": "MLUPS", "cores": threads,
            "kind": "optimised CPU step (AVX-512)" if cpu_step.host_has_avx512()
            else "optimised CPU step (AVX2)",
            "sample": "%d steps of the %dx%d FP64 RT lattice after 2 warm-up steps (%.2f s), %s"
                      % (steps, lx, ly, dt, cpu_model())}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--lx", type=int, default=1920)
    ap.add_argument("--ly", type=int, default=2048)
    ap.add_argument("--layout", default="column", choices=["soa", "column"])
    ap.add_argument("--split-steps", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=50,
                    help="steps of the full-tape adjoint timing on the headline lattice")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the headline fused FP64 step (for profiling)")
    ap.add_argument("--workloads", nargs="*", default=None,
                    choices=["parity", "fp32", "adjoint", "production"],
                    help="run these workloads (all four when none is named) and print one "
                         "JSON record each instead of the headline line")
    ap.add_argument("--rt-run", action="store_true",
                    help="a long Rayleigh-Taylor run with in-situ observables (one JSON record)")
    ap.add_argument("--rt-steps", type=int, default=20000)
    ap.add_argument("--rt-every", type=int, default=500)
    ap.add_argument("--ablations", action="store_true",
                    help="run the layout / collision / stability / FP32-shift ablations")
    ap.add_argument("--stability-steps", type=int, default=5000)
    ap.add_argument("--fp32-steps", type=int, default=2000,
                    help="steps of the 4096 x 4096 FP32-precision workload")
    ap.add_argument("--production-steps", type=int, default=5000,
                    help="steps of the 8192 x 4096 production workload")
    ap.add_argument("--forms", nargs="+", default=None,
                    choices=["fp64", "fp32l", "fp32c", "fp32s", "fp32s_f32sum"],
                    help="time only the fused step of these storage forms on the headline "
                         "lattice (one JSON record each; for profiles)")
    ap.add_argument("--variants", action="store_true",
                    help="time the split stages with each alternative kernel (LDS-staged and "
                         "16-byte propagate, matrix-core collide)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter scale reference)")
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    from paper_1703_00186_amd import workload
    from paper_1703_00186_amd.lb import LB

    if args.rt_run:
        print(json.dumps(run_rt(args, torch)), flush=True)
        return 0
    if args.variants:
        for rec in run_variants(args, torch):
            print(json.dumps(rec), flush=True)
        if args.copy_calibration:
            copy_calibration(torch)
        return 0
    if args.forms:
        for rec in run_forms(args, torch):
            print(json.dumps(rec), flush=True)
        if args.copy_calibration:
            copy_calibration(torch)
        return 0
    if args.workloads is not None or args.ablations:
        for rec in (run_workloads if args.workloads is not None else run_ablations)(args, torch):
            print(json.dumps(rec), flush=True)
        return 0

    lx, ly = args.lx, args.ly
    sites = lx * ly
    fields = workload.rt_fields(lx, ly, seed=workload.config_seed(2))[:4]
    log("bench: D2Q37 %dx%d, building FP64 lattice" % (lx, ly))
    lb = LB(lx, ly, *fields, layout=args.layout, kernel="fused")
    lb.step(args.warmup)
    t = time_steps(lb, args.steps, torch)
    ms = t / args.steps * 1e3
    value = mlups(sites * args.steps, t)
    achieved = bytes_per_site("fp64") * sites / (t / args.steps) / 1e9
    log("bench: fused FP64 %.4f ms/step, %.1f MLUPS, %.0f GB/s" % (ms, value, achieved))
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "D2Q37 thermal LB, Rayleigh-Taylor %dx%d, FP64, fused "
                               "propagate+bc+collide" % (lx, ly),
                   "lattice": [lx, ly], "tau": 0.7, "g": 1e-4, "t_bottom": 1.5,
                   "t_top": 0.5, "layout": args.layout, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "k_fused<double>",
                     "bytes_per_site": bytes_per_site("fp64")},
    }
    fps = counted_flop_per_site()
    if fps is not None:
        tflops = fps * sites / (t / args.steps) / 1e12
        out["fp64_compute"] = {"flop_per_site_counted": fps, "achieved": round(tflops, 2),
                               "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4)}
    traffic = measured_traffic(lx, ly) if args.layout == "column" else None
    if traffic is not None:
        out["roofline"]["traffic"] = traffic
        out["roofline"]["traffic_unit"] = "bytes per launch"
    if args.copy_calibration:
        copy_calibration(torch)
    if not args.no_extras:
        lb.set_params(kernel="split")
        sp = time_split_kernels(lb, args.split_steps, torch)
        tot = sum(sp.values())
        out["split_fp64"] = {
            k: {"ms": round(v * 1e3, 5), "MLUPS": round(mlups(sites, v), 1)} for k, v in sp.items()}
        out["split_fp64"]["propagate"]["GB/s"] = round(bytes_per_site() * sites / sp["propagate"] / 1e9, 1)
        out["split_fp64"]["collide"]["GB/s"] = round(bytes_per_site() * sites / sp["collide"] / 1e9, 1)
        out["split_fp64"]["step"] = {"ms": round(tot * 1e3, 5), "MLUPS": round(mlups(sites, tot), 1)}
        log("bench: split FP64 %s" % json.dumps(out["split_fp64"]))
        # the split path advanced the FP64 lattice: reinit it for the adjoint
        lb.reinit(*fields)
        lb.set_params(kernel="fused")
        lb.step(args.warmup)
        out["adjoint_fp64"] = time_adjoint(lb, args.adjoint_steps, torch)
        log("bench: adjoint %s" % json.dumps(out["adjoint_fp64"]))
        del lb
        torch.cuda.empty_cache()
        out.update(fp32_legs(lx, ly, fields, args.layout, value, torch))
        out["precision_4096x4096"] = precision_leg(torch, args.layout)
        out["production_8192x4096"] = production_leg(torch)
    if not args.no_extras:
        # launch-bound small lattice: eager launches vs one graph of 100 steps
        sl, sh = 256, 128
        fsm = workload.rt_fields(sl, sh, seed=workload.config_seed(1))[:4]
        lbs = LB(sl, sh, *fsm)
        lbs.step(20)
        te = time_steps(lbs, 1000, torch)
        graph = lbs.capture(100)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        tg = e0.elapsed_time(e1) / 1e3
        out["small_lattice_256x128"] = {
            "eager_MLUPS": round(mlups(sl * sh * 1000, te), 1),
            "graph_MLUPS": round(mlups(sl * sh * 1000, tg), 1),
            "eager_us_per_step": round(te / 1000 * 1e6, 2),
            "graph_us_per_step": round(tg / 1000 * 1e6, 2)}
        log("bench: 256x128 eager %.2f us/step, graph %.2f us/step" % (te / 1000 * 1e6,
                                                                     tg / 1000 * 1e6))
        del graph, lbs
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle (%d steps)" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(lx, ly, fields, args.cpu_steps)
        log("bench: timing the optimised CPU step")
        out["cpu_optimised"] = cpu_optimised(lx, ly, fields)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
