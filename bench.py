"""Benchmark of the D2Q37 step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the Rayleigh-Taylor lattice of the paper's Table 1, 1920 x 2048
sites (Sec. 5), FP64, tau 0.7, g = 1e-4 along -y, walls at T = 1.5 / 0.5.  A
step is one pass of the whole hot path: periodic halo, propagate, bc and
collide, run as the fused kernel (one launch per step).  Inputs are resident
in HBM before timing starts.  Printed: one JSON line with the headline FP64
MLUPS, the roofline of the fused kernel, the split kernels, the FP32-shifted
step, and the CPU oracle timed on a bounded sample on this host.
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
    """Algorithmic HBM bytes of one site update: read and write 37 populations."""
    return 2 * Q * (8 if precision == "fp64" else 4)


def mlups(sites: int, seconds: float) -> float:
    return sites / seconds / 1e6


PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_SUMMARY = os.path.join(PROFILES, "k_fused_fp64_rt1920x2048_hbm_traffic.md")
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


def measured_traffic(lx: int, ly: int):
    """HBM bytes per fused launch from the committed counter summary, or None
    when the summary is missing, is for another lattice, or the kernel
    sources changed since the counters were taken."""
    try:
        vals = {}
        for line in open(TRAFFIC_SUMMARY):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip()
        if vals.get("source_sha256_16") != kernel_source_hash():
            return None
        if vals.get("lattice") != "%dx%d" % (lx, ly):
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
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
    max|ref|; u as max|du| over max(max|u|, sqrt(min T)) (the flow or thermal
    speed, whichever is larger; rho u is a cancelling sum of thermal-speed
    terms)."""
    import numpy as np
    m = [np.asarray(a, dtype=np.float64) for a in m]
    r = [np.asarray(a, dtype=np.float64) for a in ref]
    du = np.hypot(m[1] - r[1], m[2] - r[2])
    scale_u = max(float(np.hypot(r[1], r[2]).max()), float(np.sqrt(r[3].min())))
    return {"rho": float(np.abs(m[0] - r[0]).max() / np.abs(r[0]).max()),
            "u": float(du.max() / scale_u),
            "T": float(np.abs(m[3] - r[3]).max() / np.abs(r[3]).max())}


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


def cpu_baseline(lx: int, ly: int, fields, steps: int) -> dict:
    import oracle

    threads = min(16, len(os.sched_getaffinity(0)))
    oracle.set_threads(threads)
    P = oracle.Params(tau=0.7, gx=0.0, gy=-1e-4, t_bottom=1.5, t_top=0.5)
    f = oracle.init_feq(*fields)
    f = oracle.run(f, P, 1)  # warm-up step
    t0 = time.perf_counter()
    oracle.run(f, P, steps)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(mlups(lx * ly * steps, dt), 4), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d steps of the %dx%d FP64 RT lattice after 1 warm-up step (%.1f s), %s"
                      % (steps, lx, ly, dt, cpu)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--lx", type=int, default=1920)
    ap.add_argument("--ly", type=int, default=2048)
    ap.add_argument("--layout", default="column", choices=["soa", "column"])
    ap.add_argument("--split-steps", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the headline fused FP64 step (for profiling)")
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
        # the split path advanced the FP64 lattice: rerun it for the comparison
        lb.reinit(*fields)
        lb.set_params(kernel="fused")
        lb.step(args.warmup + args.steps)
        m64 = host_moments(lb, torch)
        del lb
        torch.cuda.empty_cache()
        for key, prec in (("fp32_shifted", "fp32s"), ("fp32_shifted_f32sum", "fp32s_f32sum")):
            lb32 = LB(lx, ly, *fields, precision=prec, layout=args.layout, kernel="fused")
            lb32.step(args.warmup)
            t32 = time_steps(lb32, args.steps, torch)
            v32 = mlups(sites * args.steps, t32)
            errs = field_errors(host_moments(lb32, torch), m64)
            out[key] = {
                "MLUPS": round(v32, 2), "ms_per_step": round(t32 / args.steps * 1e3, 5),
                "ratio_vs_fp64": round(v32 / value, 3),
                "GB/s": round(bytes_per_site("fp32") * sites / (t32 / args.steps) / 1e9, 1),
                "error_vs_fp64_gpu": {k: float("%.3g" % v) for k, v in errs.items()},
                "error_after_steps": args.warmup + args.steps}
            log("bench: fused %s %.1f MLUPS (x%.2f), errors %s" % (prec, v32, v32 / value, errs))
            del lb32
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle (%d steps)" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(lx, ly, fields, args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
