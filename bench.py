"""Benchmark of the D2Q13 step on one MI355X.

Default workload: the 4096 x 4096 periodic transverse shear + acoustic wave
(ux = 0.01 sin(2 pi y/L), rho = 1 + 1e-3 cos(2 pi x/L), uniform T), FP32
deviation form, one lattice update per node per step.  A "step" is one pass of
the hot path over the grid (gather along the 13 velocities, collide, store);
FP64 diagnostics (conservation sums, Nusselt, symmetry) run once per
--diag-every steps inside the timed region.  The plain FP64 GPU step is timed
on the same workload for the precision comparison.

Prints ONE JSON line (rank 0).  `value` is MLUPS (million lattice updates per
second) over the timed region with the state resident in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BENCH_TILE = (64, 8)          # tile shape of the step kernel timed here
GRAPH_K = 100                 # steps per captured HIP graph
BYTES_PER_LU = {0: 208, 1: 104}  # 13 loads + 13 stores of populations, FP64 / FP32
HBM_PEAK_GBPS = 8000.0        # MI355X HBM3E
METRIC = "MLUPS and % of HBM roofline, FP32/batched vs plain FP64 GPU at stated error"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_4096_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1401_0188_amd", "csrc", "lbm13_kernels.hip")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(precision):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get("fp32" if precision == 1 else "fp64")
    if not rec or t.get("kernel_source_sha") != kernel_sha():
        return None
    return rec.get("bytes_per_launch")


def run_form(precision, n, steps, warmup, diag_every, tile, graph_k):
    import torch

    from paper_1401_0188_amd import lbm13, workloads
    stream = torch.cuda.current_stream()
    lat = lbm13.Lattice(n, n, precision, stream=stream)
    lat.set_tile(*tile)
    lat.set_params()
    lat.init_moments(*workloads.shear_acoustic(n))
    if graph_k:
        lat.use_graph(graph_k)
    lat.step(warmup)
    d0 = lat.diagnostics()
    torch.cuda.synchronize()
    chunk = diag_every if diag_every > 0 else steps
    ev = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.step(k)
        b.record(stream)
        ev.append((a, b, k))
        if diag_every > 0:
            lat.diagnostics()  # FP64 reductions (synchronises)
        done += k
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = sum(a.elapsed_time(b) for a, b, _ in ev)
    d1 = lat.diagnostics()
    nodes = n * n
    drift = abs(d1["sum_rho"] - d0["sum_rho"]) / d0["sum_rho"]
    lat.destroy()
    del lat
    torch.cuda.empty_cache()
    return dict(wall_s=wall, ms_per_step=wall * 1e3 / steps, kernel_ms_per_launch=kern_ms / steps,
                mlups=nodes * steps / wall / 1e6, kernel_mlups=nodes / (kern_ms / steps * 1e-3) / 1e6,
                mass_drift=drift, nodes=nodes)


def copy_bandwidth():
    import torch
    nbytes = 2 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(n, budget_s):
    """The FP64 CPU oracle on the same workload, for about budget_s seconds."""
    import oracle
    from paper_1401_0188_amd import workloads
    p = oracle.params()
    f = oracle.init(*workloads.shear_acoustic(n), p)
    s = oracle.sides()
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = oracle.step(f, p, s)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / steps * (steps + 1) > 2.5 * budget_s:
            break
    return dict(value=round(n * n * steps / el / 1e6, 3), unit="MLUPS", cores=oracle.num_threads(), kind="oracle",
                sample="%d steps of the %dx%d periodic shear + acoustic wave, FP64 oracle, %.1f s" % (steps, n, n, el))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--diag-every", type=int, default=1000)
    ap.add_argument("--fp64-steps", type=int, default=-1, help="steps of the plain FP64 form (default steps/2)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-graph", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the domain would shard as y-slabs with 2-row halos; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1401_0188_amd import lbm13
    lbm13.lib()

    n = args.size
    graph_k = 0 if args.no_graph else GRAPH_K
    log("device copy bandwidth")
    copy_gbps = copy_bandwidth()
    log("fp32-deviation %dx%d: %d warmup + %d steps" % (n, n, args.warmup, args.steps))
    r32 = run_form(lbm13.FP32_DEV, n, args.steps, args.warmup, args.diag_every, BENCH_TILE, graph_k)
    log("fp32: %.1f MLUPS, kernel %.4f ms" % (r32["mlups"], r32["kernel_ms_per_launch"]))
    fp64_steps = args.fp64_steps if args.fp64_steps >= 0 else max(1, args.steps // 2)
    log("fp64 %dx%d: %d steps" % (n, n, fp64_steps))
    r64 = run_form(lbm13.FP64, n, fp64_steps, max(1, args.warmup // 2), args.diag_every, BENCH_TILE, graph_k)
    log("fp64: %.1f MLUPS, kernel %.4f ms" % (r64["mlups"], r64["kernel_ms_per_launch"]))

    def roof(r, prec):
        achieved = BYTES_PER_LU[prec] * r["nodes"] / (r["kernel_ms_per_launch"] * 1e-3) / 1e9
        t = measured_traffic(prec)
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": t}

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) for about %.0f s" % args.cpu_seconds)
        cpu = cpu_baseline(n, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "periodic %dx%d transverse shear + acoustic wave" % (n, n), "nx": n, "ny": n,
                   "form": "fp32-deviation", "tile": list(BENCH_TILE), "graph_steps": graph_k,
                   "diag_every": args.diag_every},
        "roofline": roof(r32, 1),
        "cpu_baseline": cpu,
        "fp64": {"value": round(r64["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r64["ms_per_step"], 5),
                 "roofline": roof(r64, 0), "steps": fp64_steps},
        "speedup_vs_fp64": round(r32["mlups"] / r64["mlups"], 3),
        "kernel_ms_per_launch": {"fp32": round(r32["kernel_ms_per_launch"], 5),
                                 "fp64": round(r64["kernel_ms_per_launch"], 5)},
        "copy_GBps": round(copy_gbps, 1),
        "frac_of_copy": round(roof(r32, 1)["achieved"] / copy_gbps, 4),
        "mass_drift": {"fp32": r32["mass_drift"], "fp64": r64["mass_drift"]},
        "kernel_source_sha": kernel_sha(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
