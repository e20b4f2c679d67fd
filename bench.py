"""Benchmark of the D2Q13 step on one MI355X.

Default workload: the 4096 x 4096 periodic transverse shear + acoustic wave
(ux = 0.01 sin(2 pi y/L), rho = 1 + 1e-3 cos(2 pi x/L), uniform T), FP32
deviation form, one lattice update per node per step.  A "step" is one pass of
the hot path over the grid (gather along the 13 velocities, collide, store);
FP64 diagnostics (conservation sums, Nusselt, symmetry) run once per
--diag-every steps inside the timed region.  The FP64 form (in its own
autotuned launch) and the plain FP64 step (one step per launch) are timed on
the same workload for the precision comparison.  Other workloads
(--workload): cavities64 and channels128 (batched FP32 forms against the same
domains as sequential plain FP64 contexts), wave32 and cavity256 (the small,
cache-resident configurations, whole runs checked against the oracle).

Prints ONE JSON line (rank 0).  `value` is MLUPS (million lattice updates per
second) over the timed region with the state resident in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Starting launch configuration of each precision (the default run lets the
# library's autotuner replace it on the device; on MI355X it has kept these
# three-step shapes); its single-step tile is the one of the plain single-step
# FP64 comparison.
BENCH_CONFIG = {1: dict(spl=3, fused_tile=(64, 16), tile=(64, 8), interior_kernel=True),
                0: dict(spl=3, fused_tile=(32, 16), tile=(64, 8), interior_kernel=True)}
BENCH_TILE = BENCH_CONFIG[1]["tile"]
GRAPH_K = 120                 # steps per captured HIP graph (a multiple of 2 and 3: whole multi-step launches)
SETTLE_STEPS = 240            # set-up: steps of the chosen launches run before the state restarts
ACCURACY_STEPS = 10000        # FP32 against FP64 on the GPU after this many steps (the stated FP32 bound's horizon)
BYTES_PER_LU = {0: 208, 1: 104}  # 13 loads + 13 stores of populations, FP64 / FP32
HBM_PEAK_GBPS = 8000.0        # MI355X HBM3E
# Vector ALU of the MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, one wave64
# VALU instruction per SIMD every 4 cycles.  FMA = 2 flops: 78.6 TFLOP/s in FP64
# (the published vector peak) and in unpacked FP32 (the published 157.3 counts
# packed FP32 instructions, which the library's build excludes).
CLOCK_GHZ = 2.4
SIMDS = 256 * 4
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * CLOCK_GHZ / 1e3
# Floating-point operations of one collision (each add, subtract, multiply and
# the reciprocal of rho counted once): the pair sums and differences, the 13
# moments, the equilibria, the relaxation and the inverse of the pair-symmetric
# form; +16 with the body force and energy-source terms.
FLOPS_PER_LU = 177
METRIC = "MLUPS and % of HBM roofline, FP32/batched vs plain FP64 GPU at stated error"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_4096_traffic.json")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step3_batched_traffic.json")
# the sources that decide what the timed kernels do: the kernels, the descriptor
# layout and the host code that builds the tile tables and launches
KERNEL_SRC = [os.path.join(ROOT, "paper_1401_0188_amd", "csrc", f)
              for f in ("lbm13_kernels.hip", "lbm13_device.h", "lbm13_capi.cpp")]


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_sha():
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def launch_kernels(launch):
    """The part of a launch configuration that decides which kernels run."""
    spl = launch["steps_per_launch"]
    if spl == 1:
        return (1, tuple(launch["tile"]))
    if spl == 2:  # two steps take mode 2 as 1
        return (2, tuple(launch["fused_tile"]), bool(launch["interior_kernel"]))
    return (3, tuple(launch["fused_tile"]), int(launch["interior_kernel"]))


def measured_record(key, launch, path=None):
    """The committed rocprofv3 counter record of the timed form (HBM bytes per
    launch, VALU instructions per launch), if it was taken on the current
    kernel source with the same kernels (the configuration the default run
    chose, or one of the alternates measured beside it); else None."""
    try:
        with open(path or TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_sha():
        return None
    for rec in [t.get(key)] + t.get("alternates", {}).get(key, []):
        if rec and launch_kernels(rec["launch"]) == launch_kernels(launch):
            return dict(rec, file=os.path.relpath(path or TRAFFIC_FILE, ROOT))
    return None


def measured_traffic(key, launch, path=None):
    """HBM bytes per launch of the timed form (see measured_record), or None."""
    rec = measured_record(key, launch, path)
    return rec.get("bytes_per_launch") if rec else None


def measured_counters(key, launch, path=None):
    rec = measured_record(key, launch, path)
    if not rec or not rec.get("SQ_INSTS_VALU"):
        return None
    return {"SQ_INSTS_VALU": rec["SQ_INSTS_VALU"], "file": rec["file"]}


def next_chunk(done, steps, diag_every):
    """Steps of the next timed chunk and whether FP64 diagnostics follow it:
    chunks end where the count of timed steps reaches a multiple of diag_every
    (diagnostics then run, at exactly their stated rate) or at the end."""
    if diag_every <= 0:
        return steps - done, False
    k = min(diag_every - done % diag_every, steps - done)
    return k, (done + k) % diag_every == 0


def graph_length(graph_k, steps, spl):
    """Steps per captured graph: graph_k, or for shorter runs the largest
    multiple of 2 spl that fits (an even number of whole launches); 0: none."""
    if not graph_k:
        return 0
    if steps >= graph_k:
        return graph_k
    unit = 2 * spl
    return steps // unit * unit if steps >= unit else 0


def settle_steps(gk, spl):
    """Set-up steps before timing: SETTLE_STEPS rounded up to whole graph
    replays (or whole launches without a graph)."""
    unit = gk if gk else spl
    return max(unit, -(-SETTLE_STEPS // unit) * unit)


def run_form(precision, n, steps, warmup, diag_every, cfg, graph_k, tune_steps=0):
    """Time one form on the n x n wave.  cfg fixes the launch configuration;
    tune_steps > 0 lets the library's autotuner pick it on this device instead
    (from a fresh copy of the state) and the choice is returned as `launch`."""
    import torch

    from paper_1401_0188_amd import lbm13, workloads
    stream = torch.cuda.current_stream()
    lat = lbm13.Lattice(n, n, precision, stream=stream)
    lat.set_tile(*cfg["tile"])
    lat.set_fused_tile(*cfg["fused_tile"])
    lat.set_steps_per_launch(cfg["spl"])
    if "interior_kernel" in cfg:
        lat.set_interior_kernel(cfg["interior_kernel"])
    lat.set_params()
    lat.init_moments(*workloads.shear_acoustic(n))
    # the initial state, kept on the device: each restart below is a device copy,
    # so the GPU is not left idle (and its clock low) while the host re-uploads
    # the fields just before the timed region
    initial = lat.save()
    if tune_steps > 0:
        lat.autotune(tune_steps)
        lat.load(initial)
    launch = lat.launch_config()
    spl = launch["steps_per_launch"]
    gk = graph_length(graph_k, steps, spl)
    if gk:
        lat.use_graph(gk)  # an even number of launches, so one capture serves
    # set-up, like the autotuning: run the chosen launches for a few hundred steps
    # (a graph's first replay uploads it, and the GPU's clock rises under sustained
    # load over tens of milliseconds), then start again from the initial state
    setup = settle_steps(gk, spl)
    lat.step(setup)
    lat.load(initial)
    del initial
    lat.step(warmup)
    d0 = lat.diagnostics()
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k, diag_now = next_chunk(done, steps, diag_every)
        # whole launches of the chosen configuration, timed apart from a remainder
        # of shorter launches, so the per-launch time is that of the chosen kernel
        for part in (k // spl * spl, k % spl):
            if part == 0:
                continue
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.step(part)
            b.record(stream)
            ev.append((a, b, part, part % spl == 0))
        if diag_now:
            lat.diagnostics()  # FP64 reductions (synchronises)
        done += k
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = sum(a.elapsed_time(b) for a, b, _, _ in ev)
    whole = [(a.elapsed_time(b), k) for a, b, k, w in ev if w]
    per_launch = (sum(t for t, _ in whole) / (sum(k for _, k in whole) / spl)) if whole else kern_ms / steps * spl
    d1 = lat.diagnostics()
    nodes = n * n
    drift = abs(d1["sum_rho"] - d0["sum_rho"]) / d0["sum_rho"]
    lat.destroy()
    del lat
    torch.cuda.empty_cache()
    return dict(wall_s=wall, ms_per_step=wall * 1e3 / steps, kernel_ms_per_launch=per_launch,
                mlups=nodes * steps / wall / 1e6, kernel_mlups=nodes / (kern_ms / steps * 1e-3) / 1e6,
                mass_drift=drift, nodes=nodes, spl=spl, launch=launch, graph_steps=gk, setup_steps=setup)


def cavity_specs(count=64, seed=4):
    """Heated cavities of uneven sizes (side U{64..512}), Ra log-uniform in
    [1e3, 1e6], Pr U[0.5, 7] (one seeded draw per cavity), each with its own
    parameter set and feasible forcing (dT within the cap of
    workloads.cavity_dT_cap; Ra clamped and recorded when needed)."""
    from paper_1401_0188_amd import lbm13, workloads
    out = []
    for i, c in enumerate(workloads.cavity_batch(count=count, seed=seed)):
        kw = workloads.cavity_parameter_set(c["Pr"])
        st, d = lbm13.derive(**kw)
        cf = workloads.cavity_forcing(c["nx"], c["Ra"], c["Pr"], d["nu"], d["kappa"],
                                      dT_max=workloads.cavity_dT_cap(c["nx"]), cs=d["cs2"] ** 0.5)
        E0 = kw["E0"]
        out.append(dict(nx=c["nx"], ny=c["ny"], kw=dict(kw, g=(0.0, -cf["g"])),
                        sides=((2, 2, 1, 1), (0, 0, 0, 0), (E0 + cf["dT"] / 2, E0 - cf["dT"] / 2, 0, 0)),
                        fields=("cavity", dict(n=c["nx"], T0=E0, dT=cf["dT"], seed=seed * 1000 + i)),
                        info=dict(Pr=c["Pr"], Ra=c["Ra"], Ra_eff=cf["Ra"], clamped=cf["clamped"], dT=cf["dT"])))
    return out


def channel_specs(count=128, seed=5):
    """Couette (even index) and Poiseuille (odd index) channels, periodic along
    y, temperature walls E0 +- dT (sec. 7), viscosity from the speed limit."""
    from paper_1401_0188_amd import workloads
    out = []
    E0 = -2.0
    for c in workloads.channel_batch(count=count, seed=seed):
        if c["kind"] == "poiseuille":
            cv = workloads.channel_viscosity(c["nx"], c["F"])
            kw = dict(s_XX=workloads.s_xx_for_nu(cv["nu"]), F0=(0.0, cv["F"]), E0=E0)
            u_w = 0.0
        else:
            cv = dict(nu=0.0625, F=0.0, clamped=False)
            kw = dict(s_XX=workloads.s_xx_for_nu(0.0625), E0=E0)
            u_w = c["U"]
        out.append(dict(nx=c["nx"], ny=c["ny"], kw=kw,
                        sides=((2, 2, 0, 0), (u_w, 0, 0, 0), (E0 + c["dT"], E0 - c["dT"], 0, 0)),
                        fields=("rest", dict(nx=c["nx"], ny=c["ny"], T0=E0)),
                        info=dict(kind=c["kind"], nu=cv["nu"], clamped=cv["clamped"])))
    return out


def spec_fields(spec):
    from paper_1401_0188_amd import workloads
    kind, a = spec["fields"]
    if kind == "cavity":
        return workloads.cavity_fields(a["n"], T0=a["T0"], dT=a["dT"], seed=a["seed"])
    return workloads.rest_fields(a["nx"], a["ny"], a["T0"])


def build_batch(specs, precision):
    from paper_1401_0188_amd import lbm13
    b = lbm13.Batch([(s["nx"], s["ny"]) for s in specs], precision)
    for i, s in enumerate(specs):
        b.set_params(i, sides=lbm13.make_sides(*s["sides"]), **s["kw"])
        b.init_moments(i, *spec_fields(s))
    return b


def run_batch(specs, precision, steps, warmup, diag_every, graph_k, autotune=True, launch=None, tune_steps=40):
    """`launch`: a fixed launch configuration (a `launch` object of an earlier run) instead of autotuning."""
    import torch
    b = build_batch(specs, precision)
    cfg = dict(launch) if launch else None
    if autotune or cfg:
        if not cfg:
            b.autotune(tune_steps)
            cfg = b.launch_config()
            b.destroy()
            b = build_batch(specs, precision)  # fresh state after tuning
        b.set_tile(*cfg["tile"])
        b.set_fused_tile(*cfg["fused_tile"])
        b.set_interior_kernel(cfg["interior_kernel"])
        b.set_steps_per_launch(cfg["steps_per_launch"])
    if graph_k:
        b.use_graph(graph_k)
    # set-up as for one domain: run the chosen launches, then restore every domain
    saved = [b.save(i) for i in range(b.count)]
    setup = settle_steps(graph_k, cfg["steps_per_launch"] if cfg else 1)
    b.step(setup)
    for i, blob in enumerate(saved):
        b.load(i, blob)
    del saved
    b.step(warmup)
    b.diagnostics()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k, diag_now = next_chunk(done, steps, diag_every)
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        b.step(k)
        e.record(stream)
        ev.append((a, e, k))
        if diag_now:
            b.diagnostics()
        done += k
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = sum(a.elapsed_time(e) for a, e, _ in ev)
    diag = b.diagnostics()
    nodes = b.nodes()
    b.destroy()
    torch.cuda.empty_cache()
    spl = cfg["steps_per_launch"] if cfg else 1
    return dict(wall_s=wall, ms_per_step=wall * 1e3 / steps, kernel_ms_per_launch=kern_ms / steps * spl,
                mlups=nodes * steps / wall / 1e6, nodes=nodes, cfg=cfg, spl=spl, diag=diag, setup_steps=setup)


def run_sequential_fp64(specs, steps):
    """The same domains as separate plain FP64 contexts, stepped one after another."""
    import torch
    from paper_1401_0188_amd import lbm13
    lats = []
    for s in specs:
        lat = lbm13.Lattice(s["nx"], s["ny"], lbm13.FP64)
        lat.set_params(sides=lbm13.make_sides(*s["sides"]), **s["kw"])
        lat.init_moments(*spec_fields(s))
        lats.append(lat)
    for lat in lats:
        lat.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for lat in lats:
            lat.step(1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nodes = sum(s["nx"] * s["ny"] for s in specs)
    for lat in lats:
        lat.destroy()
    del lats
    torch.cuda.empty_cache()
    return dict(wall_s=wall, ms_per_step=wall * 1e3 / steps, mlups=nodes * steps / wall / 1e6, nodes=nodes)


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


def host_cpu():
    """Model name of the host CPU the oracle runs on."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def one_thread(rec, step, nodes, budget_s):
    """Adds to an oracle baseline record its rate on one host thread: `step`
    advances the oracle by one step, timed for about budget_s (at least once)."""
    import oracle
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        steps, t0 = 0, time.perf_counter()
        while True:
            step()
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget_s or el / steps * (steps + 1) > 2 * budget_s:
                break
    finally:
        oracle.set_num_threads(threads)
    rec["value_1_thread"] = round(nodes * steps / el / 1e6, 3)
    rec["sample_1_thread"] = "%d steps, %.1f s" % (steps, el)
    rec["cpu"] = host_cpu()
    return rec


def cpu_baseline(n, budget_s):
    """The FP64 CPU oracle on the same workload, for about budget_s seconds.
    Returns the baseline record, the number of steps and the oracle's moments
    (rho, ux, uy, T) after them (the reference of the error report)."""
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
    rec = dict(value=round(n * n * steps / el / 1e6, 3), unit="MLUPS", cores=oracle.num_threads(), kind="oracle",
               sample="%d steps of the %dx%d periodic shear + acoustic wave, FP64 oracle, %.1f s" % (steps, n, n, el))
    om = oracle.moments(f, p)
    state = [f]

    def advance():
        state[0] = oracle.step(state[0], p, s)
    one_thread(rec, advance, n * n, budget_s / 2)
    del f, state
    return rec, steps, om


def final_moments(precision, n, launch, steps, graph_k):
    """Moments (rho, ux, uy, T) on the host after `steps` steps of the wave in
    the given launch configuration (outside any timed region)."""
    import torch

    from paper_1401_0188_amd import lbm13, workloads
    lat = lbm13.Lattice(n, n, precision)
    lat.set_tile(*launch["tile"])
    lat.set_fused_tile(*launch["fused_tile"])
    lat.set_steps_per_launch(launch["steps_per_launch"])
    lat.set_interior_kernel(launch["interior_kernel"])
    lat.set_params()
    lat.init_moments(*workloads.shear_acoustic(n))
    if graph_k and steps >= graph_k:
        lat.use_graph(graph_k)
    lat.step(steps)
    m = [t.cpu().numpy() for t in lat.moments()]
    lat.destroy()
    del lat
    torch.cuda.empty_cache()
    return m


FP32_MEASURE = "max absolute error, lattice units (rho0 = 1, cs^2 = A/52 ~ 1)"
FP64_MEASURE = "max error over the field's max magnitude for rho and T, max absolute error for u"


def moment_errors(got, ref, precision):
    """Errors of (rho, ux, uy, T) against a reference, in the measure of the stated
    bound of the precision: FP32 <= 1e-5 as the max absolute error in lattice
    units (T's zero is set by the free parameter E0, so an error relative to
    max |T| would depend on that choice); FP64 <= 1e-12 relative to the field's
    max magnitude for rho and T, absolute for u.  The GPU parity tests use the
    same measures."""
    import numpy as np
    d = [float(np.abs(got[k] - ref[k]).max()) for k in range(4)]
    if precision == 0:
        return {"rho": d[0] / float(np.abs(ref[0]).max()), "u": max(d[1], d[2]),
                "T": d[3] / float(np.abs(ref[3]).max())}
    return {"rho": d[0], "u": max(d[1], d[2]), "T": d[3]}


def roofline(nodes, kernel_ms, precision, traffic=None, spl=1, counters=None, sourced=False):
    """Roofline of one launch that advances every node by spl steps.

    HBM: the least a launch must move is one read and one write of the state,
    26 populations per node (104 B FP32, 208 B FP64) whatever spl; `achieved`
    is those bytes over the launch's average duration.  ALU: the collisions'
    floating-point operations (FLOPS_PER_LU per update, spl updates per node)
    over the same time, against the unpacked vector peak.  `bound` is the
    ceiling whose lower bound on the launch time is larger (HBM for every form
    here: about 6 flop/B against a machine balance near 10).  `traffic` is the
    HBM bytes a launch moved (rocprofv3 FETCH_SIZE + WRITE_SIZE); `valu_issue`
    the measured VALU instruction issue over the issue peak of the 1024 SIMDs
    at 2.4 GHz (rocprofv3 SQ_INSTS_VALU), the resource that limits the
    multi-step kernels in practice."""
    t = kernel_ms * 1e-3
    hbm_bytes = BYTES_PER_LU[precision] * nodes
    flops = (FLOPS_PER_LU + (16 if sourced else 0)) * nodes * spl
    hbm = hbm_bytes / t / 1e9
    alu = flops / t / 1e12
    t_hbm, t_alu = hbm_bytes / (HBM_PEAK_GBPS * 1e9), flops / (ALU_PEAK_TFLOPS * 1e12)
    out = {"bound": "hbm" if t_hbm >= t_alu else "alu", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBPS,
           "unit": "GB/s", "frac": round(hbm / HBM_PEAK_GBPS, 4), "traffic": traffic,
           "steps_per_launch": spl, "bytes_per_launch": hbm_bytes,
           "alu": {"achieved": round(alu, 2), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                   "frac": round(alu / ALU_PEAK_TFLOPS, 4), "flops_per_update": flops // (nodes * spl)}}
    if out["bound"] == "alu":
        out.update(achieved=out["alu"]["achieved"], peak=out["alu"]["peak"], unit="TFLOP/s",
                   frac=out["alu"]["frac"])
    if traffic:
        out["traffic_GBps"] = round(traffic / t / 1e9, 1)
        out["traffic_over_bytes"] = round(traffic / hbm_bytes, 3)
    if counters and counters.get("SQ_INSTS_VALU"):
        cap = SIMDS * CLOCK_GHZ * 1e9 * t / 4.0
        out["valu_issue"] = {"frac": round(counters["SQ_INSTS_VALU"] / cap, 4), "clock_GHz": CLOCK_GHZ,
                             "lane_ops_per_update": round(counters["SQ_INSTS_VALU"] * 64 / (nodes * spl), 1),
                             "source": "rocprofv3 SQ_INSTS_VALU per launch, " + counters.get("file", "")}
    return out


def cpu_baseline_spec(spec, budget_s):
    """The FP64 oracle on one domain of a batched workload for about budget_s."""
    import numpy as np

    import oracle
    kw = dict(spec["kw"])
    F0 = kw.pop("F0", (0.0, 0.0))
    g = kw.pop("g", (0.0, 0.0))
    p = oracle.params(F0x=F0[0], F0y=F0[1], gx=g[0], gy=g[1], **kw)
    s = oracle.sides(*spec["sides"])
    f = oracle.init(*[np.asarray(a) for a in spec_fields(spec)], p)
    steps, t0 = 0, time.perf_counter()
    while True:
        f = oracle.step(f, p, s)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    n = spec["nx"] * spec["ny"]
    rec = dict(value=round(n * steps / el / 1e6, 3), unit="MLUPS", cores=oracle.num_threads(), kind="oracle",
               sample="%d steps of one %dx%d domain of the workload, FP64 oracle, %.1f s" % (
                   steps, spec["nx"], spec["ny"], el))
    state = [f]

    def advance():
        state[0] = oracle.step(state[0], p, s)
    return one_thread(rec, advance, n, budget_s / 2)


def batch_final_moments(specs, precision, cfg, steps, graph_k):
    """Moments of every domain on the host after `steps` steps of a batch in the
    given launch configuration (outside any timed region)."""
    import torch
    b = build_batch(specs, precision)
    if cfg:
        b.set_tile(*cfg["tile"])
        b.set_fused_tile(*cfg["fused_tile"])
        b.set_interior_kernel(cfg["interior_kernel"])
        b.set_steps_per_launch(cfg["steps_per_launch"])
    if graph_k and steps >= graph_k:
        b.use_graph(graph_k)
    b.step(steps)
    out = [[t.cpu().numpy() for t in b.moments(i)] for i in range(len(specs))]
    b.destroy()
    del b
    torch.cuda.empty_cache()
    return out


def main_batched(args, copy_gbps):
    from paper_1401_0188_amd import lbm13
    specs = cavity_specs() if args.workload == "cavities64" else channel_specs()
    graph_k = 0 if args.no_graph else GRAPH_K
    log("%s: %d domains, batched fp32-deviation, %d steps" % (args.workload, len(specs), args.steps))
    r32 = run_batch(specs, lbm13.FP32_DEV, args.steps, args.warmup, args.diag_every, graph_k, launch=args.launch_fp32,
                    tune_steps=args.tune_steps)
    log("batched fp32: %.1f MLUPS, kernel %.4f ms per launch, config %s" % (r32["mlups"], r32["kernel_ms_per_launch"],
                                                                          r32["cfg"]))
    fp64_steps = args.fp64_steps if args.fp64_steps >= 0 else max(1, args.steps // 4)
    log("sequential plain fp64: %d steps" % fp64_steps)
    r64 = run_sequential_fp64(specs, fp64_steps)
    log("sequential fp64: %.1f MLUPS" % r64["mlups"])
    cpu = None
    if not args.no_cpu:
        big = max(range(len(specs)), key=lambda i: specs[i]["nx"] * specs[i]["ny"])
        cpu = cpu_baseline_spec(specs[big], args.cpu_seconds)
    err = None
    if not args.no_accuracy:
        # stated error, outside the timed region: every domain of the FP32 batch in
        # the timed configuration against the same domains run as an FP64 batch
        log("batched fp32 against fp64 after %d steps" % ACCURACY_STEPS)
        ref = batch_final_moments(specs, lbm13.FP64, dict(r32["cfg"], fused_tile=(32, 16)), ACCURACY_STEPS, graph_k)
        got = batch_final_moments(specs, lbm13.FP32_DEV, r32["cfg"], ACCURACY_STEPS, graph_k)
        per = [moment_errors(g, r, 1) for g, r in zip(got, ref)]
        spread = [float(r[3].max() - r[3].min()) for r in ref]  # the T range of each FP64 domain
        del got, ref
        worst = max(range(len(per)), key=lambda i: max(per[i].values()))
        err = {"bounds": {"fp32": 1e-5}, "measures": {"fp32": FP32_MEASURE}, "fp32_vs_fp64_gpu": {
            "steps": ACCURACY_STEPS, "measure": FP32_MEASURE, "rho": max(e["rho"] for e in per),
            "u": max(e["u"] for e in per), "T": max(e["T"] for e in per), "domains": len(per),
            "domains_over_bound": sum(1 for e in per if max(e.values()) > 1e-5),
            "worst_domain": dict(index=worst, nx=specs[worst]["nx"], ny=specs[worst]["ny"],
                                 E0=specs[worst]["kw"].get("E0", -2.0), T_range=spread[worst],
                                 **per[worst], **specs[worst]["info"])}}
    clamped = sum(1 for s in specs if s["info"].get("clamped"))
    nonfinite = sum(1 for d in r32["diag"] if d["nonfinite"] > 0)
    # FP64 diagnostics of every domain at the end of the timed run (min, median, max), after
    # warm-up + timed steps from rest: early in a run these are start-up transients
    summary = {"steps_from_start": args.warmup + args.steps}
    # (centro-asymmetry only for the cavities: a channel with one moving wall has no such symmetry)
    for k in ("Nu_mean", "asym_rel", "u_max") if args.workload == "cavities64" else ("Nu_mean", "u_max"):
        v = sorted(float(d[k]) for d in r32["diag"])
        summary[k] = {"min": round(v[0], 6), "median": round(v[len(v) // 2], 6), "max": round(v[-1], 6)}
    return {
        "metric": METRIC, "value": round(r32["mlups"], 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r32["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s: %d domains, %d nodes" % (args.workload, len(specs), r32["nodes"]),
                   "form": "fp32-deviation batched, one launch covers every domain", "launch": r32["cfg"],
                   "launch_choice": "fixed" if args.launch_fp32 else "autotuned on this device",
                   "graph_steps": graph_k, "diag_every": args.diag_every, "clamped_domains": clamped,
                   "setup_steps": r32["setup_steps"]},
        "roofline": roofline(r32["nodes"], r32["kernel_ms_per_launch"], 1, spl=r32["spl"], sourced=True,
                             traffic=measured_traffic(args.workload, r32["cfg"], BATCH_TRAFFIC_FILE) if r32["cfg"] else None,
                             counters=measured_counters(args.workload, r32["cfg"], BATCH_TRAFFIC_FILE)
                             if r32["cfg"] else None),
        "cpu_baseline": cpu,
        "fp64_sequential": {"value": round(r64["mlups"], 1), "unit": "MLUPS",
                            "ms_per_step": round(r64["ms_per_step"], 5), "steps": fp64_steps,
                            "launches_per_step": len(specs)},
        "speedup_vs_fp64_sequential": round(r32["mlups"] / r64["mlups"], 3),
        "kernel_ms_per_launch": round(r32["kernel_ms_per_launch"], 5),
        "copy_GBps": round(copy_gbps, 1),
        "domains_nonfinite": nonfinite,
        "diagnostics_at_end": summary,
        "error": err,
        "kernel_source_sha": kernel_sha(),
    }


CAVITY_RA = (1e3, 1e4, 1e5)


def small_cases(workload):
    """The small configurations, whose state fits in the caches: the 32^2
    periodic wave in FP64 (1000 steps, checked against the oracle over the
    whole run) and the 256^2 heated cavity at Ra = 1e3, 1e4, 1e5, Pr = 0.71 in
    FP64 and FP32 (10^5 steps timed; the error against the oracle after 10^4
    steps, the horizon of the stated bounds)."""
    from paper_1401_0188_amd import workloads
    if workload == "wave32":
        return [dict(n=32, steps=1000, check_steps=1000, forms=(0,), fields=workloads.periodic_wave(32),
                     kinds=(0, 0, 0, 0), T_w=(0, 0, 0, 0), kw={}, label="wave",
                     desc="periodic 32x32 nonlinear wave (rho, ux cosine)")]
    from paper_1401_0188_amd import lbm13
    n = 256
    kw0 = dict(workloads.CAVITY_PR071_SET)
    Pr, E0 = kw0["Pr"], kw0["E0"]
    st, d = lbm13.derive(**kw0)
    out = []
    for Ra in CAVITY_RA:
        cf = workloads.cavity_forcing(n, Ra, Pr, d["nu"], d["kappa"], cs=d["cs2"] ** 0.5)
        out.append(dict(n=n, steps=100000, check_steps=10000, forms=(0, 1),
                        fields=workloads.cavity_fields(n, T0=E0, seed=0, dT=cf["dT"]), kinds=(2, 2, 1, 1),
                        T_w=(E0 + cf["dT"] / 2, E0 - cf["dT"] / 2, 0, 0),
                        kw=dict(kw0, g=(0.0, -cf["g"])), label="Ra %.0e" % Ra,
                        Ra=cf["Ra"], dT=cf["dT"], g=cf["g"],
                        desc="heated cavity 256x256, Ra 1e3, 1e4, 1e5, Pr 0.71, hot West / cold East, adiabatic S/N"))
    return out


def cpu_baseline_small(cases):
    """The FP64 CPU oracle over each small case's checked steps: its rate, and
    its moments after them (the reference of the error)."""
    import oracle
    oms, upd, el = [], 0, 0.0
    for c in cases:
        kw = dict(c["kw"])
        g = kw.pop("g", (0.0, 0.0))
        po = oracle.params(gx=g[0], gy=g[1], **kw)
        so = oracle.sides(c["kinds"], (0, 0, 0, 0), c["T_w"])
        t0 = time.perf_counter()
        f = oracle.run(oracle.init(*c["fields"], po), po, so, c["check_steps"])
        el += time.perf_counter() - t0
        upd += c["n"] * c["n"] * c["check_steps"]
        oms.append(oracle.moments(f, po))
    rec = dict(value=round(upd / el / 1e6, 3), unit="MLUPS", cores=oracle.num_threads(), kind="oracle",
               sample="%d steps of each of %d case(s) (%s), %.1f s" % (
                   cases[0]["check_steps"], len(cases), ", ".join(c["label"] for c in cases), el))
    state = [f]

    def advance():
        state[0] = oracle.step(state[0], po, so)
    one_thread(rec, advance, cases[-1]["n"] ** 2, min(3.0, max(el / len(cases), 0.05)))
    return rec, oms


def main_small(args, copy_gbps):
    """A small configuration: each form of each case timed over the case's
    steps (autotuned launch), its error against the oracle after the checked
    steps, the FP64 diagnostics (Nusselt numbers, centro-asymmetry) at the end,
    FP32 against FP64 after the whole run, and the oracle's own rate."""
    import torch

    from paper_1401_0188_amd import lbm13
    cases = small_cases(args.workload)
    log("%s: oracle, %d case(s)" % (args.workload, len(cases)))
    cpu, oms = cpu_baseline_small(cases)
    out, tot = [], {}
    for c, om in zip(cases, oms):
        n, steps = c["n"], c["steps"]
        rec = {"case": c["label"]}
        rec.update({k: round(c[k], 6) for k in ("Ra", "dT", "g") if k in c})
        finals = {}
        for prec in c["forms"]:
            name = "fp64" if prec == 0 else "fp32"
            log("%s %s: %d steps" % (c["label"], name, steps))
            lat = lbm13.Lattice(n, n, prec)
            lat.set_params(sides=lbm13.make_sides(c["kinds"], (0, 0, 0, 0), c["T_w"]), **c["kw"])
            lat.init_moments(*c["fields"])
            lat.autotune(12)
            launch = lat.launch_config()
            if not args.no_graph:
                lat.use_graph(GRAPH_K)
            if c["check_steps"] != steps:
                lat.init_moments(*c["fields"])
                lat.step(c["check_steps"])
                err = moment_errors([t.cpu().numpy() for t in lat.moments()], om, prec)
            lat.init_moments(*c["fields"])
            d0 = lat.diagnostics()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            t1 = time.perf_counter()
            a.record(lat.stream)
            lat.step(steps)
            b.record(lat.stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t1
            gm = [t.cpu().numpy() for t in lat.moments()]
            if c["check_steps"] == steps:
                err = moment_errors(gm, om, prec)
            finals[prec] = gm
            d = lat.diagnostics()
            rec[name] = {"value": round(n * n * steps / wall / 1e6, 1), "unit": "MLUPS",
                         "kernel_ms_per_step": round(a.elapsed_time(b) / steps, 5), "launch": launch,
                         "error_vs_oracle": err,
                         # change of the conserved sums over the run (FP64 reductions; a periodic box keeps them)
                         "drift": {k: float(d[k] - d0[k]) for k in ("sum_rho", "sum_jx", "sum_jy", "sum_E")}}
            if c["kinds"][0] != 0:
                rec[name].update({k: round(float(d[k]), 6) for k in ("Nu_mean", "Nu_west", "Nu_east", "asym_rel",
                                                                     "u_max")})
            t = tot.setdefault(name, [0, 0.0])
            t[0] += n * n * steps
            t[1] += wall
            lat.destroy()
            del lat
            torch.cuda.empty_cache()
        if 0 in finals and 1 in finals:
            rec["fp32_vs_fp64_gpu"] = moment_errors(finals[1], finals[0], 1)
        out.append(rec)
    head = "fp32" if "fp32" in tot else "fp64"
    value = tot[head][0] / tot[head][1] / 1e6
    n, steps, check = cases[0]["n"], cases[0]["steps"], cases[0]["check_steps"]

    def worst(errs):  # the largest error of each quantity over the cases
        return {q: max(e[q] for e in errs) for q in ("rho", "u", "T")}
    error = {"bounds": {"fp64": 1e-12, "fp32": 1e-5}, "measures": {"fp64": FP64_MEASURE, "fp32": FP32_MEASURE},
             "vs_oracle": {"steps": check, **{k: worst([r[k]["error_vs_oracle"] for r in out]) for k in tot}}}
    if len(tot) == 2:
        error["fp32_vs_fp64_gpu"] = {"steps": steps, **worst([r["fp32_vs_fp64_gpu"] for r in out])}
    return {
        "metric": METRIC, "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(n * n / value / 1e3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if head == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": cases[0]["desc"], "nx": n, "ny": n, "steps": steps, "cases": len(cases),
                   "note": "state resident in the L2 / MALL caches: no HBM roofline claim"},
        "roofline": None,
        "cpu_baseline": cpu,
        "cases": out,
        "error": error,
        "copy_GBps": round(copy_gbps, 1),
        "kernel_source_sha": kernel_sha(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2040)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="wave4096",
                    choices=["wave4096", "cavities64", "channels128", "wave32", "cavity256"])
    ap.add_argument("--size", type=int, default=4096, help="side of the periodic wave (wave4096)")
    ap.add_argument("--diag-every", type=int, default=960)
    ap.add_argument("--fp64-steps", type=int, default=-1, help="steps of the plain FP64 form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the error report (timed forms against the oracle and FP32 against FP64)")
    ap.add_argument("--tune-steps", type=int, default=40,
                    help="steps per candidate of the launch autotuner (0: fixed configuration for the wave forms)")
    ap.add_argument("--launch-fp32", type=json.loads, metavar="JSON",
                    help="fix the FP32 launch configuration (a `launch` object of an earlier run; no autotuning); "
                         "also for the batched workloads")
    ap.add_argument("--launch-fp64", type=json.loads, metavar="JSON",
                    help="fix the FP64 launch configuration (as --launch-fp32)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a domain would shard as y-slabs exchanging 2-row halos)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1401_0188_amd import lbm13
    lbm13.lib()

    log("device copy bandwidth")
    copy_gbps = copy_bandwidth()
    if args.workload in ("wave32", "cavity256"):
        print(json.dumps(main_small(args, copy_gbps)), flush=True)
        return
    if args.workload != "wave4096":
        print(json.dumps(main_batched(args, copy_gbps)), flush=True)
        return

    n = args.size
    graph_k = 0 if args.no_graph else GRAPH_K
    log("fp32-deviation %dx%d: %d warmup + %d steps" % (n, n, args.warmup, args.steps))
    def fixed(launch):
        return dict(spl=launch["steps_per_launch"], tile=tuple(launch["tile"]), fused_tile=tuple(launch["fused_tile"]),
                    interior_kernel=int(launch["interior_kernel"]))
    cfg32, cfg64 = dict(BENCH_CONFIG[1]), dict(BENCH_CONFIG[0])
    tune32 = tune64 = args.tune_steps
    if args.launch_fp32:
        cfg32, tune32 = fixed(args.launch_fp32), 0
    if args.launch_fp64:
        cfg64, tune64 = fixed(args.launch_fp64), 0
    r32 = run_form(lbm13.FP32_DEV, n, args.steps, args.warmup, args.diag_every, cfg32, graph_k, tune32)
    log("fp32: %.1f MLUPS, kernel %.4f ms per launch, %s" % (r32["mlups"], r32["kernel_ms_per_launch"],
                                                           r32["launch"]))
    fp64_steps = args.fp64_steps if args.fp64_steps >= 0 else max(2, args.steps // 2)
    log("fp64 %dx%d: %d steps" % (n, n, fp64_steps))
    r64 = run_form(lbm13.FP64, n, fp64_steps, max(2, args.warmup // 2), args.diag_every, cfg64, graph_k, tune64)
    log("fp64: %.1f MLUPS, kernel %.4f ms per launch" % (r64["mlups"], r64["kernel_ms_per_launch"]))
    plain_cfg = dict(BENCH_CONFIG[0], spl=1)
    r64p = run_form(lbm13.FP64, n, fp64_steps, max(2, args.warmup // 2), args.diag_every, plain_cfg, graph_k)
    log("fp64 one step per launch: %.1f MLUPS, kernel %.4f ms" % (r64p["mlups"], r64p["kernel_ms_per_launch"]))

    cpu = None
    err = None
    if not args.no_cpu:
        log("cpu baseline (oracle) for about %.0f s" % args.cpu_seconds)
        cpu, cpu_steps, om = cpu_baseline(n, args.cpu_seconds)
    if not args.no_accuracy:
        # stated error of the timed forms, outside the timed region: against the
        # oracle's state after the baseline's steps, and FP32 against FP64 on the
        # GPU after 10^4 steps
        err = {"bounds": {"fp64": 1e-12, "fp32": 1e-5}, "measures": {"fp64": FP64_MEASURE, "fp32": FP32_MEASURE}}
        if cpu is not None:
            log("error against the oracle after %d steps" % cpu_steps)
            err["vs_oracle"] = {"steps": cpu_steps,
                                "fp32": moment_errors(final_moments(lbm13.FP32_DEV, n, r32["launch"], cpu_steps, 0), om, 1),
                                "fp64": moment_errors(final_moments(lbm13.FP64, n, r64["launch"], cpu_steps, 0), om, 0)}
            del om
        log("fp32 against fp64 after %d steps" % ACCURACY_STEPS)
        m64 = final_moments(lbm13.FP64, n, r64["launch"], ACCURACY_STEPS, graph_k)
        err["fp32_vs_fp64_gpu"] = dict(
            steps=ACCURACY_STEPS, **moment_errors(final_moments(lbm13.FP32_DEV, n, r32["launch"], ACCURACY_STEPS,
                                                                graph_k), m64, 1))
        del m64

    roof32 = roofline(r32["nodes"], r32["kernel_ms_per_launch"], 1, measured_traffic("fp32", r32["launch"]),
                      spl=r32["spl"], counters=measured_counters("fp32", r32["launch"]))
    roof64 = roofline(r64["nodes"], r64["kernel_ms_per_launch"], 0, measured_traffic("fp64", r64["launch"]),
                      spl=r64["spl"], counters=measured_counters("fp64", r64["launch"]))
    roof64p = roofline(r64p["nodes"], r64p["kernel_ms_per_launch"], 0, measured_traffic("fp64_plain", r64p["launch"]),
                       spl=1, counters=measured_counters("fp64_plain", r64p["launch"]))
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
                   "form": "fp32-deviation", "launch": r32["launch"],
                   "launch_choice": "autotuned on this device" if tune32 else "fixed",
                   "graph_steps": r32["graph_steps"], "diag_every": args.diag_every,
                   "setup_steps": r32["setup_steps"]},
        "roofline": roof32,
        "cpu_baseline": cpu,
        "fp64": {"value": round(r64["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r64["ms_per_step"], 5),
                 "roofline": roof64, "steps": fp64_steps, "form": "fp64", "launch": r64["launch"]},
        "fp64_plain": {"value": round(r64p["mlups"], 1), "unit": "MLUPS",
                       "ms_per_step": round(r64p["ms_per_step"], 5), "roofline": roof64p,
                       "form": "fp64, one step per launch"},
        "speedup_vs_fp64": round(r32["mlups"] / r64["mlups"], 3),
        "speedup_vs_fp64_plain": round(r32["mlups"] / r64p["mlups"], 3),
        "kernel_ms_per_launch": {"fp32": round(r32["kernel_ms_per_launch"], 5),
                                 "fp64": round(r64["kernel_ms_per_launch"], 5),
                                 "fp64_plain": round(r64p["kernel_ms_per_launch"], 5)},
        "copy_GBps": round(copy_gbps, 1),
        "frac_of_copy": round(roof32["achieved"] / copy_gbps, 4) if roof32["unit"] == "GB/s" else None,
        "mass_drift": {"fp32": r32["mass_drift"], "fp64": r64["mass_drift"], "fp64_plain": r64p["mass_drift"]},
        "error": err,
        "kernel_source_sha": kernel_sha(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
