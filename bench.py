#!/usr/bin/env python3
"""Benchmark of the reversible 3D FDTD hot path on one MI355X.

A step is one complete solve of the benchmark workload: zero the fields, then
T leapfrog steps of the Yee/CPML update with the plane-wave source and the
flux detector.  The default workload is a 256^3 grid with a 10-cell CPML on
every face and T = 2000 (forward only).  The line also carries:
  - roofline: the forward sweep (one launch of the z-march over every tile
    class for K steps, timed on the same grid without the detector so no
    reduction kernel is inside the events) against the 8 TB/s HBM peak, with
    algorithmic bytes 52 B per cell plus 32 B per CPML slab cell and slab
    axis, per time step; traffic from the committed counter summary;
  - fwd_grad: the 200^3 gradient problem (CPML 10, 64^3 design cube,
    T = 1500): forward with the interface record, then the time-reversed
    adjoint pass, rated as N*T / (t_fwd + t_bwd), the fused reverse step
    against the roofline; beside it the same gradient by uniform
    checkpointing, recursive halving and treeverse (the methods time
    reversal replaces);
  - fwd_grad_large: the same on 640x640x400 (CPML 12, 4000 steps, 71.8 GB);
  - serving: the first requests of the serving mix (100 by default), one at
    a time and with continuous batching: throughput, and p50/p99 latency
    under Poisson arrivals at 0.8x the one-at-a-time rate;
  - cpu_baseline: the FP64 oracle on the host cores and on one core, timed
    on a bounded sample (the same 256^3 grid, a few time steps).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s fwd and fwd+grad (FP32, % HBM roofline); p99 latency in serving mix"
PEAK_GBS = 8000.0
# rocprofv3 counter summary of the forward sweep on this workload: HBM bytes
# per sweep (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy kernel's
# counters) and the hash of the sources it was taken on: the z-march kernel
# and the tile planner block of the library (shape, time block, tiles, march
# lengths), which together decide the sweep's traffic
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "fdtd_forward_zmarch_256cube_hbm_traffic.md")
TRAFFIC_SOURCES = ("paper_2412_12360_amd/csrc/kern_tb.hip",
                   "paper_2412_12360_amd/csrc/fdtd_api.hip [tile planner]")
PLANNER_BEGIN = b"// ------------------------------------------------------------- tile planner"
PLANNER_END = b"// ------------------------------------------------------ end of tile planner"


def source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2412_12360_amd/csrc/kern_tb.hip"), "rb") as f:
        h.update(f.read())
    with open(os.path.join(ROOT, "paper_2412_12360_amd/csrc/fdtd_api.hip"), "rb") as f:
        api = f.read()
    i, j = api.index(PLANNER_BEGIN), api.index(PLANNER_END)
    h.update(api[i:j])
    return h.hexdigest()


def measured_traffic(K: int):
    """HBM bytes per K-step sweep from the committed counter summary, or None
    when it is missing, was taken at another K, or the forward kernel source
    has changed since."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    b = re.search(r"traffic_bytes_per_sweep:\s*(\d+)", text)
    k = re.search(r"time_block:\s*(\d+)", text)
    h = re.search(r"sources_sha256:\s*([0-9a-f]{64})", text)
    if not (b and k and h) or int(k.group(1)) != K or h.group(1) != source_hash():
        return None
    return int(b.group(1))


REV_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "fdtd_reverse_zmarch_200cube_hbm_traffic.md")


def rev_source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2412_12360_amd/csrc/kern_tb_rev.hip"), "rb") as f:
        h.update(f.read())
    with open(os.path.join(ROOT, "paper_2412_12360_amd/csrc/fdtd_api.hip"), "rb") as f:
        api = f.read()
    i, j = api.index(PLANNER_BEGIN), api.index(PLANNER_END)
    h.update(api[i:j])
    return h.hexdigest()


def measured_rev_traffic(pr):
    """HBM bytes per fused reverse step of this grid from the committed
    counter summary, or None when there is none for the grid or the reverse
    kernel or tile planner has changed since it was taken."""
    try:
        with open(REV_TRAFFIC_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    h = re.search(r"sources_sha256:\s*([0-9a-f]{64})", text)
    b = re.search(r"traffic_bytes_per_step_%dx%dx%d:\s*(\d+)" % (pr.nx, pr.ny, pr.nz), text)
    if not (h and b) or h.group(1) != rev_source_hash():
        return None
    return int(b.group(1))


def slab_cell_axes(pr) -> int:
    if pr.p == 0:
        return 0
    n = (pr.nx, pr.ny, pr.nz)
    return sum(2 * pr.p * (pr.N // n[a]) for a in range(3))


def alg_bytes_fwd_step(pr, record: bool = False) -> int:
    b = 52 * pr.N + 32 * slab_cell_axes(pr)
    if record and pr.p > 0:
        Lx, Ly, Lz = pr.nx - 2 * pr.p, pr.ny - 2 * pr.p, pr.nz - 2 * pr.p
        b += 4 * 2 * 2 * (Ly * Lz + Lx * Lz + Lx * Ly)
    return b


def alg_bytes_rev_step(pr) -> int:
    """Algorithmic bytes of one fused reverse step: 100 B per interior cell
    (forward E, H read and written, adjoint E, H read and written, S/eps
    read), 52 B per CPML cell (adjoint only), 32 B per slab cell and slab
    axis (four psi-bar read and written), 8 B per design cell (dJ/deps
    accumulator read and written) and the record of one step read."""
    Lx, Ly, Lz = pr.nx - 2 * pr.p, pr.ny - 2 * pr.p, pr.nz - 2 * pr.p
    interior = Lx * Ly * Lz
    d = 1
    for a in range(3):
        d *= pr.design_hi[a] - pr.design_lo[a]
    rec = 4 * 2 * 2 * (Ly * Lz + Lx * Lz + Lx * Ly) if pr.p > 0 else 0
    return 100 * interior + 52 * (pr.N - interior) + 32 * slab_cell_axes(pr) + 8 * d + rec


def time_solves(solver, count: int, torch):
    """Events on the solver's stream around `count` full forward solves."""
    st = solver.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(count):
        solver.reset()
        solver.forward()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def tfsf_run(pr, Solver, torch, time_block: int, steps: int, W):
    """The headline forward workload with the one-sided total-field/scattered-
    field plane (Ex polarised, same plane) in place of the soft sheet: full
    solves timed like the headline value, and the material upload that reruns
    the plane's incident line (fdtd_set_inv_eps) timed on the solver's stream."""
    pt = W.with_tfsf(pr)
    s = Solver(pt, record=False, time_block=time_block)
    s.reset()
    s.forward()
    ms = time_solves(s, steps, torch)
    s.reset()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.set_inv_eps(s.inv_eps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    line_ms = e0.elapsed_time(e1)
    del s
    torch.cuda.empty_cache()
    return {
        "workload": "the same grid, materials, detector and waveform with a one-sided TFSF plane wave "
                    f"(Ex, first total-field plane k = {pt.sources[0].k}) instead of the sheet",
        "value": round(pt.N * pt.T * steps / (ms / 1e3) / 1e6, 1),
        "unit": "Mcell-updates/s",
        "ms_per_solve": round(ms / steps, 3),
        "incident_line_ms": round(line_ms, 3),
        "incident_line_note": f"material upload plus the {pt.T}-step incident line, once per create or set_inv_eps",
    }


def interp_detector_run(pr, Solver, torch, time_block: int, steps: int):
    """The headline forward workload with its flux detector in the
    interpolated (co-located) mode: raw planes written by the sweep kernels,
    E^n gathered before each sweep, the co-located density formed after it."""
    pi = dataclasses.replace(pr, detectors=[dataclasses.replace(d, interpolate=True) for d in pr.detectors])
    s = Solver(pi, record=False, time_block=time_block)
    s.reset()
    s.forward()
    ms = time_solves(s, steps, torch)
    del s
    torch.cuda.empty_cache()
    return {
        "workload": "the same solve with the flux detector interpolated (all components co-located at "
                    "(i+1/2, j+1/2, k) and time n+1/2)",
        "value": round(pi.N * pi.T * steps / (ms / 1e3) / 1e6, 1),
        "unit": "Mcell-updates/s",
        "ms_per_solve": round(ms / steps, 3),
    }


def shard_run(Solver, torch, time_block: int, steps: int, W, T: int = 100):
    """The forward step on one GPU's share of a 2400x1600x600 grid cut into
    four z-slabs (2400x1600x150, 576M cells, 12-cell CPML on all six faces):
    the field set spans 13.8 GB, so the z-march runs with a 64-bit base per
    component and plane.  A bounded sample of T steps per solve."""
    pr = W.shard_slab(T=T)
    s = Solver(pr, record=False, time_block=time_block)
    path = s.kernel_path
    s.reset()
    s.forward()
    ms = time_solves(s, steps, torch)
    fp = s.footprint
    del s
    torch.cuda.empty_cache()
    return {
        "workload": f"{pr.nx}x{pr.ny}x{pr.nz} z-slab (one of four of a {pr.nx}x{pr.ny}x{4 * pr.nz} grid), "
                    f"CPML {pr.p} on all six faces, Ex sheet, flux detector, {T} steps per solve",
        "value": round(pr.N * T * steps / (ms / 1e3) / 1e6, 1),
        "unit": "Mcell-updates/s",
        "ms_per_step": round(ms / steps / T, 3),
        "kernel_path": path,
        "footprint_gb": round(fp / 1e9, 2),
    }


def lossy_run(pg, Solver, torch, W):
    """The gradient problem with its design cube conducting (sigma ~ U[0, 1]
    per cell, seed 21): the record keeps E^n of the lossy cells every step and
    the inverse replays it (the z-marches' lossy instances).  A warm-up solve,
    then forward + gradient timed on the solver's stream."""
    pl = W.with_lossy(pg)
    g = Solver(pl, record=True)
    g.reset()
    g.forward()
    g.grad()
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(g.stream)
    g.reset()
    g.forward()
    e1.record(g.stream)
    _, recon = g.grad()
    e2.record(g.stream)
    torch.cuda.synchronize()
    tf, tb = e0.elapsed_time(e1), e1.elapsed_time(e2)
    nb = 1
    for a in range(3):
        nb *= pl.lossy_hi[a] - pl.lossy_lo[a]
    res = {
        "workload": "the same problem with the design cube conducting (sigma ~ U[0,1] per cell, seed 21); "
                    "E^n of the lossy cells recorded every step and replayed by the inverse",
        "value": round(pl.N * pl.T / ((tf + tb) / 1e3) / 1e6, 1), "unit": "Mcell-steps/s",
        "fwd_ms": round(tf, 2), "bwd_ms": round(tb, 2), "recon_err": float(recon.item()),
        "lossy_record_gb": round(12 * nb * pl.T / 1e9, 3), "hbm_footprint_gb": round(g.footprint / 1e9, 2),
        "kernel_path": g.kernel_path,
    }
    del g
    torch.cuda.empty_cache()
    return res


def fwd_grad_run(pg, Solver, torch, time_block: int, workload: str, checkpoint: bool = False,
                 warmup: bool = True):
    """A warm-up solve (unless the kernels ran already), then a timed forward
    (with the interface record) and gradient on the solver's stream:
    N*T / (t_fwd + t_bwd).  The fused reverse step is rated against the HBM
    roofline by its algorithmic bytes."""
    g = Solver(pg, record=True, time_block=time_block)
    if warmup:
        g.reset()
        g.forward()
        g.grad()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    g.reset()
    g.forward()
    e1.record(g.stream)
    dg, recon = g.grad()
    e2.record(g.stream)
    torch.cuda.synchronize()
    tf, tb = e0.elapsed_time(e1), e1.elapsed_time(e2)
    res = {
        "workload": workload,
        "value": round(pg.N * pg.T / ((tf + tb) / 1e3) / 1e6, 1), "unit": "Mcell-steps/s",
        "fwd_ms": round(tf, 2), "bwd_ms": round(tb, 2),
        "recon_err": float(recon.item()),
        "hbm_footprint_gb": round(g.footprint / 1e9, 2),
        "kernel_path": g.kernel_path,
    }
    rev_alg = alg_bytes_rev_step(pg)
    rev_ms = tb / pg.T
    res["roofline_reverse"] = {
        "bound": "hbm", "kernel": "fused reverse z-march step (inverse + adjoint, one launch per step)",
        "achieved": round(rev_alg / (rev_ms / 1e3) / 1e9, 1), "peak": PEAK_GBS, "unit": "GB/s",
        "frac": round(rev_alg / (rev_ms / 1e3) / 1e9 / PEAK_GBS, 4), "alg_bytes_per_launch": rev_alg,
        "avg_launch_ms": round(rev_ms, 5), "launches_timed": pg.T,
        "traffic": measured_rev_traffic(pg),
    }
    tr = res["roofline_reverse"]["traffic"]
    # the counted HBM bytes over the same launch time (what the memory system moved)
    res["roofline_reverse"]["traffic_gbs"] = round(tr / (rev_ms / 1e3) / 1e9, 1) if tr else None
    if checkpoint:
        # the baseline the time reversal replaces: checkpoints every sqrt(T)
        # steps, each segment recomputed and kept, adjoint-only reverse steps
        seg = max(1, int(round(math.sqrt(pg.T))))
        store = torch.empty(g.checkpoint_bytes(seg), dtype=torch.uint8, device=g.device)
        g.grad_checkpointed(seg, store=store)
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(g.stream)
        dck, _ = g.grad_checkpointed(seg, store=store)
        c1.record(g.stream)
        torch.cuda.synchronize()
        tc = c0.elapsed_time(c1)
        res["checkpointed"] = {
            "what": f"forward + gradient by checkpointing every {seg} steps (segments recomputed and kept)",
            "value": round(pg.N * pg.T / (tc / 1e3) / 1e6, 1), "unit": "Mcell-steps/s", "ms": round(tc, 2),
            "extra_hbm_gb": round(store.numel() / 1e9, 2),
            "time_reversal_speedup": round(tc / (tf + tb), 3),
            "grad_rel_diff_vs_time_reversal": float(((dck - dg).norm() / dg.norm()).item()),
        }
        del store
        # the schedules section 2.2 names: recursive halving, and treeverse
        # with a fixed number of kept states (each a complete forward state)
        from paper_2412_12360_amd.fdtd import revolve_plan
        sched = {}
        for name, k in (("halving", 0), ("treeverse", 4)):
            fsteps, peak, _ = revolve_plan(pg.T, name, k)
            store = torch.empty(g.revolve_bytes(name, k), dtype=torch.uint8, device=g.device)
            c0 = torch.cuda.Event(enable_timing=True)
            c1 = torch.cuda.Event(enable_timing=True)
            c0.record(g.stream)
            dr, _ = g.grad_revolve(name, k, store=store)
            c1.record(g.stream)
            torch.cuda.synchronize()
            tc = c0.elapsed_time(c1)
            sched[name if name == "halving" else f"treeverse_{k}"] = {
                "value": round(pg.N * pg.T / (tc / 1e3) / 1e6, 1), "unit": "Mcell-steps/s", "ms": round(tc, 2),
                "forward_steps": fsteps, "kept_states": peak, "extra_hbm_gb": round(store.numel() / 1e9, 2),
                "time_reversal_speedup": round(tc / (tf + tb), 3),
                "grad_bitwise_equal_to_segments": bool(torch.equal(dr, dck)),
            }
            del store
        res["checkpoint_schedules"] = sched
    del g
    torch.cuda.empty_cache()
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_rate(threads: int, target_s: float):
    """The FP64 oracle on the benchmark grid in a child process (its own
    OpenMP thread count; the child never touches the GPU): (Mcell-updates/s,
    steps timed)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), OMP_PROC_BIND="false")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-oracle-child", str(target_s)],
                       env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"oracle child failed: {r.stderr[-400:]}")
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return d["rate"], d["steps"]


def cpu_oracle_child(target_s: float):
    """Child of cpu_oracle_rate: times oracle steps of the benchmark grid."""
    from oracle.oracle import Oracle, build as build_oracle
    from paper_2412_12360_amd import workloads as W
    build_oracle(force=False)
    pr = W.config2()
    o = Oracle(pr)
    st = o.new_state()
    t0 = time.perf_counter()
    o.forward(st, 1, 0)
    one = time.perf_counter() - t0
    n = max(1, min(pr.T - 1, int(target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    o.forward(st, n, 1)
    dt = time.perf_counter() - t0
    print(json.dumps({"rate": pr.N * n / dt / 1e6, "steps": n}), flush=True)


def cpu_baseline(pr, target_s: float = 10.0):
    """The FP64 oracle on the host cores available to this process (their
    count from the CPU affinity, capped by OMP_NUM_THREADS when set) and on
    one core: the benchmark grid for a bounded number of steps."""
    cores = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = max(1, min(cores, int(os.environ["OMP_NUM_THREADS"])))
    rate, n = cpu_oracle_rate(cores, target_s)
    rate1, n1 = cpu_oracle_rate(1, target_s)
    return {"value": round(rate, 3), "unit": "Mcell-updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{pr.nx}x{pr.ny}x{pr.nz} grid, {n} FP64 time steps (steps 1..{n}) of the same problem "
                      f"with {cores} threads; {n1} steps with 1 thread",
            "value_1_thread": round(rate1, 3)}


def copy_calibration(torch, nbytes: int = 1 << 30, reps: int = 4):
    """Plain device kernels of known traffic: an elementwise negation reads
    and writes `nbytes` (and a runtime copy does the same); their per-dispatch
    HBM counters (FETCH_SIZE, WRITE_SIZE) against `nbytes` give the counters'
    scale factor."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.neg(a, out=b)
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def serving_bench(count: int, torch, seed_rate: float = 0.8, budget_gb: float = 0.0, max_active: int = 6,
                  chunk: int = 64, extra_rates=(), open_loops: bool = True, open_rate: float = 0.0,
                  share: int = 0, cell_cap: int = 0):
    """Serving mix: `count` requests of the Poisson mix recipe (edges U{64..256},
    50% forward / 50% gradient, T = 8 x max edge, CPML 8).  Measures saturation
    throughput one-at-a-time and with continuous batching (all queued at t=0),
    then open-loop Poisson arrivals at 0.8 x the one-at-a-time request rate for
    both systems, reporting p50/p99 latency; `extra_rates` repeats the open
    loop at further multiples of that rate (same arrival seed).  A long mix can
    be split over two runs: `open_rate` > 0 skips the closed loops and runs the
    open loops at that rate (req/s); `open_loops` = False skips the open loops."""
    from paper_2412_12360_amd import serve
    from paper_2412_12360_amd import workloads as W
    descs = W.serving_mix(count=count, rate_hz=None)
    probs = {rid: W.serving_request(e, k == "gradient", seed=1000 + rid, p=8, rid=rid) for (rid, e, k, _) in descs}
    kinds = {rid: k for (rid, _, k, _) in descs}
    budget = int(budget_gb * 1e9) if budget_gb > 0 else int(torch.cuda.mem_get_info()[0] * 0.8)

    def run(max_active, arrivals=None, limit=None):
        rids = sorted(probs)[:limit]
        reqs = [serve.Request(rid=rid, kind=kinds[rid], problem=probs[rid],
                              arrival=0.0 if arrivals is None else arrivals[i])
                for i, rid in enumerate(rids)]
        sch = serve.Scheduler(serve.GpuExecutor(), budget_bytes=budget, max_active=max_active, chunk=chunk,
                              share=share if share > 0 else None,
                              cell_cap=cell_cap if (cell_cap > 0 and max_active > 1) else None)
        t0 = time.perf_counter()
        res = sch.run(reqs, open_loop=arrivals is not None,
                      progress=lambda d, n: log(f"  {d} of {n} requests served"))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out = serve.summarize(res, wall)
        out["peak_hbm_gb"] = round(sch.peak_in_use / 1e9, 2)
        return out

    t_start = time.perf_counter()

    def log(msg):   # one line per phase (a long mix runs for minutes)
        print(f"[serving] {msg} ({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)

    run(1, limit=8)                          # warm-up (code objects, allocator)
    log("warm-up done")
    r = lambda v: None if v is None else round(v, 4)
    res = {"workload": f"{count} requests of the serving mix (edges U{{64..256}} per axis, 50% gradient, "
                       f"T = 8 x max edge, CPML 8, eps_r U[1,12.25]; seeds 6/7/1000+rid)",
           "hbm_budget_gb": round(budget / 1e9, 1), "max_active": max_active, "chunk_steps": chunk,
           "share": share if share > 0 else None, "cell_cap": cell_cap if cell_cap > 0 else None,
           "batched_launches": "one z-march launch per forward sweep and per reverse step spans all active requests"}
    if open_rate <= 0:
        seq = run(1)
        log(f"one at a time: {seq['req_per_s']:.3f} req/s")
        bat = run(max_active)
        log(f"batched: {bat['req_per_s']:.3f} req/s")
        res["one_at_a_time"] = {"throughput_mcell_steps_s": r(seq["throughput_mcell_steps_s"]),
                                "req_per_s": r(seq["req_per_s"]), "wall_s": r(seq["wall_s"])}
        res["batched"] = {"throughput_mcell_steps_s": r(bat["throughput_mcell_steps_s"]),
                          "req_per_s": r(bat["req_per_s"]), "wall_s": r(bat["wall_s"]),
                          "peak_hbm_gb": bat["peak_hbm_gb"]}
        res["speedup_throughput"] = r(bat["throughput_mcell_steps_s"] / seq["throughput_mcell_steps_s"])
        seq_rate = seq["req_per_s"]
    else:
        seq_rate = open_rate / seed_rate
    if not open_loops:
        return res
    import numpy as np

    def arrivals(factor):
        rng = np.random.Generator(np.random.PCG64(8))
        return list(np.cumsum(rng.exponential(1.0 / (factor * seq_rate), size=count)))

    rate = seed_rate * seq_rate
    arr = arrivals(seed_rate)
    seq_open = run(1, arr)
    log(f"open loop, one at a time: p99 {seq_open['p99_latency_s']:.3f} s")
    bat_open = run(max_active, arr)
    log(f"open loop, batched: p99 {bat_open['p99_latency_s']:.3f} s")
    more = []
    for f in extra_rates:
        a = arrivals(f)
        so = run(1, a)
        log(f"open loop at {f} x, one at a time: p99 {so['p99_latency_s']:.3f} s")
        bo = run(max_active, a)
        log(f"open loop at {f} x, batched: p99 {bo['p99_latency_s']:.3f} s")
        more.append({"rate_factor": f, "rate_req_s": r(f * seq_rate),
                     "one_at_a_time_open": {"p50_s": r(so["p50_latency_s"]), "p99_s": r(so["p99_latency_s"])},
                     "batched_open": {"p50_s": r(bo["p50_latency_s"]), "p99_s": r(bo["p99_latency_s"])}})
    res["open_loop_rate_req_s"] = r(rate)
    res["one_at_a_time_open"] = {"p50_s": r(seq_open["p50_latency_s"]), "p99_s": r(seq_open["p99_latency_s"])}
    res["batched_open"] = {"p50_s": r(bat_open["p50_latency_s"]), "p99_s": r(bat_open["p99_latency_s"])}
    if more:
        res["open_loop_other_rates"] = more
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed full solves")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--time-block", type=int, default=0)
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the TFSF-source and interpolated-detector variants of the forward workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-shard", action="store_true",
                    help="skip the forward step on one z-slab of a 2400x1600x600 grid (2400x1600x150)")
    ap.add_argument("--serving", type=int, default=100,
                    help="requests of the serving mix to run (0 = skip; the first requests of the 500-request mix)")
    ap.add_argument("--solve-steps", type=int, default=0,
                    help="profiling runs only: time steps per solve instead of the workload's (0 = workload)")
    ap.add_argument("--large", action="store_true",
                    help="also run the 640x640x400 forward+gradient problem (CPML 12, 4000 steps) and "
                         "forward+gradient on the 2400x1600x150 z-slab (100 steps)")
    ap.add_argument("--serving-max-active", type=int, default=6,
                    help="requests on the GPU at once in the batched runs (6 measured best on a "
                         "200-request mix: more sharing lengthens the largest requests)")
    ap.add_argument("--serving-chunk", type=int, default=64, help="serving: forward steps per scheduler iteration")
    ap.add_argument("--serving-share", type=int, default=0,
                    help="serving: younger requests take 1/share of a chunk (0 = equal chunks)")
    ap.add_argument("--serving-cell-cap", type=int, default=8_000_000,
                    help="serving: a request joins running ones only while their grid cells together stay "
                         "within this many (0 = no limit; 8M measured best on the 100-request mix: grids that "
                         "fill the device run alone, small ones share the launches)")
    ap.add_argument("--serving-closed-only", action="store_true",
                    help="serving: the two closed loops only (a long mix split over two runs)")
    ap.add_argument("--serving-open-rate", type=float, default=0.0,
                    help="serving: skip the closed loops and run the open loops at this rate (req/s)")
    ap.add_argument("--serving-extra-rates", default="",
                    help="comma-separated multiples of the one-at-a-time rate for further open-loop runs "
                         "(e.g. 0.5,1.2)")
    ap.add_argument("--serving-budget-gb", type=float, default=0.0,
                    help="HBM budget for the serving mix (0 = 80%% of free memory)")
    ap.add_argument("--cpu-oracle-child", type=float, default=0.0, help=argparse.SUPPRESS)
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 640x640x400 forward + gradient leg")
    ap.add_argument("--no-checkpoint", action="store_true",
                    help="skip the checkpointing comparators of the 200^3 gradient leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="profiling runs only: run a plain 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.cpu_oracle_child > 0:
        cpu_oracle_child(args.cpu_oracle_child)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU z-slab decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_12360_amd import workloads as W
    from paper_2412_12360_amd.fdtd import Solver

    if args.copy_calibration:
        copy_calibration(torch)
        return
    rank = int(os.environ.get("RANK", "0"))
    t_bench = time.perf_counter()

    def progress(leg):   # one stderr line per finished leg (a --large run takes minutes)
        print(f"[bench] {leg} done ({time.perf_counter() - t_bench:.0f} s)", file=sys.stderr, flush=True)

    pr = W.config2(T=args.solve_steps) if args.solve_steps else W.config2()
    s = Solver(pr, record=False, time_block=args.time_block)
    K = s.time_block
    for _ in range(args.warmup):
        s.reset()
        s.forward()
    torch.cuda.synchronize()
    ms = time_solves(s, args.steps, torch)
    cells = pr.N * pr.T * args.steps
    value = cells / (ms / 1e3) / 1e6
    del s
    torch.cuda.empty_cache()
    # The dominant kernel: one K-step sweep (the tile-class kernels, run
    # concurrently and joined on the solver's stream).  Timed on the same grid
    # without the flux detector, so that no reduction kernel falls inside the
    # events; the sweep kernels are the same ones.
    ps = dataclasses.replace(pr, detectors=[])
    sw = Solver(ps, record=False, time_block=args.time_block)
    sw.reset()
    sw.forward()
    sw.reset()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(sw.stream)
    sw.forward()
    ev1.record(sw.stream)
    torch.cuda.synchronize()
    passes = math.ceil(ps.T / K)
    pass_ms = ev0.elapsed_time(ev1) / passes
    del sw
    torch.cuda.empty_cache()
    alg = alg_bytes_fwd_step(pr) * K
    achieved = alg / (pass_ms / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "256^3 Yee grid, 10-cell CPML, 2000 steps forward, ramped Ex plane-wave sheet, "
                        "flux detector, eps_r 2.25 with a 128^3 cube U[2.25,12.25] (seed 2)",
            "grid": [pr.nx, pr.ny, pr.nz], "steps_per_solve": pr.T, "time_block": K,
            **({"profiling_run": "steps per solve overridden"} if args.solve_steps else {}),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_GBS, 4), "traffic": measured_traffic(K),
            "kernel": f"forward z-march sweep (K={K} steps, one launch over the tiles of every class)",
            "alg_bytes_per_launch": alg, "avg_launch_ms": round(pass_ms, 5),
            "launches_timed": passes,
        },
    }
    tr = out["roofline"]["traffic"]
    # the counted HBM bytes over the same launch time (what the memory system moved)
    out["roofline"]["traffic_gbs"] = round(tr / (pass_ms / 1e3) / 1e9, 1) if tr else None

    progress("headline forward")
    if not args.no_variants:
        out["tfsf"] = tfsf_run(pr, Solver, torch, args.time_block, args.steps, W)
        out["interpolated_detector"] = interp_detector_run(pr, Solver, torch, args.time_block, args.steps)
        progress("forward variants")

    if not args.no_shard:
        out["shard"] = shard_run(Solver, torch, args.time_block, args.steps, W,
                                 T=args.solve_steps if args.solve_steps else 100)
        progress("z-slab forward")

    if not args.no_grad:
        pg = W.config3(T=args.solve_steps) if args.solve_steps else W.config3()
        out["fwd_grad"] = fwd_grad_run(pg, Solver, torch, args.time_block,
                                       "200^3 grid, CPML 10, 64^3 design cube rho~U[0,1] (seed 3), eps_r = 2.25 + 10 rho, "
                                       "1500 steps, objective = time-integrated flux; forward with interface record, "
                                       "then inverse-step + adjoint backward", checkpoint=not args.no_checkpoint)
        out["fwd_grad"]["lossy"] = lossy_run(pg, Solver, torch, W)
        progress("forward + gradient")

    if not args.no_grad and not args.no_large:
        # (the kernels ran in the 200^3 leg: no warm-up solve)
        out["fwd_grad_large"] = fwd_grad_run(W.config4(T=args.solve_steps) if args.solve_steps else W.config4(),
                                             Solver, torch, args.time_block,
                                             "640x640x400 grid, CPML 12, 256x256x128 design box (blurred binary rho, "
                                             "seed 5), eps_r = 2.25 + 10 rho, 4000 steps, interface record in HBM",
                                             warmup=False)
        progress("large forward + gradient")

    if args.large and not args.no_grad:
        T = args.solve_steps if args.solve_steps else 100
        out["shard_fwd_grad"] = fwd_grad_run(W.shard_slab(T=T), Solver, torch, args.time_block,
                                             f"2400x1600x150 z-slab, CPML 12, 1200x800x75 design block, {T} steps "
                                             "with the interface record, then the gradient (a sample: the wave has "
                                             "not reached the detector yet; the kernels do the same work either way)")
        progress("z-slab forward + gradient")

    if args.serving > 0:
        out["serving"] = serving_bench(args.serving, torch, budget_gb=args.serving_budget_gb,
                                       max_active=args.serving_max_active, chunk=args.serving_chunk, share=args.serving_share,
                                       cell_cap=args.serving_cell_cap,
                                       extra_rates=[float(v) for v in args.serving_extra_rates.split(",") if v],
                                       open_loops=not args.serving_closed_only, open_rate=args.serving_open_rate)

    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
