"""Scheduler policy of the serving loop, on the CPU with a simulated executor:
admission by footprint, FIFO order, continuous admission while others run,
error isolation, cancellation, latency statistics."""
import dataclasses

import numpy as np
import pytest

from paper_2412_12360_amd import serve
from paper_2412_12360_amd import workloads as W


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


@dataclasses.dataclass
class FakeProblem:
    nx: int
    ny: int
    nz: int
    T: int

    @property
    def N(self):
        return self.nx * self.ny * self.nz


def mk(rid, edge=64, T=128, kind="forward", arrival=0.0):
    return serve.Request(rid=rid, kind=kind, problem=FakeProblem(edge, edge, edge, T), arrival=arrival)


def run(reqs, budget, max_active=8, chunk=32, open_loop=True, **exkw):
    clk = VClock()
    ex = serve.MockExecutor(clk, **exkw)
    sch = serve.Scheduler(ex, budget, max_active=max_active, chunk=chunk, clock=clk)
    inuse = []
    orig = sch.step

    def step():
        n = orig()
        inuse.append(sch.in_use)
        return n
    sch.step = step
    res = sch.run(reqs, open_loop=open_loop, sleep=clk.sleep)
    return sch, ex, res, inuse


def test_all_requests_complete_with_correct_results():
    reqs = [mk(i, edge=32 + 8 * (i % 4), T=64 + 16 * i, kind="gradient" if i % 2 else "forward") for i in range(12)]
    sch, ex, res, _ = run(reqs, budget=10**12)
    assert len(res) == 12 and all(r.ok for r in res.values())
    for r in reqs:
        assert res[r.rid].J == r.problem.N * r.problem.T
        assert (res[r.rid].grad is not None) == (r.kind == "gradient")
    assert ex.live == 0 and sch.in_use == 0


def test_progress_reported_once_per_block_of_results():
    reqs = [mk(i, edge=32, T=64) for i in range(23)]
    clk = VClock()
    sch = serve.Scheduler(serve.MockExecutor(clk), 10**12, max_active=4, chunk=32, clock=clk)
    seen = []
    res = sch.run(reqs, open_loop=False, sleep=clk.sleep, progress=lambda d, n: seen.append((d, n)),
                  progress_every=5)
    assert len(res) == 23
    assert [d // 5 for d, _ in seen] == [1, 2, 3, 4]
    assert all(n == 23 for _, n in seen)


def test_admission_never_exceeds_budget_and_is_fifo():
    reqs = [mk(i, edge=40 + 10 * (i % 5)) for i in range(20)]
    fps = [r.problem.N * 100 for r in reqs]
    budget = 3 * max(fps)
    sch, ex, res, inuse = run(reqs, budget=budget, open_loop=False)
    assert max(inuse) <= budget
    assert sch.peak_in_use <= budget
    starts = [rid for (ev, rid, t) in ex.log if ev == "start"]
    assert starts == sorted(starts)          # FIFO admission
    assert all(r.ok for r in res.values())


def test_requests_admitted_while_others_run():
    """Continuous batching: a late arrival starts before earlier ones finish."""
    reqs = [mk(0, edge=96, T=512), mk(1, edge=96, T=512), mk(2, edge=48, T=64, arrival=0.01)]
    sch, ex, res, _ = run(reqs, budget=10**12, rate_cells_per_s=1e9)
    assert res[2].t_admit < res[0].t_done and res[2].t_admit < res[1].t_done
    assert res[2].t_done < res[0].t_done      # the short request overtakes


def test_oversized_and_invalid_requests_fail_alone():
    reqs = [mk(0), mk(1, edge=400), mk(2), mk(3)]
    budget = 64 ** 3 * 100 * 2
    sch, ex, res, _ = run(reqs, budget=budget, bad_rids={3})
    assert res[0].ok and res[2].ok
    assert not res[1].ok and "exceeds" in res[1].error
    assert not res[3].ok and "rejected" in res[3].error
    assert sch.in_use == 0


def test_device_error_is_isolated():
    reqs = [mk(i, T=256) for i in range(5)]
    sch, ex, res, _ = run(reqs, budget=10**12, fail_rids={2})
    assert not res[2].ok and "device error" in res[2].error
    assert all(res[i].ok for i in (0, 1, 3, 4))
    assert ex.live == 0 and sch.in_use == 0


def test_cancellation_of_queued_and_running_requests():
    clk = VClock()
    ex = serve.MockExecutor(clk)
    sch = serve.Scheduler(ex, budget_bytes=64 ** 3 * 100, max_active=1, chunk=16, clock=clk)
    for i in range(3):
        sch.submit(mk(i, T=256))
    sch.step()                     # admits request 0 only (budget holds one)
    sch.cancel(0)
    sch.cancel(2)
    while not sch.idle():
        if sch.step() == 0:
            clk.sleep(1e-3)
    res = sch.results
    assert not res[0].ok and res[0].error == "cancelled"
    assert res[1].ok
    assert not res[2].ok and res[2].error == "cancelled"


def test_latency_summary_on_poisson_mix():
    descs = W.serving_mix(count=40, rate_hz=200.0, lo=24, hi=48)
    reqs = [mk(rid, edge=e[0], T=8 * max(e), kind=k, arrival=a) for (rid, e, k, a) in descs]
    sch, ex, res, _ = run(reqs, budget=10**12, rate_cells_per_s=2e9)
    s = serve.summarize(res, wall_s=max(r.t_done for r in res.values()))
    assert s["ok"] == 40
    assert 0 < s["p50_latency_s"] <= s["p99_latency_s"]
    assert s["throughput_mcell_steps_s"] > 0


def test_serving_mix_descriptor_recipe():
    d = W.serving_mix(count=500, rate_hz=10.0)
    edges = np.array([e for (_, e, _, _) in d])
    assert edges.min() >= 64 and edges.max() <= 256
    kinds = [k for (_, _, k, _) in d]
    assert 200 < kinds.count("gradient") < 300
    arr = np.array([a for (*_, a) in d])
    assert np.all(np.diff(arr) >= 0)
    assert abs(np.mean(np.diff(arr)) - 0.1) < 0.02


def test_scheduler_rejects_bad_configuration():
    with pytest.raises(ValueError):
        serve.Scheduler(serve.MockExecutor(VClock()), budget_bytes=0)


def test_share_gives_whole_chunks_to_the_oldest_only():
    """With share = s the oldest active request takes whole chunks and the
    younger ones 1/s of a chunk per iteration (first come, first served with
    backfill); every request still completes with its full work."""
    clk = VClock()
    ex = serve.MockExecutor(clk)
    seen = []
    orig = ex.forward

    def fwd(slot, n):
        seen.append((slot["rid"], n))
        orig(slot, n)
    ex.forward = fwd
    sch = serve.Scheduler(ex, 10**12, max_active=4, chunk=64, clock=clk, share=4)
    reqs = [mk(i, edge=32, T=256) for i in range(3)]
    res = sch.run(reqs, open_loop=False, sleep=clk.sleep)
    assert all(r.ok and r.J == r.cell_steps for r in res.values())
    first = {}
    for rid, n in seen:
        first.setdefault(rid, n)
    assert first[0] == 64 and first[1] == 16 and first[2] == 16
    with pytest.raises(ValueError):
        serve.Scheduler(ex, 10**12, share=0)


def test_cell_cap_runs_large_grids_alone_and_batches_small_ones():
    """With cell_cap, a grid at or above the cap never shares the device, and
    small grids run together up to the cap; FIFO order holds."""
    big = [mk(i, edge=100, T=64) for i in range(3)]            # 1e6 cells each
    small = [mk(10 + i, edge=40, T=64) for i in range(6)]      # 64000 cells each
    reqs = [big[0], small[0], small[1], big[1], small[2], small[3], small[4], big[2], small[5]]
    clk = VClock()
    ex = serve.MockExecutor(clk)
    sch = serve.Scheduler(ex, 10**12, max_active=8, chunk=32, clock=clk, cell_cap=400_000)
    peak = []
    orig = sch.step

    def step():
        n = orig()
        live = [a.req for a in sch.active.values()]
        peak.append((len(live), sum(r.problem.N for r in live), [r.rid for r in live]))
        return n
    sch.step = step
    res = sch.run(reqs, open_loop=False, sleep=clk.sleep)
    assert all(r.ok for r in res.values()) and len(res) == len(reqs)
    for n, cells, rids in peak:
        if any(r in (0, 1, 2) for r in rids):
            assert n == 1, rids               # a large grid runs alone
        else:
            assert cells <= 400_000
    assert max(n for n, _, _ in peak) >= 3    # small grids did share
    starts = [rid for (ev, rid, _) in ex.log if ev == "start"]
    assert starts == [r.rid for r in reqs]    # FIFO admission
    with pytest.raises(ValueError):
        serve.Scheduler(ex, 10**9, cell_cap=0)


def test_chunk_cells_scales_chunks_by_grid_size():
    """With chunk_cells, a small grid takes whole multiples of `chunk` steps
    per iteration (about chunk_cells cell-steps), a large one `chunk`."""
    clk = VClock()
    ex = serve.MockExecutor(clk)
    calls = []
    orig = ex.forward

    def fwd(slot, n):
        calls.append((slot["rid"], n))
        return orig(slot, n)
    ex.forward = fwd
    sch = serve.Scheduler(ex, 10**12, max_active=4, chunk=16, clock=clk, chunk_cells=16 * 100**3)
    reqs = [mk(0, edge=100, T=64), mk(1, edge=25, T=4096)]
    res = sch.run(reqs, open_loop=False, sleep=clk.sleep)
    assert all(r.ok for r in res.values())
    big = {n for rid, n in calls if rid == 0}
    small = [n for rid, n in calls if rid == 1]
    assert big == {16}
    assert small[0] == 16 * 64 and sum(small) == 4096
    with pytest.raises(ValueError):
        serve.Scheduler(ex, 10**9, chunk_cells=0)
