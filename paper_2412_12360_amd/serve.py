"""Continuous-batching serving loop for FDTD forward and gradient solves.

Requests of uneven grid sizes arrive at arbitrary times.  Each scheduler
iteration
  1. admits queued requests (FIFO) while the sum of the admitted requests'
     exact workspace footprints (fdtd_footprint) stays within the HBM budget
     and a slot is free (with `cell_cap`, a request joins running ones only
     while their grid cells together stay within it: grids that fill the
     device run alone, small launch-bound ones share the launches); an
     admitted request gets its own handle and workspace, so its fields and
     interface record stay resident until it finishes;
  2. gives every active request whose previous chunk has finished its next
     chunk of work: `chunk` more forward time steps, or, once a gradient
     request's forward is complete, `bchunk` more time-reversed steps of its
     backward pass (with `chunk_cells`, both scaled by whole multiples so
     that a chunk holds about chunk_cells cell-steps: a small grid takes
     more steps per iteration) (with `share` = s, only the oldest active request takes
     whole chunks and the others 1/s of them: they fill what the oldest
     leaves of the device, in the same launches, without holding it back
     much -- first-come first-served with backfill);
  3. hands the iteration's chunks to the executor at once (flush): the GPU
     executor advances all of them with batched launches -- every forward
     sweep and every reverse step is one kernel launch whose tile table
     spans all requests of the batch (fdtd_forward_batch,
     fdtd_grad_steps_batch);
  4. retires finished requests: copies their results out, releases the slot
     and its memory, records the latency.
A request that arrives while others run is admitted as soon as memory and a
slot are free and joins the next batch.  A request that cannot be served
(invalid problem, footprint above the whole budget, a device error) fails
alone with an error result and frees its slot.

The scheduler only talks to an executor object, so its policy is testable on
the CPU with a mock executor that simulates durations.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from typing import Callable, Deque, Dict, List, Optional


class BatchError(RuntimeError):
    """A batched call failed; rids: the requests whose work it held."""

    def __init__(self, rids, cause):
        super().__init__(str(cause))
        self.rids = list(rids)
        self.cause = cause


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                      # "forward" or "gradient"
    problem: object                # workloads.Problem
    arrival: float = 0.0           # seconds after the start of the run (open loop)


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    ok: bool
    J: Optional[float] = None
    trace: Optional[object] = None
    grad: Optional[object] = None
    recon: Optional[float] = None
    error: Optional[str] = None
    t_arrival: float = 0.0
    t_admit: float = math.nan
    t_done: float = math.nan
    footprint: int = 0
    cell_steps: int = 0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Executor:
    """Interface the scheduler drives (one slot per admitted request)."""

    def footprint(self, req: Request) -> int:
        raise NotImplementedError

    def start(self, req: Request):
        """Create the request's solver; returns an opaque slot.  May raise."""
        raise NotImplementedError

    def forward(self, slot, nsteps: int) -> None:
        """Enqueue nsteps forward steps (non-blocking)."""
        raise NotImplementedError

    def backward(self, slot, nsteps: int) -> None:
        """Enqueue nsteps more reverse steps of the gradient pass (non-blocking);
        the first call starts the pass, the one that reaches step 0 ends it."""
        raise NotImplementedError

    def flush(self) -> None:
        """Issue the work enqueued since the last flush (called once per
        scheduler iteration)."""

    def ready(self, slot) -> bool:
        """True when the slot can take another chunk (an executor may keep
        a chunk queued behind the running one)."""
        raise NotImplementedError

    def idle(self, slot) -> bool:
        """True when everything enqueued for the slot has finished."""
        return self.ready(slot)

    def result(self, slot) -> dict:
        """Host copies of the outputs (only after ready())."""
        raise NotImplementedError

    def release(self, slot) -> None:
        raise NotImplementedError


@dataclasses.dataclass
class _Active:
    req: Request
    slot: object
    footprint: int
    t: int = 0
    rt: int = 0                   # reverse steps left in the backward pass
    phase: str = "forward"        # forward -> backward -> done
    t_admit: float = 0.0
    cancel: bool = False


class Scheduler:
    def __init__(self, executor: Executor, budget_bytes: int, max_active: int = 32, chunk: int = 64,
                 clock: Callable[[], float] = time.perf_counter, bchunk: Optional[int] = None,
                 share: Optional[int] = None, cell_cap: Optional[int] = None,
                 chunk_cells: Optional[int] = None):
        bchunk = max(1, chunk // 2) if bchunk is None else bchunk
        if budget_bytes <= 0 or max_active <= 0 or chunk <= 0 or bchunk <= 0:
            raise ValueError("budget, max_active, chunk and bchunk must be positive")
        if share is not None and share <= 0:
            raise ValueError("share must be positive")
        if cell_cap is not None and cell_cap <= 0:
            raise ValueError("cell_cap must be positive")
        self.share = share
        # admission by size: a request joins running ones only while their
        # grid cells together stay within cell_cap (None: no limit), so that
        # grids that fill the device run alone at full speed and only small,
        # launch-bound ones share the launches
        self.cell_cap = cell_cap
        self.cells_active = 0
        # chunks by work instead of steps: a request of N cells takes
        # chunk_cells / N forward steps per iteration (at least `chunk`), so
        # that every chunk is about the same device time and small grids are
        # not held to one scheduler iteration per `chunk` steps
        if chunk_cells is not None and chunk_cells <= 0:
            raise ValueError("chunk_cells must be positive")
        self.chunk_cells = chunk_cells
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.chunk = int(chunk)
        self.bchunk = int(bchunk)
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()
        self.active: Dict[int, _Active] = {}
        self.results: Dict[int, Result] = {}
        self.in_use = 0
        self.peak_in_use = 0
        self._t0 = None
        self._lock = threading.Lock()
        self._cancelled = set()

    # ------------------------------------------------------------ clients
    def now(self) -> float:
        if self._t0 is None:
            self._t0 = self.clock()
        return self.clock() - self._t0

    def submit(self, req: Request) -> None:
        with self._lock:
            self.queue.append(req)

    def cancel(self, rid: int) -> None:
        with self._lock:
            self._cancelled.add(rid)

    def idle(self) -> bool:
        return not self.queue and not self.active

    # --------------------------------------------------------- one iteration
    def _fail(self, req: Request, msg: str, t_admit=math.nan, fp=0):
        self.results[req.rid] = Result(rid=req.rid, kind=req.kind, ok=False, error=msg, t_arrival=req.arrival,
                                       t_admit=t_admit, t_done=self.now(), footprint=fp)

    def _admit(self) -> int:
        n = 0
        while True:
            with self._lock:
                if not self.queue or len(self.active) >= self.max_active:
                    return n
                req = self.queue[0]
                if req.rid in self._cancelled:
                    self.queue.popleft()
                    self._fail(req, "cancelled")
                    continue
            try:
                fp = int(self.ex.footprint(req))
            except Exception as e:       # invalid problem: fails alone
                with self._lock:
                    self.queue.popleft()
                self._fail(req, f"rejected: {e}")
                continue
            if fp > self.budget:
                with self._lock:
                    self.queue.popleft()
                self._fail(req, f"footprint {fp} exceeds the HBM budget {self.budget}", fp=fp)
                continue
            if self.in_use + fp > self.budget:
                return n                  # FIFO: wait for memory to free up
            cells = int(req.problem.N)
            if self.cell_cap is not None and self.active and self.cells_active + cells > self.cell_cap:
                return n                  # FIFO: wait until the running grids leave room
            with self._lock:
                self.queue.popleft()
            t_admit = self.now()
            try:
                slot = self.ex.start(req)
            except Exception as e:
                self._fail(req, f"start failed: {e}", t_admit, fp)
                continue
            self.active[req.rid] = _Active(req=req, slot=slot, footprint=fp, t_admit=t_admit)
            self.in_use += fp
            self.cells_active += cells
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            n += 1

    def _retire(self, a: _Active, ok: bool, error: Optional[str] = None):
        res = Result(rid=a.req.rid, kind=a.req.kind, ok=ok, error=error, t_arrival=a.req.arrival,
                     t_admit=a.t_admit, footprint=a.footprint)
        if ok:
            try:
                out = self.ex.result(a.slot)
                res.J = out.get("J")
                res.trace = out.get("trace")
                res.grad = out.get("grad")
                res.recon = out.get("recon")
                pr = a.req.problem
                res.cell_steps = pr.N * pr.T * (2 if a.req.kind == "gradient" else 1)
            except Exception as e:
                res.ok = False
                res.error = f"result failed: {e}"
        res.t_done = self.now()
        try:
            self.ex.release(a.slot)
        finally:
            self.in_use -= a.footprint
            self.cells_active -= int(a.req.problem.N)
            del self.active[a.req.rid]
            self.results[a.req.rid] = res

    def step(self) -> int:
        """One scheduler iteration; returns how many actions it took."""
        acted = self._admit()
        for rank, rid in enumerate(list(self.active.keys())):
            a = self.active[rid]
            div = self.share if (self.share and rank > 0) else 1
            fc, bc = self.chunk, self.bchunk
            if self.chunk_cells is not None:
                scale = max(1, int(self.chunk_cells // max(1, int(a.req.problem.N))) // self.chunk)
                fc, bc = fc * scale, bc * scale
            fchunk, rchunk = max(2, fc // div), max(1, bc // div)
            if rid in self._cancelled:
                a.cancel = True
            try:
                if not self.ex.ready(a.slot):
                    continue
                if a.cancel:
                    if not self.ex.idle(a.slot):
                        continue
                    self._retire(a, False, "cancelled")
                    acted += 1
                    continue
                T = a.req.problem.T
                if a.phase == "forward" and a.t < T:
                    n = min(fchunk, T - a.t)
                    self.ex.forward(a.slot, n)
                    a.t += n
                elif a.phase == "forward":
                    if a.req.kind == "gradient":
                        a.phase = "backward"
                        a.rt = T
                        n = min(rchunk, a.rt)
                        self.ex.backward(a.slot, n)
                        a.rt -= n
                    else:
                        if not self.ex.idle(a.slot):
                            continue
                        a.phase = "done"
                        self._retire(a, True)
                elif a.phase == "backward" and a.rt > 0:
                    n = min(rchunk, a.rt)
                    self.ex.backward(a.slot, n)
                    a.rt -= n
                elif a.phase == "backward":
                    if not self.ex.idle(a.slot):
                        continue
                    a.phase = "done"
                    self._retire(a, True)
                acted += 1
            except Exception as e:          # a device or API error fails only this request
                if rid in self.active:
                    self._retire(a, False, f"{type(e).__name__}: {e}")
                acted += 1
        self._flush()
        return acted

    def _flush(self):
        """Hand the iteration's chunks to the executor; a failure there fails
        the requests whose work it held (the executor names them)."""
        try:
            self.ex.flush()
        except BatchError as e:
            for rid in e.rids:
                if rid in self.active:
                    self._retire(self.active[rid], False, f"{type(e.cause).__name__}: {e.cause}")

    # -------------------------------------------------------------- driver
    def run(self, requests: List[Request], open_loop: bool = True, poll_s: float = 2e-4,
            sleep: Callable[[float], None] = time.sleep,
            progress: Optional[Callable[[int, int], None]] = None, progress_every: int = 50) -> Dict[int, Result]:
        """Feed `requests` by their arrival times (or all at once) and serve
        until every one has a result.  `progress(done, total)` is called each
        time another `progress_every` results are in."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        total, reported = len(requests), 0
        self.now()
        while pending or not self.idle():
            if progress is not None and len(self.results) // progress_every > reported:
                reported = len(self.results) // progress_every
                progress(len(self.results), total)
            t = self.now()
            while pending and (not open_loop or pending[0].arrival <= t):
                r = pending.popleft()
                if not open_loop:
                    r = dataclasses.replace(r, arrival=t)
                self.submit(r)
            if self.step() == 0:
                if pending and self.idle():
                    sleep(max(0.0, min(pending[0].arrival - self.now(), 0.01)))
                else:
                    sleep(poll_s)
        if progress is not None and len(self.results) // progress_every > reported:
            progress(len(self.results), total)
        return self.results


def summarize(results: Dict[int, Result], wall_s: float) -> dict:
    ok = [r for r in results.values() if r.ok]
    lat = sorted(r.latency for r in ok)

    def pct(q):
        if not lat:
            return None
        i = min(len(lat) - 1, max(0, int(math.ceil(q / 100.0 * len(lat))) - 1))
        return lat[i]
    cells = sum(r.cell_steps for r in ok)
    return {
        "requests": len(results), "ok": len(ok), "failed": len(results) - len(ok),
        "wall_s": wall_s, "throughput_mcell_steps_s": cells / wall_s / 1e6 if wall_s > 0 else None,
        "req_per_s": len(ok) / wall_s if wall_s > 0 else None,
        "p50_latency_s": pct(50), "p99_latency_s": pct(99),
        "mean_latency_s": sum(lat) / len(lat) if lat else None,
    }


# ------------------------------------------------------------ GPU executor

class GpuExecutor(Executor):
    """Slots are libfdtd handles (fdtd.Solver), all on one device stream.
    forward() and backward() only queue a chunk; flush() issues the queued
    chunks of all slots as batch calls (one z-march launch per sweep and per
    reverse step spanning every queued request) and records one event that
    tells each of those slots when its chunk has finished.  A slot takes its
    next chunk while one is still running (ready), so the next batch is
    queued on the stream before the running one ends and the device does not
    wait for the host between iterations."""

    def __init__(self, time_block: int = 0, device: str = "cuda"):
        import torch
        from . import fdtd
        self.torch = torch
        self.fdtd = fdtd
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        # requests are created on a stream of their own: the uploads of a
        # creation then wait only for themselves, not for the batches queued
        # on self.stream; the handle then moves to self.stream
        self.setup = torch.cuda.Stream(device=self.device)
        self.time_block = time_block
        self._fwd = []
        self._bwd = []

    def footprint(self, req: Request) -> int:
        return self.fdtd.footprint(req.problem, record=req.kind == "gradient", time_block=self.time_block) + 256

    def start(self, req: Request):
        with self.torch.cuda.stream(self.setup):
            s = self.fdtd.Solver(req.problem, record=req.kind == "gradient", time_block=self.time_block,
                                 device=str(self.device), stream=self.setup)
        s.set_stream(self.stream)
        with self.torch.cuda.stream(self.stream):
            ev = self.torch.cuda.Event()
            ev.record(self.stream)
            slot = {"s": s, "evs": [ev], "kind": req.kind, "rid": req.rid,
                    "trace": [], "grad": None, "recon": None, "rleft": None}
        return slot

    def forward(self, slot, nsteps: int) -> None:
        self._fwd.append((slot, int(nsteps)))

    def backward(self, slot, nsteps: int) -> None:
        self._bwd.append((slot, int(nsteps)))

    def flush(self) -> None:
        fwd, bwd = self._fwd, self._bwd
        self._fwd, self._bwd = [], []
        if not fwd and not bwd:
            return
        with self.torch.cuda.stream(self.stream):
            if fwd:
                try:
                    outs = self.fdtd.forward_batch([sl["s"] for sl, _ in fwd], [n for _, n in fwd])
                except Exception as e:
                    raise BatchError([sl["rid"] for sl, _ in fwd] + [sl["rid"] for sl, _ in bwd], e)
                for (sl, _), (tr, J) in zip(fwd, outs):
                    sl["trace"].append(tr)
                    sl["J"] = J
            if bwd:
                try:
                    for sl, _ in bwd:
                        if sl["rleft"] is None:          # the pass starts
                            sl["J"] = sl["J"].clone()
                            sl["s"].grad_begin()
                            sl["rleft"] = sl["s"].t
                    self.fdtd.grad_steps_batch([sl["s"] for sl, _ in bwd], [n for _, n in bwd])
                    for sl, n in bwd:
                        sl["rleft"] -= n
                        if sl["rleft"] == 0:             # the pass ends
                            sl["grad"], sl["recon"] = sl["s"].grad_end()
                except Exception as e:
                    raise BatchError([sl["rid"] for sl, _ in bwd], e)
            ev = self.torch.cuda.Event()
            ev.record(self.stream)
        for sl, _ in fwd + bwd:
            sl["evs"].append(ev)

    def _pending(self, slot) -> int:
        evs = slot["evs"]
        while evs and evs[0].query():
            evs.pop(0)
        return len(evs)

    def ready(self, slot) -> bool:
        return self._pending(slot) <= 1

    def idle(self, slot) -> bool:
        return self._pending(slot) == 0

    def result(self, slot) -> dict:
        # (the slot is idle: its work has finished, the copies need no wait
        # on the stream, where other slots' work may be queued)
        out = {"J": float(slot["J"].item())}
        if slot["trace"]:
            out["trace"] = self.torch.cat(slot["trace"]).cpu().numpy()
        if slot["grad"] is not None:
            out["grad"] = slot["grad"].cpu().numpy()
            out["recon"] = float(slot["recon"].item())
        return out

    def release(self, slot) -> None:
        # the workspace was allocated on self.stream, so the allocator orders
        # its reuse after the slot's last (finished) work there
        slot["s"].close()
        slot.clear()


# ------------------------------------------------------------ mock executor

class MockExecutor(Executor):
    """CPU stand-in: work takes simulated time proportional to cell-steps on a
    device that runs up to `lanes` slots at once; `clock` must be the same
    virtual clock the scheduler reads.  Used to test the scheduler policy."""

    def __init__(self, clock, rate_cells_per_s: float = 1e9, lanes: int = 4, fail_rids=(), bad_rids=(),
                 bytes_per_cell: int = 100):
        self.clock = clock
        self.rate = rate_cells_per_s
        self.lanes = lanes
        self.fail_rids = set(fail_rids)      # device error during the forward
        self.bad_rids = set(bad_rids)        # invalid problem (footprint raises)
        self.bpc = bytes_per_cell
        self.live = 0
        self.log = []

    def footprint(self, req: Request) -> int:
        if req.rid in self.bad_rids:
            raise ValueError("invalid problem")
        return req.problem.N * self.bpc

    def start(self, req: Request):
        self.live += 1
        self.log.append(("start", req.rid, self.clock.t))
        return {"rid": req.rid, "busy_until": self.clock.t, "steps": 0, "req": req, "grad": False}

    def _work(self, slot, cells):
        slot["busy_until"] = max(slot["busy_until"], self.clock.t) + cells / self.rate * max(1, self.live) / self.lanes

    def forward(self, slot, nsteps: int) -> None:
        if slot["rid"] in self.fail_rids and slot["steps"] > 0:
            raise RuntimeError("simulated device error")
        slot["steps"] += nsteps
        self._work(slot, slot["req"].problem.N * nsteps)

    def backward(self, slot, nsteps: int) -> None:
        slot["rsteps"] = slot.get("rsteps", 0) + nsteps
        slot["grad"] = slot["rsteps"] == slot["req"].problem.T
        self._work(slot, 2 * slot["req"].problem.N * nsteps)

    def ready(self, slot) -> bool:
        return self.clock.t >= slot["busy_until"]

    def result(self, slot) -> dict:
        pr = slot["req"].problem
        return {"J": float(pr.N * slot["steps"]), "grad": [1.0] if slot["grad"] else None}

    def release(self, slot) -> None:
        self.live -= 1
        self.log.append(("release", slot["rid"], self.clock.t))
