"""Batches of handles (the serving loop's launches): fdtd_forward_batch and
fdtd_grad_steps_batch give every handle the bits of its own single-handle
calls, whatever the batch holds (grids of different sizes and CPML, record
on or off, a TFSF plane, an H point source, sweeps of different lengths, a
handle on the per-cell kernels); the chunked gradient (begin / steps / end)
gives the bits of fdtd_grad; and the batch calls validate their arguments."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2412_12360_amd import workloads as W

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _problems():
    a = W.small_cpml(nx=70, ny=45, nz=38, p=5, T=90, d=8, seed=41, name="a")
    b = W.with_tfsf(W.small_cpml(nx=40, ny=36, nz=44, p=6, T=90, d=8, seed=42, name="b"), comp=1)
    c = W.small_cpml(nx=134, ny=74, nz=40, p=5, T=90, d=8, seed=43, name="c")
    # (33 = 32 + 1: a one-column last x tile; nz 30, so that the wave reaches
    # the detector within the 90 steps)
    d = W.serving_request((33, 61, 30), True, seed=44, p=4, rid=3).with_steps(90)
    return [a, b, c, d]


def _state(s):
    torch.cuda.synchronize()
    return [x.cpu().numpy().copy() for x in s.fields()]


def test_forward_batch_equals_single_calls(monkeypatch):
    from paper_2412_12360_amd.fdtd import Solver, forward_batch
    prs = _problems()
    recs = [True, False, True, True]
    chunks = [[7, 12, 0, 33, 38], [2, 31, 5, 50, 2], [90, 0, 0, 0, 0], [1, 1, 40, 40, 8]]
    announce("forward batch vs single calls, 4 handles")
    single = []
    for pr, rec, ch in zip(prs, recs, chunks):
        s = Solver(pr, record=rec)
        tr = []
        for n in ch:
            t, J = s.forward(n)
            tr.append(t.cpu().numpy().copy())
        single.append((_state(s), np.concatenate(tr), float(J.item()),
                       s.record_step(pr.T - 1).cpu().numpy().copy() if rec else None))
        s.close()
    stream = torch.cuda.current_stream()
    sol = [Solver(pr, record=rec, stream=stream) for pr, rec in zip(prs, recs)]
    trs = [[] for _ in sol]
    for step in range(5):
        outs = forward_batch(sol, [ch[step] for ch in chunks])
        for i, (t, J) in enumerate(outs):
            trs[i].append(t.cpu().numpy().copy())
    for i, s in enumerate(sol):
        st, tr, J, rec = single[i]
        assert s.t == prs[i].T
        for a, b in zip(_state(s), st):
            assert np.array_equal(a, b)
        assert np.array_equal(np.concatenate(trs[i]), tr)
        assert float(s.J.item()) == J
        if rec is not None:
            assert np.array_equal(s.record_step(prs[i].T - 1).cpu().numpy(), rec)


def test_chunked_and_batched_gradient_equal_fdtd_grad(monkeypatch):
    from paper_2412_12360_amd.fdtd import Solver, forward_batch, grad_steps_batch
    prs = _problems()
    announce("gradient: fdtd_grad vs chunks vs batch, 4 handles")
    ref = []
    for pr in prs:
        s = Solver(pr, record=True)
        s.forward()
        g, r = s.grad()
        torch.cuda.synchronize()
        ref.append((g.cpu().numpy().copy(), float(r.item())))
        assert np.abs(ref[-1][0]).max() > 1e-4
        s.close()
    # chunks on one handle
    s = Solver(prs[0], record=True)
    s.forward()
    s.grad_begin()
    for n in (1, 17, 30, 0, 42):
        s.grad_steps(n)
    assert s.t == 0
    g, r = s.grad_end()
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), ref[0][0]) and float(r.item()) == ref[0][1]
    s.close()
    # a batch, with different chunkings, and one handle on the per-cell kernels
    stream = torch.cuda.current_stream()
    sol = []
    for i, pr in enumerate(prs):
        if i == 3:
            monkeypatch.setenv("FDTD_NAIVE", "1")
        sol.append(Solver(pr, record=True, stream=stream))
        monkeypatch.delenv("FDTD_NAIVE", raising=False)
    assert sol[3].kernel_path == "per-cell" and sol[0].kernel_path != "per-cell"
    forward_batch(sol, [pr.T for pr in prs])
    for s in sol:
        s.grad_begin()
    plan = [[10, 10, 70], [45, 45, 0], [1, 88, 1], [30, 30, 30]]
    for k in range(3):
        grad_steps_batch(sol, [p[k] for p in plan])
    for i, s in enumerate(sol):
        assert s.t == 0
        g, r = s.grad_end()
        torch.cuda.synchronize()
        # (the per-cell kernels of handle 3 give the z-march's bits too)
        assert np.array_equal(g.cpu().numpy(), ref[i][0])
        assert float(r.item()) == ref[i][1]


def test_batch_validation():
    from paper_2412_12360_amd.fdtd import Solver, FdtdError, forward_batch, grad_steps_batch
    pr = W.small_cpml(nx=30, ny=28, nz=36, p=5, T=20, d=6, seed=45)
    announce("batch validation")
    s1 = Solver(pr, record=True)
    other = torch.cuda.Stream()
    s2 = Solver(pr, record=True, stream=other)
    with pytest.raises(FdtdError):
        forward_batch([s1, s2], [1, 1])          # two streams
    with pytest.raises(FdtdError):
        forward_batch([s1, s1], [1, 1])          # the same handle twice
    with pytest.raises(FdtdError):
        forward_batch([s1], [-1])
    with pytest.raises(FdtdError):
        forward_batch([s1], [21])                # beyond T
    with pytest.raises(FdtdError):
        grad_steps_batch([s1], [1])              # no gradient running
    forward_batch([s1], [20])
    s1.grad_begin()
    with pytest.raises(FdtdError):
        s1.forward(1)                            # forward during a gradient
    with pytest.raises(FdtdError):
        grad_steps_batch([s1], [21])
    with pytest.raises(FdtdError):
        s1.grad_end()                            # t != 0
    grad_steps_batch([s1], [20])
    g, _ = s1.grad_end()
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()


def test_set_stream_moves_a_handle_between_streams():
    """A handle created on one stream and moved with fdtd_set_stream to
    another (the serving loop's creation stream, then its batch stream) gives
    the bits of a handle that stays on one stream, forward and gradient; a
    move during a chunked gradient is refused."""
    from paper_2412_12360_amd.fdtd import FdtdError, Solver
    pr = W.small_cpml(nx=70, ny=45, nz=38, p=5, T=90, d=8, seed=45, name="mv")
    announce("set_stream: forward + gradient on a moved handle")
    ref = Solver(pr, record=True)
    ref.forward()
    g0, _ = ref.grad()
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(a):
        s = Solver(pr, record=True, stream=a)
    s.set_stream(b)
    with torch.cuda.stream(b):
        s.forward(25)
        s.forward(65)
        g1, _ = s.grad()
        s.forward()
        s.grad_begin()
        with pytest.raises(FdtdError, match="E_STATE"):
            s.set_stream(a)
        s.grad_steps(90)
        s.grad_end()
    torch.cuda.synchronize()
    assert torch.equal(g0, g1)
    assert float(g0.abs().max()) > 1e-3
