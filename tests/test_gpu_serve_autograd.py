"""GPU: the autograd objective against the FP64 oracle, and the serving loop:
each request's result is bitwise the same alone and in the mix."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle
from paper_2412_12360_amd import workloads as W

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def test_autograd_rho_gradient_matches_oracle():
    from paper_2412_12360_amd.autograd import objective
    from paper_2412_12360_amd.fdtd import Solver
    pr = W.small_cpml(nx=30, ny=28, nz=36, p=5, T=130, d=6, seed=21)
    announce("autograd 30x28x36")
    o = Oracle(pr)
    g, J, _ = o.grad_history()
    ref = 10.0 * o.deps_design(g)
    s = Solver(pr, record=True)
    rho = torch.tensor(pr.rho, dtype=torch.float32, device="cuda", requires_grad=True)
    Jt = objective(2.25 + 10.0 * rho, s)
    Jt.backward()
    torch.cuda.synchronize()
    assert abs(float(Jt.item()) - J) <= 1e-4 * abs(J)
    got = rho.grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-3 * np.linalg.norm(ref)
    # a second evaluation at another design reuses the handle
    rho2 = (rho.detach() * 0.5).requires_grad_(True)
    J2 = objective(2.25 + 10.0 * rho2, s)
    J2.backward()
    assert torch.isfinite(rho2.grad).all() and float(J2.item()) != float(Jt.item())


def _mix(count=6):
    reqs = []
    from paper_2412_12360_amd import serve
    rng = np.random.default_rng(5)
    for i in range(count):
        e = tuple(int(v) for v in rng.integers(24, 44, size=3))
        pr = W.serving_request(e, i % 2 == 1, seed=100 + i, p=4, rid=i)
        pr = pr.with_steps(96)
        reqs.append(serve.Request(rid=i, kind="gradient" if i % 2 else "forward", problem=pr, arrival=0.0))
    return reqs


def test_serving_result_same_alone_and_in_mix():
    from paper_2412_12360_amd import serve
    reqs = _mix()
    announce("serving alone")
    alone = {}
    for r in reqs:
        sch = serve.Scheduler(serve.GpuExecutor(), budget_bytes=8 << 30, max_active=1, chunk=32)
        alone.update(sch.run([r], open_loop=False))
    announce("serving mix")
    sch = serve.Scheduler(serve.GpuExecutor(), budget_bytes=8 << 30, max_active=6, chunk=16)
    mix = sch.run(reqs, open_loop=False)
    for r in reqs:
        a, b = alone[r.rid], mix[r.rid]
        assert a.ok and b.ok, (a.error, b.error)
        assert a.J == b.J
        assert np.array_equal(a.trace, b.trace)
        if r.kind == "gradient":
            assert np.array_equal(a.grad, b.grad)
            assert a.recon == b.recon


def test_serving_admission_respects_budget_on_gpu():
    from paper_2412_12360_amd import fdtd, serve
    reqs = _mix(5)
    fps = [fdtd.footprint(r.problem, record=r.kind == "gradient") + 256 for r in reqs]
    budget = max(fps) * 2
    announce("serving budget")
    sch = serve.Scheduler(serve.GpuExecutor(), budget_bytes=budget, max_active=8, chunk=32)
    res = sch.run(reqs, open_loop=False)
    assert all(r.ok for r in res.values())
    assert sch.peak_in_use <= budget
