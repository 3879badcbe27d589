"""Parity at the benchmark sizes, in the launch configuration bench.py times
(default time block, tile classes, z chunks):
  - 256^3 with a 10-cell CPML and 640x640x400 with a 12-cell CPML: a random
    interior+PML field state advanced a few steps with the source and
    detector on, against the FP64 oracle on the whole grid;
  - 200^3 and 640x640x400: the adjoint (fused reverse kernel) is the exact
    transpose of the forward step map, <M x, y> = <x, M^T y>, on random states
    including every CPML auxiliary array;
  - 200^3 (1500 steps) and 640x640x400 (4000 steps): the time-reversal
    gradient against central differences of the GPU objective along the
    gradient direction and along its restriction to the lower half of the
    design box.  Each such check fixes one projection of the gradient only
    (the true gradient's component along v against the computed one); the
    element-wise comparison of the 200^3 gradient with the FP64 oracle is in
    test_gpu_reverse_classes.py.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import NSLOT, Oracle
from paper_2412_12360_amd import workloads as W

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def held_mask_t(pr, dev):
    k = torch.arange(pr.nz, device=dev).view(-1, 1, 1)
    j = torch.arange(pr.ny, device=dev).view(1, -1, 1)
    i = torch.arange(pr.nx, device=dev).view(1, 1, -1)
    return [(j == 0) | (k == 0), (i == 0) | (k == 0), (i == 0) | (j == 0)]


def random_fields(pr, s, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    hm = held_mask_t(pr, s.device)
    fs = s.fields(0)
    for q in range(6):
        fs[q].copy_(torch.randn(fs[q].shape, generator=g, device="cuda"))
        if q < 3:
            fs[q][hm[q].expand_as(fs[q])] = 0.0
    torch.cuda.synchronize()
    return np.stack([f.cpu().numpy().astype(np.float64) for f in fs])


@pytest.mark.parametrize("which,steps", [("c2", 12), ("c4", 6)])
def test_random_state_forward_parity_full_size(which, steps):
    from paper_2412_12360_amd.fdtd import Solver
    pr = W.config2(T=steps) if which == "c2" else W.config4(T=steps)
    announce(f"full-size forward {which} {pr.nx}x{pr.ny}x{pr.nz} steps={steps}")
    s = Solver(pr)
    f0 = random_fields(pr, s, 7)
    s.forward()
    torch.cuda.synchronize()
    got = [f.cpu().numpy() for f in s.fields()]
    del s
    torch.cuda.empty_cache()
    o = Oracle(pr)
    st = np.zeros((NSLOT, pr.nz, pr.ny, pr.nx))
    st[:6] = f0
    del f0
    J, trace, _ = o.forward(st, steps)
    num = sum(float(np.sum((got[q] - st[q]) ** 2)) for q in range(6))
    den = sum(float(np.sum(st[q] ** 2)) for q in range(6))
    assert np.sqrt(num / den) <= 1e-5
    # the PML slabs took part: their fields differ from the plain interior update
    assert np.max(np.abs(st[6:])) > 0


@pytest.mark.parametrize("which", ["c3", "c4"])
def test_adjoint_transpose_full_size(which):
    from paper_2412_12360_amd.fdtd import Solver
    pr = W.config3(T=4) if which == "c3" else W.config4(T=4)
    announce(f"full-size dot product {which}")
    s = Solver(pr, record=True)
    g = torch.Generator(device="cuda").manual_seed(11)
    hm = held_mask_t(pr, s.device)
    xs, ys = s.state_arrays(0), s.state_arrays(1)
    for arr in xs + ys:
        arr.copy_(torch.randn(arr.numel(), generator=g, device="cuda"))
    for q in range(3):
        xs[q].view(pr.nz, pr.ny, pr.nx)[hm[q].expand(pr.nz, pr.ny, pr.nx)] = 0.0
        ys[q].view(pr.nz, pr.ny, pr.nx)[hm[q].expand(pr.nz, pr.ny, pr.nx)] = 0.0
    x0 = [a.clone() for a in xs]
    y0 = [a.clone() for a in ys]
    s.linear_steps(2, adjoint=False)
    s.linear_steps(2, adjoint=True)
    torch.cuda.synchronize()
    Mx, Mty = s.state_arrays(0), s.state_arrays(1)
    dot = lambda a, b: float(torch.dot(a.double(), b.double()))
    lhs = sum(dot(a, b) for a, b in zip(Mx, y0))
    rhs = sum(dot(a, b) for a, b in zip(x0, Mty))
    scale = np.sqrt(sum(dot(a, a) for a in Mx) * sum(dot(b, b) for b in y0))
    assert abs(lhs - rhs) <= 2e-6 * scale


@pytest.mark.parametrize("which", ["c3", "c4"])
def test_directional_fd_full_size(which):
    """c3 (200^3, CPML 10, 1500 steps) and c4 (640x640x400, CPML 12, 4000
    steps, 54 GB of interface record): the time-reversal gradient against a
    central difference of the GPU objective in eps_r along the gradient's
    own direction v = g/|g| and along its restriction to the lower half of
    the design cube.  Agreement says g_true . v = g . v for those two
    directions: a consistency check of the whole pipeline at size, not a
    proof that g equals g_true (a g with an error orthogonal to g_true can
    pass).  A random direction is not resolvable here: it moves J by about
    one float32 ulp.  The step is chosen so that J changes by about 1e-3 of
    itself, in the linear regime."""
    from paper_2412_12360_amd.fdtd import Solver
    from paper_2412_12360_amd.autograd import objective
    pr = W.config3() if which == "c3" else W.config4()
    announce(f"full-size directional finite difference {which}")
    s = Solver(pr, record=True)
    eps = torch.tensor(W.eps_from_rho(pr.rho), dtype=torch.float32, device=s.device).requires_grad_(True)
    J = objective(eps, s)
    J.backward()
    g = eps.grad.detach().double()
    J0 = float(J.item())
    half = g.clone()
    half[g.shape[0] // 2:] = 0.0
    for name, v in (("gradient", g.clone()), ("lower half", half)):
        v = v / v.norm()
        dJ = float((g * v).sum().item())
        h = min(2.0, 1e-3 * abs(J0) / max(abs(dJ), 1e-30))
        with torch.no_grad():
            Jp = float(objective((eps.double() + h * v).float(), s).item())
            Jm = float(objective((eps.double() - h * v).float(), s).item())
        fd = (Jp - Jm) / (2 * h)
        print(f"[gpu-case] {which} {name}: J {J0:.6e} h {h:.3e} adjoint {dJ:.6e} fd {fd:.6e}", flush=True)
        assert abs(Jp - Jm) > 1e-5 * abs(J0)          # resolvable in float32 (about 90 ulps of J)
        assert abs(fd - dJ) <= 2e-2 * abs(dJ)
