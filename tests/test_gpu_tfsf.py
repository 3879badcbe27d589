"""H-field sources and the one-sided total-field/scattered-field plane on the
GPU (arXiv 2412.12360, section 2.1 names TFSF as its source type), through
the C ABI:
  - fields, flux trace and objective against the FP64 oracle, which runs its
    own incident line (both polarisations, ragged multi-tile grids);
  - below the plane of a wide PEC box the GPU field stays at rounding level
    (the wave is launched one way);
  - the z-march at every time-block size gives the per-cell kernels' bits,
    and the fused reverse gives the per-cell reverse step's bits;
  - the time-reversal gradient against the oracle's stored-history gradient;
  - fdtd_set_inv_eps reruns the incident line with the plane's new material.
Tolerances as in the other parity tests: fields rel-L2 <= 1e-4, gradients
rel-L2 <= 1e-3.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle
from paper_2412_12360_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-4
GRAD_TOL = 1e-3


def _solver(*a, **k):
    from paper_2412_12360_amd.fdtd import Solver
    return Solver(*a, **k)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def gpu_fields(s):
    torch.cuda.synchronize()
    return np.stack([f.cpu().numpy().astype(np.float64) for f in s.fields()])


def tfsf_cpml(shape, p, T, pol=0, d=8, seed=11):
    pr = W.small_cpml(nx=shape[0], ny=shape[1], nz=shape[2], p=p, T=T, d=d, seed=seed)
    return W.with_tfsf(pr, comp=pol)


def with_h_point(pr, comp=5):
    """An extra H point source in the interior (Gaussian pulse)."""
    q = W.Source(kind=0, comp=comp, i=pr.nx // 3, j=pr.ny // 2 + 1, k=pr.nz // 2 + 3,
                 amp=W.gaussian_pulse(pr.T, 16, 5))
    return dataclasses.replace(pr, sources=list(pr.sources) + [q])


@pytest.mark.parametrize("shape,p,T,pol", [((40, 36, 44), 6, 160, 0), ((67, 29, 23), 4, 90, 1)])
def test_tfsf_forward_parity(shape, p, T, pol):
    pr = tfsf_cpml(shape, p, T, pol)
    announce(f"tfsf forward {shape} p={p} T={T} pol={pol}")
    st, J, trace, _ = Oracle(pr).run()
    s = _solver(pr)
    tr, Jg = s.forward()
    f = gpu_fields(s)
    assert rel_l2(f, st[:6]) <= FIELD_TOL
    assert rel_l2(tr.cpu().numpy(), trace) <= FIELD_TOL
    assert abs(float(Jg.item()) - J) <= FIELD_TOL * abs(J)


def test_h_point_source_parity():
    pr = with_h_point(W.small_cpml(nx=45, ny=38, nz=41, p=5, T=120))
    announce("H point source + sheet 45x38x41 p=5 T=120")
    st, J, trace, _ = Oracle(pr).run()
    s = _solver(pr)
    tr, Jg = s.forward()
    f = gpu_fields(s)
    assert rel_l2(f, st[:6]) <= FIELD_TOL
    assert abs(float(Jg.item()) - J) <= FIELD_TOL * abs(J)


def test_tfsf_one_sided_on_gpu():
    """A PEC box wide enough that the central columns cannot see a side wall
    within T steps: there the field below the plane is zero in exact
    arithmetic; on the GPU it stays at FP32 rounding level, and the whole
    field matches the oracle."""
    T, k0 = 60, 6
    n, nz = 2 * T + 10, k0 + T + 6
    inv = np.full((nz, n, n), 1.0 / 2.25, np.float32)
    src = W.Source(kind=2, comp=0, i=0, j=0, k=k0, amp=W.ramped_sine(T, W.courant(), lambda0=12.0, periods=1))
    pr = W.Problem(name="tfsf_pec", nx=n, ny=n, nz=nz, S=W.courant(), p=0, pml_m=3.0, pml_sigma_max=0.0,
                   pml_kappa_max=1.0, pml_alpha_max=0.0, inv_eps=inv, sources=[src], detectors=[],
                   design_lo=(0, 0, 0), design_hi=(1, 1, 1), T=T)
    announce(f"tfsf one-sided PEC {n}x{n}x{nz} T={T}")
    st, _, _, _ = Oracle(pr).run()
    s = _solver(pr)
    s.forward()
    f = gpu_fields(s)
    assert rel_l2(f, st[:6]) <= FIELD_TOL
    c = slice(T + 3, n - T - 3)
    scale = np.max(np.abs(f[0][:, c, c]))
    assert scale > 0.1
    assert np.max(np.abs(f[:, :k0, c, c])) <= 1e-5 * scale


def run(pr, K, naive, monkeypatch):
    monkeypatch.setenv("FDTD_NAIVE", "1" if naive else "0")
    s = _solver(pr, record=True, time_block=K)
    tr, J = s.forward()
    torch.cuda.synchronize()
    return {
        "fields": torch.stack([f.clone() for f in s.fields()]),
        "psi": [a.clone() for a in s.state_arrays(0)[6:]],
        "trace": tr.clone(),
        "J": J.clone(),
        "rec": torch.stack([s.record_step(i).clone() for i in range(pr.T)]),
    }


# (step counts long enough for the wave to reach the detector)
@pytest.mark.parametrize("shape,p,T", [((70, 45, 38), 5, 90), ((33, 61, 70), 6, 200)])
def test_tfsf_and_h_source_bitwise_all_K(shape, p, T, monkeypatch):
    pr = with_h_point(tfsf_cpml(shape, p, T))
    announce(f"tfsf + H point bitwise {shape} p={p} T={T} naive")
    ref = run(pr, 1, True, monkeypatch)
    assert float(ref["trace"].abs().max()) > 1.0
    for K in (1, 2, 3, 4):
        announce(f"tfsf + H point bitwise {shape} p={p} T={T} K={K}")
        out = run(pr, K, False, monkeypatch)
        assert torch.equal(out["fields"], ref["fields"])
        for x, y in zip(out["psi"], ref["psi"]):
            assert torch.equal(x, y)
        assert torch.equal(out["trace"], ref["trace"])
        assert torch.equal(out["J"], ref["J"])
        assert torch.equal(out["rec"], ref["rec"])


def test_tfsf_gradient_parity():
    pr = with_h_point(tfsf_cpml((40, 36, 44), 6, 160, seed=12))
    announce("tfsf + H point gradient 40x36x44 p=6 T=160")
    o = Oracle(pr)
    g, J, _ = o.grad_history()
    ref = o.deps_design(g)
    assert np.linalg.norm(ref) > 1e-8 * abs(J)
    s = _solver(pr, record=True)
    _, Jg = s.forward()
    dg, recon = s.grad()
    torch.cuda.synchronize()
    assert abs(float(Jg.item()) - J) <= FIELD_TOL * abs(J)
    assert rel_l2(dg.cpu().numpy(), ref) <= GRAD_TOL
    assert float(recon.item()) < 1e-3


def test_tfsf_fused_reverse_bitwise_equal_to_per_cell(monkeypatch):
    pr = with_h_point(tfsf_cpml((70, 45, 38), 5, 100, seed=31))
    announce("tfsf + H point fused reverse bitwise 70x45x38")
    outs = []
    for naive in (True, False):
        monkeypatch.setenv("FDTD_NAIVE", "1" if naive else "0")
        s = _solver(pr, record=True)
        _, J = s.forward()
        g, r = s.grad()
        torch.cuda.synchronize()
        outs.append((J.clone(), g.clone(), r.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    assert float(outs[1][1].abs().max()) > 1e-3


def test_set_inv_eps_reruns_incident_line():
    """Changing the plane's material through fdtd_set_inv_eps gives the bits
    of a solver created with that material (the incident line is rerun)."""
    pr = tfsf_cpml((40, 36, 44), 6, 80)
    k0 = pr.sources[0].k
    inv2 = pr.inv_eps.copy()
    inv2[k0 - 1: k0 + 1] = np.float32(1.0 / 4.0)
    pr2 = dataclasses.replace(pr, inv_eps=inv2)
    announce("tfsf set_inv_eps 40x36x44")
    a = _solver(pr)
    a.fdtd_set_inv_eps(torch.from_numpy(inv2).to(a.device))
    a.forward()
    b = _solver(pr2)
    b.forward()
    c = _solver(pr)
    c.forward()
    torch.cuda.synchronize()
    fa, fb, fc = (torch.stack([f.clone() for f in x.fields()]) for x in (a, b, c))
    assert torch.equal(fa, fb)
    assert not torch.equal(fa, fc)
