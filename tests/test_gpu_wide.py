"""Forward and reverse z-marches with a 64-bit base per component and plane,
the instances a handle runs when one field set spans 4 GiB or more (above
about 179M cells), through the C ABI:
  - forced onto small ragged grids (FDTD_TB_WIDE), they give the bits of the
    32-bit-offset instances: the forward at every time-block size, and the
    recorded forward plus the time-reversal gradient, with the one-sided
    plane wave, an H point source, a plain and an interpolated flux detector;
  - on a PEC box, fdtd_inverse gives the bits of the 32-bit instance;
  - at full size, one GPU's z-slab of a 2400x1600x600 grid (2400x1600x150,
    576M cells, 12-cell CPML), they are chosen by themselves and give the
    bits of the per-cell kernels, forward alone and forward plus gradient.
All comparisons are bitwise: the instances differ only in addressing.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2412_12360_amd import workloads as W

pytestmark = pytest.mark.gpu


def _solver(*a, **k):
    from paper_2412_12360_amd.fdtd import Solver
    return Solver(*a, **k)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def problem(shape, p, T):
    pr = W.with_tfsf(W.small_cpml(nx=shape[0], ny=shape[1], nz=shape[2], p=p, T=T, d=8, seed=21))
    q = W.Source(kind=0, comp=4, i=pr.nx // 3, j=pr.ny // 2 + 1, k=pr.nz // 2 + 3,
                 amp=W.gaussian_pulse(pr.T, 16, 5))
    d0 = pr.detectors[0]
    d1 = dataclasses.replace(d0, k=d0.k - 2, i0=d0.i0 + 1, j0=d0.j0 + 2, weight=0.5, interpolate=True)
    return dataclasses.replace(pr, sources=list(pr.sources) + [q], detectors=[d0, d1])


def shard_probe(T):
    """The 2400x1600x150 slab with the sheet (unit amplitude) and the flux
    plane three cells apart inside the design box, so that a few steps give a
    nonzero trace, objective and gradient."""
    pr = W.shard_slab(T=T)
    src = W.Source(kind=1, comp=0, i=0, j=0, k=108, amp=np.ones(T, np.float32))
    det = dataclasses.replace(pr.detectors[0], k=111)
    return dataclasses.replace(pr, sources=[src], detectors=[det])


def run(pr, K, wide, monkeypatch, naive=False):
    monkeypatch.setenv("FDTD_TB_WIDE", "1" if wide else "0")
    monkeypatch.setenv("FDTD_NAIVE", "1" if naive else "0")
    s = _solver(pr, record=False, time_block=K)
    want = "per-cell" if naive else ("z-march-wide" if wide else "z-march")
    assert s.kernel_path == want
    tr, J = s.forward()
    torch.cuda.synchronize()
    return s, {
        "fields": torch.stack([f.clone() for f in s.fields()]),
        "psi": [a.clone() for a in s.state_arrays(0)[6:]],
        "trace": tr.clone(),
        "J": J.clone(),
    }


# (step counts long enough for the wave to reach the detector; the PEC box
# has no detector)
@pytest.mark.parametrize("shape,p,T", [((70, 45, 38), 5, 90), ((33, 61, 70), 6, 200), ((40, 36, 44), 0, 25)])
def test_wide_instance_bitwise_all_K(shape, p, T, monkeypatch):
    pr = problem(shape, p, T) if p > 0 else W.config1(T=T, n=shape[0])
    for K in (1, 2, 3, 4):
        announce(f"wide vs narrow z-march {shape} p={p} T={T} K={K}")
        _, ref = run(pr, K, False, monkeypatch)
        assert p == 0 or float(ref["trace"].abs().max()) > 1.0
        _, out = run(pr, K, True, monkeypatch)
        assert torch.equal(out["fields"], ref["fields"])
        for x, y in zip(out["psi"], ref["psi"]):
            assert torch.equal(x, y)
        assert torch.equal(out["trace"], ref["trace"])
        assert torch.equal(out["J"], ref["J"])


# (enough steps for the wave to pass the design cube and reach the detector)
@pytest.mark.parametrize("shape,p,T", [((70, 45, 38), 5, 100), ((33, 61, 70), 6, 220)])
def test_wide_gradient_bitwise(shape, p, T, monkeypatch):
    pr = problem(shape, p, T)
    outs = []
    for wide in (False, True):
        announce(f"{'wide' if wide else 'narrow'} recorded forward + gradient {shape} p={p} T={T}")
        monkeypatch.setenv("FDTD_TB_WIDE", "1" if wide else "0")
        monkeypatch.setenv("FDTD_NAIVE", "0")
        s = _solver(pr, record=True, time_block=2)
        assert s.kernel_path == ("z-march-wide" if wide else "z-march")
        _, J = s.forward()
        rec = torch.stack([s.record_step(i).clone() for i in range(pr.T)])
        g, r = s.grad()
        torch.cuda.synchronize()
        outs.append((J.clone(), rec, g.clone(), r.clone(), torch.stack([f.clone() for f in s.fields()])))
    assert float(outs[0][2].abs().max().item()) > 1e-3
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_wide_inverse_on_pec_box(monkeypatch):
    pr = W.config1(T=60)
    announce("wide forward + inverse on the 32^3 PEC box")
    outs = []
    for wide in (False, True):
        s, _ = run(pr, 2, wide, monkeypatch)
        s.inverse(pr.T // 2)
        torch.cuda.synchronize()
        outs.append(torch.stack([f.clone() for f in s.fields()]))
    assert torch.equal(outs[0], outs[1])


def test_wide_chosen_and_bitwise_at_shard_size(monkeypatch):
    """2400x1600x150 (the field set is 13.8 GB): eight steps of the wide
    z-march against eight steps of the per-cell kernels."""
    pr = shard_probe(8)
    announce("wide z-march at 2400x1600x150, 8 steps")
    monkeypatch.delenv("FDTD_TB_WIDE", raising=False)
    monkeypatch.setenv("FDTD_NAIVE", "0")
    s = _solver(pr, record=False, time_block=2)
    assert s.kernel_path == "z-march-wide"
    tr, J = s.forward()
    torch.cuda.synchronize()
    wide = [f.clone() for f in s.fields()]
    tw, Jw = tr.clone(), J.clone()
    del s, tr, J
    torch.cuda.empty_cache()
    announce("per-cell kernels at 2400x1600x150, 8 steps")
    monkeypatch.setenv("FDTD_NAIVE", "1")
    s = _solver(pr, record=False, time_block=2)
    assert s.kernel_path == "per-cell"
    tr, J = s.forward()
    torch.cuda.synchronize()
    assert float(wide[0].abs().max().item()) > 0.0
    assert float(tw.abs().max().item()) > 0.0
    for a, b in zip(wide, s.fields()):
        assert torch.equal(a, b)
    assert torch.equal(tw, tr)
    assert torch.equal(Jw, J)


def test_wide_gradient_at_shard_size(monkeypatch):
    """2400x1600x150 with the record: eight steps forward and back on the wide
    marches against the per-cell kernels (J, dJ/deps over the 1200x800x75
    design box, reconstruction error)."""
    pr = shard_probe(8)
    monkeypatch.delenv("FDTD_TB_WIDE", raising=False)
    outs = []
    for naive in (False, True):
        announce(f"{'per-cell' if naive else 'wide'} forward + gradient at 2400x1600x150, 8 steps")
        monkeypatch.setenv("FDTD_NAIVE", "1" if naive else "0")
        s = _solver(pr, record=True, time_block=2)
        assert s.kernel_path == ("per-cell" if naive else "z-march-wide")
        _, J = s.forward()
        g, r = s.grad()
        torch.cuda.synchronize()
        outs.append((J.clone(), g.clone(), r.clone()))
        del s, g, r, J
        torch.cuda.empty_cache()
    assert float(outs[0][0].abs().item()) > 0.0
    assert float(outs[0][1].abs().max().item()) > 0.0
    for a, b in zip(*outs):
        assert torch.equal(a, b)
