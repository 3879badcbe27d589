"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/fdtd.h declares, and validates arguments before touching a device."""
import ctypes as C
import dataclasses
import os
import re

import pytest

from paper_2412_12360_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _F():
    from paper_2412_12360_amd import fdtd as F
    return F


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "fdtd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:fdtd_status|const char \*|size_t)\s*(fdtd_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    F = _F()
    L = F.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert sorted(F.ENTRY_POINTS) == names


def _fp(prob, **kw):
    F = _F()
    return F.footprint(prob, **kw)


def test_footprint_grows_with_record():
    pr = W.small_cpml()
    a = _fp(pr)
    b = _fp(pr, record=True)
    N = pr.N
    assert a >= 4 * (12 * N + N)          # two field buffers + coefficients
    assert b > a + 4 * 6 * N              # adjoint fields + record


def test_footprint_record_bytes_match_six_slices():
    pr = W.small_cpml(nx=40, ny=36, nz=44, p=6, T=100)
    a = _fp(pr, record=True)
    b = _fp(pr.with_steps(200), record=True)
    Lx, Ly, Lz = 28, 24, 32
    per_step = 2 * 2 * (Ly * Lz + Lx * Lz + Lx * Ly) * 4
    # 100 more steps: record + trace + amplitudes
    extra = b - a
    assert per_step * 100 <= extra <= per_step * 100 + 100 * 4 * 8 + 4096


@pytest.mark.parametrize("mutate,what", [
    (lambda d: setattr(d, "courant", 0.6), "courant"),
    (lambda d: setattr(d, "nx", 2), "grid size"),
    (lambda d: setattr(d, "pml_cells", 30), "PML"),
    (lambda d: setattr(d, "time_block", 9), "time_block"),
    (lambda d: setattr(d, "n_steps", 0), "n_steps"),
])
def test_invalid_descriptor_rejected(mutate, what):
    F = _F()
    pr = W.small_cpml()
    d = F.make_desc(pr, 1, record=True)
    mutate(d)
    out = C.c_size_t(0)
    st = F.lib().fdtd_footprint(C.byref(d), F.make_sources(pr, [1]), 1, F.make_detectors(pr), 1, C.byref(out))
    assert st == F.FDTD_E_INVALID
    assert what.lower() in F.lib().fdtd_last_error(None).decode().lower()


def test_detector_outside_interior_rejected_when_recording():
    F = _F()
    pr = W.small_cpml()
    det = F.make_detectors(pr)
    det[0].k = 1
    d = F.make_desc(pr, 1, record=True)
    out = C.c_size_t(0)
    st = F.lib().fdtd_footprint(C.byref(d), F.make_sources(pr, [1]), 1, det, 1, C.byref(out))
    assert st == F.FDTD_E_INVALID
    d = F.make_desc(pr, 1, record=False)
    assert F.lib().fdtd_footprint(C.byref(d), F.make_sources(pr, [1]), 1, det, 1, C.byref(out)) == F.FDTD_OK


def test_bad_source_and_create_arguments():
    F = _F()
    pr = W.small_cpml()
    d = F.make_desc(pr, 1)
    src = F.make_sources(pr, [1])
    src[0].comp = 6
    out = C.c_size_t(0)
    assert F.lib().fdtd_footprint(C.byref(d), src, 1, F.make_detectors(pr), 1, C.byref(out)) == F.FDTD_E_INVALID
    # a too-small workspace is refused before any device work
    h = C.c_void_p(0)
    st = F.lib().fdtd_create(C.byref(d), F.make_sources(pr, [1]), 1, F.make_detectors(pr), 1,
                             C.c_void_p(256), C.c_size_t(1024), None, C.byref(h))
    assert st == F.FDTD_E_NOMEM and not h.value
    assert F.lib().fdtd_forward(None, 1, None, None) == F.FDTD_E_INVALID


def _status(pr, record=False):
    F = _F()
    d = F.make_desc(pr, 1, record=record)
    out = C.c_size_t(0)
    st = F.lib().fdtd_footprint(C.byref(d), F.make_sources(pr, [1] * len(pr.sources)), len(pr.sources),
                                F.make_detectors(pr), len(pr.detectors), C.byref(out))
    return st, int(out.value)


def test_h_sources_and_tfsf_accepted():
    F = _F()
    pr = W.small_cpml(nx=40, ny=36, nz=44, p=6, T=100)
    amp = pr.sources[0].amp
    for comp in range(6):
        q = W.Source(kind=0, comp=comp, i=20, j=18, k=22, amp=amp)
        assert _status(W.dataclasses.replace(pr, sources=[q]))[0] == F.FDTD_OK
    st, fp_tfsf = _status(W.with_tfsf(pr), record=True)
    assert st == F.FDTD_OK
    # the TFSF waveform and its incident line live in the workspace
    assert fp_tfsf > _status(pr, record=True)[1]


@pytest.mark.parametrize("change,what", [
    (dict(comp=2), "polarisation"),       # only Ex or Ey
    (dict(k=6), "[p+1, nz-p)"),           # H layer k-1 inside the CPML
    (dict(k=38), "[p+1, nz-p)"),          # E plane inside the CPML
    (dict(k=19), "design box"),           # layer k-1 = 18 is the design box's first layer
])
def test_tfsf_placement_validated(change, what):
    F = _F()
    pr = W.with_tfsf(W.small_cpml(nx=40, ny=36, nz=44, p=6, T=100))   # design z in [18, 26)
    src = W.dataclasses.replace(pr.sources[0], **change)
    st, _ = _status(W.dataclasses.replace(pr, sources=[src]))
    assert st == F.FDTD_E_INVALID
    assert what.lower() in F.lib().fdtd_last_error(None).decode().lower()


def test_tfsf_takes_two_source_slots():
    F = _F()
    pr = W.with_tfsf(W.small_cpml(nx=40, ny=36, nz=44, p=6, T=100))
    extra = [W.Source(kind=0, comp=2, i=20, j=18, k=30, amp=pr.sources[0].amp)] * 3
    assert _status(W.dataclasses.replace(pr, sources=pr.sources + extra[:2]))[0] == F.FDTD_OK
    st, _ = _status(W.dataclasses.replace(pr, sources=pr.sources + extra))
    assert st == F.FDTD_E_INVALID
    assert "slots" in F.lib().fdtd_last_error(None).decode()


@pytest.mark.parametrize("change", [dict(k=0), dict(i1=40), dict(j1=36), dict(interpolate=2)])
def test_interpolated_detector_placement_validated(change):
    F = _F()
    pr = W.small_cpml(nx=40, ny=36, nz=44, p=0, T=50)
    det = W.Detector(k=10, i0=0, i1=39, j0=0, j1=35, interpolate=True)
    assert _status(W.dataclasses.replace(pr, detectors=[det]))[0] == F.FDTD_OK
    bad = W.dataclasses.replace(det, **change)
    st, _ = _status(W.dataclasses.replace(pr, detectors=[bad]))
    assert st == F.FDTD_E_INVALID


@pytest.mark.parametrize("change,ok", [(dict(quantity=1), True), (dict(quantity=1, interpolate=False), False),
                                       (dict(quantity=2), False)])
def test_energy_detector_validated(change, ok):
    F = _F()
    pr = W.small_cpml(nx=40, ny=36, nz=44, p=0, T=50)
    det = W.dataclasses.replace(W.Detector(k=10, i0=0, i1=39, j0=0, j1=35, interpolate=True), **change)
    st, _ = _status(W.dataclasses.replace(pr, detectors=[det]))
    assert st == (F.FDTD_OK if ok else F.FDTD_E_INVALID)


def test_lossy_box_record_and_validation():
    """Conducting cells add E^n of the lossy box to each step's record (three
    floats per box cell) plus sigma and ca per box cell; the box must lie in
    the interior and off the layers of a TFSF plane."""
    F = _F()
    pr = W.small_cpml(nx=40, ny=36, nz=44, p=6, T=100, d=8)
    lp = W.with_lossy(pr)
    nb = 8 * 8 * 8
    a = _fp(pr, record=True)
    b = _fp(lp, record=True)
    assert 4 * (3 * nb * 100 + 2 * nb) <= b - a <= 4 * (3 * nb * 100 + 2 * nb) + 3 * 256
    # forward only: no record, just the coefficients
    assert 0 < _fp(lp) - _fp(pr) <= 4 * 2 * nb + 2 * 256

    def status(prob):
        d = F.make_desc(prob, 1, record=True, sigma_ptr=1)
        out = C.c_size_t(0)
        return F.lib().fdtd_footprint(C.byref(d), F.make_sources(prob, [1] * len(prob.sources)),
                                      len(prob.sources), F.make_detectors(prob), len(prob.detectors), C.byref(out))
    import dataclasses
    for lo, hi in [((5, 14, 14), (13, 22, 22)),      # x below the interior
                   ((14, 14, 14), (14, 22, 22)),     # empty along x
                   ((14, 14, 30), (22, 22, 39))]:    # z beyond nz - p
        bad = dataclasses.replace(lp, lossy_lo=lo, lossy_hi=hi)
        assert status(bad) == F.FDTD_E_INVALID
        assert "lossy box" in F.lib().fdtd_last_error(None).decode()
    # a TFSF plane whose layers meet the lossy box's z range
    t = W.with_tfsf(dataclasses.replace(lp, lossy_lo=(14, 14, 8), lossy_hi=(22, 22, 16)), k=10)
    assert status(t) == F.FDTD_E_INVALID
    assert "lossy box" in F.lib().fdtd_last_error(None).decode()
    assert status(lp) == F.FDTD_OK



@pytest.mark.parametrize("K", [1, 2, 3])
def test_footprint_holds_64_steps_of_detector_planes(K):
    """The flux planes of the z-march wait in the workspace for up to 64 steps
    (the largest multiple of K within 64), then one fixed-order launch sums
    them: a detector window larger by dL cells costs 64 / K * K planes of dL
    floats more (plus the sums' scratch of ceil(L / 4096) floats per step and
    the workspace's 256-byte alignment)."""
    pr = W.small_cpml(nx=40, ny=36, nz=44, p=6, T=100)
    d = pr.detectors[0]
    small = dataclasses.replace(pr, detectors=[dataclasses.replace(d, i1=d.i0 + 5, j1=d.j0 + 4)])
    a = _fp(small, time_block=K)
    b = _fp(pr, time_block=K)
    dL = (d.i1 - d.i0) * (d.j1 - d.j0) - 5 * 4
    cap = 64 // K * K
    assert cap * dL * 4 <= b - a <= cap * dL * 4 + cap * 4 + 8 * 256
