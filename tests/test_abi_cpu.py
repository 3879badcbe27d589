"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/fdtd.h declares, and validates arguments before touching a device."""
import ctypes as C
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
    return sorted(set(re.findall(r"^\s*(?:fdtd_status|const char \*)\s*(fdtd_\w+)\s*\(", txt, re.M)))


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
    src[0].comp = 4
    out = C.c_size_t(0)
    assert F.lib().fdtd_footprint(C.byref(d), src, 1, F.make_detectors(pr), 1, C.byref(out)) == F.FDTD_E_INVALID
    # a too-small workspace is refused before any device work
    h = C.c_void_p(0)
    st = F.lib().fdtd_create(C.byref(d), F.make_sources(pr, [1]), 1, F.make_detectors(pr), 1,
                             C.c_void_p(256), C.c_size_t(1024), None, C.byref(h))
    assert st == F.FDTD_E_NOMEM and not h.value
    assert F.lib().fdtd_forward(None, 1, None, None) == F.FDTD_E_INVALID
