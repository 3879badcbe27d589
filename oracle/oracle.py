"""ctypes front end of the FP64 CPU oracle (fdtd_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the GPU product path never imports it.  It takes
a problem description object (grid, Courant number, CPML grading, 1/eps_r,
sources, detectors, design box; float32 inputs promoted to float64) and runs
the plain reference recursions of the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fdtd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
MAXSRC = 4
MAXDET = 4
NSLOT = 18


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, strict IEEE: no fast-math, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("S", C.c_double),
        ("p", C.c_int),
        ("m", C.c_double), ("sigma_max", C.c_double), ("kappa_max", C.c_double), ("alpha_max", C.c_double),
        ("d", C.POINTER(C.c_double)),
        ("nsrc", C.c_int),
        ("src_kind", C.c_int * MAXSRC), ("src_comp", C.c_int * MAXSRC),
        ("src_i", C.c_int * MAXSRC), ("src_j", C.c_int * MAXSRC), ("src_k", C.c_int * MAXSRC),
        ("src_amp", C.POINTER(C.c_double) * MAXSRC),
        ("ndet", C.c_int),
        ("det_k", C.c_int * MAXDET),
        ("det_i0", C.c_int * MAXDET), ("det_i1", C.c_int * MAXDET),
        ("det_j0", C.c_int * MAXDET), ("det_j1", C.c_int * MAXDET),
        ("det_w", C.c_double * MAXDET),
        ("det_interp", C.c_int * MAXDET),
        ("det_energy", C.c_int * MAXDET),
        ("dlo", C.c_int * 3), ("dhi", C.c_int * 3),
        ("sig", C.POINTER(C.c_double)),
        ("llo", C.c_int * 3), ("lhi", C.c_int * 3),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        P = C.POINTER(_Problem)
        L.or_forward.argtypes = [P, dp, C.c_int, C.c_int, dp, dp]
        L.or_forward.restype = C.c_double
        L.or_inverse.argtypes = [P, dp, C.c_int, C.c_int, dp]
        L.or_step_linear.argtypes = [P, dp, C.c_int]
        L.or_adjoint_linear.argtypes = [P, dp, C.c_int]
        L.or_grad_history.argtypes = [P, C.c_int, C.c_int, dp, dp]
        L.or_grad_history.restype = C.c_double
        L.or_grad_reversed.argtypes = [P, C.c_int, dp, dp, dp]
        L.or_grad_reversed.restype = C.c_double
        L.or_record_floats.argtypes = [P]
        L.or_record_floats.restype = C.c_size_t
        L.or_grade.argtypes = [P, C.c_int, C.c_double, dp]
        _lib = L
    return _lib


def tfsf_incident(S: float, d: float, amp: np.ndarray, pol: int):
    """Incident fields of a one-sided total-field/scattered-field plane along +z
    (section 2.1 names the source type; the formulation here is the textbook
    one for a Yee grid).

    A 1D Yee line along z carries the incident wave, with the grid's Courant
    number S and the plane's 1/eps_r d, so that for a wave uniform in x and y
    it is exactly the 3D update restricted to z.  E lives on its nodes, H
    between them.  Node 0 is driven, E_0^{n+1} = amp[n] (a hard source), one
    cell below the plane; node 1 is the first total-field E plane k0.  At step n
    the 3D curl across the boundary misses the incident part on each side:
      - the scattered-field H layer k0-1 reads total E at k0, so after its H
        half step it takes +S E_1^n (Hy, Ex polarisation) or -S E_1^n (Hx, Ey);
      - the total-field E plane k0 reads scattered H at k0-1, so after its E
        half step it takes +S d H_0^{n+1/2} (on the polarisation component).
    The line has T/2 + 8 nodes and a conducting far end, which a wave from
    node 0 cannot reach and return from within T steps (a Yee update moves
    information at most one cell per step).

    Returns (aE, aH, E_line, H_line): the two amplitude series and the line
    after len(amp) steps."""
    T = len(amp)
    L = T // 2 + 8
    E = np.zeros(L)
    H = np.zeros(L - 1)
    aE = np.zeros(T)
    aH = np.zeros(T)
    sg = 1.0 if pol == 0 else -1.0
    for n in range(T):
        aH[n] = sg * S * E[1]
        H -= S * (E[1:] - E[:-1])
        aE[n] = S * d * H[0]
        E[1:-1] -= S * d * (H[1:] - H[:-1])
        E[0] = float(amp[n])
    return aE, aH, E, H


def expand_sources(prob, d: np.ndarray):
    """The problem's sources as plain additive sources (kind 0 point, kind 1
    plane; components 0..5): a TFSF source becomes its E plane source on k0 and
    its H plane source on k0-1, fed by tfsf_incident with 1/eps_r of the plane's
    centre cell."""
    out = []
    for src in prob.sources:
        if src.kind != 2:
            out.append((src.kind, src.comp, src.i, src.j, src.k, np.asarray(src.amp, np.float64)))
            continue
        assert src.comp in (0, 1)
        dc = float(d[src.k, prob.ny // 2, prob.nx // 2])
        aE, aH, _, _ = tfsf_incident(float(prob.S), dc, np.asarray(src.amp, np.float64), src.comp)
        out.append((1, src.comp, 0, 0, src.k, aE))
        out.append((1, 4 if src.comp == 0 else 3, 0, 0, src.k - 1, aH))
    return out


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """FP64 reference for one problem.  `d` overrides 1/eps_r (float64, [nz,ny,nx])."""

    def __init__(self, prob, d: np.ndarray | None = None):
        self.prob = prob
        self.L = _load()
        self.d = np.ascontiguousarray(prob.inv_eps, dtype=np.float64) if d is None else \
            np.ascontiguousarray(d, dtype=np.float64)
        assert self.d.shape == (prob.nz, prob.ny, prob.nx)
        s = _Problem()
        s.nx, s.ny, s.nz = prob.nx, prob.ny, prob.nz
        s.S = float(prob.S)
        s.p = int(prob.p)
        s.m, s.sigma_max = float(prob.pml_m), float(prob.pml_sigma_max)
        s.kappa_max, s.alpha_max = float(prob.pml_kappa_max), float(prob.pml_alpha_max)
        s.d = _ptr(self.d)
        srcs = expand_sources(prob, self.d)
        assert len(srcs) <= MAXSRC and len(prob.detectors) <= MAXDET
        self._amps = []
        s.nsrc = len(srcs)
        for i, (kind, comp, si, sj, sk, amp) in enumerate(srcs):
            a = np.ascontiguousarray(amp, dtype=np.float64)
            self._amps.append(a)
            s.src_kind[i], s.src_comp[i] = kind, comp
            s.src_i[i], s.src_j[i], s.src_k[i] = si, sj, sk
            s.src_amp[i] = _ptr(a)
        self.sources = srcs
        s.ndet = len(prob.detectors)
        for i, det in enumerate(prob.detectors):
            s.det_k[i] = det.k
            s.det_i0[i], s.det_i1[i], s.det_j0[i], s.det_j1[i] = det.i0, det.i1, det.j0, det.j1
            s.det_w[i] = float(det.weight)
            s.det_interp[i] = int(getattr(det, "interpolate", False))
            s.det_energy[i] = int(getattr(det, "quantity", 0) == 1)
            assert not s.det_energy[i] or s.det_interp[i], "the energy detector is co-located (interpolate)"
            if s.det_interp[i]:
                # the co-located flux reads layer k-1 and the cells at i1, j1
                assert det.k >= 1 and det.i1 < prob.nx and det.j1 < prob.ny
        for a in range(3):
            s.dlo[a], s.dhi[a] = prob.design_lo[a], prob.design_hi[a]
        # conducting cells: sigma over the whole grid, zero outside the lossy box
        self.sig = None
        if getattr(prob, "sigma", None) is not None:
            n = (prob.nx, prob.ny, prob.nz)
            for a in range(3):
                lo, hi = prob.lossy_lo[a], prob.lossy_hi[a]
                assert prob.p <= lo < hi <= n[a] - prob.p, "the lossy box lies in the interior"
            assert prob.sigma.shape == prob.lossy_shape()
            self.sig = np.zeros(prob.shape, np.float64)
            self.sig[prob.lossy_slices()] = np.asarray(prob.sigma, np.float64)
            s.sig = _ptr(self.sig)
            for a in range(3):
                s.llo[a], s.lhi[a] = prob.lossy_lo[a], prob.lossy_hi[a]
        self.s = s

    # -------------------------------------------------------------- helpers
    def new_state(self) -> np.ndarray:
        p = self.prob
        return np.zeros((NSLOT, p.nz, p.ny, p.nx), np.float64)

    def record_floats(self) -> int:
        return int(self.L.or_record_floats(C.byref(self.s)))

    def grade(self, axis: int, u: float):
        out = np.zeros(3)
        self.L.or_grade(C.byref(self.s), axis, float(u), _ptr(out))
        return out  # b, a, 1/kappa

    def _check_T(self, n0, T):
        for a in self._amps:
            assert len(a) >= n0 + T, "source amplitude shorter than the run"

    # ------------------------------------------------------------- forward
    def forward(self, state: np.ndarray, T: int, n0: int = 0, record: bool = False):
        """Advance `state` in place by T steps from step n0.  Returns (J, trace[T, ndet], rec)."""
        self._check_T(n0, T)
        nd = max(1, len(self.prob.detectors))
        trace = np.zeros((max(T, 1), nd), np.float64)
        rec = np.zeros((max(T, 1), self.record_floats()), np.float64) if record else None
        J = self.L.or_forward(C.byref(self.s), _ptr(state), n0, T, _ptr(trace),
                              _ptr(rec) if record else None)
        return J, trace[:T, :len(self.prob.detectors)], (rec[:T] if record else None)

    def run(self, T: int | None = None, record: bool = False):
        T = self.prob.T if T is None else T
        st = self.new_state()
        J, trace, rec = self.forward(st, T, 0, record)
        return st, J, trace, rec

    def inverse(self, state: np.ndarray, rec: np.ndarray | None, T: int, n0: int = 0):
        """Undo steps n0+T-1 .. n0 on the interior (in place).  The record is
        needed with a CPML and with conducting cells."""
        assert rec is not None or self.record_floats() == 0, "this problem's inverse reads the record"
        self.L.or_inverse(C.byref(self.s), _ptr(state), n0, T, _ptr(rec) if rec is not None else None)

    def step_linear(self, state: np.ndarray, T: int = 1):
        self.L.or_step_linear(C.byref(self.s), _ptr(state), T)

    def adjoint_linear(self, adj: np.ndarray, T: int = 1):
        self.L.or_adjoint_linear(C.byref(self.s), _ptr(adj), T)

    # ----------------------------------------------------------- gradients
    def _check_grad(self):
        lo, hi = self.prob.design_lo[2], self.prob.design_hi[2]
        for det in self.prob.detectors:
            if getattr(det, "quantity", 0) == 1 and det.weight != 0.0:
                # the energy reads eps_r: its gradient omits that explicit term
                assert not (lo <= det.k < hi), "a weighted energy detector lies outside the design box in z"

    def grad_history(self, T: int | None = None, seg: int | None = None):
        """dJ/dd over the grid by the stored-history VJP; returns (g, J, trace)."""
        self._check_grad()
        T = self.prob.T if T is None else T
        self._check_T(0, T)
        seg = seg or max(1, int(np.ceil(np.sqrt(T))))
        g = np.zeros(self.prob.shape, np.float64)
        nd = max(1, len(self.prob.detectors))
        trace = np.zeros((max(T, 1), nd), np.float64)
        J = self.L.or_grad_history(C.byref(self.s), T, seg, _ptr(g), _ptr(trace))
        return g, J, trace[:T, :len(self.prob.detectors)]

    def grad_reversed(self, T: int | None = None):
        """dJ/dd by time reversal; returns (g, J, trace, recon)."""
        self._check_grad()
        T = self.prob.T if T is None else T
        self._check_T(0, T)
        g = np.zeros(self.prob.shape, np.float64)
        nd = max(1, len(self.prob.detectors))
        trace = np.zeros((max(T, 1), nd), np.float64)
        recon = np.zeros(1)
        J = self.L.or_grad_reversed(C.byref(self.s), T, _ptr(g), _ptr(trace), _ptr(recon))
        return g, J, trace[:T, :len(self.prob.detectors)], float(recon[0])

    def deps_design(self, g: np.ndarray) -> np.ndarray:
        """dJ/deps_r over the design box from dJ/dd: -d^2 g."""
        sl = self.prob.design_slices()
        return -(self.d[sl] ** 2) * g[sl]
