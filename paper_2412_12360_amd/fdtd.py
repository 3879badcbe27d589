"""Python binding of libfdtd (include/fdtd.h): ctypes marshalling only.

Every step of the FDTD path runs in the HIP kernels of libfdtd.so; this module
converts problem descriptions into the C structs, owns the device workspace as
a torch tensor (PyTorch is used for device memory and streams only) and exposes
the C entry points under their own names.  If the library is missing the
import of `lib()` raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")
MAX_SOURCES = 4
MAX_DETECTORS = 4

FDTD_OK, FDTD_E_INVALID, FDTD_E_NOMEM, FDTD_E_DEVICE, FDTD_E_STATE, FDTD_E_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_STATE", 5: "E_UNSUPPORTED"}


class fdtd_desc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("courant", C.c_float),
        ("pml_cells", C.c_int32),
        ("pml_order", C.c_float), ("pml_sigma_max", C.c_float), ("pml_kappa_max", C.c_float),
        ("pml_alpha_max", C.c_float), ("pml_eps_bg", C.c_float),
        ("inv_eps", C.c_void_p),
        ("design_lo", C.c_int32 * 3), ("design_hi", C.c_int32 * 3),
        ("n_steps", C.c_int32),
        ("record", C.c_int32),
        ("time_block", C.c_int32),
        ("sigma", C.c_void_p),
        ("lossy_lo", C.c_int32 * 3), ("lossy_hi", C.c_int32 * 3),
    ]


class fdtd_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("comp", C.c_int32), ("i", C.c_int32), ("j", C.c_int32),
                ("k", C.c_int32), ("amp", C.c_void_p)]


class fdtd_flux_detector(C.Structure):
    _fields_ = [("k", C.c_int32), ("i0", C.c_int32), ("i1", C.c_int32), ("j0", C.c_int32),
                ("j1", C.c_int32), ("weight", C.c_float), ("interpolate", C.c_int32),
                ("quantity", C.c_int32)]


ENTRY_POINTS = [
    "fdtd_footprint", "fdtd_create", "fdtd_forward", "fdtd_inverse", "fdtd_grad", "fdtd_set_inv_eps",
    "fdtd_reset", "fdtd_destroy", "fdtd_time", "fdtd_last_error", "fdtd_field_ptr", "fdtd_state_arrays",
    "fdtd_linear_steps", "fdtd_record_ptr", "fdtd_time_block", "fdtd_checkpoint_bytes",
    "fdtd_grad_checkpointed", "fdtd_kernel_path", "fdtd_tile_classes", "fdtd_grad_checkpointed_noalloc",
    "fdtd_noalloc_store_bytes", "fdtd_grad_begin", "fdtd_grad_steps", "fdtd_grad_end", "fdtd_forward_batch",
    "fdtd_grad_steps_batch", "fdtd_revolve_plan", "fdtd_revolve_bytes", "fdtd_grad_revolve", "fdtd_set_stream",
]

_lib = None


def lib():
    """The loaded libfdtd.so with argument types set.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2412_12360_amd/build.py "
                           "(the FDTD path has no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    D = C.POINTER(fdtd_desc)
    Sp = C.POINTER(fdtd_source)
    Dp = C.POINTER(fdtd_flux_detector)
    fp = C.c_void_p
    L.fdtd_footprint.argtypes = [D, Sp, C.c_int32, Dp, C.c_int32, C.POINTER(C.c_size_t)]
    L.fdtd_create.argtypes = [D, Sp, C.c_int32, Dp, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                              C.POINTER(H)]
    L.fdtd_forward.argtypes = [H, C.c_int32, fp, fp]
    L.fdtd_inverse.argtypes = [H, C.c_int32]
    L.fdtd_grad.argtypes = [H, fp, fp]
    L.fdtd_grad_begin.argtypes = [H]
    L.fdtd_grad_steps.argtypes = [H, C.c_int32]
    L.fdtd_grad_end.argtypes = [H, fp, fp]
    L.fdtd_forward_batch.argtypes = [C.POINTER(H), C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p)]
    L.fdtd_grad_steps_batch.argtypes = [C.POINTER(H), C.c_int32, C.POINTER(C.c_int32)]
    L.fdtd_revolve_plan.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]
    L.fdtd_revolve_bytes.argtypes = [H, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
    L.fdtd_grad_revolve.argtypes = [H, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, fp, fp]
    L.fdtd_checkpoint_bytes.argtypes = [H, C.c_int32, C.POINTER(C.c_size_t)]
    L.fdtd_grad_checkpointed.argtypes = [H, C.c_int32, C.c_void_p, C.c_size_t, fp, fp]
    L.fdtd_grad_checkpointed_noalloc.argtypes = [H, C.c_int32, fp, fp]
    L.fdtd_noalloc_store_bytes.argtypes = []
    L.fdtd_set_inv_eps.argtypes = [H, fp]
    L.fdtd_reset.argtypes = [H]
    L.fdtd_set_stream.argtypes = [H, C.c_void_p]
    L.fdtd_destroy.argtypes = [H]
    L.fdtd_time.argtypes = [H, C.POINTER(C.c_int32)]
    L.fdtd_last_error.argtypes = [H]
    L.fdtd_last_error.restype = C.c_char_p
    L.fdtd_field_ptr.argtypes = [H, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]
    L.fdtd_state_arrays.argtypes = [H, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_size_t), C.c_int32,
                                    C.POINTER(C.c_int32)]
    L.fdtd_linear_steps.argtypes = [H, C.c_int32, C.c_int32]
    L.fdtd_record_ptr.argtypes = [H, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_size_t)]
    L.fdtd_time_block.argtypes = [H, C.POINTER(C.c_int32)]
    L.fdtd_kernel_path.argtypes = [H, C.POINTER(C.c_int32)]
    L.fdtd_tile_classes.argtypes = [H, C.c_int32, C.POINTER(C.c_int32)]
    for name in ENTRY_POINTS:
        if name not in ("fdtd_last_error", "fdtd_noalloc_store_bytes"):
            getattr(L, name).restype = C.c_int
    L.fdtd_noalloc_store_bytes.restype = C.c_size_t
    _lib = L
    return L


class FdtdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, handle=None):
    if status != FDTD_OK:
        m = lib().fdtd_last_error(handle)
        raise FdtdError(status, m.decode() if m else "")


def make_desc(prob, inv_eps_ptr: int = 0, record: bool = False, time_block: int = 0, T: Optional[int] = None,
              sigma_ptr: int = 0):
    d = fdtd_desc()
    d.nx, d.ny, d.nz = prob.nx, prob.ny, prob.nz
    d.courant = prob.S
    d.pml_cells = prob.p
    d.pml_order = prob.pml_m
    d.pml_sigma_max = prob.pml_sigma_max
    d.pml_kappa_max = prob.pml_kappa_max
    d.pml_alpha_max = prob.pml_alpha_max
    d.pml_eps_bg = 1.0
    d.inv_eps = inv_eps_ptr
    for a in range(3):
        d.design_lo[a] = prob.design_lo[a]
        d.design_hi[a] = prob.design_hi[a]
    d.n_steps = prob.T if T is None else T
    d.record = 1 if record else 0
    d.time_block = time_block
    # conducting cells (sigma over the lossy box), if the problem has them
    if getattr(prob, "sigma", None) is not None:
        d.sigma = sigma_ptr
        for a in range(3):
            d.lossy_lo[a] = prob.lossy_lo[a]
            d.lossy_hi[a] = prob.lossy_hi[a]
    return d


def make_sources(prob, amp_ptrs: Sequence[int]):
    arr = (fdtd_source * MAX_SOURCES)()
    for i, (s, ptr) in enumerate(zip(prob.sources, amp_ptrs)):
        arr[i].kind, arr[i].comp, arr[i].i, arr[i].j, arr[i].k = s.kind, s.comp, s.i, s.j, s.k
        arr[i].amp = ptr
    return arr


def make_detectors(prob):
    arr = (fdtd_flux_detector * MAX_DETECTORS)()
    for i, d in enumerate(prob.detectors):
        arr[i].k, arr[i].i0, arr[i].i1, arr[i].j0, arr[i].j1 = d.k, d.i0, d.i1, d.j0, d.j1
        arr[i].weight = d.weight
        arr[i].interpolate = int(getattr(d, "interpolate", False))
        arr[i].quantity = int(getattr(d, "quantity", 0))
    return arr


def footprint(prob, record: bool = False, time_block: int = 0, T: Optional[int] = None) -> int:
    """Workspace bytes of a problem (no device work)."""
    d = make_desc(prob, 1, record, time_block, T, sigma_ptr=1)
    srcs = make_sources(prob, [1] * len(prob.sources))
    dets = make_detectors(prob)
    out = C.c_size_t(0)
    check(lib().fdtd_footprint(C.byref(d), srcs, len(prob.sources), dets, len(prob.detectors), C.byref(out)))
    return int(out.value)


def _handles(solvers):
    return (C.c_void_p * max(1, len(solvers)))(*[s.handle.value for s in solvers])


SCHEDULES = {"halving": 0, "treeverse": 1}


def revolve_plan(T: int, schedule: str, snapshots: int = 0, actions: bool = False):
    """fdtd_revolve_plan: (forward steps, most kept states, [(op, a, b), ...]
    or None) of a checkpoint schedule for T steps (host only)."""
    f = C.c_int64(0)
    pk = C.c_int32(0)
    n = C.c_int32(0)
    check(lib().fdtd_revolve_plan(int(T), SCHEDULES[schedule], int(snapshots), C.byref(f), C.byref(pk), None, 0,
                                  C.byref(n)))
    acts = None
    if actions:
        buf = (C.c_int32 * (3 * max(1, n.value)))()
        check(lib().fdtd_revolve_plan(int(T), SCHEDULES[schedule], int(snapshots), None, None, buf, n.value,
                                      C.byref(n)))
        acts = [(buf[3 * i], buf[3 * i + 1], buf[3 * i + 2]) for i in range(n.value)]
    return int(f.value), int(pk.value), acts


def _batch_check(status: int, solvers):
    """A failed batch call: the batch-level message and every handle's last
    message (a handle's message may predate this call)."""
    if status == FDTD_OK:
        return
    parts = []
    m = lib().fdtd_last_error(None)
    if m:
        parts.append(m.decode())
    for i, s in enumerate(solvers):
        m = lib().fdtd_last_error(s.handle)
        if m:
            parts.append(f"handle {i}: {m.decode()}")
    raise FdtdError(status, "; ".join(parts))


def forward_batch(solvers, n_steps):
    """fdtd_forward_batch: advance solvers[i] by n_steps[i] (all created on one
    stream) with one z-march launch per sweep spanning all of them; returns
    per solver (trace [n, ndet], J) device tensors, as Solver.forward."""
    import torch
    nh = len(solvers)
    if nh == 0:
        return []
    counts = (C.c_int32 * nh)(*[int(n) for n in n_steps])
    outs, tptr, jptr = [], (C.c_void_p * nh)(), (C.c_void_p * nh)()
    for i, (s, n) in enumerate(zip(solvers, n_steps)):
        tr = torch.zeros((max(int(n), 1), max(s.ndet, 1)), dtype=torch.float32, device=s.device)
        outs.append((tr, s.J))
        tptr[i] = tr.data_ptr()
        jptr[i] = s.J.data_ptr()
    _batch_check(lib().fdtd_forward_batch(_handles(solvers), nh, counts, tptr, jptr), solvers)
    return [(tr[:int(n), :s.ndet], J) for (tr, J), s, n in zip(outs, solvers, n_steps)]


def grad_steps_batch(solvers, n_steps):
    """fdtd_grad_steps_batch: n_steps[i] reverse steps of solvers[i]'s running
    gradient, one launch per reverse step spanning all of them."""
    nh = len(solvers)
    if nh == 0:
        return
    counts = (C.c_int32 * nh)(*[int(n) for n in n_steps])
    _batch_check(lib().fdtd_grad_steps_batch(_handles(solvers), nh, counts), solvers)


class Solver:
    """One FDTD problem resident on the GPU.  Holds the workspace (a torch
    uint8 tensor), the material and amplitude inputs, and the C handle."""

    def __init__(self, prob, record: bool = False, time_block: int = 0, device: str = "cuda",
                 T: Optional[int] = None, stream=None, workspace=None):
        import torch
        self.torch = torch
        self.prob = prob
        self.T = prob.T if T is None else T
        self.record = record
        dev = torch.device(device)
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.inv_eps = torch.from_numpy(np.ascontiguousarray(prob.inv_eps, np.float32)).to(dev)
        self.amps = []
        for s in prob.sources:
            a = np.zeros(self.T, np.float32)
            m = min(self.T, len(s.amp))
            a[:m] = s.amp[:m]
            self.amps.append(torch.from_numpy(a).to(dev))
        self.sigma = None
        if getattr(prob, "sigma", None) is not None:
            if tuple(np.shape(prob.sigma)) != tuple(prob.lossy_shape()):
                raise ValueError(f"sigma has shape {np.shape(prob.sigma)}, the lossy box {prob.lossy_shape()}")
            self.sigma = torch.from_numpy(np.ascontiguousarray(prob.sigma, np.float32)).to(dev)
        self.desc = make_desc(prob, self.inv_eps.data_ptr(), record, time_block, self.T,
                              sigma_ptr=self.sigma.data_ptr() if self.sigma is not None else 0)
        self.srcs = make_sources(prob, [a.data_ptr() for a in self.amps])
        self.dets = make_detectors(prob)
        self.ndet = len(prob.detectors)
        nbytes = C.c_size_t(0)
        check(lib().fdtd_footprint(C.byref(self.desc), self.srcs, len(prob.sources), self.dets, self.ndet,
                                   C.byref(nbytes)))
        self.footprint = int(nbytes.value)
        if workspace is None:
            workspace = torch.empty(self.footprint + 256, dtype=torch.uint8, device=dev)
        self.ws_tensor = workspace
        base = workspace.data_ptr()
        self.ws_off = (-base) % 256
        self.ws_ptr = base + self.ws_off
        self.handle = C.c_void_p(0)
        # The inputs were written on the current stream; fdtd_create enqueues
        # its uploads on self.stream.  Order the two streams (no host wait, so
        # other streams' queued work keeps running), and tell the caching
        # allocator that the workspace is used on self.stream.
        cur = torch.cuda.current_stream(dev)
        if self.stream != cur:
            self.stream.wait_stream(cur)
            workspace.record_stream(self.stream)
        with torch.cuda.stream(self.stream):
            check(lib().fdtd_create(C.byref(self.desc), self.srcs, len(prob.sources), self.dets, self.ndet,
                                    C.c_void_p(self.ws_ptr), C.c_size_t(workspace.numel() - self.ws_off),
                                    C.c_void_p(self.stream.cuda_stream), C.byref(self.handle)))
        self._fws = workspace[self.ws_off:].view(torch.float32) if (workspace.numel() - self.ws_off) % 4 == 0 \
            else workspace[self.ws_off: self.ws_off + ((workspace.numel() - self.ws_off) // 4) * 4].view(torch.float32)
        self.J = torch.zeros(1, dtype=torch.float32, device=dev)

    # ------------------------------------------------------------ helpers
    def _view(self, ptr: int, count: int):
        off = ptr - self.ws_ptr
        assert off % 4 == 0 and 0 <= off and off // 4 + count <= self._fws.numel()
        return self._fws[off // 4: off // 4 + count]

    def close(self):
        if self.handle:
            lib().fdtd_destroy(self.handle)
            self.handle = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------- entry points
    def fdtd_forward(self, n: Optional[int] = None, trace=None, J=None):
        n = self.T - self.t if n is None else n
        check(lib().fdtd_forward(self.handle, n, C.c_void_p(trace.data_ptr() if trace is not None else 0),
                                 C.c_void_p(J.data_ptr() if J is not None else 0)), self.handle)

    def forward(self, n: Optional[int] = None):
        """Advance n steps; returns (trace [n, ndet], J) as device tensors."""
        n = self.T - self.t if n is None else n
        trace = self.torch.zeros((max(n, 1), max(self.ndet, 1)), dtype=self.torch.float32, device=self.device)
        self.fdtd_forward(n, trace, self.J)
        return trace[:n, :self.ndet], self.J

    def fdtd_inverse(self, n: int):
        check(lib().fdtd_inverse(self.handle, n), self.handle)

    inverse = fdtd_inverse

    def fdtd_grad(self, dJ_deps, recon=None):
        check(lib().fdtd_grad(self.handle, C.c_void_p(dJ_deps.data_ptr()),
                              C.c_void_p(recon.data_ptr() if recon is not None else 0)), self.handle)

    def grad(self):
        """dJ/deps_r over the design box [dz, dy, dx] and the reconstruction error."""
        g = self.torch.empty(self.prob.design_shape(), dtype=self.torch.float32, device=self.device)
        r = self.torch.zeros(1, dtype=self.torch.float32, device=self.device)
        self.fdtd_grad(g, r)
        return g, r

    # the gradient in chunks (fdtd_grad_begin / _steps / _end)
    def grad_begin(self):
        check(lib().fdtd_grad_begin(self.handle), self.handle)

    def grad_steps(self, n: int):
        check(lib().fdtd_grad_steps(self.handle, int(n)), self.handle)

    def grad_end(self):
        """dJ/deps_r and the reconstruction error once the chunks reached t = 0."""
        g = self.torch.empty(self.prob.design_shape(), dtype=self.torch.float32, device=self.device)
        r = self.torch.zeros(1, dtype=self.torch.float32, device=self.device)
        check(lib().fdtd_grad_end(self.handle, C.c_void_p(g.data_ptr()), C.c_void_p(r.data_ptr())), self.handle)
        return g, r

    def checkpoint_bytes(self, segment: int) -> int:
        """Device bytes the checkpointed gradient keeps for this segment length."""
        v = C.c_size_t(0)
        check(lib().fdtd_checkpoint_bytes(self.handle, int(segment), C.byref(v)), self.handle)
        return int(v.value)

    def grad_checkpointed(self, segment: int, store=None):
        """The checkpointed gradient (comparator of grad()): runs the forward
        pass itself; returns dJ/deps_r over the design box [dz, dy, dx] and J.
        `store`: optional preallocated uint8 device tensor of at least
        checkpoint_bytes(segment) bytes (256-byte aligned)."""
        nbytes = self.checkpoint_bytes(segment)
        if store is None:
            store = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        g = self.torch.empty(self.prob.design_shape(), dtype=self.torch.float32, device=self.device)
        J = self.torch.zeros(1, dtype=self.torch.float32, device=self.device)
        check(lib().fdtd_grad_checkpointed(self.handle, int(segment), C.c_void_p(store.data_ptr()),
                                           C.c_size_t(store.numel() * store.element_size()),
                                           C.c_void_p(g.data_ptr()), C.c_void_p(J.data_ptr())), self.handle)
        self._keep_store = store
        return g, J

    def revolve_bytes(self, schedule: str, snapshots: int = 0) -> int:
        v = C.c_size_t(0)
        check(lib().fdtd_revolve_bytes(self.handle, SCHEDULES[schedule], int(snapshots), C.byref(v)), self.handle)
        return int(v.value)

    def grad_revolve(self, schedule: str, snapshots: int = 0, store=None):
        """The gradient by recursive halving ("halving") or treeverse with
        `snapshots` kept states ("treeverse"): runs the forward pass itself;
        returns dJ/deps_r over the design box and J."""
        nbytes = self.revolve_bytes(schedule, snapshots)
        if store is None:
            store = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        g = self.torch.empty(self.prob.design_shape(), dtype=self.torch.float32, device=self.device)
        J = self.torch.zeros(1, dtype=self.torch.float32, device=self.device)
        check(lib().fdtd_grad_revolve(self.handle, SCHEDULES[schedule], int(snapshots), C.c_void_p(store.data_ptr()),
                                      C.c_size_t(store.numel() * store.element_size()), C.c_void_p(g.data_ptr()),
                                      C.c_void_p(J.data_ptr())), self.handle)
        self._keep_store = store
        return g, J

    def grad_checkpointed_noalloc(self, segment: int):
        """grad_checkpointed with the library's fixed device store (no
        allocation by the library or for the store); outputs as there."""
        g = self.torch.empty(self.prob.design_shape(), dtype=self.torch.float32, device=self.device)
        J = self.torch.zeros(1, dtype=self.torch.float32, device=self.device)
        check(lib().fdtd_grad_checkpointed_noalloc(self.handle, int(segment), C.c_void_p(g.data_ptr()),
                                                   C.c_void_p(J.data_ptr())), self.handle)
        return g, J

    def fdtd_set_inv_eps(self, inv_eps):
        self._keep = inv_eps
        check(lib().fdtd_set_inv_eps(self.handle, C.c_void_p(inv_eps.data_ptr())), self.handle)

    set_inv_eps = fdtd_set_inv_eps

    def fdtd_set_stream(self, stream):
        """Move the handle to `stream` (a torch stream), ordered after the
        work of its current stream; the workspace is marked as used there."""
        stream.wait_stream(self.stream)
        self.ws_tensor.record_stream(stream)
        self.J.record_stream(stream)
        check(lib().fdtd_set_stream(self.handle, C.c_void_p(stream.cuda_stream)), self.handle)
        self.stream = stream

    set_stream = fdtd_set_stream

    def fdtd_reset(self):
        check(lib().fdtd_reset(self.handle), self.handle)

    reset = fdtd_reset

    @property
    def t(self) -> int:
        v = C.c_int32(0)
        check(lib().fdtd_time(self.handle, C.byref(v)), self.handle)
        return int(v.value)

    @property
    def time_block(self) -> int:
        v = C.c_int32(0)
        check(lib().fdtd_time_block(self.handle, C.byref(v)), self.handle)
        return int(v.value)

    @property
    def kernel_path(self) -> str:
        """Kernels the forward and reverse steps run on: "per-cell", "z-march" (32-bit
        offsets from one base per field set) or "z-march-wide" (a 64-bit base
        per component and plane, for field sets of 4 GiB or more)."""
        v = C.c_int32(0)
        check(lib().fdtd_kernel_path(self.handle, C.byref(v)), self.handle)
        return ("per-cell", "z-march", "z-march-wide")[v.value]

    def tile_classes(self, march: int = 0):
        """Tiles per z-march class [interior, x slab, y slab, both] of the fused
        reverse march (march = 0) or of a forward sweep of `march` steps."""
        v = (C.c_int32 * 4)()
        check(lib().fdtd_tile_classes(self.handle, int(march), v), self.handle)
        return [int(x) for x in v]

    def field(self, comp: int, which: int = 0):
        """Device view [nz, ny, nx] of field component comp (0..5) of the
        forward (which = 0) or adjoint (which = 1) state."""
        p = C.c_void_p(0)
        check(lib().fdtd_field_ptr(self.handle, which, comp, C.byref(p)), self.handle)
        pr = self.prob
        return self._view(p.value, pr.N).view(pr.nz, pr.ny, pr.nx)

    def fields(self, which: int = 0):
        return [self.field(c, which) for c in range(6)]

    def state_arrays(self, which: int = 0):
        ptrs = (C.c_void_p * 32)()
        counts = (C.c_size_t * 32)()
        n = C.c_int32(0)
        check(lib().fdtd_state_arrays(self.handle, which, ptrs, counts, 32, C.byref(n)), self.handle)
        return [self._view(ptrs[i], counts[i]) for i in range(n.value)]

    def linear_steps(self, n: int, adjoint: bool = False):
        check(lib().fdtd_linear_steps(self.handle, n, 1 if adjoint else 0), self.handle)

    def record_step(self, n: int):
        p = C.c_void_p(0)
        cnt = C.c_size_t(0)
        check(lib().fdtd_record_ptr(self.handle, n, C.byref(p), C.byref(cnt)), self.handle)
        return self._view(p.value, cnt.value)
