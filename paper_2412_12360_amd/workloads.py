"""Seeded synthetic inputs for the FDTD hot path.

This module only *describes problems*: grid sizes, permittivity maps, source
waveforms, detector and design-box placement, CPML grading parameters.  It
holds none of the update arithmetic, so both the GPU path and the CPU oracle
consume exactly the same float32 inputs from here.

The paper's own workloads (a silicon coupler of Shen et al., a waveguide bend,
a 2PP stitching device; section 3) rely on geometries that are not public
here.  The problems below keep their scale instead: the cell counts of the
speed table (section 3.1, Table 2), the Courant factor 0.99 applied to the 3D
limit, the paper's materials (eps_r 1, 2.25, 12.25: air, polymer/silica,
silicon) and a plane-wave excitation of 1 um wavelength at 25 nm cells
(40 cells per wavelength; appendix A).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

C0 = 299_792_458.0


def courant() -> float:
    """S = c dt / dx = 0.99 / sqrt(3): the paper's "Courant factor 0.99"
    applied to the 3D stability limit (section 3.1), rounded to float32."""
    return float(np.float32(0.99 / math.sqrt(3.0)))


def steps_for(duration_s: float, dx_m: float) -> int:
    """Number of time steps for a simulated duration at cell size dx with the
    0.99 Courant factor, rounded to nearest (reproduces every step count that
    section 3.1, Table 2 and sections 3.2-3.3 print)."""
    dt = 0.99 * dx_m / (C0 * math.sqrt(3.0))
    return int(round(duration_s / dt))


# ------------------------------------------------------------------ records

@dataclasses.dataclass
class Source:
    kind: int            # 0 = point, 1 = whole z-normal plane, 2 = TFSF plane wave along +z
    comp: int            # 0..5 = Ex, Ey, Ez, Hx, Hy, Hz; kind 2: 0 (Ex) or 1 (Ey) polarisation
    i: int
    j: int
    k: int               # kind 2: the first total-field E plane
    amp: np.ndarray      # float32, one value per step (kind 2: the incident waveform)


@dataclasses.dataclass
class Detector:
    k: int               # z-normal plane
    i0: int
    i1: int
    j0: int
    j1: int
    weight: float = 1.0
    interpolate: bool = False   # components co-located at (i+1/2, j+1/2, k), time n+1/2
    quantity: int = 0           # 0 = Poynting flux, 1 = energy density (co-located, forward only)


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    S: float
    p: int                           # CPML cells per face (0 = bare PEC box)
    pml_m: float
    pml_sigma_max: float
    pml_kappa_max: float
    pml_alpha_max: float
    inv_eps: np.ndarray              # float32 [nz, ny, nx]
    sources: List[Source]
    detectors: List[Detector]
    design_lo: Tuple[int, int, int]  # (x, y, z), half-open box
    design_hi: Tuple[int, int, int]
    T: int
    rho: Optional[np.ndarray] = None  # design parameters [dz, dy, dx] when eps = 2.25 + 10 rho
    # conducting (lossy) cells: sigma over the half-open box [lossy_lo, lossy_hi)
    # (x, y, z), float32 [lz, ly, lx] in normalised units (eps dE/dt = curl H - sigma E);
    # None = lossless
    sigma: Optional[np.ndarray] = None
    lossy_lo: Tuple[int, int, int] = (0, 0, 0)
    lossy_hi: Tuple[int, int, int] = (0, 0, 0)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    def design_shape(self) -> Tuple[int, int, int]:
        lo, hi = self.design_lo, self.design_hi
        return (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])

    def design_slices(self):
        lo, hi = self.design_lo, self.design_hi
        return (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))

    def lossy_shape(self) -> Tuple[int, int, int]:
        lo, hi = self.lossy_lo, self.lossy_hi
        return (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])

    def lossy_slices(self):
        lo, hi = self.lossy_lo, self.lossy_hi
        return (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))

    def with_steps(self, T: int) -> "Problem":
        """The same problem truncated (or extended with zero amplitude) to T steps."""
        srcs = []
        for s in self.sources:
            a = np.zeros(T, np.float32)
            m = min(T, len(s.amp))
            a[:m] = s.amp[:m]
            srcs.append(dataclasses.replace(s, amp=a))
        return dataclasses.replace(self, T=T, sources=srcs)


# ----------------------------------------------------------------- waveforms

def gaussian_pulse(T: int, n0: float = 48.0, tau: float = 12.0) -> np.ndarray:
    n = np.arange(T, dtype=np.float64)
    return np.exp(-((n - n0) / tau) ** 2).astype(np.float32)


def ramped_sine(T: int, S: float, lambda0: float = 40.0, periods: int = 3) -> np.ndarray:
    """sin(w n) with a raised-cosine ramp over `periods` periods; w = 2 pi S / lambda0."""
    w = 2.0 * math.pi * S / lambda0
    nr = int(round(periods * 2.0 * math.pi / w))
    n = np.arange(T, dtype=np.float64)
    ramp = np.where(n < nr, 0.5 * (1.0 - np.cos(math.pi * n / nr)), 1.0)
    return (np.sin(w * n) * ramp).astype(np.float32)


def pml_grading(S: float, eps_bg: float, m: float = 3.0, kappa_max: float = 1.0,
                alpha_max: float = 0.01) -> Tuple[float, float, float, float]:
    """CFS-CPML grading in per-step units: sigma_max = 0.8 (m+1) S / sqrt(eps_bg)
    (the usual optimum for a polynomial grading), kappa_max, alpha_max."""
    sig = 0.8 * (m + 1.0) * S / math.sqrt(eps_bg)
    f = lambda v: float(np.float32(v))
    return f(m), f(sig), f(kappa_max), f(alpha_max)


def eps_from_rho(rho: np.ndarray) -> np.ndarray:
    return (2.25 + 10.0 * rho.astype(np.float64))


# ------------------------------------------------------------------- configs

def _sheet_problem(name, nx, ny, nz, p, T, eps, eps_bg, design_lo, design_hi, rho=None, inv=None):
    S = courant()
    m, sig, kap, alp = pml_grading(S, eps_bg)
    if inv is None:
        inv = (1.0 / eps).astype(np.float32)
    src = Source(kind=1, comp=0, i=0, j=0, k=p + 2, amp=ramped_sine(T, S))
    det = Detector(k=nz - p - 3, i0=p, i1=nx - p, j0=p, j1=ny - p, weight=1.0)
    return Problem(name=name, nx=nx, ny=ny, nz=nz, S=S, p=p, pml_m=m, pml_sigma_max=sig,
                   pml_kappa_max=kap, pml_alpha_max=alp, inv_eps=inv, sources=[src],
                   detectors=[det], design_lo=design_lo, design_hi=design_hi, T=T, rho=rho)


def with_tfsf(prob: Problem, k: Optional[int] = None, comp: int = 0) -> Problem:
    """The same problem with its first source replaced by a one-sided
    total-field/scattered-field plane wave along +z (section 2.1 names this
    source type) with the same waveform, on the plane k (default: that
    source's plane)."""
    s0 = prob.sources[0]
    src = Source(kind=2, comp=comp, i=0, j=0, k=s0.k if k is None else k, amp=s0.amp)
    return dataclasses.replace(prob, name=prob.name + "_tfsf", sources=[src] + list(prob.sources[1:]))


def with_lossy(prob: Problem, lo=None, hi=None, sigma_max: float = 1.0, seed: int = 21) -> Problem:
    """The same problem with conducting cells: per-cell sigma ~ U[0, sigma_max]
    (seed) over the box [lo, hi) (default: the design box, so the lossy
    region is also the design region).  In normalised units a cell with
    sigma and eps_r damps E by (1 - u)/(1 + u) per step, u = sigma S / (2 eps_r);
    sigma = 1 at eps_r = 2.25 gives u = 0.13, a 1/e length of a few cells."""
    lo = tuple(prob.design_lo) if lo is None else tuple(lo)
    hi = tuple(prob.design_hi) if hi is None else tuple(hi)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])
    sig = rng.uniform(0.0, sigma_max, size=shape).astype(np.float32)
    return dataclasses.replace(prob, name=prob.name + "_lossy", sigma=sig, lossy_lo=lo, lossy_hi=hi)


def config1(T: int = 500, n: int = 32) -> Problem:
    """32^3 bare PEC box, eps_r = 1 except a centred 8^3 block with per-cell
    eps_r ~ U[1, 12.25] (seed 1); Ez point dipole at the centre, Gaussian pulse."""
    rng = np.random.Generator(np.random.PCG64(1))
    eps = np.ones((n, n, n))
    lo, hi = n // 2 - 4, n // 2 + 4
    eps[lo:hi, lo:hi, lo:hi] = rng.uniform(1.0, 12.25, size=(8, 8, 8))
    S = courant()
    src = Source(kind=0, comp=2, i=n // 2, j=n // 2, k=n // 2, amp=gaussian_pulse(T))
    return Problem(name="c1_pec32", nx=n, ny=n, nz=n, S=S, p=0, pml_m=3.0, pml_sigma_max=0.0,
                   pml_kappa_max=1.0, pml_alpha_max=0.0, inv_eps=(1.0 / eps).astype(np.float32),
                   sources=[src], detectors=[], design_lo=(lo, lo, lo), design_hi=(hi, hi, hi), T=T)


def config2(T: int = 2000, n: int = 256, p: int = 10) -> Problem:
    """Forward-only n^3 with p-cell CPML, background eps_r 2.25, design cube of
    edge n/2 with per-cell eps_r ~ U[2.25, 12.25] (seed 2); Ex sheet source."""
    rng = np.random.Generator(np.random.PCG64(2))
    eps = np.full((n, n, n), 2.25)
    a, b = n // 4, n // 4 + n // 2
    eps[a:b, a:b, a:b] = rng.uniform(2.25, 12.25, size=(b - a,) * 3)
    return _sheet_problem(f"c2_fwd{n}", n, n, n, p, T, eps, 2.25, (a, a, a), (b, b, b))


def config3(T: int = 1500, n: int = 200, p: int = 10, d: int = 64) -> Problem:
    """Gradient solve n^3, p-cell CPML, centred design cube of edge d with
    rho ~ U[0,1] (seed 3), eps_r = 2.25 + 10 rho, background 2.25."""
    rng = np.random.Generator(np.random.PCG64(3))
    eps = np.full((n, n, n), 2.25)
    a = (n - d) // 2
    b = a + d
    rho = rng.uniform(0.0, 1.0, size=(d, d, d))
    eps[a:b, a:b, a:b] = eps_from_rho(rho)
    return _sheet_problem(f"c3_grad{n}", n, n, n, p, T, eps, 2.25, (a, a, a), (b, b, b), rho=rho)


def fd_cells(prob: Problem, count: int = 16, seed: int = 4) -> np.ndarray:
    """`count` distinct design cells (z, y, x offsets inside the design box)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dz, dy, dx = prob.design_shape()
    flat = rng.choice(dz * dy * dx, size=count, replace=False)
    return np.stack(np.unravel_index(flat, (dz, dy, dx)), axis=1)


def blurred_binary(shape, sigma: float, seed: int) -> np.ndarray:
    """Gaussian blur (reflecting edges) of a Bernoulli(0.5) field."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.integers(0, 2, size=shape).astype(np.float64)
    return gaussian_filter(x, sigma=sigma, mode="reflect")


def config4(T: int = 4000, nx: int = 640, ny: int = 640, nz: int = 400, p: int = 12,
            dbox=(256, 256, 128)) -> Problem:
    """Large forward+gradient problem: 640x640x400, 12-cell CPML, centred
    256x256x128 design box with a blurred binary rho (seed 5)."""
    lo = ((nx - dbox[0]) // 2, (ny - dbox[1]) // 2, (nz - dbox[2]) // 2)
    hi = (lo[0] + dbox[0], lo[1] + dbox[1], lo[2] + dbox[2])
    rho = blurred_binary((dbox[2], dbox[1], dbox[0]), 2.0, 5)
    eps = np.full((nz, ny, nx), 2.25, np.float32)
    eps[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = eps_from_rho(rho)
    return _sheet_problem(f"c4_large{nx}x{ny}x{nz}", nx, ny, nz, p, T, eps, 2.25, lo, hi, rho=rho)


def shard_slab(T: int = 100, nx: int = 2400, ny: int = 1600, nz: int = 150, p: int = 12) -> Problem:
    """One GPU's share of a 2400x1600x600 grid (about 2.3e9 cells, the size
    the paper's largest runs reach) cut into four z-slabs: 2400x1600x150 with a
    12-cell CPML on all six faces (a slab of a decomposed grid has it on the x
    and y faces only, and exchanges one plane with each z neighbour instead),
    background eps_r 2.25 with a centred half-edge block of per-cell
    eps_r ~ U[2.25, 12.25] (seed 9); Ex sheet source and flux detector as in
    the other configurations.  1/eps_r is built directly in FP32 (the field
    set alone is 13.8 GB)."""
    rng = np.random.Generator(np.random.PCG64(9))
    lo = (nx // 4, ny // 4, nz // 4)
    hi = (lo[0] + nx // 2, lo[1] + ny // 2, lo[2] + nz // 2)
    inv = np.full((nz, ny, nx), 1.0 / 2.25, np.float32)
    block = rng.uniform(2.25, 12.25, size=(hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0]))
    inv[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = 1.0 / block
    return _sheet_problem(f"shard{nx}x{ny}x{nz}", nx, ny, nz, p, T, None, 2.25, lo, hi, inv=inv)


def small_cpml(nx=40, ny=36, nz=44, p=6, T=160, d=8, seed=11, name="small_cpml") -> Problem:
    """A small CPML problem with ragged sizes: a design cube with rho ~ U[0,1]
    near the centre, the sheet source and the flux detector of the large configs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = np.full((nz, ny, nx), 2.25)
    lo = ((nx - d) // 2, (ny - d) // 2, (nz - d) // 2)
    hi = (lo[0] + d, lo[1] + d, lo[2] + d)
    rho = rng.uniform(0.0, 1.0, size=(d, d, d))
    eps[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = eps_from_rho(rho)
    pr = _sheet_problem(name, nx, ny, nz, p, T, eps, 2.25, lo, hi, rho=rho)
    # a short wavelength so that a few hundred steps carry signal across the box
    pr.sources[0].amp = ramped_sine(T, pr.S, lambda0=12.0, periods=1)
    return pr


# ----------------------------------------------------------- serving requests

@dataclasses.dataclass
class Request:
    rid: int
    kind: str            # "forward" or "gradient"
    arrival: float       # seconds after start (open loop)
    problem: Problem


def serving_request(edges, kind_grad: bool, seed: int, p: int = 8, rid: int = 0) -> Problem:
    """One request of the serving mix: eps_r ~ U[1, 12.25] in the interior, 1 in
    the CPML; sheet source at k = p+2; flux detector at nz-p-3; centred design
    box of half the edge on each axis; T = 8 * max edge."""
    nx, ny, nz = edges
    T = 8 * max(edges)
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = np.ones((nz, ny, nx))
    eps[p:nz - p, p:ny - p, p:nx - p] = rng.uniform(1.0, 12.25, size=(nz - 2 * p, ny - 2 * p, nx - 2 * p))
    lo = (nx // 4, ny // 4, nz // 4)
    hi = (lo[0] + nx // 2, lo[1] + ny // 2, lo[2] + nz // 2)
    pr = _sheet_problem(f"req{rid}_{nx}x{ny}x{nz}", nx, ny, nz, p, T, eps, 1.0, lo, hi)
    return pr


def serving_mix(count: int = 500, rate_hz: Optional[float] = None, lo: int = 64, hi: int = 256,
                p: int = 8, seeds=(6, 7, 8)) -> List[Tuple[int, Tuple[int, int, int], str, float]]:
    """Request descriptors (rid, edges, kind, arrival time) of the Poisson serving
    mix: edges uniform in {lo..hi} per axis (seed 6), 50% forward / 50% gradient
    (seed 7), exponential inter-arrival times at rate_hz (seed 8; all at t=0 if
    rate_hz is None).  Materials are generated per request with seed 1000+rid."""
    r_size = np.random.Generator(np.random.PCG64(seeds[0]))
    r_kind = np.random.Generator(np.random.PCG64(seeds[1]))
    r_arr = np.random.Generator(np.random.PCG64(seeds[2]))
    edges = r_size.integers(lo, hi + 1, size=(count, 3))
    kinds = r_kind.random(count) < 0.5
    if rate_hz is None:
        arr = np.zeros(count)
    else:
        arr = np.cumsum(r_arr.exponential(1.0 / rate_hz, size=count))
    return [(i, tuple(int(e) for e in edges[i]), "gradient" if kinds[i] else "forward", float(arr[i]))
            for i in range(count)]
