"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test would fail on a plausible mistake in the oracle: a dropped curl
term, a wrong sign, a transposed difference, a misplaced boundary, a wrong
Courant scaling, a broken record or inverse, a non-transposed adjoint.
"""
import dataclasses
import decimal
import math
import pathlib

import numpy as np
import pytest

from oracle.oracle import NSLOT, Oracle, tfsf_incident
from paper_2412_12360_amd import workloads as W


# ------------------------------------------------------------------ helpers

def pec_problem(nx, ny, nz, d=None, sources=(), detectors=(), T=1, design=None):
    S = W.courant()
    inv = np.ones((nz, ny, nx), np.float32) if d is None else d.astype(np.float32)
    lo, hi = design if design else ((0, 0, 0), (nx, ny, nz))
    return W.Problem(name="pec", nx=nx, ny=ny, nz=nz, S=S, p=0, pml_m=3.0, pml_sigma_max=0.0,
                     pml_kappa_max=1.0, pml_alpha_max=0.0, inv_eps=inv, sources=list(sources),
                     detectors=list(detectors), design_lo=lo, design_hi=hi, T=T)


def held_mask(nx, ny, nz):
    """Boolean [3, nz, ny, nx]: tangential E on the index-0 planes."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([(j == 0) | (k == 0), (i == 0) | (k == 0), (i == 0) | (j == 0)])


def random_state(prob, seed, with_psi=False):
    rng = np.random.default_rng(seed)
    st = np.zeros((NSLOT, prob.nz, prob.ny, prob.nx))
    st[:6] = rng.standard_normal(st[:6].shape)
    st[:3][held_mask(prob.nx, prob.ny, prob.nz)] = 0.0
    if with_psi:
        st[6:] = rng.standard_normal(st[6:].shape)
    return st


# ---------------------------------------------------- P13: step-count rule

GOLDEN = pathlib.Path(__file__).parent / "golden" / "paper_step_and_cell_counts.txt"


def printed_counts():
    rows = []
    for line in GOLDEN.read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            f = line.split()
            rows.append(dict(dx_nm=float(f[0]), L_um=tuple(float(v) for v in f[1:4]),
                             fs=float(f[4]), cells=decimal.Decimal(f[5]), steps=int(f[6]),
                             where=f[7]))
    return rows


def test_golden_table_is_complete():
    """Table 2 has five resolutions; sections 3.2 and 3.3 one scene each."""
    where = [r["where"] for r in printed_counts()]
    assert where.count("Table2") == 5 and "Sec3.2" in where and "Sec3.3" in where


@pytest.mark.parametrize("row", printed_counts(), ids=lambda r: f"{r['where']}-{r['dx_nm']}nm")
def test_step_counts_match_paper(row):
    """The 0.99 Courant factor on the 3D limit, rounded to nearest, gives every
    printed step count (section 3.1 Table 2, sections 3.2 and 3.3)."""
    assert W.steps_for(row["fs"] * 1e-15, row["dx_nm"] * 1e-9) == row["steps"]


@pytest.mark.parametrize("row", printed_counts(), ids=lambda r: f"{r['where']}-{r['dx_nm']}nm")
def test_cell_counts_match_paper(row):
    """Volume / dx^3 gives the printed cell count to its last printed digit."""
    cells = 1
    for L in row["L_um"]:
        n = L * 1000.0 / row["dx_nm"]
        assert abs(n - round(n)) < 1e-9          # the volume is a whole number of cells
        cells *= int(round(n))
    unit = decimal.Decimal(1).scaleb(row["cells"].as_tuple().exponent)
    assert abs(decimal.Decimal(cells) - row["cells"]) <= unit / 2


# ------------------------------------------------- P1: discrete energy

def test_energy_invariant_pec():
    """W^n = sum |E^n|^2/d + sum H^{n-1/2} . H^{n+1/2} is conserved exactly by
    the lossless leapfrog in a conducting box (no sources)."""
    nx, ny, nz = 13, 11, 9
    rng = np.random.default_rng(5)
    d = 1.0 / rng.uniform(1.0, 12.25, size=(nz, ny, nx))
    pr = pec_problem(nx, ny, nz, d=d)
    o = Oracle(pr)
    st = random_state(pr, 6)
    dd = o.d
    Ws = []
    for n in range(200):
        H_prev = st[3:6].copy()
        E_now = st[:3].copy()
        o.step_linear(st, 1)
        Ws.append(np.sum(E_now ** 2 / dd) + np.sum(H_prev * st[3:6]))
    Ws = np.array(Ws)
    assert np.max(np.abs(Ws - Ws[0])) / abs(Ws[0]) < 1e-12
    # the naive energy sum |E|^2/d + |H|^2 is not conserved: the invariant is not vacuous
    naive = np.sum(st[:3] ** 2 / dd) + np.sum(st[3:6] ** 2)
    assert abs(naive - Ws[0]) / Ws[0] > 1e-6


# ----------------------------------------- P2: cavity eigenmode recurrence

@pytest.mark.parametrize("comp,modes", [(2, (2, 3, 0)), (0, (0, 1, 2)), (1, (3, 0, 1))])
def test_cavity_mode_recurrence(comp, modes):
    """For a box eigenmode, E^{n+1} + E^{n-1} = (2 - 4 S^2 sum sin^2(pi m_a / 2 n_a)) E^n
    at every cell: Yee's numerical dispersion for standing waves.  Ez mode
    varies in x,y; Ex in y,z; Ey in x,z."""
    nx, ny, nz = 12, 10, 8
    pr = pec_problem(nx, ny, nz)
    o = Oracle(pr)
    st = np.zeros((NSLOT, nz, ny, nx))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = [i, j, k]
    n_ = [nx, ny, nz]
    f = np.ones((nz, ny, nx))
    lam = 0.0
    for a in range(3):
        if a == comp:
            continue
        f = f * np.sin(modes[a] * math.pi * pos[a] / n_[a])
        lam += 4 * math.sin(modes[a] * math.pi / (2 * n_[a])) ** 2
    st[comp] = f
    S = pr.S
    coef = 2 - S * S * lam
    hist = [st[comp].copy()]
    for n in range(40):
        o.step_linear(st, 1)
        hist.append(st[comp].copy())
        # the other E components stay zero
        for q in range(3):
            if q != comp:
                assert np.max(np.abs(st[q])) < 1e-13
    for n in range(1, 40):
        res = hist[n + 1] + hist[n - 1] - coef * hist[n]
        assert np.max(np.abs(res)) < 1e-12 * max(1.0, np.max(np.abs(hist[n])))


def _fit_omega(series):
    """2 cos(w) from E^{n+1} + E^{n-1} = 2cos(w) E^n by least squares."""
    x = series[1:-1]
    y = series[2:] + series[:-2]
    return float(np.arccos(np.dot(x, y) / np.dot(x, x) / 2.0))


def test_resonance_converges_to_continuum():
    """The lowest TM_110 resonance of a unit square cavity (uniform in z),
    measured from the oracle's time series, approaches the continuum value
    w = pi c sqrt(1/Lx^2 + 1/Ly^2) with O(dx^2) error."""
    errs = []
    for n in (8, 16, 32):
        pr = pec_problem(n, n, 2)
        o = Oracle(pr)
        st = np.zeros((NSLOT, 2, n, n))
        k, j, i = np.meshgrid(np.arange(2), np.arange(n), np.arange(n), indexing="ij")
        st[2] = np.sin(math.pi * i / n) * np.sin(math.pi * j / n)
        series = []
        for _ in range(60):
            o.step_linear(st, 1)
            series.append(st[2, 0, n // 2, n // 2])
        w_step = _fit_omega(np.array(series))
        dx = 1.0 / n
        dt = pr.S * dx
        w = w_step / dt
        errs.append(abs(w - math.pi * math.sqrt(2.0)) / (math.pi * math.sqrt(2.0)))
    assert errs[0] < 0.05
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5


# ------------------------------------------ P4: forward then inverse

@pytest.mark.parametrize("comp", [2, 4])
def test_inverse_recovers_pec_state(comp):
    """On a closed conducting box the whole update is reversible (section 2.2):
    T forward steps with a source (on E, or on H), then T inverse steps,
    recover the start."""
    nx, ny, nz = 14, 12, 10
    rng = np.random.default_rng(7)
    d = 1.0 / rng.uniform(1.0, 12.25, size=(nz, ny, nx))
    T = 80
    src = W.Source(kind=0, comp=comp, i=7, j=6, k=5, amp=W.gaussian_pulse(T, 20, 6))
    pr = pec_problem(nx, ny, nz, d=d, sources=[src], T=T)
    o = Oracle(pr)
    st = random_state(pr, 8)
    s0 = st.copy()
    o.forward(st, T)
    assert np.max(np.abs(st[:6] - s0[:6])) > 0.1
    o.inverse(st, None, T)
    assert np.max(np.abs(st[:6] - s0[:6])) < 1e-12 * np.max(np.abs(s0[:6])) * T


@pytest.mark.parametrize("tfsf", [False, True])
def test_inverse_recovers_cpml_interior_with_record(tfsf):
    """With CPML only the interior is reversible; the six face records (2
    tangential components each) make the interior exactly recoverable (with
    the sheet source, and with the TFSF plane's E and H sources)."""
    pr = W.small_cpml(nx=26, ny=24, nz=28, p=5, T=120)
    pr = W.with_tfsf(pr) if tfsf else pr
    o = Oracle(pr)
    st = o.new_state()
    # a nonzero start inside the interior
    rng = np.random.default_rng(9)
    p = pr.p
    st[:6, p:-p, p:-p, p:-p] = rng.standard_normal((6, pr.nz - 2 * p, pr.ny - 2 * p, pr.nx - 2 * p))
    s0 = st.copy()
    J, tr, rec = o.forward(st, pr.T, record=True)
    # without the record the reconstruction is wrong
    bad = st.copy()
    o.inverse(bad, np.zeros_like(rec), pr.T)
    inner = (slice(0, 6), slice(p, -p), slice(p, -p), slice(p, -p))
    assert np.max(np.abs(bad[inner] - s0[inner])) > 1e-3
    o.inverse(st, rec, pr.T)
    assert np.max(np.abs(st[inner] - s0[inner])) < 1e-11


def test_record_size_matches_six_slices():
    pr = W.small_cpml(nx=26, ny=24, nz=28, p=5)
    o = Oracle(pr)
    Lx, Ly, Lz = 26 - 10, 24 - 10, 28 - 10
    assert o.record_floats() == 2 * 2 * (Ly * Lz + Lx * Lz + Lx * Ly)


# ------------------------------------------- P5: adjoint = transpose

@pytest.mark.parametrize("T", [1, 3])
def test_adjoint_is_transpose_with_cpml(T):
    """<M x, y> = <x, M^T y> for the full step map including every psi."""
    pr = W.small_cpml(nx=17, ny=15, nz=19, p=4, T=4)
    # a non-trivial kappa exercises the 1/kappa scaling too
    pr.pml_kappa_max = 3.0
    o = Oracle(pr)
    x = random_state(pr, 10, with_psi=True)
    y = random_state(pr, 11, with_psi=True)
    Mx = x.copy()
    o.step_linear(Mx, T)
    Mty = y.copy()
    o.adjoint_linear(Mty, T)
    lhs = np.sum(Mx * y)
    rhs = np.sum(x * Mty)
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(Mx ** 2) * np.sum(y ** 2)) * 10


# --------------------------------------- P6, P7: gradient by VJP vs FD

def tiny_grad_problem(T=60):
    return W.small_cpml(nx=16, ny=16, nz=16, p=3, T=T, d=4, seed=12, name="tiny")


@pytest.mark.parametrize("tfsf", [False, True])
def test_history_gradient_equals_reversed_gradient(tfsf):
    """Time reversal reaches exactly the plain stored-history VJP (section 2.2)."""
    pr = W.small_cpml(nx=22, ny=20, nz=24, p=4, T=90, d=6, seed=13)
    pr = W.with_tfsf(pr) if tfsf else pr
    o = Oracle(pr)
    g1, J1, tr1 = o.grad_history(seg=7)
    g2, J2, tr2, recon = o.grad_reversed()
    assert abs(J1 - J2) <= 1e-13 * abs(J1)
    assert np.max(np.abs(g1)) > 0
    assert np.linalg.norm(g1 - g2) <= 1e-10 * np.linalg.norm(g1)
    assert recon < 1e-12
    # segment length does not change the stored-history result
    g3, _, _ = o.grad_history(seg=90)
    assert np.linalg.norm(g1 - g3) <= 1e-13 * np.linalg.norm(g1)


@pytest.mark.parametrize("tfsf", [False, True])
def test_gradient_matches_central_differences_all_design_cells(tfsf):
    """Central differences in rho (h = 1e-3) against the adjoint dJ/drho = 10 dJ/deps
    on every design cell of a tiny CPML problem (sheet source, or TFSF plane)."""
    pr = tiny_grad_problem()
    pr = W.with_tfsf(pr) if tfsf else pr
    o = Oracle(pr)
    g, J, _ = o.grad_history()
    # dJ/drho = dJ/deps * 10 with eps = 2.25 + 10 rho, evaluated at the exact float64 d
    eps0 = W.eps_from_rho(pr.rho)
    sl = pr.design_slices()
    d_exact = o.d.copy()
    d_exact[sl] = 1.0 / eps0
    o = Oracle(pr, d=d_exact)
    g, J, _ = o.grad_history()
    adj = 10.0 * o.deps_design(g)
    h = 1e-3
    fd = np.zeros_like(adj)
    for idx in np.ndindex(*adj.shape):
        vals = []
        for sgn in (1, -1):
            rho = pr.rho.copy()
            rho[idx] += sgn * h
            d = d_exact.copy()
            d[sl] = 1.0 / W.eps_from_rho(rho)
            Jp, _, _ = Oracle(pr, d=d).forward(Oracle(pr, d=d).new_state(), pr.T)
            vals.append(Jp)
        fd[idx] = (vals[0] - vals[1]) / (2 * h)
    assert np.max(np.abs(adj)) > 0
    assert np.linalg.norm(fd - adj) <= 1e-6 * np.linalg.norm(adj)


# ------------------------------------------------ P10: CPML special case

def test_cpml_with_zero_grading_is_plain_yee_bitwise():
    pr = W.small_cpml(nx=18, ny=16, nz=20, p=5, T=50)
    pr.pml_sigma_max = 0.0
    pr.pml_alpha_max = 0.0
    pr.pml_kappa_max = 1.0
    st1, J1, tr1, _ = Oracle(pr).run()
    import dataclasses
    plain = dataclasses.replace(pr, p=0)
    st2, J2, tr2, _ = Oracle(plain).run()
    assert np.array_equal(st1[:6], st2[:6])
    assert np.array_equal(tr1, tr2)
    assert np.all(st1[6:] == 0.0)


def test_grading_profile_values():
    """b, a, 1/kappa at a few coordinates against the CFS-CPML formulas."""
    pr = W.small_cpml(nx=30, ny=30, nz=30, p=6)
    pr.pml_kappa_max = 2.0
    o = Oracle(pr)
    # interior: no stretching
    assert np.allclose(o.grade(0, 15.0), [1.0, 0.0, 1.0])
    assert np.allclose(o.grade(0, 6.0), [1.0, 0.0, 1.0])
    assert np.allclose(o.grade(0, 24.0), [1.0, 0.0, 1.0])
    # the outer wall (delta = 1): alpha = 0
    sig, kap = pr.pml_sigma_max, 2.0
    b = math.exp(-sig / kap)
    assert np.allclose(o.grade(0, 0.0), [b, (b - 1) / kap, 1 / kap])
    # half depth on the high side
    delta = 3.0 / 6
    s = sig * delta ** 3
    k = 1 + (kap - 1) * delta ** 3
    al = pr.pml_alpha_max * (1 - delta)
    b = math.exp(-(s / k + al))
    a = s / (s * k + k * k * al) * (b - 1)
    assert np.allclose(o.grade(0, 27.0), [b, a, 1 / k])


# --------------------------------------------------- P11: reflection

def _point_pulse_probe(n, p, T, probe_offset):
    """Ez at `probe_offset` cells below a centred point source (zero-mean
    derivative-of-Gaussian drive) in an n^3 box with a p-cell CPML."""
    c = n // 2
    t = np.arange(T, dtype=np.float64)
    amp = (-(t - 30) / 8.0 * np.exp(-((t - 30) / 8.0) ** 2)).astype(np.float32)
    src = W.Source(kind=0, comp=2, i=c, j=c, k=c, amp=amp)
    S = W.courant()
    m, sig, kap, alp = W.pml_grading(S, 1.0)
    pr = W.Problem(name="refl", nx=n, ny=n, nz=n, S=S, p=p, pml_m=m, pml_sigma_max=sig,
                   pml_kappa_max=kap, pml_alpha_max=alp, inv_eps=np.ones((n, n, n), np.float32),
                   sources=[src], detectors=[], design_lo=(c, c, c), design_hi=(c + 1,) * 3, T=T)
    o = Oracle(pr)
    st = o.new_state()
    out = []
    for n_ in range(T):
        o.forward(st, 1, n0=n_)
        out.append(st[2, c - probe_offset, c, c])
    return np.array(out)


def test_cpml_reflection_small():
    """Probe 2 cells in front of the CPML of a 30^3 box versus the same probe in
    a 60^3 box, over the window before the large box's own reflection returns:
    the CPML reflection stays below 2% of the pulse peak (empirical bound; the
    paper prints none).  A plain conducting wall (no CPML) fails the same bound."""
    T = 85
    small = _point_pulse_probe(30, 6, T, 7)
    big = _point_pulse_probe(60, 6, T, 7)
    bare = _point_pulse_probe(30, 0, T, 7)
    peak = np.max(np.abs(big))
    assert peak > 0
    err = np.max(np.abs(small - big)) / peak
    assert err < 0.02, err
    assert np.max(np.abs(bare - big)) / peak > 0.1


# ------------------------------------------------- P12: reciprocity

def test_reciprocity_point_sources():
    """Ez at B from an impulse at A equals Ez at A from an impulse at B when
    1/eps_r is equal at A and B (lossless, conducting box)."""
    nx, ny, nz = 12, 11, 10
    rng = np.random.default_rng(14)
    d = 1.0 / rng.uniform(1.0, 12.25, size=(nz, ny, nx))
    A, B = (3, 4, 5), (8, 6, 3)
    d[A[2], A[1], A[0]] = d[B[2], B[1], B[0]] = 0.5
    T = 60
    imp = np.zeros(T, np.float32)
    imp[0] = 1.0

    def trace(src, rcv):
        s = W.Source(kind=0, comp=2, i=src[0], j=src[1], k=src[2], amp=imp)
        pr = pec_problem(nx, ny, nz, d=d, sources=[s], T=T)
        o = Oracle(pr)
        st = o.new_state()
        out = []
        for t in range(T):
            o.forward(st, 1, n0=t)
            out.append(st[2, rcv[2], rcv[1], rcv[0]])
        return np.array(out)
    ab = trace(A, B)
    ba = trace(B, A)
    assert np.max(np.abs(ab)) > 1e-3
    assert np.max(np.abs(ab - ba)) < 1e-12


# ----------------------------------------------------- detector sign

def test_plane_wave_flux_is_positive_upward():
    """The sheet source radiates a +z wave through the detector plane, so the
    non-interpolated flux integrates to J > 0; a detector below the sheet
    sees a -z wave and J < 0."""
    pr = W.small_cpml(nx=24, ny=24, nz=40, p=5, T=200)
    o = Oracle(pr)
    _, J, tr, _ = o.run()
    assert J > 0
    import dataclasses
    below = dataclasses.replace(pr.detectors[0], k=pr.p + 1)
    pr2 = dataclasses.replace(pr, detectors=[below])
    _, J2, _, _ = Oracle(pr2).run()
    assert J2 < 0


# ------------------------------------ P14: total-field/scattered-field plane

def tfsf_box(T, k0, pol, n_extra=10):
    """A conducting box wide enough that no column within T+3 cells of the
    centre can see a side wall within T steps (a Yee update moves information
    at most one cell per step), and tall enough that the incident wave does not
    reach the top wall; eps_r = 2.25 everywhere."""
    n = 2 * T + n_extra
    nz = k0 + T + 6
    inv = np.full((nz, n, n), 1.0 / 2.25, np.float32)
    amp = W.ramped_sine(T, W.courant(), lambda0=12.0, periods=1)
    src = W.Source(kind=2, comp=pol, i=0, j=0, k=k0, amp=amp)
    return pec_problem(n, n, nz, d=inv, sources=[src], T=T), amp


@pytest.mark.parametrize("pol", [0, 1])
def test_tfsf_total_field_is_the_incident_line_scattered_field_is_zero(pol):
    """Away from the side walls a plane wave along z is exactly a 1D problem:
    above the plane the 3D field equals the incident line (E on its nodes, the
    matching H between them), below it every component stays zero.  A wrong
    sign, a wrong time level of either correction or a line with other
    coefficients than the grid leaks 0.3-1.5 of the field below the plane."""
    T, k0 = 24, 6
    pr, amp = tfsf_box(T, k0, pol)
    o = Oracle(pr)
    st = o.new_state()
    o.forward(st, T)
    n = pr.nx
    _, _, El, Hl = tfsf_incident(pr.S, float(o.d[k0, n // 2, n // 2]), amp.astype(np.float64), pol)
    c = slice(T + 3, n - T - 3)
    assert c.stop > c.start
    Ecomp = st[pol][:, c, c]
    Hcomp = st[4 if pol == 0 else 3][:, c, c]
    hsign = 1.0 if pol == 0 else -1.0
    scale = np.max(np.abs(El))
    assert scale > 0.1
    j = np.arange(k0, pr.nz) - (k0 - 1)          # line node of each total-field plane
    Eref = np.array([El[q] if q < len(El) else 0.0 for q in j])
    Href = np.array([Hl[q] if q < len(Hl) else 0.0 for q in j])
    assert np.max(np.abs(Ecomp[k0:] - Eref[:, None, None])) <= 1e-13 * scale
    assert np.max(np.abs(Hcomp[k0:] - hsign * Href[:, None, None])) <= 1e-13 * scale
    for q in range(6):
        assert np.max(np.abs(st[q][:k0, c, c])) <= 1e-14 * scale
    for q in {0, 1, 2, 3, 4, 5} - {pol, 4 if pol == 0 else 3}:
        assert np.max(np.abs(st[q][:, c, c])) == 0.0


@pytest.mark.parametrize("lam,d", [(20.0, 1 / 2.25), (12.0, 1.0), (30.0, 1 / 12.25)])
def test_tfsf_line_obeys_discrete_dispersion(lam, d):
    """The incident line is a 1D Yee grid: behind the switched-on front its
    field is a sinusoid whose wavenumber kk obeys the closed-form discrete
    dispersion sin(w/2) = S sqrt(d) sin(kk/2), so E[k-1] + E[k+1] = 2 cos(kk) E[k].
    The continuum value cos(w / (S sqrt(d))) differs by 2e-3 to 1e-2."""
    S = W.courant()
    T = 1200
    amp = W.ramped_sine(T, S, lambda0=lam, periods=2).astype(np.float64)
    w = 2 * math.pi * S / lam
    _, _, E, _ = tfsf_incident(S, d, amp, 0)
    v = S * math.sqrt(d)
    settled = int(0.8 * v * (T - round(2 * 2 * math.pi / w)))
    k = np.arange(2, settled)
    c_fit = np.sum((E[k - 1] + E[k + 1]) * E[k]) / (2 * np.sum(E[k] ** 2))
    c_discrete = 1 - 2 * (math.sin(w / 2) / v) ** 2
    c_continuum = math.cos(w / v)
    assert abs(c_fit - c_discrete) <= 1e-4
    assert abs(c_fit - c_continuum) >= 1e-3


def test_tfsf_is_one_sided_sheet_is_not():
    """In a CPML box the TFSF plane radiates only upward: the flux through a
    plane below it is below 1e-6 of the flux above (8e-9 measured), while the
    soft sheet radiates as much downward as upward."""
    S = W.courant()
    n, nz, p, T, k0 = 40, 64, 8, 260, 24
    m, sig, kap, alp = W.pml_grading(S, 2.25)
    inv = np.full((nz, n, n), 1.0 / 2.25, np.float32)
    amp = W.ramped_sine(T, S, lambda0=16.0, periods=2)
    dets = [W.Detector(k=k0 - 6, i0=p, i1=n - p, j0=p, j1=n - p), W.Detector(k=k0 + 14, i0=p, i1=n - p, j0=p, j1=n - p)]
    ratio = {}
    for kind in (1, 2):
        src = W.Source(kind=kind, comp=0, i=0, j=0, k=k0, amp=amp)
        pr = W.Problem(name="one_sided", nx=n, ny=n, nz=nz, S=S, p=p, pml_m=m, pml_sigma_max=sig,
                       pml_kappa_max=kap, pml_alpha_max=alp, inv_eps=inv, sources=[src], detectors=dets,
                       design_lo=(16, 16, 34), design_hi=(24, 24, 40), T=T)
        _, _, trace, _ = Oracle(pr).run()
        up = np.sum(trace[:, 1])
        assert up > 0
        ratio[kind] = abs(np.sum(trace[:, 0])) / up
    assert ratio[2] < 1e-6
    assert ratio[1] > 0.5


# ------------------------------------------- P15: interpolated flux detector

OFFSETS = {0: (0.5, 0.0, 0.0), 1: (0.0, 0.5, 0.0), 3: (0.0, 0.5, 0.5), 4: (0.5, 0.0, 0.5)}   # Ex, Ey, Hx, Hy


def trilinear(F, off, x, y, z):
    """A staggered component F[z, y, x] whose node (i, j, k) sits at
    (i, j, k) + off, interpolated trilinearly at (x, y, z)."""
    axes = []
    for u, o in zip((x, y, z), off):
        t = u - o
        lo = math.floor(t)
        w = t - lo
        axes.append([(lo, 1.0 - w), (lo + 1, w)])
    v = 0.0
    for i, wi in axes[0]:
        for j, wj in axes[1]:
            for k, wk in axes[2]:
                if wi * wj * wk != 0.0:
                    v += wi * wj * wk * F[k, j, i]
    return v


def test_interpolated_flux_is_the_colocated_product():
    """Section 2.1: composite metrics need all components at one point and
    time.  Against a generic trilinear interpolation of each component from
    its own Yee position (E at integer steps, H at half steps) onto the points
    (i+1/2, j+1/2, k) at time n+1/2, on random CPML states stepped with a
    source: a wrong axis, layer, neighbour or time level fails it."""
    pr = W.small_cpml(nx=14, ny=13, nz=12, p=3, T=6, d=4, seed=41)
    k = 6
    pr = dataclasses.replace(pr, detectors=[
        W.Detector(k=k, i0=2, i1=12, j0=1, j1=11, weight=0.0, interpolate=True),
        W.Detector(k=k, i0=2, i1=12, j0=1, j1=11, weight=0.0)])
    o = Oracle(pr)
    st = random_state(pr, 42, with_psi=True)
    for n in range(pr.T):
        before = st.copy()
        _, trace, _ = o.forward(st, 1, n0=n)
        got = trace[0, 0]
        want = plain = 0.0
        for j in range(1, 11):
            for i in range(2, 12):
                x, y = i + 0.5, j + 0.5
                ex = 0.5 * (trilinear(before[0], OFFSETS[0], x, y, k) + trilinear(st[0], OFFSETS[0], x, y, k))
                ey = 0.5 * (trilinear(before[1], OFFSETS[1], x, y, k) + trilinear(st[1], OFFSETS[1], x, y, k))
                hx = trilinear(st[3], OFFSETS[3], x, y, k)
                hy = trilinear(st[4], OFFSETS[4], x, y, k)
                want += ex * hy - ey * hx
                plain += st[0][k, j, i] * st[4][k, j, i] - st[1][k, j, i] * st[3][k, j, i]
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want))
        assert abs(trace[0, 1] - plain) <= 1e-12 * max(1.0, abs(plain))
        assert abs(got - plain) > 1e-3 * abs(want)


def test_interpolated_flux_of_a_plane_wave_is_in_phase():
    """A steady plane wave (TFSF in a conducting box, central columns that
    cannot see a side wall): the co-located flux is C sin^2(w(n+1/2) - phase),
    so its oscillation equals its mean, with C = cos(w/2) cos(kk/2) / sqrt(d)
    from the discrete dispersion (E amplitude 1).  The non-interpolated flux,
    whose E and H sit half a step and half a cell apart, oscillates 1.2 times
    its mean and turns negative."""
    S = W.courant()
    T, k0, lam = 80, 6, 8.0
    n, nz = 2 * T + 10, k0 + T + 6
    d = 1.0 / 2.25
    inv = np.full((nz, n, n), d, np.float32)
    src = W.Source(kind=2, comp=0, i=0, j=0, k=k0, amp=W.ramped_sine(T, S, lambda0=lam, periods=2))
    c0, c1 = T + 3, n - T - 4
    dets = [W.Detector(k=k0 + 3, i0=c0, i1=c1, j0=c0, j1=c1, interpolate=True),
            W.Detector(k=k0 + 3, i0=c0, i1=c1, j0=c0, j1=c1)]
    pr = pec_problem(n, n, nz, d=inv, sources=[src], detectors=dets, T=T)
    _, _, trace, _ = Oracle(pr).run()
    cells = (c1 - c0) ** 2
    w = 2 * math.pi * S / lam
    kk = 2 * math.asin(math.sin(w / 2) / (S * math.sqrt(d)))
    C = math.cos(w / 2) * math.cos(kk / 2) / math.sqrt(d)
    steady = np.arange(45, T)
    X = np.stack([np.ones(len(steady)), np.cos(2 * w * steady), np.sin(2 * w * steady)], 1)
    fit = lambda P: np.linalg.lstsq(X, P[steady] / cells, rcond=None)[0]
    a, b, c = fit(trace[:, 0])
    assert abs(a - C / 2) <= 2e-3 * C
    assert abs(math.hypot(b, c) - a) <= 2e-3 * a
    assert np.min(trace[steady, 0]) >= -1e-3 * C * cells
    ap, bp, cp = fit(trace[:, 1])
    assert math.hypot(bp, cp) > 1.1 * ap
    assert np.min(trace[steady, 1]) < -0.05 * C * cells


def with_interp_objective(pr):
    """The objective from an interpolated detector (weight 1) and the plain
    flux of the same window (weight 0.3)."""
    d = pr.detectors[0]
    return dataclasses.replace(pr, detectors=[dataclasses.replace(d, weight=0.3),
                                              dataclasses.replace(d, weight=1.0, interpolate=True)])


def test_interpolated_objective_history_equals_reversed_gradient():
    pr = with_interp_objective(W.small_cpml(nx=22, ny=20, nz=24, p=4, T=90, d=6, seed=13))
    o = Oracle(pr)
    g1, J1, _ = o.grad_history(seg=7)
    g2, J2, _, recon = o.grad_reversed()
    assert abs(J1 - J2) <= 1e-13 * abs(J1)
    assert np.max(np.abs(g1)) > 0
    assert np.linalg.norm(g1 - g2) <= 1e-10 * np.linalg.norm(g1)
    # the interpolated detector's own adjoint source matters
    g0, _, _ = Oracle(dataclasses.replace(pr, detectors=pr.detectors[:1])).grad_history(seg=7)
    assert np.linalg.norm(g1 - g0) > 0.1 * np.linalg.norm(g1)


def test_interpolated_objective_gradient_matches_central_differences():
    """Central differences of the interpolated-flux objective in rho on every
    design cell against the adjoint (the detector's adjoint source covers
    E^{n+1} in two flux terms and H^{n+1/2} on both layers)."""
    pr = with_interp_objective(tiny_grad_problem())
    sl = pr.design_slices()
    o = Oracle(pr)
    d_exact = o.d.copy()
    d_exact[sl] = 1.0 / W.eps_from_rho(pr.rho)
    o = Oracle(pr, d=d_exact)
    g, J, _ = o.grad_history()
    adj = 10.0 * o.deps_design(g)
    h = 1e-3
    fd = np.zeros_like(adj)
    for idx in np.ndindex(*adj.shape):
        vals = []
        for sgn in (1, -1):
            rho = pr.rho.copy()
            rho[idx] += sgn * h
            d = d_exact.copy()
            d[sl] = 1.0 / W.eps_from_rho(rho)
            oo = Oracle(pr, d=d)
            vals.append(oo.forward(oo.new_state(), pr.T)[0])
        fd[idx] = (vals[0] - vals[1]) / (2 * h)
    assert np.max(np.abs(adj)) > 0
    assert np.linalg.norm(fd - adj) <= 1e-6 * np.linalg.norm(adj)


OFFSETS.update({2: (0.0, 0.0, 0.5), 5: (0.5, 0.5, 0.0)})   # Ez, Hz


def test_colocated_energy_is_the_trilinear_interpolation():
    """The co-located energy 1/2 (eps_r |E|^2 + |H|^2) at (i+1/2, j+1/2, k),
    time n+1/2 (eps_r of cell (i,j,k)), against the generic trilinear
    interpolation of all six staggered components, on random CPML states with
    per-cell eps_r, stepped with a source."""
    pr = W.small_cpml(nx=14, ny=13, nz=12, p=3, T=5, d=6, seed=43)
    k = 6
    pr = dataclasses.replace(pr, detectors=[
        W.Detector(k=k, i0=3, i1=12, j0=2, j1=11, weight=0.0, interpolate=True, quantity=1)])
    o = Oracle(pr)
    eps = 1.0 / o.d
    st = random_state(pr, 44, with_psi=True)
    for n in range(pr.T):
        before = st.copy()
        _, trace, _ = o.forward(st, 1, n0=n)
        want = 0.0
        for j in range(2, 11):
            for i in range(3, 12):
                x, y = i + 0.5, j + 0.5
                e2 = sum((0.5 * (trilinear(before[q], OFFSETS[q], x, y, k) +
                                 trilinear(st[q], OFFSETS[q], x, y, k))) ** 2 for q in (0, 1, 2))
                h2 = sum(trilinear(st[q], OFFSETS[q], x, y, k) ** 2 for q in (3, 4, 5))
                want += 0.5 * (eps[k, j, i] * e2 + h2)
        assert abs(trace[0, 0] - want) <= 1e-12 * want


def test_colocated_energy_of_a_plane_wave():
    """Steady plane wave (as above): E amplitude 1 and H amplitude sqrt(eps_r)
    (from the discrete update and dispersion), so the co-located energy is
    1/2 eps (cos^2(w/2) + cos^2(kk/2)) sin^2(w(n+1/2) - phase) per cell: mean
    equal to its oscillation, both a quarter of eps (cos^2(w/2) + cos^2(kk/2))."""
    S = W.courant()
    T, k0, lam = 80, 6, 8.0
    n, nz = 2 * T + 10, k0 + T + 6
    d = 1.0 / 2.25
    inv = np.full((nz, n, n), d, np.float32)
    src = W.Source(kind=2, comp=0, i=0, j=0, k=k0, amp=W.ramped_sine(T, S, lambda0=lam, periods=2))
    c0, c1 = T + 3, n - T - 4
    dets = [W.Detector(k=k0 + 3, i0=c0, i1=c1, j0=c0, j1=c1, interpolate=True, quantity=1, weight=0.0)]
    pr = pec_problem(n, n, nz, d=inv, sources=[src], detectors=dets, T=T)
    o = Oracle(pr)
    _, _, trace, _ = o.run()
    cells = (c1 - c0) ** 2
    w = 2 * math.pi * S / lam
    kk = 2 * math.asin(math.sin(w / 2) / (S * math.sqrt(d)))
    eps = 1.0 / float(o.d[k0 + 3, n // 2, n // 2])
    mean = 0.25 * eps * (math.cos(w / 2) ** 2 + math.cos(kk / 2) ** 2)
    steady = np.arange(45, T)
    X = np.stack([np.ones(len(steady)), np.cos(2 * w * steady), np.sin(2 * w * steady)], 1)
    a, b, c = np.linalg.lstsq(X, trace[steady, 0] / cells, rcond=None)[0]
    assert abs(a - mean) <= 2e-3 * mean
    assert abs(math.hypot(b, c) - a) <= 2e-3 * a


def with_energy_objective(pr):
    """Objective: the co-located energy (weight 1) on the flux detector's
    window (outside the design box in z) plus the plain flux (weight 0.3)."""
    d = pr.detectors[0]
    assert not (pr.design_lo[2] <= d.k < pr.design_hi[2])
    return dataclasses.replace(pr, detectors=[dataclasses.replace(d, weight=0.3),
                                              dataclasses.replace(d, weight=1.0, interpolate=True, quantity=1)])


def test_energy_objective_history_equals_reversed_gradient():
    pr = with_energy_objective(W.small_cpml(nx=22, ny=20, nz=24, p=4, T=90, d=6, seed=13))
    o = Oracle(pr)
    g1, J1, _ = o.grad_history(seg=7)
    g2, J2, _, _ = o.grad_reversed()
    assert abs(J1 - J2) <= 1e-13 * abs(J1)
    assert np.linalg.norm(g1 - g2) <= 1e-10 * np.linalg.norm(g1)
    g0, _, _ = Oracle(dataclasses.replace(pr, detectors=pr.detectors[:1])).grad_history(seg=7)
    assert np.linalg.norm(g1 - g0) > 0.1 * np.linalg.norm(g1)


def test_energy_objective_gradient_matches_central_differences():
    """Central differences of an objective holding the co-located energy, on
    every design cell (the energy's adjoint source covers E^{n+1} in two energy
    terms, Ez on two layers and all three H components)."""
    pr = with_energy_objective(tiny_grad_problem())
    sl = pr.design_slices()
    o = Oracle(pr)
    d_exact = o.d.copy()
    d_exact[sl] = 1.0 / W.eps_from_rho(pr.rho)
    o = Oracle(pr, d=d_exact)
    g, J, _ = o.grad_history()
    adj = 10.0 * o.deps_design(g)
    h = 5e-4   # the energy is quadratic in the fields: a smaller step keeps O(h^2) below 1e-6
    fd = np.zeros_like(adj)
    for idx in np.ndindex(*adj.shape):
        vals = []
        for sgn in (1, -1):
            rho = pr.rho.copy()
            rho[idx] += sgn * h
            d = d_exact.copy()
            d[sl] = 1.0 / W.eps_from_rho(rho)
            oo = Oracle(pr, d=d)
            vals.append(oo.forward(oo.new_state(), pr.T)[0])
        fd[idx] = (vals[0] - vals[1]) / (2 * h)
    assert np.max(np.abs(adj)) > 0
    assert np.linalg.norm(fd - adj) <= 1e-6 * np.linalg.norm(adj)


# ------------------------------------ P10b: CPML along each axis, in 1D

def _grading_1d(n, p, u, m, smax, kmax, amax):
    """The CFS-CPML grading at staggered coordinate u (reading R7: depth
    delta = max(p-u, u-(n-p), 0)/p, sigma = smax delta^m, kappa = 1 + (kmax-1)
    delta^m, alpha = amax (1-delta), b = exp(-(sigma/kappa + alpha)),
    a = sigma (b-1) / (sigma kappa + kappa^2 alpha))."""
    delta = max(p - u, u - (n - p), 0.0) / p
    if delta <= 0.0:
        return 1.0, 0.0, 1.0
    dm = delta ** m
    sig, kap, alp = smax * dm, 1.0 + (kmax - 1.0) * dm, amax * (1.0 - delta)
    b = math.exp(-(sig / kap + alp))
    return b, sig * (b - 1.0) / (sig * kap + kap * kap * alp), 1.0 / kap


def _line_1d(n, p, S, d, pr, E0, T):
    """A separate 1D recursion along one axis: H at i + 1/2 from the forward
    difference of E, E at i from the backward difference of H, each difference
    wrapped by its own psi recursion, E held at index 0 and read as 0 at n."""
    gE = np.array([_grading_1d(n, p, float(i), pr.pml_m, pr.pml_sigma_max, pr.pml_kappa_max, pr.pml_alpha_max)
                   for i in range(n)])
    gH = np.array([_grading_1d(n, p, i + 0.5, pr.pml_m, pr.pml_sigma_max, pr.pml_kappa_max, pr.pml_alpha_max)
                   for i in range(n)])
    E, H = E0.astype(np.float64).copy(), np.zeros(n)
    pE, pH = np.zeros(n), np.zeros(n)
    out = []
    for _ in range(T):
        dH = np.append(E[1:], 0.0) - E
        pH = gH[:, 0] * pH + gH[:, 1] * dH
        H = H - S * (dH * gH[:, 2] + pH)
        dE = H - np.concatenate(([0.0], H[:-1]))
        pE = gE[:, 0] * pE + gE[:, 1] * dE
        E = E - S * d * (dE * gE[:, 2] + pE)
        E[0] = 0.0
        out.append(E.copy())
    return np.array(out)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cpml_along_each_axis_matches_1d_recursion(axis):
    """A pulse uniform across the two other axes, travelling along `axis` into
    the graded CPML (kappa_max 3, so every term of the recursion acts): the
    oracle's central line equals a separately written 1D recursion with the
    grading evaluated at integer (E) and half-integer (H) coordinates, until
    the transverse conducting walls can reach the line (one cell per step)."""
    n, p, T = 40, 8, 56
    w = 2 * T + 6
    shape = [w, w, w]
    shape[axis] = n
    nx, ny, nz = shape
    S = W.courant()
    m, sig, kap, alp = W.pml_grading(S, 2.25, kappa_max=3.0, alpha_max=0.05)
    pr = W.Problem(name="cpml1d", nx=nx, ny=ny, nz=nz, S=S, p=p, pml_m=m, pml_sigma_max=sig,
                   pml_kappa_max=kap, pml_alpha_max=alp,
                   inv_eps=np.full((nz, ny, nx), 1.0 / 2.25, np.float32), sources=[], detectors=[],
                   design_lo=(p, p, p), design_hi=(p + 1, p + 1, p + 1), T=T)
    o = Oracle(pr)
    e = (axis + 1) % 3                      # E component across the line; H is (axis + 2) % 3
    i = np.arange(n, dtype=np.float64)
    E0 = np.exp(-((i - n / 2) / 3.0) ** 2)
    E0[0] = 0.0
    st = o.new_state()
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    st[e] = np.broadcast_to(E0.reshape(bshape), (nz, ny, nx))
    st[e][held_mask(nx, ny, nz)[e]] = 0.0
    ref = _line_1d(n, p, S, float(np.float32(1.0 / 2.25)), pr, E0, T)
    c = [w // 2, w // 2, w // 2]
    got = []
    for _ in range(T):
        o.step_linear(st, 1)
        idx = [c[2], c[1], c[0]]
        idx[2 - axis] = slice(None)
        got.append(st[e][tuple(idx)].copy())
    got = np.array(got)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the pulse has entered the CPML and been damped there
    assert np.max(np.abs(ref[-1])) < 0.5 * np.max(np.abs(E0))
