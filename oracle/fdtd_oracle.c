/*
 * fdtd_oracle.c -- plain, slow, FP64 CPU reference of the reversible 3D FDTD
 * hot path of Mahlau et al., "A flexible framework for large-scale FDTD
 * simulations: open-source inverse design for 3D nanostructures"
 * (arXiv 2412.12360).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code, headers or tables with the GPU library; each side computes its own
 * CPML coefficients from the same explicit parameters.
 *
 * What it computes (paper section 2.1, eqs. 1-2; section 2.2):
 *   - the Yee leapfrog in normalised units (dx = c = eps0 = mu0 = 1, dt = S):
 *       H^{n+1/2} = H^{n-1/2} - S * C E^n
 *       E^{n+1}   = E^n + S * D * C^T H^{n+1/2}          (D = diag(1/eps_r))
 *     H is updated over the whole grid before any E cell (state (E^n, H^{n-1/2})).
 *   - a perfectly conducting box: tangential E on the index-0 planes is held at
 *     zero and never updated; any read at index n_a is outside the box and is 0.
 *   - convolutional PML (the CFS-CPML that section 2.1 cites) on all six faces,
 *     written in its plain recursive form for every (component, derivative axis)
 *     pair; psi arrays exist on the whole grid and stay exactly 0 where the
 *     profile is zero (b = 1, a = 0, kappa = 1).
 *   - additive sources on any field component, at one cell or on a whole
 *     z-normal plane: E sources after the E half step, H sources after the H
 *     half step (a total-field/scattered-field plane is one E and one H plane
 *     source, see oracle.py); a non-interpolated Poynting-flux detector on a
 *     z-normal plane and the objective J = S * sum_n w * P[n] (section 2.1,
 *     detectors without interpolation).
 *   - the interpolated flux of section 2.1: Ex, Ey, Hx, Hy each averaged onto
 *     the point (i+1/2, j+1/2, k) of the detector plane at time n+1/2 (E of
 *     steps n and n+1; H^{n+1/2} of layers k-1 and k), and its adjoint source;
 *     the co-located energy density 1/2 (eps_r |E|^2 + |H|^2) at the same point
 *     and time, and its adjoint source (detector outside the design box).
 *   - the interface record (section 2.2): every step, tangential H^{n+1/2} on
 *     the PML-side layer p-1 of the three low faces and tangential E^{n+1} on
 *     layer n_a-p of the three high faces, over the interior window.
 *   - the inverse step on the interior I = [p, n-p)^3 (section 2.2): E then H
 *     un-updated, the out-of-interior neighbours taken from the record.
 *   - the exact reverse-mode VJP of one step (section 2.2, "vector Jacobian
 *     product"), including the transposed CPML recursions, the detector
 *     adjoint source and dJ/dd accumulated over the design box.
 *   - gradients by stored history (checkpointed segments, recomputation with
 *     the forward step only) and by time reversal (inverse steps plus the
 *     interface record).
 *   - conducting cells in a box inside the interior: eps dE/dt = curl H - sigma E
 *     with E averaged over the two time levels, E^{n+1} = ca E^n + cb curl H,
 *     u = sigma S d / 2, ca = (1-u)/(1+u), cb = S d/(1+u).  The update divides
 *     by nothing but damps, so it is not inverted: section 2.2 bases the time
 *     reversal on lossless media, and, as for the PML, the record keeps what
 *     the inverse cannot rebuild -- E^n of every cell of the lossy box, per
 *     step, after the interface layers.  The VJP carries ca, cb and their
 *     derivatives in d.
 *
 * Layout: every 3D array is [nz][ny][nx], x fastest.  A state buffer holds 18
 * arrays of N doubles: slots 0..5 = Ex,Ey,Ez,Hx,Hy,Hz; slot 6+2c+s = psi of
 * component c along derivative axis (c%3+1+s)%3.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXSRC 4
#define OR_MAXDET 4
#define OR_NSLOT 18
/* grids smaller than this run their sweeps on one thread: thread start-up
 * would cost more than the sweep */
#define OR_PAR_MIN 65536

typedef struct {
    int nx, ny, nz;
    double S;                       /* Courant number c*dt/dx */
    int p;                          /* CPML cells per face; 0 = bare PEC box */
    double m, sigma_max, kappa_max, alpha_max;  /* CPML grading (per-step units) */
    const double *d;                /* N values of 1/eps_r */
    int nsrc;
    int src_kind[OR_MAXSRC];        /* 0 = point, 1 = full z-normal plane */
    int src_comp[OR_MAXSRC];        /* 0..5 = Ex,Ey,Ez,Hx,Hy,Hz */
    int src_i[OR_MAXSRC], src_j[OR_MAXSRC], src_k[OR_MAXSRC];
    const double *src_amp[OR_MAXSRC];   /* amplitude per step, length >= T */
    int ndet;
    int det_k[OR_MAXDET];
    int det_i0[OR_MAXDET], det_i1[OR_MAXDET], det_j0[OR_MAXDET], det_j1[OR_MAXDET];
    double det_w[OR_MAXDET];
    int det_interp[OR_MAXDET];      /* 1: co-located (interpolated) flux */
    int det_energy[OR_MAXDET];      /* 1: co-located energy density instead of flux */
    int dlo[3], dhi[3];             /* half-open design box */
    const double *sig;              /* N values of the conductivity sigma (NULL: lossless);
                                       zero outside the lossy box */
    int llo[3], lhi[3];             /* half-open lossy box inside the interior; E^n of
                                       its cells is part of the record of step n */
} or_problem;

/* ---------------------------------------------------------------- helpers */

static size_t ncell(const or_problem *P) { return (size_t)P->nx * P->ny * P->nz; }
static int dim(const or_problem *P, int a) { return a == 0 ? P->nx : a == 1 ? P->ny : P->nz; }
static size_t idx(const or_problem *P, int i, int j, int k)
{
    return ((size_t)k * P->ny + j) * P->nx + i;
}
static double *slot(double *st, const or_problem *P, int s) { return st + (size_t)s * ncell(P); }
static double *psi(double *st, const or_problem *P, int c, int s) { return slot(st, P, 6 + 2 * c + s); }

/* a field value; anything outside the box reads as zero */
static double at(const double *F, const or_problem *P, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= P->nx || j >= P->ny || k >= P->nz) return 0.0;
    return F[idx(P, i, j, k)];
}

static const int E_OFF[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

/* F(x + e_a) - F(x): the difference H-type updates take of E */
static double dfwd(const double *F, const or_problem *P, int a, int i, int j, int k)
{
    return at(F, P, i + E_OFF[a][0], j + E_OFF[a][1], k + E_OFF[a][2]) - at(F, P, i, j, k);
}
/* F(x) - F(x - e_a): the difference E-type updates take of H */
static double dbwd(const double *F, const or_problem *P, int a, int i, int j, int k)
{
    return at(F, P, i, j, k) - at(F, P, i - E_OFF[a][0], j - E_OFF[a][1], k - E_OFF[a][2]);
}

static int coord(int a, int i, int j, int k) { return a == 0 ? i : a == 1 ? j : k; }

/* tangential E held at zero on the index-0 planes of the conducting box */
static int e_held(int q, int i, int j, int k)
{
    int r = (q + 1) % 3, t = (q + 2) % 3;
    return coord(r, i, j, k) == 0 || coord(t, i, j, k) == 0;
}

/* ------------------------------------------------------------- CPML grading
 * Depth delta(u) = max(p-u, u-(n-p), 0)/p at a component's own staggered
 * coordinate u; sigma = sigma_max*delta^m, kappa = 1+(kappa_max-1)*delta^m,
 * alpha = alpha_max*(1-delta); b = exp(-(sigma/kappa+alpha)),
 * a = sigma/(sigma*kappa + kappa^2*alpha) * (b-1).                          */
typedef struct { double *b[3], *a[3], *kinv[3]; } or_prof;   /* per axis, per index */

static void grade(const or_problem *P, int n, double u, double *b, double *a, double *kinv)
{
    double delta = 0.0;
    if (P->p > 0) {
        double lo = P->p - u, hi = u - (n - P->p);
        delta = fmax(fmax(lo, hi), 0.0) / P->p;
    }
    if (delta <= 0.0) { *b = 1.0; *a = 0.0; *kinv = 1.0; return; }
    double dm = pow(delta, P->m);
    double sig = P->sigma_max * dm;
    double kap = 1.0 + (P->kappa_max - 1.0) * dm;
    double alp = P->alpha_max * (1.0 - delta);
    *b = exp(-(sig / kap + alp));
    *a = sig > 0.0 ? sig / (sig * kap + kap * kap * alp) * (*b - 1.0) : 0.0;
    *kinv = 1.0 / kap;
}

/* E-type pairs sit at integer coordinates along their derivative axis,
 * H-type pairs at half-integer ones. */
static void prof_make(const or_problem *P, or_prof *E, or_prof *H)
{
    for (int a = 0; a < 3; a++) {
        int n = dim(P, a);
        E->b[a] = malloc(sizeof(double) * n); E->a[a] = malloc(sizeof(double) * n);
        E->kinv[a] = malloc(sizeof(double) * n);
        H->b[a] = malloc(sizeof(double) * n); H->a[a] = malloc(sizeof(double) * n);
        H->kinv[a] = malloc(sizeof(double) * n);
        for (int i = 0; i < n; i++) {
            grade(P, n, (double)i, &E->b[a][i], &E->a[a][i], &E->kinv[a][i]);
            grade(P, n, i + 0.5, &H->b[a][i], &H->a[a][i], &H->kinv[a][i]);
        }
    }
}
static void prof_free(or_prof *X)
{
    for (int a = 0; a < 3; a++) { free(X->b[a]); free(X->a[a]); free(X->kinv[a]); }
}

/* exported for tests: the grading at one coordinate */
void or_grade(const or_problem *P, int axis, double u, double *out3)
{
    grade(P, dim(P, axis), u, &out3[0], &out3[1], &out3[2]);
}

/* --------------------------------------------------------------- forward */

static void h_sweep(const or_problem *P, double *st, const or_prof *PH)
{
    const double S = P->S;
    double *E[3] = {slot(st, P, 0), slot(st, P, 1), slot(st, P, 2)};
#pragma omp parallel for schedule(static) if (ncell(P) >= OR_PAR_MIN)
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = idx(P, i, j, k);
                for (int q = 0; q < 3; q++) {
                    int r = (q + 1) % 3, t = (q + 2) % 3;
                    int ir = coord(r, i, j, k), it = coord(t, i, j, k);
                    double dr = dfwd(E[t], P, r, i, j, k);   /* d_r E_t */
                    double dt = dfwd(E[r], P, t, i, j, k);   /* d_t E_r */
                    double *pr = psi(st, P, 3 + q, 0) + c, *pt = psi(st, P, 3 + q, 1) + c;
                    *pr = PH->b[r][ir] * *pr + PH->a[r][ir] * dr;
                    *pt = PH->b[t][it] * *pt + PH->a[t][it] * dt;
                    double Tr = dr * PH->kinv[r][ir] + *pr;
                    double Tt = dt * PH->kinv[t][it] + *pt;
                    slot(st, P, 3 + q)[c] -= S * (Tr - Tt);
                }
            }
}

static void e_sweep(const or_problem *P, double *st, const or_prof *PE)
{
    const double S = P->S;
    double *H[3] = {slot(st, P, 3), slot(st, P, 4), slot(st, P, 5)};
#pragma omp parallel for schedule(static) if (ncell(P) >= OR_PAR_MIN)
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = idx(P, i, j, k);
                for (int q = 0; q < 3; q++) {
                    if (e_held(q, i, j, k)) continue;
                    int r = (q + 1) % 3, t = (q + 2) % 3;
                    int ir = coord(r, i, j, k), it = coord(t, i, j, k);
                    double dr = dbwd(H[t], P, r, i, j, k);   /* d_r H_t */
                    double dt = dbwd(H[r], P, t, i, j, k);   /* d_t H_r */
                    double *pr = psi(st, P, q, 0) + c, *pt = psi(st, P, q, 1) + c;
                    *pr = PE->b[r][ir] * *pr + PE->a[r][ir] * dr;
                    *pt = PE->b[t][it] * *pt + PE->a[t][it] * dt;
                    double Tr = dr * PE->kinv[r][ir] + *pr;
                    double Tt = dt * PE->kinv[t][it] + *pt;
                    double sg = P->sig ? P->sig[c] : 0.0;
                    if (sg == 0.0) {
                        slot(st, P, q)[c] += S * P->d[c] * (Tr - Tt);
                    } else {
                        /* conducting cell: eps dE/dt = curl H - sigma E with E
                         * averaged over the two time levels */
                        double u = 0.5 * sg * S * P->d[c];
                        double *Eq = slot(st, P, q) + c;
                        *Eq = (1.0 - u) / (1.0 + u) * *Eq + S * P->d[c] / (1.0 + u) * (Tr - Tt);
                    }
                }
            }
}

/* sources on the E components (hfield = 0) or on the H components (hfield = 1);
 * held E cells take no source */
static void add_sources(const or_problem *P, double *st, int n, double sign, int hfield)
{
    for (int s = 0; s < P->nsrc; s++) {
        int q = P->src_comp[s];
        if ((q >= 3) != hfield) continue;
        double A = sign * P->src_amp[s][n];
        double *F = slot(st, P, q);
        if (P->src_kind[s] == 0) {
            int i = P->src_i[s], j = P->src_j[s], k = P->src_k[s];
            if (q >= 3 || !e_held(q, i, j, k)) F[idx(P, i, j, k)] += A;
        } else {
            int k = P->src_k[s];
            for (int j = 0; j < P->ny; j++)
                for (int i = 0; i < P->nx; i++)
                    if (q >= 3 || !e_held(q, i, j, k)) F[idx(P, i, j, k)] += A;
        }
    }
}

/* inverse-step variant: subtract only on interior cells */
static void sub_sources_interior(const or_problem *P, double *st, int n, int hfield)
{
    int p = P->p;
    for (int s = 0; s < P->nsrc; s++) {
        int q = P->src_comp[s];
        if ((q >= 3) != hfield) continue;
        double A = P->src_amp[s][n];
        double *F = slot(st, P, q);
        for (int k = p; k < P->nz - p; k++)
            for (int j = p; j < P->ny - p; j++)
                for (int i = p; i < P->nx - p; i++) {
                    int hit = P->src_kind[s] == 0
                                  ? (i == P->src_i[s] && j == P->src_j[s] && k == P->src_k[s])
                                  : (k == P->src_k[s]);
                    if (hit && (q >= 3 || !e_held(q, i, j, k))) F[idx(P, i, j, k)] -= A;
                }
    }
}

static double det_flux(const or_problem *P, const double *st, int m)
{
    const double *Ex = st, *Ey = st + ncell(P);
    const double *Hx = st + 3 * ncell(P), *Hy = st + 4 * ncell(P);
    double s = 0.0;
    int k = P->det_k[m];
    for (int j = P->det_j0[m]; j < P->det_j1[m]; j++)
        for (int i = P->det_i0[m]; i < P->det_i1[m]; i++) {
            size_t c = idx(P, i, j, k);
            s += Ex[c] * Hy[c] - Ey[c] * Hx[c];
        }
    return s;
}

/* Interpolated flux of detector m (section 2.1: composite metrics need the
 * components at one point in space and time).  Target point (i+1/2, j+1/2, k)
 * at time n+1/2.  Ex(i+1/2, j, k) is averaged over j, j+1 and over the steps
 * n, n+1; Ey(i, j+1/2, k) over i, i+1 and the two steps; Hx(i, j+1/2, k+-1/2)
 * over i, i+1 and the layers k-1, k; Hy(i+1/2, j, k+-1/2) over j, j+1 and the
 * two layers; H^{n+1/2} is already at time n+1/2.  eprev holds Ex^n then Ey^n
 * of plane k, [ny][nx] each; st holds E^{n+1}, H^{n+1/2}. */
static double det_flux_interp(const or_problem *P, const double *st, const double *eprev, int m)
{
    size_t N = ncell(P), A = (size_t)P->nx * P->ny;
    const double *Ex = st, *Ey = st + N, *Hx = st + 3 * N, *Hy = st + 4 * N;
    const double *Px = eprev, *Py = eprev + A;
    int k = P->det_k[m];
    double s = 0.0;
    for (int j = P->det_j0[m]; j < P->det_j1[m]; j++)
        for (int i = P->det_i0[m]; i < P->det_i1[m]; i++) {
            size_t p00 = (size_t)j * P->nx + i, p01 = p00 + P->nx, p10 = p00 + 1;
            double ex = 0.25 * (Px[p00] + Px[p01] + Ex[idx(P, i, j, k)] + Ex[idx(P, i, j + 1, k)]);
            double ey = 0.25 * (Py[p00] + Py[p10] + Ey[idx(P, i, j, k)] + Ey[idx(P, i + 1, j, k)]);
            double hx = 0.25 * (Hx[idx(P, i, j, k - 1)] + Hx[idx(P, i + 1, j, k - 1)] +
                                Hx[idx(P, i, j, k)] + Hx[idx(P, i + 1, j, k)]);
            double hy = 0.25 * (Hy[idx(P, i, j, k - 1)] + Hy[idx(P, i, j + 1, k - 1)] +
                                Hy[idx(P, i, j, k)] + Hy[idx(P, i, j + 1, k)]);
            s += ex * hy - ey * hx;
        }
    return s;
}

/* Co-located energy of detector m: 1/2 (eps_r |E|^2 + |H|^2) at the point
 * (i+1/2, j+1/2, k) and time n+1/2, summed over the window, eps_r of cell
 * (i,j,k).  Ex, Ey, Hx, Hy as for the interpolated flux; Ez(i, j, k+-1/2) is
 * averaged over i, i+1, j, j+1, the layers k-1, k and the steps n, n+1;
 * Hz(i+1/2, j+1/2, k) is already at the point.  eprev holds Ex^n, Ey^n, Ez^n
 * of plane k and Ez^n of layer k-1, [ny][nx] each. */
static double det_energy_interp(const or_problem *P, const double *st, const double *eprev, int m)
{
    size_t N = ncell(P), A = (size_t)P->nx * P->ny;
    const double *Ex = st, *Ey = st + N, *Ez = st + 2 * N, *Hx = st + 3 * N, *Hy = st + 4 * N, *Hz = st + 5 * N;
    const double *Px = eprev, *Py = eprev + A, *Pz = eprev + 2 * A, *Pzm = eprev + 3 * A;
    int k = P->det_k[m];
    double s = 0.0;
    for (int j = P->det_j0[m]; j < P->det_j1[m]; j++)
        for (int i = P->det_i0[m]; i < P->det_i1[m]; i++) {
            size_t p00 = (size_t)j * P->nx + i, p01 = p00 + P->nx, p10 = p00 + 1, p11 = p01 + 1;
            double ex = 0.25 * (Px[p00] + Px[p01] + Ex[idx(P, i, j, k)] + Ex[idx(P, i, j + 1, k)]);
            double ey = 0.25 * (Py[p00] + Py[p10] + Ey[idx(P, i, j, k)] + Ey[idx(P, i + 1, j, k)]);
            double ez = 0.0;
            for (int kk = k - 1; kk <= k; kk++)
                ez += Ez[idx(P, i, j, kk)] + Ez[idx(P, i + 1, j, kk)] + Ez[idx(P, i, j + 1, kk)] +
                      Ez[idx(P, i + 1, j + 1, kk)];
            const double *Q = Pz, *Qm = Pzm;
            ez += Q[p00] + Q[p10] + Q[p01] + Q[p11] + Qm[p00] + Qm[p10] + Qm[p01] + Qm[p11];
            ez /= 16.0;
            double hx = 0.25 * (Hx[idx(P, i, j, k - 1)] + Hx[idx(P, i + 1, j, k - 1)] +
                                Hx[idx(P, i, j, k)] + Hx[idx(P, i + 1, j, k)]);
            double hy = 0.25 * (Hy[idx(P, i, j, k - 1)] + Hy[idx(P, i, j + 1, k - 1)] +
                                Hy[idx(P, i, j, k)] + Hy[idx(P, i, j + 1, k)]);
            double hz = Hz[idx(P, i, j, k)];
            double eps = 1.0 / P->d[idx(P, i, j, k)];
            s += 0.5 * (eps * (ex * ex + ey * ey + ez * ez) + hx * hx + hy * hy + hz * hz);
        }
    return s;
}

/* ------------------------------------------------------- interface record
 * Face f = 2a + side.  side 0 (low): tangential H at layer p-1; side 1 (high):
 * tangential E at layer n_a - p.  Components (a+1)%3 then (a+2)%3.  Window over
 * the two other axes u < v, each restricted to [p, n-p), stored [comp][v][u]. */
static void face_axes(int a, int *u, int *v) { *u = a == 0 ? 1 : 0; *v = a == 2 ? 1 : 2; }

static size_t iface_floats(const or_problem *P)
{
    size_t tot = 0;
    if (P->p == 0) return 0;
    for (int a = 0; a < 3; a++) {
        int u, v; face_axes(a, &u, &v);
        tot += 2 * 2 * (size_t)(dim(P, u) - 2 * P->p) * (dim(P, v) - 2 * P->p);
    }
    return tot;
}

/* cells of the lossy box (0 without conductivity) */
static size_t lossy_cells(const or_problem *P)
{
    if (!P->sig) return 0;
    size_t c = 1;
    for (int a = 0; a < 3; a++) c *= (size_t)(P->lhi[a] > P->llo[a] ? P->lhi[a] - P->llo[a] : 0);
    return c;
}

/* the record of one step: the interface layers, then E^n of the lossy box */
size_t or_record_floats(const or_problem *P)
{
    return iface_floats(P) + 3 * lossy_cells(P);
}

/* position of component q of cell (i,j,k) in a lossy-box array */
static size_t lossy_index(const or_problem *P, int q, int i, int j, int k)
{
    size_t lx = P->lhi[0] - P->llo[0], ly = P->lhi[1] - P->llo[1], lz = P->lhi[2] - P->llo[2];
    return (((size_t)q * lz + (k - P->llo[2])) * ly + (j - P->llo[1])) * lx + (i - P->llo[0]);
}

/* E of the lossy box, [comp][z][y][x] over the box: dir = 0 state -> buf,
 * dir = 1 buf -> state */
static void lossy_io(const or_problem *P, double *st, double *buf, int dir)
{
    size_t r = 0;
    for (int q = 0; q < 3; q++) {
        double *F = slot(st, P, q);
        for (int k = P->llo[2]; k < P->lhi[2]; k++)
            for (int j = P->llo[1]; j < P->lhi[1]; j++)
                for (int i = P->llo[0]; i < P->lhi[0]; i++, r++) {
                    size_t c = idx(P, i, j, k);
                    if (dir == 0) buf[r] = F[c]; else F[c] = buf[r];
                }
    }
}

/* dir = 0: state -> record; dir = 1: record -> state.  which = 0 low (H) faces, 1 high (E) faces */
static void record_io(const or_problem *P, double *st, double *rec, int which, int dir)
{
    int p = P->p;
    size_t off = 0;
    for (int a = 0; a < 3; a++) {
        int u, v; face_axes(a, &u, &v);
        int Lu = dim(P, u) - 2 * p, Lv = dim(P, v) - 2 * p;
        for (int side = 0; side < 2; side++) {
            int layer = side == 0 ? p - 1 : dim(P, a) - p;
            for (int cc = 0; cc < 2; cc++) {
                int comp = (side == 0 ? 3 : 0) + (a + 1 + cc) % 3;
                double *F = slot(st, P, comp);
                for (int iv = 0; iv < Lv; iv++)
                    for (int iu = 0; iu < Lu; iu++) {
                        int x[3];
                        x[a] = layer; x[u] = p + iu; x[v] = p + iv;
                        size_t c = idx(P, x[0], x[1], x[2]);
                        size_t r = off + (size_t)iv * Lu + iu;
                        if (side == which) {
                            if (dir == 0) rec[r] = F[c]; else F[c] = rec[r];
                        }
                    }
                off += (size_t)Lu * Lv;
            }
        }
    }
}

/* one forward step n: psi_H, H, H sources, psi_E, E, E sources, detectors, record */
/* trow (ndet values, may be NULL) receives this step's fluxes; rec (may be
 * NULL) this step's record. */
static void step_fwd(const or_problem *P, double *st, int n, const or_prof *PE, const or_prof *PH,
                     double *trow, double *rec, int with_src)
{
    /* E^n of the interpolated detectors' planes, before the step */
    double *eprev = NULL;
    size_t A = (size_t)P->nx * P->ny;
    if (trow)
        for (int m = 0; m < P->ndet; m++)
            if (P->det_interp[m]) {
                if (!eprev) eprev = malloc(sizeof(double) * 4 * A * OR_MAXDET);
                /* Ex, Ey, Ez of plane k and Ez of layer k-1 */
                for (int q = 0; q < 3; q++)
                    memcpy(eprev + (4 * (size_t)m + q) * A, slot(st, P, q) + (size_t)P->det_k[m] * A,
                           sizeof(double) * A);
                memcpy(eprev + (4 * (size_t)m + 3) * A, slot(st, P, 2) + (size_t)(P->det_k[m] - 1) * A,
                       sizeof(double) * A);
            }
    if (rec && lossy_cells(P)) lossy_io(P, st, rec + iface_floats(P), 0);
    h_sweep(P, st, PH);
    if (with_src) add_sources(P, st, n, 1.0, 1);
    if (rec && P->p > 0) record_io(P, st, rec, 0, 0);
    e_sweep(P, st, PE);
    if (with_src) add_sources(P, st, n, 1.0, 0);
    if (rec && P->p > 0) record_io(P, st, rec, 1, 0);
    if (trow)
        for (int m = 0; m < P->ndet; m++)
            trow[m] = !P->det_interp[m] ? det_flux(P, st, m)
                      : P->det_energy[m] ? det_energy_interp(P, st, eprev + 4 * (size_t)m * A, m)
                                         : det_flux_interp(P, st, eprev + 4 * (size_t)m * A, m);
    free(eprev);
}

/* Advance st by T steps starting at step n0.  trace: [T][ndet] or NULL.
 * rec: [T][or_record_floats] or NULL.  Returns J = S * sum w * P over the run. */
/* Adjoint of the interpolated flux.  The gradient passes keep, per step n and
 * interpolated detector m, the planes the co-located flux of step n reads:
 * E^{n+1} x, y of plane k, H^{n+1/2} x, y of layer k-1, H^{n+1/2} x, y of
 * layer k (six [ny][nx] planes), and E^0 x, y of plane k. */
#define OR_DSTORE 9   /* planes per step and detector */
#define OR_DE0 4      /* E planes of step 0 per detector */

static size_t dstore_floats(const or_problem *P, int T)
{
    return (size_t)T * P->ndet * OR_DSTORE * (size_t)P->nx * P->ny;
}

static int any_interp(const or_problem *P)
{
    for (int m = 0; m < P->ndet; m++)
        if (P->det_interp[m]) return 1;
    return 0;
}

/* planes 0..8: Ex, Ey (plane k), Hx, Hy (layer k-1), Hx, Hy (layer k), Ez,
 * Hz (plane k), Ez (layer k-1); with e_only the E planes Ex, Ey, Ez (k), Ez
 * (k-1) */
static void dstore_planes(const or_problem *P, const double *st, double *dst, int m, int e_only)
{
    size_t A = (size_t)P->nx * P->ny;
    int k = P->det_k[m];
    const int comp[OR_DSTORE] = {0, 1, 3, 4, 3, 4, 2, 5, 2};
    const int layer[OR_DSTORE] = {k, k, k - 1, k - 1, k, k, k, k, k - 1};
    const int eq[OR_DE0] = {0, 1, 6, 8};
    for (int q = 0; q < (e_only ? OR_DE0 : OR_DSTORE); q++) {
        int qq = e_only ? eq[q] : q;
        memcpy(dst + q * A, slot((double *)st, P, comp[qq]) + (size_t)layer[qq] * A, sizeof(double) * A);
    }
}

/* Energy detector m, J = S sum_n w U[n] with U the co-located energy sum:
 * dU/d(node) = eps_r * (co-located E) or (co-located H) times the node's
 * averaging weight, for every cell the node enters (eps_r of the cell; the
 * detector lies outside the design box, so U has no explicit eps_r term in
 * the gradient).  E^{n+1} enters U[n] and U[n+1], H^{n+1/2} U[n]. */
static void det_energy_adjoint(const or_problem *P, double *adj, const double *store, const double *e0, int n,
                               int T, int m, double sw)
{
    size_t N = ncell(P), A = (size_t)P->nx * P->ny;
    int k = P->det_k[m];
    const double *R = store + ((size_t)n * P->ndet + m) * OR_DSTORE * A;
    const double *Ep = n == 0 ? e0 + (size_t)m * OR_DE0 * A : store + ((size_t)(n - 1) * P->ndet + m) * OR_DSTORE * A;
    const double *Epz = n == 0 ? Ep + 2 * A : Ep + 6 * A, *Epzm = n == 0 ? Ep + 3 * A : Ep + 8 * A;
    const double *R1 = n + 1 < T ? store + ((size_t)(n + 1) * P->ndet + m) * OR_DSTORE * A : NULL;
    double *aE[3] = {adj, adj + N, adj + 2 * N}, *aH[3] = {adj + 3 * N, adj + 4 * N, adj + 5 * N};
    for (int j = P->det_j0[m]; j < P->det_j1[m]; j++)
        for (int i = P->det_i0[m]; i < P->det_i1[m]; i++) {
            size_t p00 = (size_t)j * P->nx + i, p01 = p00 + P->nx, p10 = p00 + 1, p11 = p01 + 1;
            const size_t q4[4] = {p00, p10, p01, p11};
            double eps = 1.0 / P->d[idx(P, i, j, k)];
            double ex = 0.25 * (Ep[p00] + Ep[p01] + R[p00] + R[p01]);
            double ey = 0.25 * (Ep[A + p00] + Ep[A + p10] + R[A + p00] + R[A + p10]);
            double ez = 0.0;
            for (int c = 0; c < 4; c++) ez += Epz[q4[c]] + Epzm[q4[c]] + R[6 * A + q4[c]] + R[8 * A + q4[c]];
            ez /= 16.0;
            double hx = 0.25 * (R[2 * A + p00] + R[2 * A + p10] + R[4 * A + p00] + R[4 * A + p10]);
            double hy = 0.25 * (R[3 * A + p00] + R[3 * A + p01] + R[5 * A + p00] + R[5 * A + p01]);
            double hz = R[7 * A + p00];
            double ex1 = 0.0, ey1 = 0.0, ez1 = 0.0;
            if (R1) {
                ex1 = 0.25 * (R[p00] + R[p01] + R1[p00] + R1[p01]);
                ey1 = 0.25 * (R[A + p00] + R[A + p10] + R1[A + p00] + R1[A + p10]);
                for (int c = 0; c < 4; c++)
                    ez1 += R[6 * A + q4[c]] + R[8 * A + q4[c]] + R1[6 * A + q4[c]] + R1[8 * A + q4[c]];
                ez1 /= 16.0;
            }
            double gx = 0.25 * sw * eps * (ex + ex1), gy = 0.25 * sw * eps * (ey + ey1);
            double gz = sw * eps * (ez + ez1) / 16.0;
            aE[0][idx(P, i, j, k)] += gx;
            aE[0][idx(P, i, j + 1, k)] += gx;
            aE[1][idx(P, i, j, k)] += gy;
            aE[1][idx(P, i + 1, j, k)] += gy;
            for (int kk = k - 1; kk <= k; kk++) {
                aE[2][idx(P, i, j, kk)] += gz;
                aE[2][idx(P, i + 1, j, kk)] += gz;
                aE[2][idx(P, i, j + 1, kk)] += gz;
                aE[2][idx(P, i + 1, j + 1, kk)] += gz;
                aH[0][idx(P, i, j, kk)] += 0.25 * sw * hx;
                aH[0][idx(P, i + 1, j, kk)] += 0.25 * sw * hx;
                aH[1][idx(P, i, j, kk)] += 0.25 * sw * hy;
                aH[1][idx(P, i, j + 1, kk)] += 0.25 * sw * hy;
            }
            aH[2][idx(P, i, j, k)] += sw * hz;
        }
}

/* Before reverse step n: add dJ/dE^{n+1} and dJ/dH^{n+1/2} of the interpolated
 * detectors, J = S sum_n w P[n] with P[n] the co-located sum.  E^{n+1} enters
 * P[n] (as the later of its two steps) and P[n+1] (as the earlier); H^{n+1/2}
 * enters P[n] only.  Each co-located value is a quarter of four nodes, so each
 * node receives a quarter of the partner value of every cell it enters. */
static void det_interp_adjoint(const or_problem *P, double *adj, const double *store, const double *e0, int n,
                               int T)
{
    size_t N = ncell(P), A = (size_t)P->nx * P->ny;
    for (int m = 0; m < P->ndet; m++) {
        if (!P->det_interp[m]) continue;
        double sw = P->S * P->det_w[m];
        if (sw == 0.0) continue;
        if (P->det_energy[m]) {
            det_energy_adjoint(P, adj, store, e0, n, T, m, sw);
            continue;
        }
        int k = P->det_k[m];
        const double *R = store + ((size_t)n * P->ndet + m) * OR_DSTORE * A;
        const double *Ep = n == 0 ? e0 + (size_t)m * OR_DE0 * A : store + ((size_t)(n - 1) * P->ndet + m) * OR_DSTORE * A;
        const double *R1 = n + 1 < T ? store + ((size_t)(n + 1) * P->ndet + m) * OR_DSTORE * A : NULL;
        for (int j = P->det_j0[m]; j < P->det_j1[m]; j++)
            for (int i = P->det_i0[m]; i < P->det_i1[m]; i++) {
                size_t p00 = (size_t)j * P->nx + i, p01 = p00 + P->nx, p10 = p00 + 1;
                double exc = 0.25 * (Ep[p00] + Ep[p01] + R[p00] + R[p01]);
                double eyc = 0.25 * (Ep[A + p00] + Ep[A + p10] + R[A + p00] + R[A + p10]);
                double hxc = 0.25 * (R[2 * A + p00] + R[2 * A + p10] + R[4 * A + p00] + R[4 * A + p10]);
                double hyc = 0.25 * (R[3 * A + p00] + R[3 * A + p01] + R[5 * A + p00] + R[5 * A + p01]);
                double hxc1 = 0.0, hyc1 = 0.0;
                if (R1) {
                    hxc1 = 0.25 * (R1[2 * A + p00] + R1[2 * A + p10] + R1[4 * A + p00] + R1[4 * A + p10]);
                    hyc1 = 0.25 * (R1[3 * A + p00] + R1[3 * A + p01] + R1[5 * A + p00] + R1[5 * A + p01]);
                }
                double *aEx = adj, *aEy = adj + N, *aHx = adj + 3 * N, *aHy = adj + 4 * N;
                double gx = 0.25 * sw * (hyc + hyc1), gy = -0.25 * sw * (hxc + hxc1);
                aEx[idx(P, i, j, k)] += gx;
                aEx[idx(P, i, j + 1, k)] += gx;
                aEy[idx(P, i, j, k)] += gy;
                aEy[idx(P, i + 1, j, k)] += gy;
                double ghy = 0.25 * sw * exc, ghx = -0.25 * sw * eyc;
                for (int kk = k - 1; kk <= k; kk++) {
                    aHy[idx(P, i, j, kk)] += ghy;
                    aHy[idx(P, i, j + 1, kk)] += ghy;
                    aHx[idx(P, i, j, kk)] += ghx;
                    aHx[idx(P, i + 1, j, kk)] += ghx;
                }
            }
    }
}

/* forward loop shared by or_forward and the gradients; store/e0 (may be NULL)
 * receive the interpolated detectors' planes */
static double forward_run(const or_problem *P, double *st, int n0, int T, double *trace, double *rec,
                          double *store, double *e0)
{
    or_prof PE, PH;
    prof_make(P, &PE, &PH);
    size_t rf = rec ? or_record_floats(P) : 0, A = (size_t)P->nx * P->ny;
    double J = 0.0;
    double *tr = trace ? trace : malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * (P->ndet > 0 ? P->ndet : 1));
    if (e0)
        for (int m = 0; m < P->ndet; m++)
            if (P->det_interp[m]) dstore_planes(P, st, e0 + (size_t)m * OR_DE0 * A, m, 1);
    for (int n = 0; n < T; n++) {
        step_fwd(P, st, n0 + n, &PE, &PH, tr + (size_t)n * P->ndet, rec ? rec + (size_t)n * rf : NULL, 1);
        for (int m = 0; m < P->ndet; m++) J += P->S * P->det_w[m] * tr[(size_t)n * P->ndet + m];
        if (store)
            for (int m = 0; m < P->ndet; m++)
                if (P->det_interp[m]) dstore_planes(P, st, store + ((size_t)n * P->ndet + m) * OR_DSTORE * A, m, 0);
    }
    if (!trace) free(tr);
    prof_free(&PE); prof_free(&PH);
    return J;
}

double or_forward(const or_problem *P, double *st, int n0, int T, double *trace, double *rec)
{
    return forward_run(P, st, n0, T, trace, rec, NULL, NULL);
}

/* the linear step map M (no source, no detector), T times */
void or_step_linear(const or_problem *P, double *st, int T)
{
    or_prof PE, PH;
    prof_make(P, &PE, &PH);
    for (int n = 0; n < T; n++) step_fwd(P, st, 0, &PE, &PH, NULL, NULL, 0);
    prof_free(&PE); prof_free(&PH);
}

/* ----------------------------------------------------------- inverse step
 * Undo step n on the interior I = [p, n-p)^3 (the whole box when p == 0):
 * E^n = E^{n+1} - srcE_n - S*D*C^T H^{n+1/2}, then
 * H^{n-1/2} = H^{n+1/2} - srcH_n + S*C E^n.
 * Before each half the out-of-interior neighbours are written from the record:
 * H^{n+1/2} on the low faces from rec_n, E^n on the high faces from rec_{n-1}
 * (E^0 = 0).  PML cells are not reconstructed. */
static void inverse_step(const or_problem *P, double *st, int n, const double *rec)
{
    const double S = P->S;
    int p = P->p;
    size_t rf = or_record_floats(P);
    if (p > 0) record_io(P, st, (double *)(rec + (size_t)n * rf), 0, 1);
    sub_sources_interior(P, st, n, 0);
    double *H[3] = {slot(st, P, 3), slot(st, P, 4), slot(st, P, 5)};
    double *E[3] = {slot(st, P, 0), slot(st, P, 1), slot(st, P, 2)};
#pragma omp parallel for schedule(static) if (ncell(P) >= OR_PAR_MIN)
    for (int k = p; k < P->nz - p; k++)
        for (int j = p; j < P->ny - p; j++)
            for (int i = p; i < P->nx - p; i++) {
                size_t c = idx(P, i, j, k);
                for (int q = 0; q < 3; q++) {
                    if (e_held(q, i, j, k)) continue;
                    int r = (q + 1) % 3, t = (q + 2) % 3;
                    double curl = dbwd(H[t], P, r, i, j, k) - dbwd(H[r], P, t, i, j, k);
                    E[q][c] -= S * P->d[c] * curl;
                }
            }
    if (p > 0) {
        if (n > 0) {
            record_io(P, st, (double *)(rec + (size_t)(n - 1) * rf), 1, 1);
        } else {
            double *zero = calloc(rf, sizeof(double));
            record_io(P, st, zero, 1, 1);
            free(zero);
        }
    }
    /* conducting cells are not inverted (their update divides by a factor
     * below one): E^n of the lossy box comes from the record of step n */
    if (lossy_cells(P)) lossy_io(P, st, (double *)(rec + (size_t)n * rf + iface_floats(P)), 1);
    sub_sources_interior(P, st, n, 1);
#pragma omp parallel for schedule(static) if (ncell(P) >= OR_PAR_MIN)
    for (int k = p; k < P->nz - p; k++)
        for (int j = p; j < P->ny - p; j++)
            for (int i = p; i < P->nx - p; i++) {
                size_t c = idx(P, i, j, k);
                for (int q = 0; q < 3; q++) {
                    int r = (q + 1) % 3, t = (q + 2) % 3;
                    double curl = dfwd(E[t], P, r, i, j, k) - dfwd(E[r], P, t, i, j, k);
                    H[q][c] += S * curl;
                }
            }
}

/* Undo steps n0+T-1 ... n0 (st holds s_{n0+T} on entry, s_{n0} on I on exit). */
void or_inverse(const or_problem *P, double *st, int n0, int T, const double *rec)
{
    for (int n = n0 + T - 1; n >= n0; n--) inverse_step(P, st, n, rec);
}

/* ------------------------------------------------------------ adjoint step
 * Reverse of forward step n.  adj holds the adjoint of s_{n+1} on entry and of
 * s_n on exit (same slot layout, psi-bar in the psi slots).  fwd holds s_{n+1}
 * (E^{n+1}, H^{n+1/2}, psi^{n+1}); it is read only at the detector planes and in
 * the design box.  g (N values, may be NULL) accumulates dJ/dd.  With
 * with_det = 0 and g == NULL this is exactly the transpose of the linear map. */
static void adjoint_step(const or_problem *P, double *adj, const double *fwd, double *g,
                         int with_det, const or_prof *PE, const or_prof *PH, double *tmp,
                         const double *lE)
{
    const double S = P->S;
    size_t N = ncell(P);
    /* detector adjoint source: dJ/dE^{n+1}, dJ/dH^{n+1/2} */
    if (with_det) {
        const double *Ex = fwd, *Ey = fwd + N, *Hx = fwd + 3 * N, *Hy = fwd + 4 * N;
        double *aEx = adj, *aEy = adj + N, *aHx = adj + 3 * N, *aHy = adj + 4 * N;
        for (int m = 0; m < P->ndet; m++) {
            if (P->det_interp[m]) continue;   /* its adjoint source: det_interp_adjoint */
            double sw = S * P->det_w[m];
            int k = P->det_k[m];
            for (int j = P->det_j0[m]; j < P->det_j1[m]; j++)
                for (int i = P->det_i0[m]; i < P->det_i1[m]; i++) {
                    size_t c = idx(P, i, j, k);
                    aEx[c] += sw * Hy[c];
                    aEy[c] -= sw * Hx[c];
                    aHy[c] += sw * Ex[c];
                    aHx[c] -= sw * Ey[c];
                }
        }
    }
    /* dJ/dd: E^{n+1} = E^n + S*d*(curl_kappa^T H + psi_E); in a conducting
     * cell E^{n+1} = ca(d) E^n + cb(d) (curl H) with u = sigma*S*d/2,
     * ca = (1-u)/(1+u), cb = S*d/(1+u), so dca/dd = -sigma*S/(1+u)^2 and
     * dcb/dd = S/(1+u)^2 (E^n of the lossy box in lE) */
    if (g) {
        const double *fH[3] = {fwd + 3 * N, fwd + 4 * N, fwd + 5 * N};
        for (int k = P->dlo[2]; k < P->dhi[2]; k++)
            for (int j = P->dlo[1]; j < P->dhi[1]; j++)
                for (int i = P->dlo[0]; i < P->dhi[0]; i++) {
                    size_t c = idx(P, i, j, k);
                    for (int q = 0; q < 3; q++) {
                        if (e_held(q, i, j, k)) continue;
                        int r = (q + 1) % 3, t = (q + 2) % 3;
                        int ir = coord(r, i, j, k), it = coord(t, i, j, k);
                        double Tr = dbwd(fH[t], P, r, i, j, k) * PE->kinv[r][ir] + fwd[(size_t)(6 + 2 * q) * N + c];
                        double Tt = dbwd(fH[r], P, t, i, j, k) * PE->kinv[t][it] + fwd[(size_t)(7 + 2 * q) * N + c];
                        double sg = P->sig ? P->sig[c] : 0.0;
                        if (sg == 0.0) {
                            g[c] += S * adj[(size_t)q * N + c] * (Tr - Tt);
                        } else {
                            double u = 0.5 * sg * S * P->d[c];
                            double En = lE[lossy_index(P, q, i, j, k)];
                            g[c] += S / ((1.0 + u) * (1.0 + u)) * adj[(size_t)q * N + c] * ((Tr - Tt) - sg * En);
                        }
                    }
                }
    }
    /* reverse of the E half: per E pair (q, s) along axis ax with sign +/-S*d,
     * psibar_tot = psibar + w; Q = w*kinv + a*psibar_tot multiplies
     * H(x) - H(x - e_ax); psibar <- b*psibar_tot.  tmp[6][N] holds Q. */
#pragma omp parallel for schedule(static) if (ncell(P) >= OR_PAR_MIN)
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = idx(P, i, j, k);
                double sg = P->sig ? P->sig[c] : 0.0;
                double u = 0.5 * sg * S * P->d[c];
                for (int q = 0; q < 3; q++) {
                    for (int s = 0; s < 2; s++) {
                        int ax = (q + 1 + s) % 3, ia = coord(ax, i, j, k);
                        double *pb = adj + (size_t)(6 + 2 * q + s) * N + c;
                        double Q = 0.0;
                        if (!e_held(q, i, j, k)) {
                            double cb = sg == 0.0 ? S * P->d[c] : S * P->d[c] / (1.0 + u);
                            double w = (s == 0 ? 1.0 : -1.0) * cb * adj[(size_t)q * N + c];
                            double tot = *pb + w;
                            Q = w * PE->kinv[ax][ia] + PE->a[ax][ia] * tot;
                            *pb = PE->b[ax][ia] * tot;
                        }
                        tmp[(size_t)(2 * q + s) * N + c] = Q;
                    }
                    /* a conducting cell passes ca Ebar' on to E^n */
                    if (sg != 0.0 && !e_held(q, i, j, k)) adj[(size_t)q * N + c] *= (1.0 - u) / (1.0 + u);
                }
            }
    /* H_F is differenced by pair (q = F+1, s = 0, axis F+2) and (q = F+2, s = 1, axis F+1) */
#pragma omp parallel for schedule(static) if (ncell(P) >= OR_PAR_MIN)
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = idx(P, i, j, k);
                for (int F = 0; F < 3; F++) {
                    int q0 = (F + 1) % 3, a0 = (F + 2) % 3;
                    int q1 = (F + 2) % 3, a1 = (F + 1) % 3;
                    const double *Q0 = tmp + (size_t)(2 * q0 + 0) * N;
                    const double *Q1 = tmp + (size_t)(2 * q1 + 1) * N;
                    double v = (at(Q0, P, i, j, k) - at(Q0, P, i + E_OFF[a0][0], j + E_OFF[a0][1], k + E_OFF[a0][2]))
                             + (at(Q1, P, i, j, k) - at(Q1, P, i + E_OFF[a1][0], j + E_OFF[a1][1], k + E_OFF[a1][2]));
                    adj[(size_t)(3 + F) * N + c] += v;
                }
            }
    /* reverse of the H half: H_q -= S*(T_r - T_t), so pair s = 0 has weight -S,
     * s = 1 weight +S; R multiplies E(x + e_ax) - E(x). */
#pragma omp parallel for schedule(static) if (ncell(P) >= OR_PAR_MIN)
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = idx(P, i, j, k);
                for (int q = 0; q < 3; q++)
                    for (int s = 0; s < 2; s++) {
                        int ax = (q + 1 + s) % 3, ia = coord(ax, i, j, k);
                        double *pb = adj + (size_t)(6 + 2 * (3 + q) + s) * N + c;
                        double w = (s == 0 ? -1.0 : 1.0) * S * adj[(size_t)(3 + q) * N + c];
                        double tot = *pb + w;
                        tmp[(size_t)(2 * q + s) * N + c] = w * PH->kinv[ax][ia] + PH->a[ax][ia] * tot;
                        *pb = PH->b[ax][ia] * tot;
                    }
            }
    /* E_F is differenced by pair (q = F+1, s = 0, axis F+2) and (q = F+2, s = 1, axis F+1) */
#pragma omp parallel for schedule(static) if (ncell(P) >= OR_PAR_MIN)
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = idx(P, i, j, k);
                for (int F = 0; F < 3; F++) {
                    if (e_held(F, i, j, k)) continue;
                    int q0 = (F + 1) % 3, a0 = (F + 2) % 3;
                    int q1 = (F + 2) % 3, a1 = (F + 1) % 3;
                    const double *R0 = tmp + (size_t)(2 * q0 + 0) * N;
                    const double *R1 = tmp + (size_t)(2 * q1 + 1) * N;
                    double v = (at(R0, P, i - E_OFF[a0][0], j - E_OFF[a0][1], k - E_OFF[a0][2]) - at(R0, P, i, j, k))
                             + (at(R1, P, i - E_OFF[a1][0], j - E_OFF[a1][1], k - E_OFF[a1][2]) - at(R1, P, i, j, k));
                    adj[(size_t)F * N + c] += v;
                }
            }
}

/* the transpose of or_step_linear, T times */
void or_adjoint_linear(const or_problem *P, double *adj, int T)
{
    or_prof PE, PH;
    prof_make(P, &PE, &PH);
    double *tmp = malloc(sizeof(double) * 6 * ncell(P));
    for (int n = 0; n < T; n++) adjoint_step(P, adj, NULL, NULL, 0, &PE, &PH, tmp, NULL);
    free(tmp);
    prof_free(&PE); prof_free(&PH);
}

/* --------------------------------------------------------------- gradients */

/* Stored-history gradient: forward from zero, checkpoint every `seg` steps,
 * then walk back segment by segment, recomputing each segment's states with
 * the forward step and storing them all.  g: N values of dJ/dd (zero outside
 * the design box).  Returns J; trace [T][ndet] may be NULL. */
double or_grad_history(const or_problem *P, int T, int seg, double *g, double *trace)
{
    size_t N = ncell(P), SZ = OR_NSLOT * N;
    if (seg < 1) seg = 1;
    int nck = (T + seg - 1) / seg + 1;
    double *ck = calloc((size_t)nck * SZ, sizeof(double));
    double *buf = malloc(sizeof(double) * (size_t)(seg + 1) * SZ);
    double *st = calloc(SZ, sizeof(double));
    or_prof PE, PH;
    prof_make(P, &PE, &PH);
    double J = 0.0;
    double *tr = malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * (P->ndet > 0 ? P->ndet : 1));
    size_t A = (size_t)P->nx * P->ny;
    double *store = any_interp(P) ? calloc(dstore_floats(P, T) + 1, sizeof(double)) : NULL;
    double *e0 = any_interp(P) ? calloc((size_t)P->ndet * OR_DE0 * A, sizeof(double)) : NULL;
    if (e0)
        for (int m = 0; m < P->ndet; m++)
            if (P->det_interp[m]) dstore_planes(P, st, e0 + (size_t)m * OR_DE0 * A, m, 1);
    for (int n = 0; n < T; n++) {
        if (n % seg == 0) memcpy(ck + (size_t)(n / seg) * SZ, st, sizeof(double) * SZ);
        step_fwd(P, st, n, &PE, &PH, tr + (size_t)n * P->ndet, NULL, 1);
        for (int m = 0; m < P->ndet; m++) J += P->S * P->det_w[m] * tr[(size_t)n * P->ndet + m];
        if (store)
            for (int m = 0; m < P->ndet; m++)
                if (P->det_interp[m]) dstore_planes(P, st, store + ((size_t)n * P->ndet + m) * OR_DSTORE * A, m, 0);
    }
    if (trace) memcpy(trace, tr, sizeof(double) * (size_t)T * P->ndet);
    double *adj = calloc(SZ, sizeof(double));
    double *tmp = malloc(sizeof(double) * 6 * N);
    double *lE = lossy_cells(P) ? malloc(sizeof(double) * 3 * lossy_cells(P)) : NULL;
    memset(g, 0, sizeof(double) * N);
    for (int s0 = ((T - 1) / seg) * seg; s0 >= 0; s0 -= seg) {
        int len = T - s0 < seg ? T - s0 : seg;
        memcpy(buf, ck + (size_t)(s0 / seg) * SZ, sizeof(double) * SZ);
        for (int m = 0; m < len; m++) {
            memcpy(buf + (size_t)(m + 1) * SZ, buf + (size_t)m * SZ, sizeof(double) * SZ);
            step_fwd(P, buf + (size_t)(m + 1) * SZ, s0 + m, &PE, &PH, NULL, NULL, 1);
        }
        for (int m = len - 1; m >= 0; m--) {
            if (store) det_interp_adjoint(P, adj, store, e0, s0 + m, T);
            /* E^n of the conducting cells, from the stored state s_n */
            if (lE) lossy_io(P, buf + (size_t)m * SZ, lE, 0);
            adjoint_step(P, adj, buf + (size_t)(m + 1) * SZ, g, 1, &PE, &PH, tmp, lE);
        }
    }
    free(ck); free(buf); free(st); free(adj); free(tmp); free(tr); free(store); free(e0); free(lE);
    prof_free(&PE); prof_free(&PH);
    return J;
}

/* Time-reversal gradient (section 2.2): forward with the interface record,
 * then per step n = T-1..0 the adjoint step (reading the reconstructed s_{n+1})
 * followed by the inverse step.  recon (may be NULL) receives the RMS of the
 * reconstructed interior E and H after reaching n = 0, where the exact state is
 * zero, divided by the RMS of the interior at n = T. */
double or_grad_reversed(const or_problem *P, int T, double *g, double *trace, double *recon)
{
    size_t N = ncell(P), SZ = OR_NSLOT * N, rf = or_record_floats(P);
    double *st = calloc(SZ, sizeof(double));
    double *rec = rf > 0 ? malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * rf) : NULL;
    size_t A = (size_t)P->nx * P->ny;
    double *store = any_interp(P) ? calloc(dstore_floats(P, T) + 1, sizeof(double)) : NULL;
    double *e0 = any_interp(P) ? calloc((size_t)P->ndet * OR_DE0 * A, sizeof(double)) : NULL;
    double J = forward_run(P, st, 0, T, trace, rec, store, e0);
    int p = P->p;
    double nT = 0.0;
    for (int f = 0; f < 6; f++)
        for (int k = p; k < P->nz - p; k++)
            for (int j = p; j < P->ny - p; j++)
                for (int i = p; i < P->nx - p; i++) { double v = st[(size_t)f * N + idx(P, i, j, k)]; nT += v * v; }
    or_prof PE, PH;
    prof_make(P, &PE, &PH);
    double *adj = calloc(SZ, sizeof(double));
    double *tmp = malloc(sizeof(double) * 6 * N);
    memset(g, 0, sizeof(double) * N);
    for (int n = T - 1; n >= 0; n--) {
        if (store) det_interp_adjoint(P, adj, store, e0, n, T);
        adjoint_step(P, adj, st, g, 1, &PE, &PH, tmp,
                     lossy_cells(P) ? rec + (size_t)n * rf + iface_floats(P) : NULL);
        inverse_step(P, st, n, rec);
    }
    if (recon) {
        double n0 = 0.0;
        for (int f = 0; f < 6; f++)
            for (int k = p; k < P->nz - p; k++)
                for (int j = p; j < P->ny - p; j++)
                    for (int i = p; i < P->nx - p; i++) { double v = st[(size_t)f * N + idx(P, i, j, k)]; n0 += v * v; }
        *recon = nT > 0.0 ? sqrt(n0 / nT) : 0.0;
    }
    free(st); free(rec); free(adj); free(tmp); free(store); free(e0);
    prof_free(&PE); prof_free(&PH);
    return J;
}
