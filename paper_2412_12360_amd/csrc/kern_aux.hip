// Auxiliary kernels: the interface record (arXiv 2412.12360, section 2.2),
// detector flux planes and their fixed-order reductions (section 2.1),
// the detector adjoint source, the objective, reconstruction norms and small
// element-wise helpers.  No atomics: every sum has one fixed order.
#include "fdtd_internal.h"

namespace {

constexpr int NT = 256;

__device__ __forceinline__ long long cidx(const Grid &g, int i, int j, int k)
{
    return (long long)k * g.nxy + (long long)j * g.nx + i;
}

// Record layout per step: faces f = 2a + side, each [comp 0..1][v][u] over the
// interior window of axes u < v.  side 0: H comps (a+1)%3, (a+2)%3 at layer
// p-1; side 1: E comps at layer n_a - p.  restore = 1 writes the record back
// into the fields (rec == nullptr writes zeros).
__global__ __launch_bounds__(NT) void k_record(Grid g, Fields F, RecGeom R, float *rec, int side, int restore,
                                               long long total)
{
    long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= total) return;
    int a = 0;
    for (; a < 3; a++) {
        const long long sz = 2LL * R.Lu[a] * R.Lv[a];
        if (t < sz) break;
        t -= sz;
    }
    const long long face = (long long)R.Lu[a] * R.Lv[a];
    const int comp = (int)(t / face);
    const long long rem = t - comp * face;
    const int v = (int)(rem / R.Lu[a]);
    const int u = (int)(rem - (long long)v * R.Lu[a]);
    const int na[3] = {g.nx, g.ny, g.nz};
    int x[3];
    const int ua = a == 0 ? 1 : 0, va = a == 2 ? 1 : 2;
    x[a] = side == 0 ? g.p - 1 : na[a] - g.p;
    x[ua] = g.p + u;
    x[va] = g.p + v;
    const int fc = (side == 0 ? 3 : 0) + (a + 1 + comp) % 3;
    const long long c = cidx(g, x[0], x[1], x[2]);
    const long long r = R.off[2 * a + side] + t;
    if (restore)
        F.c[fc][c] = rec ? rec[r] : 0.f;
    else
        rec[r] = F.c[fc][c];
}

__global__ __launch_bounds__(NT) void k_det_planes(Grid g, Fields F, Detectors D, float *planes)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= D.per_step) return;
    int m = 0;
    while (m + 1 < D.ndet && t >= D.off[m + 1]) m++;
    const long long e = t - D.off[m];
    const int w = D.i1[m] - D.i0[m];
    const int j = D.j0[m] + (int)(e / w);
    const int i = D.i0[m] + (int)(e - (long long)(j - D.j0[m]) * w);
    const long long c = cidx(g, i, j, D.k[m]);
    planes[t] = flux_density(F.c[0][c], F.c[1][c], F.c[3][c], F.c[4][c]);
}

// Interpolated detectors (section 2.1: composite metrics need all components
// at one point and time).  Cell t of detector m's extended window
// [i0, i1] x [j0, j1] (one more cell in x and y than the flux window).
__device__ __forceinline__ bool ext_cell(const Detectors &D, long long t, int &m, int &i, int &j, long long &e,
                                         long long &L)
{
    long long base = 0;
    for (m = 0; m < D.ndet; m++) {
        if (!D.interp[m]) continue;
        const int w = D.i1[m] - D.i0[m] + 1;
        L = (long long)w * (D.j1[m] - D.j0[m] + 1);
        if (t < base + L) {
            e = t - base;
            j = D.j0[m] + (int)(e / w);
            i = D.i0[m] + (int)(e - (long long)(j - D.j0[m]) * w);
            return true;
        }
        base += L;
    }
    return false;
}

// E^n (Ex, Ey) of the interpolated detectors' planes, before the step
__global__ __launch_bounds__(NT) void k_det_eprev(Grid g, Fields F, Detectors D, float *eprev, long long total)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= total) return;
    int m, i, j;
    long long e, L;
    if (!ext_cell(D, t, m, i, j, e, L)) return;
    const long long c = cidx(g, i, j, D.k[m]);
    eprev[D.eoff[m] + e] = F.c[0][c];
    eprev[D.eoff[m] + L + e] = F.c[1][c];
    if (D.energy[m]) {   // Ez of plane k and of layer k-1
        eprev[D.eoff[m] + 2 * L + e] = F.c[2][c];
        eprev[D.eoff[m] + 3 * L + e] = F.c[2][c - g.nxy];
    }
}

// the six raw planes of one step from the fields (per-cell path)
__global__ __launch_bounds__(NT) void k_det_raw(Grid g, Fields F, Detectors D, float *raw, long long total)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= total) return;
    int m, i, j;
    long long e, L;
    if (!ext_cell(D, t, m, i, j, e, L)) return;
    const long long c = cidx(g, i, j, D.k[m]), cm = c - g.nxy;
    float *r = raw + D.roff[m] + e;
    r[0] = F.c[0][c];
    r[L] = F.c[1][c];
    r[2 * L] = F.c[3][cm];
    r[3 * L] = F.c[4][cm];
    r[4 * L] = F.c[3][c];
    r[5 * L] = F.c[4][c];
    if (D.energy[m]) {   // Ez, Hz of plane k, Ez of layer k-1
        r[6 * L] = F.c[2][c];
        r[7 * L] = F.c[5][c];
        r[8 * L] = F.c[2][cm];
    }
}

// co-located flux density of detector m at step level s: E of steps n, n+1
// (from eprev for s = 0, else from the raw planes of level s-1) and
// H^{n+1/2} of layers k-1, k, each averaged onto (i+1/2, j+1/2, k)
__global__ __launch_bounds__(NT) void k_det_interp(Grid g, Detectors D, int m, int s, const float *raw,
                                                   const float *eprev, float *planes)
{
    const long long e = (long long)blockIdx.x * NT + threadIdx.x;
    const int w = D.i1[m] - D.i0[m];
    const long long n = (long long)w * (D.j1[m] - D.j0[m]);
    if (e >= n) return;
    const int jj = (int)(e / w), ii = (int)(e - (long long)jj * w);
    const int wx = w + 1;
    const long long L = (long long)wx * (D.j1[m] - D.j0[m] + 1);
    const long long p00 = (long long)jj * wx + ii, p10 = p00 + 1, p01 = p00 + wx;
    const float *Rb = raw + s * D.raw_per_step + D.roff[m];
    const float *Ea = s == 0 ? eprev + D.eoff[m] : raw + (s - 1) * D.raw_per_step + D.roff[m];
    const float ex = 0.25f * ((Ea[p00] + Ea[p01]) + (Rb[p00] + Rb[p01]));
    const float ey = 0.25f * ((Ea[L + p00] + Ea[L + p10]) + (Rb[L + p00] + Rb[L + p10]));
    const float hx = 0.25f * ((Rb[2 * L + p00] + Rb[2 * L + p10]) + (Rb[4 * L + p00] + Rb[4 * L + p10]));
    const float hy = 0.25f * ((Rb[3 * L + p00] + Rb[3 * L + p01]) + (Rb[5 * L + p00] + Rb[5 * L + p01]));
    if (!D.energy[m]) {
        planes[s * D.per_step + D.off[m] + e] = flux_density(ex, ey, hx, hy);
        return;
    }
    // energy: Ez over the four (i, j) neighbours of layers k-1, k and the two
    // steps, Hz at the point; eps_r of cell (i,j,k) from S/eps_r
    const long long p11 = p01 + 1;
    const float *Ez = Rb + 6 * L, *Ezm = Rb + 8 * L;
    const float *Pz = s == 0 ? Ea + 2 * L : Ea + 6 * L;
    const float *Pzm = s == 0 ? Ea + 3 * L : Ea + 8 * L;
    const float ez = 0.0625f * (((Ez[p00] + Ez[p10]) + (Ez[p01] + Ez[p11])) + ((Ezm[p00] + Ezm[p10]) + (Ezm[p01] + Ezm[p11])) +
                                ((Pz[p00] + Pz[p10]) + (Pz[p01] + Pz[p11])) + ((Pzm[p00] + Pzm[p10]) + (Pzm[p01] + Pzm[p11])));
    const float hz = Rb[7 * L + p00];
    const float eps = g.S / g.ce[cidx(g, D.i0[m] + ii, D.j0[m] + jj, D.k[m])];
    planes[s * D.per_step + D.off[m] + e] =
        0.5f * (eps * ((ex * ex + ey * ey) + ez * ez) + ((hx * hx + hy * hy) + hz * hz));
}

// Adjoint source of interpolated detector m before reverse step n, for
// J = S sum_n w P[n] with P[n] the co-located sum: E^{n+1} enters P[n] (as the
// later of its two steps) and P[n+1] (as the earlier), H^{n+1/2} enters P[n].
// Each co-located value is a quarter of four nodes, so a node receives a
// quarter of the partner value of every cell it enters.  drec holds the six
// raw planes of every step, e0 the E planes of step 0.  One thread per node of
// the extended window gathers its (at most two) cells: no two threads write
// one address, and the order of the sums is fixed.
struct CoVals {
    float exc, eyc, hxc, hyc, hxc1, hyc1;
};
__device__ __forceinline__ CoVals co_vals(const float *Ep, const float *R, const float *R1, long long L, int wx, int ci,
                                          int cj)
{
    const long long p00 = (long long)cj * wx + ci, p10 = p00 + 1, p01 = p00 + wx;
    CoVals v;
    v.exc = 0.25f * ((Ep[p00] + Ep[p01]) + (R[p00] + R[p01]));
    v.eyc = 0.25f * ((Ep[L + p00] + Ep[L + p10]) + (R[L + p00] + R[L + p10]));
    v.hxc = 0.25f * ((R[2 * L + p00] + R[2 * L + p10]) + (R[4 * L + p00] + R[4 * L + p10]));
    v.hyc = 0.25f * ((R[3 * L + p00] + R[3 * L + p01]) + (R[5 * L + p00] + R[5 * L + p01]));
    v.hxc1 = R1 ? 0.25f * ((R1[2 * L + p00] + R1[2 * L + p10]) + (R1[4 * L + p00] + R1[4 * L + p10])) : 0.f;
    v.hyc1 = R1 ? 0.25f * ((R1[3 * L + p00] + R1[3 * L + p01]) + (R1[5 * L + p00] + R1[5 * L + p01])) : 0.f;
    return v;
}

__global__ __launch_bounds__(NT) void k_det_interp_adjoint(Grid g, Detectors D, int m, const float *drec,
                                                           const float *e0, int n, int T, float sw, Fields A)
{
    const int w = D.i1[m] - D.i0[m], h = D.j1[m] - D.j0[m], wx = w + 1;
    const long long L = (long long)wx * (h + 1);
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= L) return;
    const int jj = (int)(t / wx), ii = (int)(t - (long long)jj * wx);
    const float *R = drec + (long long)n * D.raw_per_step + D.roff[m];
    const float *Ep = n == 0 ? e0 + D.eoff[m] : drec + (long long)(n - 1) * D.raw_per_step + D.roff[m];
    const float *R1 = n + 1 < T ? drec + (long long)(n + 1) * D.raw_per_step + D.roff[m] : nullptr;
    const bool in00 = ii < w && jj < h, in0m = ii < w && jj >= 1, inm0 = ii >= 1 && jj < h;
    CoVals c00{}, c0m{}, cm0{};
    if (in00) c00 = co_vals(Ep, R, R1, L, wx, ii, jj);
    if (in0m) c0m = co_vals(Ep, R, R1, L, wx, ii, jj - 1);
    if (inm0) cm0 = co_vals(Ep, R, R1, L, wx, ii - 1, jj);
    // Ex node (cells (i,j), (i,j-1)), Ey node (cells (i,j), (i-1,j)), Hy nodes
    // of both layers (cells (i,j), (i,j-1)), Hx nodes (cells (i,j), (i-1,j))
    const float gx = (c00.hyc + c00.hyc1) + (c0m.hyc + c0m.hyc1);
    const float gy = (c00.hxc + c00.hxc1) + (cm0.hxc + cm0.hxc1);
    const float ghy = c00.exc + c0m.exc;
    const float ghx = c00.eyc + cm0.eyc;
    const float q = 0.25f * sw;
    const long long c = cidx(g, D.i0[m] + ii, D.j0[m] + jj, D.k[m]), cm = c - g.nxy;
    A.c[0][c] = fmaf(q, gx, A.c[0][c]);
    A.c[1][c] = fmaf(-q, gy, A.c[1][c]);
    A.c[4][cm] = fmaf(q, ghy, A.c[4][cm]);
    A.c[4][c] = fmaf(q, ghy, A.c[4][c]);
    A.c[3][cm] = fmaf(-q, ghx, A.c[3][cm]);
    A.c[3][c] = fmaf(-q, ghx, A.c[3][c]);
}

// Adjoint source of energy detector m before reverse step n, J = S sum_n w
// U[n] with U the co-located energy sum: a node receives eps_r (co-located E)
// or (co-located H) times its averaging weight from every cell it enters
// (E^{n+1} in U[n] and U[n+1], H^{n+1/2} in U[n]; the detector lies outside
// the design box, so U adds no explicit eps_r term).  Raw planes of a step:
// Ex, Ey (k), Hx, Hy (k-1), Hx, Hy (k), Ez, Hz (k), Ez (k-1); step 0 keeps Ex,
// Ey, Ez (k), Ez (k-1).  One thread per node of the extended window.
struct CoAll {
    float ex, ey, ez, hx, hy, hz, ex1, ey1, ez1;
};
__device__ __forceinline__ CoAll co_all(const float *Ep, const float *Epz, const float *Epzm, const float *R,
                                        const float *R1, long long L, int wx, int ci, int cj)
{
    const long long p00 = (long long)cj * wx + ci, p10 = p00 + 1, p01 = p00 + wx, p11 = p01 + 1;
    CoAll v;
    v.ex = 0.25f * ((Ep[p00] + Ep[p01]) + (R[p00] + R[p01]));
    v.ey = 0.25f * ((Ep[L + p00] + Ep[L + p10]) + (R[L + p00] + R[L + p10]));
    const float *Rz = R + 6 * L, *Rzm = R + 8 * L;
    v.ez = 0.0625f * (((Rz[p00] + Rz[p10]) + (Rz[p01] + Rz[p11])) + ((Rzm[p00] + Rzm[p10]) + (Rzm[p01] + Rzm[p11])) +
                      ((Epz[p00] + Epz[p10]) + (Epz[p01] + Epz[p11])) + ((Epzm[p00] + Epzm[p10]) + (Epzm[p01] + Epzm[p11])));
    v.hx = 0.25f * ((R[2 * L + p00] + R[2 * L + p10]) + (R[4 * L + p00] + R[4 * L + p10]));
    v.hy = 0.25f * ((R[3 * L + p00] + R[3 * L + p01]) + (R[5 * L + p00] + R[5 * L + p01]));
    v.hz = R[7 * L + p00];
    v.ex1 = v.ey1 = v.ez1 = 0.f;
    if (R1) {
        v.ex1 = 0.25f * ((R[p00] + R[p01]) + (R1[p00] + R1[p01]));
        v.ey1 = 0.25f * ((R[L + p00] + R[L + p10]) + (R1[L + p00] + R1[L + p10]));
        const float *Sz = R1 + 6 * L, *Szm = R1 + 8 * L;
        v.ez1 = 0.0625f * (((Sz[p00] + Sz[p10]) + (Sz[p01] + Sz[p11])) + ((Szm[p00] + Szm[p10]) + (Szm[p01] + Szm[p11])) +
                           ((Rz[p00] + Rz[p10]) + (Rz[p01] + Rz[p11])) + ((Rzm[p00] + Rzm[p10]) + (Rzm[p01] + Rzm[p11])));
    }
    return v;
}

__global__ __launch_bounds__(NT) void k_det_energy_adjoint(Grid g, Detectors D, int m, const float *drec,
                                                           const float *e0, int n, int T, float sw, Fields A)
{
    const int w = D.i1[m] - D.i0[m], h = D.j1[m] - D.j0[m], wx = w + 1;
    const long long L = (long long)wx * (h + 1);
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= L) return;
    const int jj = (int)(t / wx), ii = (int)(t - (long long)jj * wx);
    const float *R = drec + (long long)n * D.raw_per_step + D.roff[m];
    const float *Ep = n == 0 ? e0 + D.eoff[m] : drec + (long long)(n - 1) * D.raw_per_step + D.roff[m];
    const float *Epz = n == 0 ? Ep + 2 * L : Ep + 6 * L, *Epzm = n == 0 ? Ep + 3 * L : Ep + 8 * L;
    const float *R1 = n + 1 < T ? drec + (long long)(n + 1) * D.raw_per_step + D.roff[m] : nullptr;
    const int k = D.k[m];
    auto eps_of = [&](int ci, int cj) { return g.S / g.ce[cidx(g, D.i0[m] + ci, D.j0[m] + cj, k)]; };
    // the cells this node enters: (i,j), (i-1,j), (i,j-1), (i-1,j-1)
    const bool c00 = ii < w && jj < h, cm0 = ii >= 1 && jj < h, c0m = ii < w && jj >= 1, cmm = ii >= 1 && jj >= 1;
    CoAll v00{}, vm0{}, v0m{}, vmm{};
    float e00 = 0.f, em0 = 0.f, e0m = 0.f, emm = 0.f;
    if (c00) { v00 = co_all(Ep, Epz, Epzm, R, R1, L, wx, ii, jj); e00 = eps_of(ii, jj); }
    if (cm0) { vm0 = co_all(Ep, Epz, Epzm, R, R1, L, wx, ii - 1, jj); em0 = eps_of(ii - 1, jj); }
    if (c0m) { v0m = co_all(Ep, Epz, Epzm, R, R1, L, wx, ii, jj - 1); e0m = eps_of(ii, jj - 1); }
    if (cmm) { vmm = co_all(Ep, Epz, Epzm, R, R1, L, wx, ii - 1, jj - 1); emm = eps_of(ii - 1, jj - 1); }
    const float gx = e00 * (v00.ex + v00.ex1) + e0m * (v0m.ex + v0m.ex1);                       // Ex: (i,j), (i,j-1)
    const float gy = e00 * (v00.ey + v00.ey1) + em0 * (vm0.ey + vm0.ey1);                       // Ey: (i,j), (i-1,j)
    const float gz = (e00 * (v00.ez + v00.ez1) + em0 * (vm0.ez + vm0.ez1)) +
                     (e0m * (v0m.ez + v0m.ez1) + emm * (vmm.ez + vmm.ez1));                       // Ez: all four
    const float ghx = v00.hx + vm0.hx, ghy = v00.hy + v0m.hy;
    const long long c = cidx(g, D.i0[m] + ii, D.j0[m] + jj, k), cm = c - g.nxy;
    const float q = 0.25f * sw, q16 = 0.0625f * sw;
    A.c[0][c] = fmaf(q, gx, A.c[0][c]);
    A.c[1][c] = fmaf(q, gy, A.c[1][c]);
    A.c[2][c] = fmaf(q16, gz, A.c[2][c]);
    A.c[2][cm] = fmaf(q16, gz, A.c[2][cm]);
    A.c[3][c] = fmaf(q, ghx, A.c[3][c]);
    A.c[3][cm] = fmaf(q, ghx, A.c[3][cm]);
    A.c[4][c] = fmaf(q, ghy, A.c[4][c]);
    A.c[4][cm] = fmaf(q, ghy, A.c[4][cm]);
    A.c[5][c] = fmaf(sw, v00.hz, A.c[5][c]);
}

// dJ/dE^{n+1} and dJ/dH^{n+1/2} of J += S w sum (Ex Hy - Ey Hx)
__global__ __launch_bounds__(NT) void k_det_adjoint(Grid g, Fields F, Fields A, Detectors D, int m, float sw)
{
    const long long e = (long long)blockIdx.x * NT + threadIdx.x;
    const int w = D.i1[m] - D.i0[m];
    const long long L = (long long)w * (D.j1[m] - D.j0[m]);
    if (e >= L) return;
    const int j = D.j0[m] + (int)(e / w);
    const int i = D.i0[m] + (int)(e - (long long)(j - D.j0[m]) * w);
    const long long c = cidx(g, i, j, D.k[m]);
    const float ex = F.c[0][c], ey = F.c[1][c], hx = F.c[3][c], hy = F.c[4][c];
    A.c[0][c] = fmaf(sw, hy, A.c[0][c]);
    A.c[1][c] = fmaf(-sw, hx, A.c[1][c]);
    A.c[4][c] = fmaf(sw, ex, A.c[4][c]);
    A.c[3][c] = fmaf(-sw, ey, A.c[3][c]);
}

__device__ __forceinline__ float block_sum(float v, float *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// out[r * out_stride] = sum of in[r * row_stride + 0 .. len), fixed order
__global__ __launch_bounds__(NT) void k_reduce_rows(const float *in, long long len, long long row_stride,
                                                    float *out, int out_stride)
{
    __shared__ float sh[NT];
    const float *row = in + (long long)blockIdx.x * row_stride;
    float acc = 0.f;
    for (long long e = threadIdx.x; e < len; e += NT) acc = acc + row[e];
    const float s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[(long long)blockIdx.x * out_stride] = s;
}

// first level of a two-level row sum: block (c, r) sums elements
// [c*CH, (c+1)*CH) of row r in a fixed order
constexpr long long CH = 4096;
__global__ __launch_bounds__(NT) void k_reduce_chunks(const float *in, long long len, long long row_stride,
                                                      float *part, int nch)
{
    __shared__ float sh[NT];
    const float *row = in + (long long)blockIdx.y * row_stride;
    const long long a = (long long)blockIdx.x * CH;
    const long long b = a + CH < len ? a + CH : len;
    float acc = 0.f;
    for (long long e = a + threadIdx.x; e < b; e += NT) acc = acc + row[e];
    const float s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.y * nch + blockIdx.x] = s;
}

__global__ __launch_bounds__(NT) void k_objective(const float *trace, int steps, int ndet, const float *w,
                                                  float S, float *J)
{
    __shared__ float sh[NT];
    float acc = 0.f;
    const long long tot = (long long)steps * ndet;
    for (long long e = threadIdx.x; e < tot; e += NT) acc = fmaf(w[e % ndet], trace[e], acc);
    const float s = block_sum(acc, sh);
    if (threadIdx.x == 0) J[0] = S * s;
}

// per-block sums of squares of the six fields over the interior
__global__ __launch_bounds__(NT) void k_sumsq(Grid g, Fields F, float *partials)
{
    __shared__ float sh[NT];
    const int p = g.p;
    const int Lx = g.nx - 2 * p, Ly = g.ny - 2 * p, Lz = g.nz - 2 * p;
    const long long tot = (long long)Lx * Ly * Lz;
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    float acc = 0.f;
    if (t < tot) {
        const int i = p + (int)(t % Lx);
        const int j = p + (int)((t / Lx) % Ly);
        const int k = p + (int)(t / ((long long)Lx * Ly));
        const long long c = cidx(g, i, j, k);
        for (int q = 0; q < 6; q++) acc = fmaf(F.c[q][c], F.c[q][c], acc);
    }
    const float s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(NT) void k_recon(const float *pT, const float *p0, int n, float *out)
{
    __shared__ float sh[NT];
    float a = 0.f, b = 0.f;
    for (int e = threadIdx.x; e < n; e += NT) { a = a + pT[e]; b = b + p0[e]; }
    const float sT = block_sum(a, sh);
    __syncthreads();
    const float s0 = block_sum(b, sh);
    if (threadIdx.x == 0) out[0] = sT > 0.f ? sqrtf(s0 / sT) : 0.f;
}

__global__ __launch_bounds__(NT) void k_deps(const float *gacc, const float *dd, long long D, float S, float *out)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= D) return;
    const float d = dd[t];
    out[t] = -(d * d) * (S * gacc[t]);
}

// Incident fields of a one-sided total-field/scattered-field plane along +z
// (section 2.1 names the source type).  A 1D Yee line along z with the grid's
// S and the plane's S/eps_r carries the incident wave; for a wave uniform in
// x and y it is the 3D update restricted to z, here with the same update
// expressions (zero transverse differences).  Node 0 is driven,
// E_0^{n+1} = amp[n]; node 1 is the first total-field E plane k0.  Step n
// writes the two corrections the grid's curl misses across the plane:
//     outH[n] = hsign * S * E_1^n       (after the H half step, layer k0-1)
//     outE[n] = S/eps * H_0^{n+1/2}     (after the E half step, plane k0)
// The line has L nodes (E) and L-1 edges (H) in `line` and a conducting far
// end; with L >= T/2 + 8 no wave from node 0 returns from it within T steps
// (an update moves information at most one cell per step).  One workgroup.
constexpr int LINE_NT = 1024;
__global__ __launch_bounds__(LINE_NT) void k_tfsf_line(const float *amp, int T, float S, const float *ce_at,
                                                       float hsign, float *line, int L, float *outE, float *outH)
{
    float *E = line, *H = line + L;
    const float ce = *ce_at;
    for (int c = threadIdx.x; c < 2 * L - 1; c += LINE_NT) line[c] = 0.f;
    __syncthreads();
    for (int n = 0; n < T; n++) {
        // H phase: reads E only
        if (threadIdx.x == 0) outH[n] = hsign * (S * E[1]);
        for (int c = threadIdx.x; c < L - 1; c += LINE_NT) H[c] = h_update(H[c], S, E[c + 1] - E[c], 0.f);
        __syncthreads();
        // E phase: reads H only; node L-1 stays 0
        if (threadIdx.x == 0) {
            outE[n] = ce * H[0];
            E[0] = amp[n];
        }
        for (int c = 1 + threadIdx.x; c < L - 1; c += LINE_NT) E[c] = e_update(E[c], ce, 0.f, H[c] - H[c - 1]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(NT) void k_fill(float *p, long long n, float v)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ __launch_bounds__(NT) void k_copy(float *dst, const float *src, long long n)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t < n) dst[t] = src[t];
}

__global__ __launch_bounds__(NT) void k_scale(const float *x, float S, float *y, long long n)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t < n) y[t] = S * x[t];
}

__global__ __launch_bounds__(NT) void k_gather_box(const float *src, Grid g, int3 lo, int3 hi, float *dst)
{
    const int dx = hi.x - lo.x, dy = hi.y - lo.y, dz = hi.z - lo.z;
    const long long tot = (long long)dx * dy * dz;
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= tot) return;
    const int i = lo.x + (int)(t % dx);
    const int j = lo.y + (int)((t / dx) % dy);
    const int k = lo.z + (int)(t / ((long long)dx * dy));
    dst[t] = src[cidx(g, i, j, k)];
}

// conducting cells: u = sigma S d / 2, ca = (1-u)/(1+u), cb = S d/(1+u) into ce
__global__ __launch_bounds__(NT) void k_lossy_coef(Grid g, const float *inv_eps, float *ce, float *lca)
{
    const int dx = g.lhi[0] - g.llo[0], dy = g.lhi[1] - g.llo[1], dz = g.lhi[2] - g.llo[2];
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= (long long)dx * dy * dz) return;
    const int i = g.llo[0] + (int)(t % dx);
    const int j = g.llo[1] + (int)((t / dx) % dy);
    const int k = g.llo[2] + (int)(t / ((long long)dx * dy));
    const long long c = cidx(g, i, j, k);
    const float d = inv_eps[c];
    const float u = 0.5f * (g.lsig[t] * (g.S * d));
    lca[t] = (1.f - u) / (1.f + u);
    ce[c] = (g.S * d) / (1.f + u);
}

// dJ/deps = -d^2 dJ/dd with dJ/dd = S/(1+u)^2 g in the design cells that conduct
__global__ __launch_bounds__(NT) void k_deps_lossy(Grid g, const float *gacc, const float *dd, int3 lo, int3 hi,
                                                   float *out)
{
    const int dx = hi.x - lo.x, dy = hi.y - lo.y, dz = hi.z - lo.z;
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= (long long)dx * dy * dz) return;
    const int i = lo.x + (int)(t % dx);
    const int j = lo.y + (int)((t / dx) % dy);
    const int k = lo.z + (int)(t / ((long long)dx * dy));
    const long long li = lossy_index(g, i, j, k);
    if (li < 0) return;
    const float d = dd[t];
    const float u = 0.5f * (g.lsig[li] * (g.S * d));
    const float f = 1.f / ((1.f + u) * (1.f + u));
    out[t] = -(d * d) * ((g.S * f) * gacc[t]);
}

unsigned nblk(long long n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

hipError_t launch_record(const Grid &g, const Fields &F, const RecGeom &R, float *rec, int side, int restore,
                         hipStream_t s)
{
    long long total = 0;
    for (int a = 0; a < 3; a++) total += 2LL * R.Lu[a] * R.Lv[a];
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_record, dim3(nblk(total)), dim3(NT), 0, s, g, F, R, rec, side, restore, total);
    return hipGetLastError();
}

hipError_t launch_record_zero_e(const Grid &g, const Fields &F, const RecGeom &R, hipStream_t s)
{
    return launch_record(g, F, R, nullptr, 1, 1, s);
}

hipError_t launch_det_planes(const Grid &g, const Fields &F, const Detectors &D, float *planes, hipStream_t s)
{
    if (D.ndet == 0 || D.per_step == 0) return hipSuccess;
    hipLaunchKernelGGL(k_det_planes, dim3(nblk(D.per_step)), dim3(NT), 0, s, g, F, D, planes);
    return hipGetLastError();
}

hipError_t launch_det_adjoint(const Grid &g, const Fields &F, const Fields &A, const Detectors &D,
                              const float *weights_S, hipStream_t s)
{
    for (int m = 0; m < D.ndet; m++) {
        const long long L = (long long)(D.i1[m] - D.i0[m]) * (D.j1[m] - D.j0[m]);
        if (L <= 0) continue;
        hipLaunchKernelGGL(k_det_adjoint, dim3(nblk(L)), dim3(NT), 0, s, g, F, A, D, m, weights_S[m]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_reduce_rows(const float *in, long long len, int rows, long long row_stride, float *out,
                              int out_stride, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(NT), 0, s, in, len, row_stride, out, out_stride);
    return hipGetLastError();
}

long long reduce_scratch_floats(long long len, int rows) { return (long long)rows * ((len + CH - 1) / CH); }

hipError_t launch_reduce_rows2(const float *in, long long len, int rows, long long row_stride, float *out,
                               int out_stride, float *scratch, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    const int nch = (int)((len + CH - 1) / CH);
    if (nch <= 1) return launch_reduce_rows(in, len, rows, row_stride, out, out_stride, s);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nch, rows), dim3(NT), 0, s, in, len, row_stride, scratch, nch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_rows(scratch, nch, rows, nch, out, out_stride, s);
}

hipError_t launch_objective(const float *trace, int steps, int ndet, const float *w, float S, float *J,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(NT), 0, s, trace, steps, ndet, w, S, J);
    return hipGetLastError();
}

hipError_t launch_interior_sumsq(const Grid &g, const Fields &F, float *partials, int *nparts, hipStream_t s)
{
    const long long tot = (long long)(g.nx - 2 * g.p) * (g.ny - 2 * g.p) * (g.nz - 2 * g.p);
    *nparts = (int)nblk(tot);
    hipLaunchKernelGGL(k_sumsq, dim3(*nparts), dim3(NT), 0, s, g, F, partials);
    return hipGetLastError();
}

hipError_t launch_recon(const float *pT, const float *p0, int n, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_recon, dim3(1), dim3(NT), 0, s, pT, p0, n, out);
    return hipGetLastError();
}

hipError_t launch_deps(const float *gacc, const float *dd, long long D, float S, float *out, hipStream_t s)
{
    if (D == 0) return hipSuccess;
    hipLaunchKernelGGL(k_deps, dim3(nblk(D)), dim3(NT), 0, s, gacc, dd, D, S, out);
    return hipGetLastError();
}

long long ext_total(const Detectors &D)
{
    long long tot = 0;
    for (int m = 0; m < D.ndet; m++)
        if (D.interp[m]) tot += (long long)(D.i1[m] - D.i0[m] + 1) * (D.j1[m] - D.j0[m] + 1);
    return tot;
}

hipError_t launch_det_eprev(const Grid &g, const Fields &F, const Detectors &D, float *eprev, hipStream_t s)
{
    const long long tot = ext_total(D);
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_det_eprev, dim3(nblk(tot)), dim3(NT), 0, s, g, F, D, eprev, tot);
    return hipGetLastError();
}

hipError_t launch_det_raw(const Grid &g, const Fields &F, const Detectors &D, float *raw, hipStream_t s)
{
    const long long tot = ext_total(D);
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_det_raw, dim3(nblk(tot)), dim3(NT), 0, s, g, F, D, raw, tot);
    return hipGetLastError();
}

hipError_t launch_det_interp(const Grid &g, const Detectors &D, const float *raw, const float *eprev, int levels,
                             float *planes, hipStream_t s)
{
    for (int m = 0; m < D.ndet; m++) {
        if (!D.interp[m]) continue;
        const long long n = (long long)(D.i1[m] - D.i0[m]) * (D.j1[m] - D.j0[m]);
        for (int l = 0; l < levels; l++) {
            hipLaunchKernelGGL(k_det_interp, dim3(nblk(n)), dim3(NT), 0, s, g, D, m, l, raw, eprev, planes);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_det_interp_adjoint(const Grid &g, const Detectors &D, const float *drec, const float *e0, int n,
                                    int T, const float *wS, const Fields &A, hipStream_t s)
{
    for (int m = 0; m < D.ndet; m++) {
        if (!D.interp[m] || wS[m] == 0.f) continue;
        const long long L = (long long)(D.i1[m] - D.i0[m] + 1) * (D.j1[m] - D.j0[m] + 1);
        if (D.energy[m])
            hipLaunchKernelGGL(k_det_energy_adjoint, dim3(nblk(L)), dim3(NT), 0, s, g, D, m, drec, e0, n, T, wS[m], A);
        else
            hipLaunchKernelGGL(k_det_interp_adjoint, dim3(nblk(L)), dim3(NT), 0, s, g, D, m, drec, e0, n, T, wS[m], A);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int tfsf_line_nodes(int T) { return T / 2 + 8; }

hipError_t launch_tfsf_line(const float *amp, int T, float S, const float *ce_at, float hsign, float *line,
                            float *outE, float *outH, hipStream_t s)
{
    hipLaunchKernelGGL(k_tfsf_line, dim3(1), dim3(LINE_NT), 0, s, amp, T, S, ce_at, hsign, line,
                       tfsf_line_nodes(T), outE, outH);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, long long n, float v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(NT), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, long long n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(NT), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_scale_ce(const float *inv_eps, float S, float *ce, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(NT), 0, s, inv_eps, S, ce, n);
    return hipGetLastError();
}

hipError_t launch_lossy_coef(const Grid &g, const float *inv_eps, float *ce, float *lca, hipStream_t s)
{
    if (!g.lca) return hipSuccess;
    const long long tot = (long long)(g.lhi[0] - g.llo[0]) * (g.lhi[1] - g.llo[1]) * (g.lhi[2] - g.llo[2]);
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lossy_coef, dim3(nblk(tot)), dim3(NT), 0, s, g, inv_eps, ce, lca);
    return hipGetLastError();
}

hipError_t launch_deps_lossy(const Grid &g, const float *gacc, const float *d_design, const int *dlo, const int *dhi,
                             float *out, hipStream_t s)
{
    if (!g.lca) return hipSuccess;
    const long long tot = (long long)(dhi[0] - dlo[0]) * (dhi[1] - dlo[1]) * (dhi[2] - dlo[2]);
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_deps_lossy, dim3(nblk(tot)), dim3(NT), 0, s, g, gacc, d_design,
                       make_int3(dlo[0], dlo[1], dlo[2]), make_int3(dhi[0], dhi[1], dhi[2]), out);
    return hipGetLastError();
}

hipError_t launch_gather_box(const float *src, const Grid &g, const int *lo, const int *hi, float *dst,
                             hipStream_t s)
{
    const long long tot = (long long)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_box, dim3(nblk(tot)), dim3(NT), 0, s, src, g, make_int3(lo[0], lo[1], lo[2]),
                       make_int3(hi[0], hi[1], hi[2]), dst);
    return hipGetLastError();
}
