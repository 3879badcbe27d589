// One-thread-per-cell kernels: the H and E half steps of the Yee leapfrog
// with CPML (arXiv 2412.12360, section 2.1) and the two phases of a reverse
// step -- inverse update plus adjoint (section 2.2).  These update in place,
// one half step per launch; they are the K = 1 reference path and the
// building blocks of the backward pass.
#include "fdtd_internal.h"

namespace {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ long long cidx(const Grid &g, int i, int j, int k)
{
    return (long long)k * g.nxy + (long long)j * g.nx + i;
}

// ----------------------------------------------------------- forward, H half
__global__ __launch_bounds__(256) void k_h_naive(Grid g, Fields F, Psi P, int n, int with_src)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long c = cidx(g, i, j, k);
    const float *Ex = F.c[0], *Ey = F.c[1], *Ez = F.c[2];
    const float ex = Ex[c], ey = Ey[c], ez = Ez[c];
    const bool xi = i + 1 < g.nx, yj = j + 1 < g.ny, zk = k + 1 < g.nz;
    const float ey_x = xi ? Ey[c + 1] : 0.f, ez_x = xi ? Ez[c + 1] : 0.f;
    const float ex_y = yj ? Ex[c + g.nx] : 0.f, ez_y = yj ? Ez[c + g.nx] : 0.f;
    const float ex_z = zk ? Ex[c + g.nxy] : 0.f, ey_z = zk ? Ey[c + g.nxy] : 0.f;
    float dy_ez = ez_y - ez, dz_ey = ey_z - ey;   // Hx
    float dz_ex = ex_z - ex, dx_ez = ez_x - ez;   // Hy
    float dx_ey = ey_x - ey, dy_ex = ex_y - ex;   // Hz
    if (g.p > 0) {
        const int sx = slab_coord(i, g.nx, g.p), sy = slab_coord(j, g.ny, g.p), sz = slab_coord(k, g.nz, g.p);
        if (sx >= 0) {   // Hy (idx 2), Hz (idx 3) along x
            const float b = g.prof[1][0][0][i], a = g.prof[1][0][1][i], kv = g.prof[1][0][2][i];
            const long long s = slab_index(g, 0, sx, i, j, k);
            float p2 = P.a[0][2][s], p3 = P.a[0][3][s];
            dx_ez = cpml_term(dx_ez, p2, b, a, kv);
            dx_ey = cpml_term(dx_ey, p3, b, a, kv);
            P.a[0][2][s] = p2; P.a[0][3][s] = p3;
        }
        if (sy >= 0) {   // Hz (idx 2), Hx (idx 3) along y
            const float b = g.prof[1][1][0][j], a = g.prof[1][1][1][j], kv = g.prof[1][1][2][j];
            const long long s = slab_index(g, 1, sy, i, j, k);
            float p2 = P.a[1][2][s], p3 = P.a[1][3][s];
            dy_ex = cpml_term(dy_ex, p2, b, a, kv);
            dy_ez = cpml_term(dy_ez, p3, b, a, kv);
            P.a[1][2][s] = p2; P.a[1][3][s] = p3;
        }
        if (sz >= 0) {   // Hx (idx 2), Hy (idx 3) along z
            const float b = g.prof[1][2][0][k], a = g.prof[1][2][1][k], kv = g.prof[1][2][2][k];
            const long long s = slab_index(g, 2, sz, i, j, k);
            float p2 = P.a[2][2][s], p3 = P.a[2][3][s];
            dz_ey = cpml_term(dz_ey, p2, b, a, kv);
            dz_ex = cpml_term(dz_ex, p3, b, a, kv);
            P.a[2][2][s] = p2; P.a[2][3][s] = p3;
        }
    }
    float hx = h_update(F.c[3][c], g.S, dy_ez, dz_ey);
    float hy = h_update(F.c[4][c], g.S, dz_ex, dx_ez);
    float hz = h_update(F.c[5][c], g.S, dx_ey, dy_ex);
    // H sources (components 3..5), after the H half step
    if (with_src) {
        for (int s = 0; s < g.nsrc; s++) {
            if (k != g.sk[s] || g.scomp[s] < 3) continue;
            if (g.skind[s] == 0 && (i != g.si[s] || j != g.sj[s])) continue;
            const float A = g.samp[s][n];
            if (g.scomp[s] == 3) hx = hx + A;
            if (g.scomp[s] == 4) hy = hy + A;
            if (g.scomp[s] == 5) hz = hz + A;
        }
    }
    F.c[3][c] = hx; F.c[4][c] = hy; F.c[5][c] = hz;
}

// ----------------------------------------------------------- forward, E half
__global__ __launch_bounds__(256) void k_e_naive(Grid g, Fields F, Psi P, int n, int with_src, float *lrec)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long c = cidx(g, i, j, k);
    const float *Hx = F.c[3], *Hy = F.c[4], *Hz = F.c[5];
    const float hx = Hx[c], hy = Hy[c], hz = Hz[c];
    const float hy_x = i > 0 ? Hy[c - 1] : 0.f, hz_x = i > 0 ? Hz[c - 1] : 0.f;
    const float hx_y = j > 0 ? Hx[c - g.nx] : 0.f, hz_y = j > 0 ? Hz[c - g.nx] : 0.f;
    const float hx_z = k > 0 ? Hx[c - g.nxy] : 0.f, hy_z = k > 0 ? Hy[c - g.nxy] : 0.f;
    float dy_hz = hz - hz_y, dz_hy = hy - hy_z;   // Ex
    float dz_hx = hx - hx_z, dx_hz = hz - hz_x;   // Ey
    float dx_hy = hy - hy_x, dy_hx = hx - hx_y;   // Ez
    const bool hex = held_ex(i, j, k), hey = held_ey(i, j, k), hez = held_ez(i, j, k);
    if (g.p > 0) {
        const int sx = slab_coord(i, g.nx, g.p), sy = slab_coord(j, g.ny, g.p), sz = slab_coord(k, g.nz, g.p);
        if (sx >= 0) {   // Ey (idx 0), Ez (idx 1) along x
            const float b = g.prof[0][0][0][i], a = g.prof[0][0][1][i], kv = g.prof[0][0][2][i];
            const long long s = slab_index(g, 0, sx, i, j, k);
            if (!hey) { float q = P.a[0][0][s]; dx_hz = cpml_term(dx_hz, q, b, a, kv); P.a[0][0][s] = q; }
            if (!hez) { float q = P.a[0][1][s]; dx_hy = cpml_term(dx_hy, q, b, a, kv); P.a[0][1][s] = q; }
        }
        if (sy >= 0) {   // Ez (idx 0), Ex (idx 1) along y
            const float b = g.prof[0][1][0][j], a = g.prof[0][1][1][j], kv = g.prof[0][1][2][j];
            const long long s = slab_index(g, 1, sy, i, j, k);
            if (!hez) { float q = P.a[1][0][s]; dy_hx = cpml_term(dy_hx, q, b, a, kv); P.a[1][0][s] = q; }
            if (!hex) { float q = P.a[1][1][s]; dy_hz = cpml_term(dy_hz, q, b, a, kv); P.a[1][1][s] = q; }
        }
        if (sz >= 0) {   // Ex (idx 0), Ey (idx 1) along z
            const float b = g.prof[0][2][0][k], a = g.prof[0][2][1][k], kv = g.prof[0][2][2][k];
            const long long s = slab_index(g, 2, sz, i, j, k);
            if (!hex) { float q = P.a[2][0][s]; dz_hy = cpml_term(dz_hy, q, b, a, kv); P.a[2][0][s] = q; }
            if (!hey) { float q = P.a[2][1][s]; dz_hx = cpml_term(dz_hx, q, b, a, kv); P.a[2][1][s] = q; }
        }
    }
    const float ce = g.ce[c];
    float ex = F.c[0][c], ey = F.c[1][c], ez = F.c[2][c];
    const long long li = lossy_index(g, i, j, k);
    if (li >= 0) {
        // a conducting cell: E^n into the record, then ca E^n + cb curl H
        if (lrec) {
            const long long nb = (long long)(g.lhi[0] - g.llo[0]) * (g.lhi[1] - g.llo[1]) * (g.lhi[2] - g.llo[2]);
            lrec[li] = ex; lrec[nb + li] = ey; lrec[2 * nb + li] = ez;
        }
        const float ca = g.lca[li];
        ex = ca * ex; ey = ca * ey; ez = ca * ez;
    }
    if (!hex) ex = e_update(ex, ce, dy_hz, dz_hy);
    if (!hey) ey = e_update(ey, ce, dz_hx, dx_hz);
    if (!hez) ez = e_update(ez, ce, dx_hy, dy_hx);
    if (with_src) {
        for (int s = 0; s < g.nsrc; s++) {
            if (k != g.sk[s]) continue;
            if (g.skind[s] == 0 && (i != g.si[s] || j != g.sj[s])) continue;
            const float A = g.samp[s][n];
            if (g.scomp[s] == 0 && !hex) ex = ex + A;
            if (g.scomp[s] == 1 && !hey) ey = ey + A;
            if (g.scomp[s] == 2 && !hez) ez = ez + A;
        }
    }
    F.c[0][c] = ex; F.c[1][c] = ey; F.c[2][c] = ez;
}

// ------------------------------------------------------------ reverse helpers

struct AdjCtx {
    const Grid &g;
    const Fields &A;
    const Psi &P;
};

// Adjoint coefficient of an E pair at (i,j,k): w = sgn * ce * Ebar_q,
// wrapped by the pair's CPML when the cell lies in that axis' slab.
__device__ __forceinline__ float q_epair(const Grid &g, const Fields &A, const Psi &P, int q, int axis,
                                         int idx, float sgn, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k >= g.nz) return 0.f;
    const bool held = q == 0 ? held_ex(i, j, k) : q == 1 ? held_ey(i, j, k) : held_ez(i, j, k);
    if (held) return 0.f;
    const long long c = cidx(g, i, j, k);
    const float w = sgn * (g.ce[c] * A.c[q][c]);
    if (g.p > 0) {
        const int cc = axis == 0 ? i : axis == 1 ? j : k;
        const int na = axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz;
        const int s = slab_coord(cc, na, g.p);
        if (s >= 0) {
            const float pb = P.a[axis][idx][slab_index(g, axis, s, i, j, k)];
            return cpml_adj_coef(w, pb, g.prof[0][axis][1][cc], g.prof[0][axis][2][cc]);
        }
    }
    return w;
}

// Adjoint coefficient of an H pair: w = sgn * S * Hbar_q, CPML-wrapped in slabs.
__device__ __forceinline__ float r_hpair(const Grid &g, const Fields &A, const Psi &P, int q, int axis,
                                         int idx, float sgn, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k >= g.nz) return 0.f;
    const long long c = cidx(g, i, j, k);
    const float w = sgn * (g.S * A.c[3 + q][c]);
    if (g.p > 0) {
        const int cc = axis == 0 ? i : axis == 1 ? j : k;
        const int na = axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz;
        const int s = slab_coord(cc, na, g.p);
        if (s >= 0) {
            const float pb = P.a[axis][idx][slab_index(g, axis, s, i, j, k)];
            return cpml_adj_coef(w, pb, g.prof[1][axis][1][cc], g.prof[1][axis][2][cc]);
        }
    }
    return w;
}

__device__ __forceinline__ bool in_interior(const Grid &g, int i, int j, int k)
{
    const int p = g.p;
    return i >= p && i < g.nx - p && j >= p && j < g.ny - p && k >= p && k < g.nz - p;
}

// ---------------------------------------------------------- reverse, phase A
// inverse E on the interior: E^n = E^{n+1} - src_n - S/eps * curl H^{n+1/2}
// dJ/dd: gacc += Ebar . curl H^{n+1/2} on the design box (times S later)
// adjoint H: Hbar += S C (D Ebar), CPML-wrapped
__global__ __launch_bounds__(256) void k_bwd_a(Grid g, Fields F, Fields A, Psi Pb, int n, int do_inv,
                                              int do_adj, float *gacc, int3 dlo, int3 dhi, const float *lrec)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long c = cidx(g, i, j, k);
    if (do_inv && in_interior(g, i, j, k)) {
        const float *Hx = F.c[3], *Hy = F.c[4], *Hz = F.c[5];
        const float hx = Hx[c], hy = Hy[c], hz = Hz[c];
        const float hy_x = i > 0 ? Hy[c - 1] : 0.f, hz_x = i > 0 ? Hz[c - 1] : 0.f;
        const float hx_y = j > 0 ? Hx[c - g.nx] : 0.f, hz_y = j > 0 ? Hz[c - g.nx] : 0.f;
        const float hx_z = k > 0 ? Hx[c - g.nxy] : 0.f, hy_z = k > 0 ? Hy[c - g.nxy] : 0.f;
        const float dy_hz = hz - hz_y, dz_hy = hy - hy_z;
        const float dz_hx = hx - hx_z, dx_hz = hz - hz_x;
        const float dx_hy = hy - hy_x, dy_hx = hx - hx_y;
        const bool hex = held_ex(i, j, k), hey = held_ey(i, j, k), hez = held_ez(i, j, k);
        // a conducting cell is not inverted: E^n comes from the record
        const long long li = lrec ? lossy_index(g, i, j, k) : -1;
        float en[3] = {0.f, 0.f, 0.f}, sg = 0.f;
        if (li >= 0) {
            const long long nb = (long long)(g.lhi[0] - g.llo[0]) * (g.lhi[1] - g.llo[1]) * (g.lhi[2] - g.llo[2]);
            en[0] = lrec[li]; en[1] = lrec[nb + li]; en[2] = lrec[2 * nb + li];
            sg = g.lsig[li];
        }
        if (do_adj && gacc && i >= dlo.x && i < dhi.x && j >= dlo.y && j < dhi.y && k >= dlo.z && k < dhi.z) {
            const long long dc = ((long long)(k - dlo.z) * (dhi.y - dlo.y) + (j - dlo.y)) * (dhi.x - dlo.x) + (i - dlo.x);
            float acc = gacc[dc];
            if (li < 0) {
                if (!hex) acc = fmaf(A.c[0][c], dy_hz - dz_hy, acc);
                if (!hey) acc = fmaf(A.c[1][c], dz_hx - dx_hz, acc);
                if (!hez) acc = fmaf(A.c[2][c], dx_hy - dy_hx, acc);
            } else {
                // E^{n+1} = ca E^n + cb curl H: dJ/dd = S/(1+u)^2 Ebar'.(curl H - sigma E^n)
                if (!hex) acc = fmaf(A.c[0][c], fmaf(-sg, en[0], dy_hz - dz_hy), acc);
                if (!hey) acc = fmaf(A.c[1][c], fmaf(-sg, en[1], dz_hx - dx_hz), acc);
                if (!hez) acc = fmaf(A.c[2][c], fmaf(-sg, en[2], dx_hy - dy_hx), acc);
            }
            gacc[dc] = acc;
        }
        float ex = F.c[0][c], ey = F.c[1][c], ez = F.c[2][c];
        for (int s = 0; s < g.nsrc; s++) {
            if (k != g.sk[s]) continue;
            if (g.skind[s] == 0 && (i != g.si[s] || j != g.sj[s])) continue;
            const float Am = g.samp[s][n];
            if (g.scomp[s] == 0 && !hex) ex = ex - Am;
            if (g.scomp[s] == 1 && !hey) ey = ey - Am;
            if (g.scomp[s] == 2 && !hez) ez = ez - Am;
        }
        const float ce = g.ce[c];
        if (!hex) ex = e_unupdate(ex, ce, dy_hz, dz_hy);
        if (!hey) ey = e_unupdate(ey, ce, dz_hx, dx_hz);
        if (!hez) ez = e_unupdate(ez, ce, dx_hy, dy_hx);
        if (li >= 0) { ex = en[0]; ey = en[1]; ez = en[2]; }
        F.c[0][c] = ex; F.c[1][c] = ey; F.c[2][c] = ez;
    }
    if (do_adj) {
        // Hbar_x: Ey along z (+, z idx 1), Ez along y (-, y idx 0)
        const float qa = q_epair(g, A, Pb, 1, 2, 1, 1.f, i, j, k) - q_epair(g, A, Pb, 1, 2, 1, 1.f, i, j, k + 1);
        const float qb = q_epair(g, A, Pb, 2, 1, 0, -1.f, i, j, k) - q_epair(g, A, Pb, 2, 1, 0, -1.f, i, j + 1, k);
        // Hbar_y: Ex along z (-, z idx 0), Ez along x (+, x idx 1)
        const float qc = q_epair(g, A, Pb, 0, 2, 0, -1.f, i, j, k) - q_epair(g, A, Pb, 0, 2, 0, -1.f, i, j, k + 1);
        const float qd = q_epair(g, A, Pb, 2, 0, 1, 1.f, i, j, k) - q_epair(g, A, Pb, 2, 0, 1, 1.f, i + 1, j, k);
        // Hbar_z: Ex along y (+, y idx 1), Ey along x (-, x idx 0)
        const float qe = q_epair(g, A, Pb, 0, 1, 1, 1.f, i, j, k) - q_epair(g, A, Pb, 0, 1, 1, 1.f, i, j + 1, k);
        const float qf = q_epair(g, A, Pb, 1, 0, 0, -1.f, i, j, k) - q_epair(g, A, Pb, 1, 0, 0, -1.f, i + 1, j, k);
        A.c[3][c] = A.c[3][c] + (qa + qb);
        A.c[4][c] = A.c[4][c] + (qc + qd);
        A.c[5][c] = A.c[5][c] + (qe + qf);
    }
}

// ---------------------------------------------------------- reverse, phase B
// psibar <- b (psibar + w), read from `Pc`, written to `Pn`; inverse H on
// the interior: H^{n-1/2} = H^{n+1/2} - srcH_n + S curl E^n; adjoint E:
// Ebar -= S C^T Hbar, CPML wrapped.
__global__ __launch_bounds__(256) void k_bwd_b(Grid g, Fields F, Fields A, Psi Pc, Psi Pn, int n, int do_inv,
                                              int do_adj)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long c = cidx(g, i, j, k);
    if (do_adj && g.p > 0) {
        // E-type psibar of this cell into the next buffer, before Ebar changes
        const bool hq[3] = {held_ex(i, j, k), held_ey(i, j, k), held_ez(i, j, k)};
        const float ce = g.ce[c];
        const int cc[3] = {i, j, k};
        const int na[3] = {g.nx, g.ny, g.nz};
        for (int ax = 0; ax < 3; ax++) {
            const int s = slab_coord(cc[ax], na[ax], g.p);
            if (s < 0) continue;
            const long long si = slab_index(g, ax, s, i, j, k);
            const float b = g.prof[0][ax][0][cc[ax]];
            // idx 0: E comp (ax+1)%3, sign -, idx 1: E comp (ax+2)%3, sign +
            const int q0 = (ax + 1) % 3, q1 = (ax + 2) % 3;
            const float w0 = -1.f * (ce * A.c[q0][c]);
            const float w1 = 1.f * (ce * A.c[q1][c]);
            Pn.a[ax][0][si] = hq[q0] ? Pc.a[ax][0][si] : b * (Pc.a[ax][0][si] + w0);
            Pn.a[ax][1][si] = hq[q1] ? Pc.a[ax][1][si] : b * (Pc.a[ax][1][si] + w1);
        }
    }
    if (do_inv && in_interior(g, i, j, k)) {
        const float *Ex = F.c[0], *Ey = F.c[1], *Ez = F.c[2];
        const float ex = Ex[c], ey = Ey[c], ez = Ez[c];
        const bool xi = i + 1 < g.nx, yj = j + 1 < g.ny, zk = k + 1 < g.nz;
        const float ey_x = xi ? Ey[c + 1] : 0.f, ez_x = xi ? Ez[c + 1] : 0.f;
        const float ex_y = yj ? Ex[c + g.nx] : 0.f, ez_y = yj ? Ez[c + g.nx] : 0.f;
        const float ex_z = zk ? Ex[c + g.nxy] : 0.f, ey_z = zk ? Ey[c + g.nxy] : 0.f;
        float hx = F.c[3][c], hy = F.c[4][c], hz = F.c[5][c];
        for (int s = 0; s < g.nsrc; s++) {
            if (k != g.sk[s] || g.scomp[s] < 3) continue;
            if (g.skind[s] == 0 && (i != g.si[s] || j != g.sj[s])) continue;
            const float Am = g.samp[s][n];
            if (g.scomp[s] == 3) hx = hx - Am;
            if (g.scomp[s] == 4) hy = hy - Am;
            if (g.scomp[s] == 5) hz = hz - Am;
        }
        F.c[3][c] = h_unupdate(hx, g.S, ez_y - ez, ey_z - ey);
        F.c[4][c] = h_unupdate(hy, g.S, ex_z - ex, ez_x - ez);
        F.c[5][c] = h_unupdate(hz, g.S, ey_x - ey, ex_y - ex);
    }
    if (do_adj) {
        // a conducting cell passes ca Ebar' on to E^n (its psi-bar is zero:
        // the lossy box lies in the interior)
        const long long li = lossy_index(g, i, j, k);
        if (li >= 0) {
            const float ca = g.lca[li];
            if (!held_ex(i, j, k)) A.c[0][c] = ca * A.c[0][c];
            if (!held_ey(i, j, k)) A.c[1][c] = ca * A.c[1][c];
            if (!held_ez(i, j, k)) A.c[2][c] = ca * A.c[2][c];
        }
        // Ebar_x: Hy along z (-S, z idx 3), Hz along y (+S, y idx 2)
        if (!held_ex(i, j, k)) {
            const float ra = r_hpair(g, A, Pc, 1, 2, 3, -1.f, i, j, k - 1) - r_hpair(g, A, Pc, 1, 2, 3, -1.f, i, j, k);
            const float rb = r_hpair(g, A, Pc, 2, 1, 2, 1.f, i, j - 1, k) - r_hpair(g, A, Pc, 2, 1, 2, 1.f, i, j, k);
            A.c[0][c] = A.c[0][c] + (ra + rb);
        }
        // Ebar_y: Hz along x (-S, x idx 3), Hx along z (+S, z idx 2)
        if (!held_ey(i, j, k)) {
            const float ra = r_hpair(g, A, Pc, 2, 0, 3, -1.f, i - 1, j, k) - r_hpair(g, A, Pc, 2, 0, 3, -1.f, i, j, k);
            const float rb = r_hpair(g, A, Pc, 0, 2, 2, 1.f, i, j, k - 1) - r_hpair(g, A, Pc, 0, 2, 2, 1.f, i, j, k);
            A.c[1][c] = A.c[1][c] + (ra + rb);
        }
        // Ebar_z: Hx along y (-S, y idx 3), Hy along x (+S, x idx 2)
        if (!held_ez(i, j, k)) {
            const float ra = r_hpair(g, A, Pc, 0, 1, 3, -1.f, i, j - 1, k) - r_hpair(g, A, Pc, 0, 1, 3, -1.f, i, j, k);
            const float rb = r_hpair(g, A, Pc, 1, 0, 2, 1.f, i - 1, j, k) - r_hpair(g, A, Pc, 1, 0, 2, 1.f, i, j, k);
            A.c[2][c] = A.c[2][c] + (ra + rb);
        }
        // H-type psibar of this cell into the next buffer
        if (g.p > 0) {
            const int cc[3] = {i, j, k};
            const int na[3] = {g.nx, g.ny, g.nz};
            for (int ax = 0; ax < 3; ax++) {
                const int s = slab_coord(cc[ax], na[ax], g.p);
                if (s < 0) continue;
                const long long si = slab_index(g, ax, s, i, j, k);
                const float b = g.prof[1][ax][0][cc[ax]];
                // idx 2: H comp (ax+1)%3 whose pair along ax has weight +S
                // idx 3: H comp (ax+2)%3 whose pair along ax has weight -S
                const int q2 = (ax + 1) % 3, q3 = (ax + 2) % 3;
                const float w2 = 1.f * (g.S * A.c[3 + q2][c]);
                const float w3 = -1.f * (g.S * A.c[3 + q3][c]);
                Pn.a[ax][2][si] = b * (Pc.a[ax][2][si] + w2);
                Pn.a[ax][3][si] = b * (Pc.a[ax][3][si] + w3);
            }
        }
    }
}

dim3 cell_grid(const Grid &g) { return dim3((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz); }

}  // namespace

hipError_t launch_h_naive(const Grid &g, const Fields &F, const Psi &P, int n, int with_src, hipStream_t s)
{
    hipLaunchKernelGGL(k_h_naive, cell_grid(g), dim3(BX, BY), 0, s, g, F, P, n, with_src);
    return hipGetLastError();
}

hipError_t launch_e_naive(const Grid &g, const Fields &F, const Psi &P, int n, int with_src, float *lrec,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_e_naive, cell_grid(g), dim3(BX, BY), 0, s, g, F, P, n, with_src, lrec);
    return hipGetLastError();
}

hipError_t launch_bwd_a(const Grid &g, const Fields &F, const Fields &A, const Psi &Pb, int n, int do_inv,
                        int do_adj, float *gacc, const int *dlo, const int *dhi, const float *lrec, hipStream_t s)
{
    hipLaunchKernelGGL(k_bwd_a, cell_grid(g), dim3(BX, BY), 0, s, g, F, A, Pb, n, do_inv, do_adj, gacc,
                       make_int3(dlo[0], dlo[1], dlo[2]), make_int3(dhi[0], dhi[1], dhi[2]), lrec);
    return hipGetLastError();
}

hipError_t launch_bwd_b(const Grid &g, const Fields &F, const Fields &A, const Psi &Pc, const Psi &Pn,
                        int n, int do_inv, int do_adj, hipStream_t s)
{
    hipLaunchKernelGGL(k_bwd_b, cell_grid(g), dim3(BX, BY), 0, s, g, F, A, Pc, Pn, n, do_inv, do_adj);
    return hipGetLastError();
}
