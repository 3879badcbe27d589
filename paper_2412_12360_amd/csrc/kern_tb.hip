// Temporally blocked forward pass: K leapfrog steps (arXiv 2412.12360,
// section 2.1) per sweep over the grid.
//
// Each workgroup owns a tile of TX x TY columns and a z range [z0, z1).  It
// loads the tile plus a K-cell halo in x and y and K planes below and above,
// and marches up in z one plane per iteration.  Level s (1..K) of the
// pipeline advances the fields from step n0+s-1 to n0+s and trails level s-1
// by one plane: its H update at plane k needs E of level s-1 at k and k+1, its
// E update needs its own H at k and k-1.  The x/y neighbours of a plane come
// from LDS, the z neighbours are held in registers.  The halo shrinks by one
// cell per level, so after K levels the owned tile is exact.  Fields and CPML
// auxiliaries are read from one buffer and written to the other (ping-pong).
// Sources, detector flux planes and the interface record are emitted at every
// level for owned cells, so the result is bitwise the same for every K.
#include "fdtd_internal.h"

namespace {

constexpr int EX = 64;

template <int K> struct TbShape;
template <> struct TbShape<1> { static constexpr int W = 8, R = 2; };
template <> struct TbShape<2> { static constexpr int W = 8, R = 2; };
template <> struct TbShape<3> { static constexpr int W = 8, R = 2; };
template <> struct TbShape<4> { static constexpr int W = 8, R = 2; };

__device__ __forceinline__ int remap_xcd(int b, int nb)
{
    const int q = nb / 8, rem = nb % 8;
    const int xcd = b % 8, slot = b / 8;
    return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

// CPML auxiliaries of one column at one plane: z-slab pairs (always present in
// the registers) and, for tiles that touch the x/y slabs, x- and y-slab pairs.
// Index order per axis as in the slab arrays: E (a+1)%3, E (a+2)%3, H (a+1)%3, H (a+2)%3.
template <bool XY> struct PsiReg;
template <> struct PsiReg<false> { float z[4]; };
template <> struct PsiReg<true> { float z[4], x[4], y[4]; };

template <bool XY> __device__ __forceinline__ void psi_zero(PsiReg<XY> &p)
{
#pragma unroll
    for (int q = 0; q < 4; q++) p.z[q] = 0.f;
    if constexpr (XY) {
#pragma unroll
        for (int q = 0; q < 4; q++) { p.x[q] = 0.f; p.y[q] = 0.f; }
    }
}

template <int K, bool XY>
__global__ __launch_bounds__(EX * TbShape<K>::W) void k_tb_forward(TbArgs A)
{
    constexpr int W = TbShape<K>::W, R = TbShape<K>::R;
    constexpr int EY = W * R, TX = EX - 2 * K, TY = EY - 2 * K;
    __shared__ float sE[3][EY][EX];
    __shared__ float sH[3][EY][EX];

    const Grid &g = A.g;
    int b = blockIdx.x;
    if (A.xcd_remap) b = remap_xcd(b, gridDim.x);
    const int4 tl = A.tiles[b];
    const int x0 = tl.x, y0 = tl.y, z0 = tl.z, z1 = tl.w;
    const int lane = threadIdx.x & (EX - 1);
    const int wv = threadIdx.x / EX;
    const int x = x0 - K + lane;
    const bool inx = x >= 0 && x < g.nx;
    const bool ownx = x >= x0 && x < x0 + TX && x < g.nx;
    const int p = g.p;
    const int sx = (XY && inx && p > 0) ? slab_coord(x, g.nx, p) : -1;

    int ys[R], row[R], sy[R];
    bool incol[R], own[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        row[r] = wv * R + r;
        ys[r] = y0 - K + row[r];
        incol[r] = inx && ys[r] >= 0 && ys[r] < g.ny;
        own[r] = ownx && ys[r] >= y0 && ys[r] < y0 + TY && ys[r] < g.ny;
        sy[r] = (XY && incol[r] && p > 0) ? slab_coord(ys[r], g.ny, p) : -1;
    }

    // pipeline registers: Eo[s], Ho[s], Po[s] = output of level s at the plane
    // level s+1 works on next; Ho[K] = last H of level K; cd[s] = S/eps of the
    // plane level s works on.
    float Eo[K][R][3], Ho[K + 1][R][3], cd[K + 1][R];
    PsiReg<XY> Po[K][R];
#pragma unroll
    for (int s = 0; s <= K; s++)
#pragma unroll
        for (int r = 0; r < R; r++) {
            cd[s][r] = 0.f;
#pragma unroll
            for (int q = 0; q < 3; q++) {
                Ho[s][r][q] = 0.f;
                if (s < K) Eo[s][r][q] = 0.f;
            }
            if (s < K) psi_zero<XY>(Po[s][r]);
        }

    const long long nxy = g.nxy;
    const int zlo = z0 - K;

    for (int t = zlo; t < z1 + K; t++) {
        // ---------------------------------------------------- level 0: load plane t
        float nE[R][3], nH[R][3];
        PsiReg<XY> nP[R];
        const bool tin = t >= 0 && t < g.nz;
        const int szt = (tin && p > 0) ? slab_coord(t, g.nz, p) : -1;
#pragma unroll
        for (int r = 0; r < R; r++) {
            psi_zero<XY>(nP[r]);
            float ce = 0.f;
            if (incol[r] && tin) {
                const long long c = (long long)t * nxy + (long long)ys[r] * g.nx + x;
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    nE[r][q] = A.in.c[q][c];
                    nH[r][q] = A.in.c[3 + q][c];
                }
                ce = g.ce[c];
                if (szt >= 0) {
                    const long long zi = slab_index(g, 2, szt, x, ys[r], t);
#pragma unroll
                    for (int q = 0; q < 4; q++) nP[r].z[q] = A.pin.a[2][q][zi];
                }
                if constexpr (XY) {
                    if (sx >= 0) {
                        const long long xi = slab_index(g, 0, sx, x, ys[r], t);
#pragma unroll
                        for (int q = 0; q < 4; q++) nP[r].x[q] = A.pin.a[0][q][xi];
                    }
                    if (sy[r] >= 0) {
                        const long long yi = slab_index(g, 1, sy[r], x, ys[r], t);
#pragma unroll
                        for (int q = 0; q < 4; q++) nP[r].y[q] = A.pin.a[1][q][yi];
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < 3; q++) { nE[r][q] = 0.f; nH[r][q] = 0.f; }
            }
#pragma unroll
            for (int s = K; s > 0; s--) cd[s][r] = cd[s - 1][r];
            cd[0][r] = ce;
        }

        // ------------------------------------------------------ levels 1..K
#pragma unroll
        for (int s = 1; s <= K; s++) {
            const int k = t - s;
            float mE[R][3], mH[R][3];
            PsiReg<XY> mP[R];
            if (k >= zlo) {
                const bool kin = k >= 0 && k < g.nz;
                const int szk = (kin && p > 0) ? slab_coord(k, g.nz, p) : -1;
                // E of level s-1 at plane k into LDS
#pragma unroll
                for (int r = 0; r < R; r++)
#pragma unroll
                    for (int q = 0; q < 3; q++) sE[q][row[r]][lane] = Eo[s - 1][r][q];
                __syncthreads();
                // ---- H half step at plane k
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const float ex = Eo[s - 1][r][0], ey = Eo[s - 1][r][1], ez = Eo[s - 1][r][2];
                    const float ex_z = nE[r][0], ey_z = nE[r][1];
                    const bool up = row[r] + 1 < EY, rt = lane + 1 < EX;
                    const float ez_y = up ? sE[2][row[r] + 1][lane] : 0.f;
                    const float ex_y = up ? sE[0][row[r] + 1][lane] : 0.f;
                    const float ey_x = rt ? sE[1][row[r]][lane + 1] : 0.f;
                    const float ez_x = rt ? sE[2][row[r]][lane + 1] : 0.f;
                    float dy_ez = ez_y - ez, dz_ey = ey_z - ey;
                    float dz_ex = ex_z - ex, dx_ez = ez_x - ez;
                    float dx_ey = ey_x - ey, dy_ex = ex_y - ex;
                    mP[r] = Po[s - 1][r];
                    if (szk >= 0) {   // Hx (idx 2), Hy (idx 3) along z
                        const float bb = g.prof[1][2][0][k], aa = g.prof[1][2][1][k], kv = g.prof[1][2][2][k];
                        dz_ey = cpml_term(dz_ey, mP[r].z[2], bb, aa, kv);
                        dz_ex = cpml_term(dz_ex, mP[r].z[3], bb, aa, kv);
                    }
                    if constexpr (XY) {
                        if (sx >= 0) {   // Hy (idx 2), Hz (idx 3) along x
                            const float bb = g.prof[1][0][0][x], aa = g.prof[1][0][1][x], kv = g.prof[1][0][2][x];
                            dx_ez = cpml_term(dx_ez, mP[r].x[2], bb, aa, kv);
                            dx_ey = cpml_term(dx_ey, mP[r].x[3], bb, aa, kv);
                        }
                        if (sy[r] >= 0) {   // Hz (idx 2), Hx (idx 3) along y
                            const int yy = ys[r];
                            const float bb = g.prof[1][1][0][yy], aa = g.prof[1][1][1][yy], kv = g.prof[1][1][2][yy];
                            dy_ex = cpml_term(dy_ex, mP[r].y[2], bb, aa, kv);
                            dy_ez = cpml_term(dy_ez, mP[r].y[3], bb, aa, kv);
                        }
                    }
                    const bool live = incol[r] && kin;
                    mH[r][0] = live ? h_update(Ho[s - 1][r][0], g.S, dy_ez, dz_ey) : 0.f;
                    mH[r][1] = live ? h_update(Ho[s - 1][r][1], g.S, dz_ex, dx_ez) : 0.f;
                    mH[r][2] = live ? h_update(Ho[s - 1][r][2], g.S, dx_ey, dy_ex) : 0.f;
#pragma unroll
                    for (int q = 0; q < 3; q++) sH[q][row[r]][lane] = mH[r][q];
                }
                __syncthreads();
                // ---- E half step at plane k
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const float hx = mH[r][0], hy = mH[r][1], hz = mH[r][2];
                    const float hx_z = Ho[s][r][0], hy_z = Ho[s][r][1];
                    const bool dn = row[r] > 0, lf = lane > 0;
                    const float hz_y = dn ? sH[2][row[r] - 1][lane] : 0.f;
                    const float hx_y = dn ? sH[0][row[r] - 1][lane] : 0.f;
                    const float hz_x = lf ? sH[2][row[r]][lane - 1] : 0.f;
                    const float hy_x = lf ? sH[1][row[r]][lane - 1] : 0.f;
                    float dy_hz = hz - hz_y, dz_hy = hy - hy_z;
                    float dz_hx = hx - hx_z, dx_hz = hz - hz_x;
                    float dx_hy = hy - hy_x, dy_hx = hx - hx_y;
                    const int yy = ys[r];
                    const bool hex = yy == 0 || k == 0, hey = x == 0 || k == 0, hez = x == 0 || yy == 0;
                    if (szk >= 0) {   // Ex (idx 0), Ey (idx 1) along z
                        const float bb = g.prof[0][2][0][k], aa = g.prof[0][2][1][k], kv = g.prof[0][2][2][k];
                        if (!hex) dz_hy = cpml_term(dz_hy, mP[r].z[0], bb, aa, kv);
                        if (!hey) dz_hx = cpml_term(dz_hx, mP[r].z[1], bb, aa, kv);
                    }
                    if constexpr (XY) {
                        if (sx >= 0) {   // Ey (idx 0), Ez (idx 1) along x
                            const float bb = g.prof[0][0][0][x], aa = g.prof[0][0][1][x], kv = g.prof[0][0][2][x];
                            if (!hey) dx_hz = cpml_term(dx_hz, mP[r].x[0], bb, aa, kv);
                            if (!hez) dx_hy = cpml_term(dx_hy, mP[r].x[1], bb, aa, kv);
                        }
                        if (sy[r] >= 0) {   // Ez (idx 0), Ex (idx 1) along y
                            const float bb = g.prof[0][1][0][yy], aa = g.prof[0][1][1][yy], kv = g.prof[0][1][2][yy];
                            if (!hez) dy_hx = cpml_term(dy_hx, mP[r].y[0], bb, aa, kv);
                            if (!hex) dy_hz = cpml_term(dy_hz, mP[r].y[1], bb, aa, kv);
                        }
                    }
                    const float ce = cd[s][r];
                    float ex = Eo[s - 1][r][0], ey = Eo[s - 1][r][1], ez = Eo[s - 1][r][2];
                    if (!hex) ex = e_update(ex, ce, dy_hz, dz_hy);
                    if (!hey) ey = e_update(ey, ce, dz_hx, dx_hz);
                    if (!hez) ez = e_update(ez, ce, dx_hy, dy_hx);
                    if (A.with_src) {
                        for (int q = 0; q < g.nsrc; q++) {
                            if (k != g.sk[q]) continue;
                            if (g.skind[q] == 0 && (x != g.si[q] || yy != g.sj[q])) continue;
                            const float am = g.samp[q][A.n0 + s - 1];
                            if (g.scomp[q] == 0 && !hex) ex = ex + am;
                            if (g.scomp[q] == 1 && !hey) ey = ey + am;
                            if (g.scomp[q] == 2 && !hez) ez = ez + am;
                        }
                    }
                    const bool live = incol[r] && kin;
                    mE[r][0] = live ? ex : 0.f;
                    mE[r][1] = live ? ey : 0.f;
                    mE[r][2] = live ? ez : 0.f;

                    // ---- outputs of this step for owned cells
                    if (own[r] && k >= z0 && k < z1) {
                        const long long step = A.n0 + s - 1;
                        if (A.planes) {
                            for (int m = 0; m < A.D.ndet; m++) {
                                if (k != A.D.k[m] || x < A.D.i0[m] || x >= A.D.i1[m] || yy < A.D.j0[m] ||
                                    yy >= A.D.j1[m])
                                    continue;
                                const long long e = A.D.off[m] + (long long)(yy - A.D.j0[m]) * (A.D.i1[m] - A.D.i0[m]) +
                                                    (x - A.D.i0[m]);
                                A.planes[(long long)(s - 1) * A.D.per_step + e] =
                                    flux_density(mE[r][0], mE[r][1], mH[r][0], mH[r][1]);
                            }
                        }
                        if (A.rec && p > 0) {
                            float *rs = A.rec + (long long)(s - 1) * A.R.per_step;
                            const bool wx = x >= p && x < g.nx - p, wy = yy >= p && yy < g.ny - p,
                                       wz = k >= p && k < g.nz - p;
                            // z faces: u = x, v = y
                            if (wx && wy && (k == p - 1 || k == g.nz - p)) {
                                const int side = k == p - 1 ? 0 : 1;
                                const long long fs = (long long)A.R.Lu[2] * A.R.Lv[2];
                                const long long e = A.R.off[4 + side] + (long long)(yy - p) * A.R.Lu[2] + (x - p);
                                rs[e] = side ? mE[r][0] : mH[r][0];
                                rs[e + fs] = side ? mE[r][1] : mH[r][1];
                            }
                            // x faces: u = y, v = z; comps (y, z)
                            if (wy && wz && (x == p - 1 || x == g.nx - p)) {
                                const int side = x == p - 1 ? 0 : 1;
                                const long long fs = (long long)A.R.Lu[0] * A.R.Lv[0];
                                const long long e = A.R.off[0 + side] + (long long)(k - p) * A.R.Lu[0] + (yy - p);
                                rs[e] = side ? mE[r][1] : mH[r][1];
                                rs[e + fs] = side ? mE[r][2] : mH[r][2];
                            }
                            // y faces: u = x, v = z; comps (z, x)
                            if (wx && wz && (yy == p - 1 || yy == g.ny - p)) {
                                const int side = yy == p - 1 ? 0 : 1;
                                const long long fs = (long long)A.R.Lu[1] * A.R.Lv[1];
                                const long long e = A.R.off[2 + side] + (long long)(k - p) * A.R.Lu[1] + (x - p);
                                rs[e] = side ? mE[r][2] : mH[r][2];
                                rs[e + fs] = side ? mE[r][0] : mH[r][0];
                            }
                        }
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; r++) {
#pragma unroll
                    for (int q = 0; q < 3; q++) { mE[r][q] = 0.f; mH[r][q] = 0.f; }
                    psi_zero<XY>(mP[r]);
                }
            }
            // rotate level s-1: its new plane becomes the one level s reads next
#pragma unroll
            for (int r = 0; r < R; r++) {
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    Eo[s - 1][r][q] = nE[r][q];
                    Ho[s - 1][r][q] = nH[r][q];
                    nE[r][q] = mE[r][q];
                    nH[r][q] = mH[r][q];
                }
                Po[s - 1][r] = nP[r];
                nP[r] = mP[r];
            }
        }

        // ---------------------------------------------------- level K: store
        const int kK = t - K;
#pragma unroll
        for (int r = 0; r < R; r++) {
#pragma unroll
            for (int q = 0; q < 3; q++) Ho[K][r][q] = nH[r][q];
            if (own[r] && kK >= z0 && kK < z1) {
                const long long c = (long long)kK * nxy + (long long)ys[r] * g.nx + x;
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    A.out.c[q][c] = nE[r][q];
                    A.out.c[3 + q][c] = nH[r][q];
                }
                const int szo = p > 0 ? slab_coord(kK, g.nz, p) : -1;
                if (szo >= 0) {
                    const long long zi = slab_index(g, 2, szo, x, ys[r], kK);
#pragma unroll
                    for (int q = 0; q < 4; q++) A.pout.a[2][q][zi] = nP[r].z[q];
                }
                if constexpr (XY) {
                    if (sx >= 0) {
                        const long long xi = slab_index(g, 0, sx, x, ys[r], kK);
#pragma unroll
                        for (int q = 0; q < 4; q++) A.pout.a[0][q][xi] = nP[r].x[q];
                    }
                    if (sy[r] >= 0) {
                        const long long yi = slab_index(g, 1, sy[r], x, ys[r], kK);
#pragma unroll
                        for (int q = 0; q < 4; q++) A.pout.a[1][q][yi] = nP[r].y[q];
                    }
                }
            }
        }
    }
}

template <int K>
hipError_t launch_k(const TbArgs &a, bool xy, hipStream_t s)
{
    constexpr int threads = EX * TbShape<K>::W;
    if (a.ntiles <= 0) return hipSuccess;
    if (xy)
        hipLaunchKernelGGL((k_tb_forward<K, true>), dim3(a.ntiles), dim3(threads), 0, s, a);
    else
        hipLaunchKernelGGL((k_tb_forward<K, false>), dim3(a.ntiles), dim3(threads), 0, s, a);
    return hipGetLastError();
}

}  // namespace

int tb_tile_x(int K) { return EX - 2 * K; }

int tb_tile_y(int K)
{
    switch (K) {
    case 1: return TbShape<1>::W * TbShape<1>::R - 2;
    case 2: return TbShape<2>::W * TbShape<2>::R - 4;
    case 3: return TbShape<3>::W * TbShape<3>::R - 6;
    default: return TbShape<4>::W * TbShape<4>::R - 8;
    }
}

// a.ntiles > 0 tiles of one class; xy selects the instance with x/y CPML
hipError_t launch_tb_forward_class(const TbArgs &a, int K, bool xy, hipStream_t s)
{
    switch (K) {
    case 1: return launch_k<1>(a, xy, s);
    case 2: return launch_k<2>(a, xy, s);
    case 3: return launch_k<3>(a, xy, s);
    case 4: return launch_k<4>(a, xy, s);
    default: return hipErrorInvalidValue;
    }
}
