// Temporally blocked forward pass: K leapfrog steps (arXiv 2412.12360,
// section 2.1) per sweep over the grid.
//
// Each workgroup owns a tile of columns [x0,x1) x [y0,y1) and a z range
// [z0, z1).  It reads the tile plus a K-cell halo in x and y and K planes
// below and above, and marches up in z one plane per iteration, fetching the
// next plane from HBM while it computes on the current one.  Level s (1..K)
// of the pipeline advances the fields from step n0+s-1 to n0+s and trails
// level s-1 by one plane: its H update at plane k needs E of level s-1 at k
// and k+1, its E update needs its own H at k and k-1.  The x/y neighbours of
// a plane come from LDS, the z neighbours are held in registers.  The halo
// shrinks by one cell per level, so after K levels the owned tile is exact.
// Fields and CPML auxiliaries are read from one buffer and written to the
// other (ping-pong).  Sources, detector flux planes and the interface record
// are emitted at every level for owned cells, so the result is bitwise the
// same for every K and equal to the per-cell kernels.
//
// Tiles come in four classes by which CPML slabs (x, y) reach into their
// halo-extended footprint; each class is its own instance so interior tiles
// carry no x/y auxiliary registers.  z-slab planes are handled in every tile.
//
// Cost notes: cell addresses are 32-bit byte offsets from one base per field
// set (one uniform plane term plus one per-row offset; grids whose field set
// spans 4 GiB or more take the WIDE instance instead: a 64-bit uniform base
// per component and plane, 32-bit offsets within the plane), the
// conducting-wall rule is folded into the
// update coefficient (a held component gets coefficient 0, which leaves it
// bit-for-bit unchanged), and records, detectors and sources are gated by
// uniform plane tests so the common plane pays nothing for them.
#include "fdtd_internal.h"

namespace {

constexpr int TB_MAXP = 64;   // largest CPML thickness the z-march kernel stages


// a float at a 32-bit byte offset from a uniform base (lets the compiler use
// the scalar-base + vector-offset addressing form)
__device__ __forceinline__ float ldo(const float *__restrict__ base, unsigned byteoff)
{
    return *(const float *)((const char *)base + byteoff);
}
// (non-temporal: the march never reads back what it writes in this sweep;
// 0.3-0.8% faster than plain stores)
__device__ __forceinline__ void sto(float *__restrict__ base, unsigned byteoff, float v)
{
    __builtin_nontemporal_store(v, (float *)((char *)base + byteoff));
}

__device__ __forceinline__ int remap_xcd(int b, int nb)
{
    const int q = nb / 8, rem = nb % 8;
    const int xcd = b % 8, slot = b / 8;
    return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

// CPML auxiliaries of one column at one plane.  Per axis, as in the slab
// arrays: E (a+1)%3, E (a+2)%3, H (a+1)%3, H (a+2)%3.
template <bool XP, bool YP> struct PsiReg {
    float z[4];
    float x[XP ? 4 : 1];
    float y[YP ? 4 : 1];
};

template <int R, bool XP, bool YP> struct Plane {
    float e[R][3], h[R][3], ce[R];
    PsiReg<XP, YP> p[R];
};

template <bool XP, bool YP> __device__ __forceinline__ void psi_zero(PsiReg<XP, YP> &p)
{
#pragma unroll
    for (int q = 0; q < 4; q++) p.z[q] = 0.f;
    if constexpr (XP) {
#pragma unroll
        for (int q = 0; q < 4; q++) p.x[q] = 0.f;
    }
    if constexpr (YP) {
#pragma unroll
        for (int q = 0; q < 4; q++) p.y[q] = 0.f;
    }
}

// psi of a held component is not advanced
__device__ __forceinline__ float cpml_term_h(float d, float &psi, float b, float a, float kinv, bool held)
{
    const float np = fmaf(b, psi, a * d);
    psi = held ? psi : np;
    return fmaf(d, kinv, psi);
}

// The handle's fixed arguments and the launch's per-request arguments, read
// with scalar loads from constant memory.
typedef const __attribute__((address_space(4))) TbArgs KArgs;
typedef const __attribute__((address_space(4))) TbReq KReq;
typedef const __attribute__((address_space(4))) TbLaunch KLaunch;

// One tile's march.  TX lanes of a wave row span x; W waves; R rows per
// thread.  The LDS arrays belong to the kernel (one set whatever the class).
// LOSSY: the instance for handles with conducting cells: in the lossy box E
// is damped, E' = ca E + cb curl H (cb in place of S/eps in the coefficient
// array), and E^n of the box goes into the record before the update.
template <int K, bool XP, bool YP, int PD, int W, int R, int TX, bool WIDE, bool LOSSY>
__device__ __forceinline__ void tb_march(KArgs &A, KArgs *Kp, KReq *Rq, const int4 tl, const int4 tz,
                                         float (*sE)[(64 * W / TX) * R + 1][TX],
                                         float (*sH)[(64 * W / TX) * R + 1][TX], float (*sGz)[6],
                                         float (*sAmp)[K])
{
    constexpr int EX = TX;
    constexpr int EY = (64 * W / TX) * R;
    const int n0 = Rq->n0;
    const unsigned ic = Rq->flags & TB_CUR;   // input buffer set
    const bool with_src = (Rq->flags & TB_SRC) != 0;
    float *const rec_n0 = Rq->rec;
    float *const planes = Rq->planes;
    float *const raw_n0 = Rq->raw;

    const int nx = A.g.nx, ny = A.g.ny, nz = A.g.nz, p = A.g.p;
    for (int e = threadIdx.x; e < 2 * p; e += blockDim.x) {
        const int kk = e < p ? e : nz - 2 * p + e;
        const float4 gE = A.profv[2][2 * kk], gH = A.profv[2][2 * kk + 1];
        sGz[e][0] = gE.x; sGz[e][1] = gE.y; sGz[e][2] = gE.z;
        sGz[e][3] = gH.x; sGz[e][4] = gH.y; sGz[e][5] = gH.z;
    }
    if ((int)threadIdx.x < FD_MAXSRC * K) {
        const int q = threadIdx.x / K, s = threadIdx.x % K;
        sAmp[q][s] = (with_src && q < A.g.nsrc) ? A.g.samp[q][n0 + s] : 0.f;
    }
    __syncthreads();
    const unsigned nxy = (unsigned)A.g.nxy;
    const float S = A.g.S;
    const int x0 = tl.x, x1 = tl.y, y0 = tl.z, y1 = tl.w, z0 = tz.x, z1 = tz.y;
    const bool active = (int)threadIdx.x < EX * (EY / R);
    const int lane = active ? (int)threadIdx.x % EX : 0;
    const int wv = active ? (int)threadIdx.x / EX : EY / R;
    const int x = x0 - K + lane;
    const bool inx = active && x >= 0 && x < nx;
    const int xc = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
    const int sx = (XP && inx) ? slab_coord(x, nx, p) : -1;

    // per-column CPML grading along x and y (E then H: b, a, 1/kappa)
    float4 gxE = make_float4(1.f, 0.f, 1.f, 0.f), gxH = gxE;
    if constexpr (XP) {
        if (sx >= 0) { gxE = A.profv[0][2 * x]; gxH = A.profv[0][2 * x + 1]; }
    }
    int ys[R], row[R], sy[R];
    unsigned off[R], soff_x[R], soff_y[R];
    bool incol[R], own[R];
    float mex[R], mey[R], mez[R];   // 1 unless a conducting wall holds the component
    float4 gyE[YP ? R : 1], gyH[YP ? R : 1];
#pragma unroll
    for (int r = 0; r < R; r++) {
        row[r] = active ? wv * R + r : EY;   // idle threads share the spare row
        ys[r] = y0 - K + row[r];
        incol[r] = inx && ys[r] >= 0 && ys[r] < ny;
        own[r] = x >= x0 && x < x1 && ys[r] >= y0 && ys[r] < y1;
        const int yc = ys[r] < 0 ? 0 : (ys[r] >= ny ? ny - 1 : ys[r]);
        off[r] = (unsigned)yc * (unsigned)nx + (unsigned)xc;
        sy[r] = (YP && incol[r]) ? slab_coord(ys[r], ny, p) : -1;
        mex[r] = ys[r] == 0 ? 0.f : 1.f;
        mey[r] = x == 0 ? 0.f : 1.f;
        mez[r] = (x == 0 || ys[r] == 0) ? 0.f : 1.f;
        // slab offsets without the plane term
        soff_x[r] = sx >= 0 ? (unsigned)yc * (unsigned)(2 * p) + (unsigned)sx : 0u;
        soff_y[r] = sy[r] >= 0 ? (unsigned)sy[r] * (unsigned)nx + (unsigned)xc : 0u;
        if constexpr (YP) {
            gyE[r] = make_float4(1.f, 0.f, 1.f, 0.f);
            gyH[r] = gyE[r];
            if (sy[r] >= 0) { gyE[r] = A.profv[1][2 * ys[r]]; gyH[r] = A.profv[1][2 * ys[r] + 1]; }
        }
    }

    // one base per buffer set: component q of a field set at q * fs bytes,
    // CPML auxiliary q of axis a at q * A.pstride[a] bytes (32-bit offsets)
    const float *__restrict__ iF = A.fld[ic][0];
    const float *__restrict__ ice = A.g.ce;
    const unsigned fs = A.fstride;

    // Arguments used only now and then are read through a copy of the
    // argument pointer that is made opaque on every plane, so they are fetched
    // where they are used instead of being held in scalar registers for the
    // whole march (the argument block is the kernel's only parameter, at
    // offset 0 of the kernel-argument segment): the source arguments, and the
    // component bases of the WIDE instance.

    auto load_plane = [&](int t, Plane<R, XP, YP> &P) {
        const bool tin = t >= 0 && t < nz;
        if constexpr (WIDE) {
            const size_t pb = (size_t)(tin ? t : 0) * (size_t)Kp->g.nxy;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const unsigned c = off[r] * 4u;
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    P.e[r][q] = ldo(Kp->fld[ic][q] + pb, c);
                    P.h[r][q] = ldo(Kp->fld[ic][3 + q] + pb, c);
                }
                P.ce[r] = ldo(Kp->g.ce + pb, c);
                psi_zero<XP, YP>(P.p[r]);
            }
        } else {
            const unsigned base = (unsigned)(tin ? t : 0) * nxy;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const unsigned c = (base + off[r]) * 4u;
                // raw values: columns and planes outside the grid are zeroed where
                // the plane is consumed, so the fetch stays in flight until then
                P.e[r][0] = ldo(iF, c); P.e[r][1] = ldo(iF, c + fs); P.e[r][2] = ldo(iF, c + 2 * fs);
                P.h[r][0] = ldo(iF, c + 3 * fs); P.h[r][1] = ldo(iF, c + 4 * fs); P.h[r][2] = ldo(iF, c + 5 * fs);
                P.ce[r] = ldo(ice, c);
                psi_zero<XP, YP>(P.p[r]);
            }
        }
        if (p > 0 && tin) {
            const int szt = slab_coord(t, nz, p);
            if (szt >= 0) {
                const unsigned zb = (unsigned)szt * nxy;
                const unsigned ps = A.pstride[2];
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const unsigned o = (zb + off[r]) * 4u;
#pragma unroll
                    for (int q = 0; q < 4; q++) P.p[r].z[q] = ldo(A.psi[ic][2], o + q * ps);
                }
            }
            if constexpr (XP) {
                const unsigned xb = (unsigned)t * (unsigned)ny * (unsigned)(2 * p);
                const unsigned ps = A.pstride[0];
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const unsigned o = (xb + soff_x[r]) * 4u;
#pragma unroll
                    for (int q = 0; q < 4; q++) P.p[r].x[q] = ldo(A.psi[ic][0], o + q * ps);
                }
            }
            if constexpr (YP) {
                const unsigned yb = (unsigned)t * (unsigned)(2 * p) * (unsigned)nx;
                const unsigned ps = A.pstride[1];
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const unsigned o = (yb + soff_y[r]) * 4u;
#pragma unroll
                    for (int q = 0; q < 4; q++) P.p[r].y[q] = ldo(A.psi[ic][1], o + q * ps);
                }
            }
        }
    };

    // source planes (uniform; -2^31 for an absent source), hoisted so the
    // per-level test issues no scalar memory load
    int skq[FD_MAXSRC];
#pragma unroll
    for (int q = 0; q < FD_MAXSRC; q++) skq[q] = (with_src && q < A.g.nsrc) ? A.g.sk[q] : (-2147483647 - 1);
    // The other source arguments are read through the opaque argument
    // pointer Kp (below).

    // pipeline registers: Eo[s], Ho[s]/Hc[s], Po[s] = output of level s at the
    // plane level s+1 works on next; Ho[K] = last Hx, Hy of level K; cd[s] =
    // S/eps of the plane level s works on.
    float Eo[K][R][3], Ho[K + 1][R][2], Hc[K][R], cd[K + 1][R];
    PsiReg<XP, YP> Po[K][R];
#pragma unroll
    for (int s = 0; s <= K; s++)
#pragma unroll
        for (int r = 0; r < R; r++) {
            cd[s][r] = 0.f;
            Ho[s][r][0] = Ho[s][r][1] = 0.f;
            if (s < K) {
                Eo[s][r][0] = Eo[s][r][1] = Eo[s][r][2] = 0.f;
                Hc[s][r] = 0.f;
                psi_zero<XP, YP>(Po[s][r]);
            }
        }

    const int zlo = z0 - K;
    const int zend = z1 + K;

    auto body = [&](const int t, const Plane<R, XP, YP> &cur) {
        float nE[R][3], nH[R][3];
        PsiReg<XP, YP> nP[R];
        const bool tin = t >= 0 && t < nz;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const bool v = tin && incol[r];
#pragma unroll
            for (int q = 0; q < 3; q++) {
                nE[r][q] = v ? cur.e[r][q] : 0.f;
                nH[r][q] = v ? cur.h[r][q] : 0.f;
            }
            nP[r] = cur.p[r];
#pragma unroll
            for (int s = K; s > 0; s--) cd[s][r] = cd[s - 1][r];
            cd[0][r] = v ? cur.ce[r] : 0.f;
        }
#pragma unroll
        for (int s = 1; s <= K; s++) {
            const int k = t - s;
            float mE[R][3], mH[R][3];
            PsiReg<XP, YP> mP[R];
            if (k >= zlo) {
                const bool kin = k >= 0 && k < nz;
                const int szk = (kin && p > 0) ? slab_coord(k, nz, p) : -1;
                float4 gzE = make_float4(1.f, 0.f, 1.f, 0.f), gzH = gzE;
                if (szk >= 0) {
                    gzE = make_float4(sGz[szk][0], sGz[szk][1], sGz[szk][2], 0.f);
                    gzH = make_float4(sGz[szk][3], sGz[szk][4], sGz[szk][5], 0.f);
                }
                const float mk = k == 0 ? 0.f : 1.f;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    sE[0][row[r]][lane] = Eo[s - 1][r][0];
                    sE[1][row[r]][lane] = Eo[s - 1][r][1];
                    sE[2][row[r]][lane] = Eo[s - 1][r][2];
                }
                __syncthreads();
                // ---- H half step at plane k
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const float ex = Eo[s - 1][r][0], ey = Eo[s - 1][r][1], ez = Eo[s - 1][r][2];
                    const float ex_z = nE[r][0], ey_z = nE[r][1];
                    const int ru = row[r] + 1 < EY ? row[r] + 1 : row[r];
                    const int lr = lane + 1 < EX ? lane + 1 : lane;
                    const float ez_y = sE[2][ru][lane], ex_y = sE[0][ru][lane];
                    const float ey_x = sE[1][row[r]][lr], ez_x = sE[2][row[r]][lr];
                    float dy_ez = ez_y - ez, dz_ey = ey_z - ey;
                    float dz_ex = ex_z - ex, dx_ez = ez_x - ez;
                    float dx_ey = ey_x - ey, dy_ex = ex_y - ex;
                    mP[r] = Po[s - 1][r];
                    if (szk >= 0) {   // Hx (idx 2), Hy (idx 3) along z
                        dz_ey = cpml_term(dz_ey, mP[r].z[2], gzH.x, gzH.y, gzH.z);
                        dz_ex = cpml_term(dz_ex, mP[r].z[3], gzH.x, gzH.y, gzH.z);
                    }
                    if constexpr (XP) {
                        if (sx >= 0) {   // Hy (idx 2), Hz (idx 3) along x
                            dx_ez = cpml_term(dx_ez, mP[r].x[2], gxH.x, gxH.y, gxH.z);
                            dx_ey = cpml_term(dx_ey, mP[r].x[3], gxH.x, gxH.y, gxH.z);
                        }
                    }
                    if constexpr (YP) {
                        if (sy[r] >= 0) {   // Hz (idx 2), Hx (idx 3) along y
                            dy_ex = cpml_term(dy_ex, mP[r].y[2], gyH[r].x, gyH[r].y, gyH[r].z);
                            dy_ez = cpml_term(dy_ez, mP[r].y[3], gyH[r].x, gyH[r].y, gyH[r].z);
                        }
                    }
                    const bool live = incol[r] && kin;
                    mH[r][0] = live ? h_update(Ho[s - 1][r][0], S, dy_ez, dz_ey) : 0.f;
                    mH[r][1] = live ? h_update(Ho[s - 1][r][1], S, dz_ex, dx_ez) : 0.f;
                    mH[r][2] = live ? h_update(Hc[s - 1][r], S, dx_ey, dy_ex) : 0.f;
                }
                // ---- H sources (components 3..5), before any E update reads
                // this plane's H; same uniform plane test as the E sources
#pragma unroll
                for (int q = 0; q < FD_MAXSRC; q++) {
                    if (k == skq[q]) {
                        const float am = sAmp[q][s - 1];
                        const int comp = Kp->g.scomp[q];
#pragma unroll
                        for (int r = 0; r < R; r++) {
                            const bool hit = incol[r] && kin &&
                                             (Kp->g.skind[q] == 1 || (x == Kp->g.si[q] && ys[r] == Kp->g.sj[q]));
                            mH[r][0] = (hit && comp == 3) ? mH[r][0] + am : mH[r][0];
                            mH[r][1] = (hit && comp == 4) ? mH[r][1] + am : mH[r][1];
                            mH[r][2] = (hit && comp == 5) ? mH[r][2] + am : mH[r][2];
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < R; r++) {
                    sH[0][row[r]][lane] = mH[r][0];
                    sH[1][row[r]][lane] = mH[r][1];
                    sH[2][row[r]][lane] = mH[r][2];
                }
                __syncthreads();
                // ---- E half step at plane k
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const float hx = mH[r][0], hy = mH[r][1], hz = mH[r][2];
                    const float hx_z = Ho[s][r][0], hy_z = Ho[s][r][1];
                    const int rd = row[r] > 0 ? row[r] - 1 : row[r];
                    const int ll = lane > 0 ? lane - 1 : lane;
                    const float hz_y = sH[2][rd][lane], hx_y = sH[0][rd][lane];
                    const float hz_x = sH[2][row[r]][ll], hy_x = sH[1][row[r]][ll];
                    float dy_hz = hz - hz_y, dz_hy = hy - hy_z;
                    float dz_hx = hx - hx_z, dx_hz = hz - hz_x;
                    float dx_hy = hy - hy_x, dy_hx = hx - hx_y;
                    const float ax = mex[r] * mk, ay = mey[r] * mk, az = mez[r];
                    if (szk >= 0) {   // Ex (idx 0), Ey (idx 1) along z
                        dz_hy = cpml_term_h(dz_hy, mP[r].z[0], gzE.x, gzE.y, gzE.z, ax == 0.f);
                        dz_hx = cpml_term_h(dz_hx, mP[r].z[1], gzE.x, gzE.y, gzE.z, ay == 0.f);
                    }
                    if constexpr (XP) {
                        if (sx >= 0) {   // Ey (idx 0), Ez (idx 1) along x
                            dx_hz = cpml_term_h(dx_hz, mP[r].x[0], gxE.x, gxE.y, gxE.z, ay == 0.f);
                            dx_hy = cpml_term_h(dx_hy, mP[r].x[1], gxE.x, gxE.y, gxE.z, az == 0.f);
                        }
                    }
                    if constexpr (YP) {
                        if (sy[r] >= 0) {   // Ez (idx 0), Ex (idx 1) along y
                            dy_hx = cpml_term_h(dy_hx, mP[r].y[0], gyE[r].x, gyE[r].y, gyE[r].z, az == 0.f);
                            dy_hz = cpml_term_h(dy_hz, mP[r].y[1], gyE[r].x, gyE[r].y, gyE[r].z, ax == 0.f);
                        }
                    }
                    const float ce = cd[s][r];
                    const bool live = incol[r] && kin;
                    float e0 = Eo[s - 1][r][0], e1 = Eo[s - 1][r][1], e2 = Eo[s - 1][r][2];
                    if constexpr (LOSSY) {
                        // a conducting cell: E^n into the record (owned cells), then ca E^n
                        if (live && k >= A.g.llo[2] && k < A.g.lhi[2] && x >= A.g.llo[0] && x < A.g.lhi[0] &&
                            ys[r] >= A.g.llo[1] && ys[r] < A.g.lhi[1]) {
                            const int bx = A.g.lhi[0] - A.g.llo[0], by = A.g.lhi[1] - A.g.llo[1];
                            const long long li = ((long long)(k - A.g.llo[2]) * by + (ys[r] - A.g.llo[1])) * bx +
                                                 (x - A.g.llo[0]);
                            if (own[r] && rec_n0 && k >= z0 && k < z1) {
                                const long long nb = (long long)bx * by * (A.g.lhi[2] - A.g.llo[2]);
                                float *lr = rec_n0 + (long long)(s - 1) * A.R.per_step + A.R.loff + li;
                                lr[0] = e0; lr[nb] = e1; lr[2 * nb] = e2;
                            }
                            const float ca = ldo(A.g.lca, (unsigned)li * 4u);
                            e0 = ca * e0; e1 = ca * e1; e2 = ca * e2;
                        }
                    }
                    const float ex = e_update(e0, ce * ax, dy_hz, dz_hy);
                    const float ey = e_update(e1, ce * ay, dz_hx, dx_hz);
                    const float ez = e_update(e2, ce * az, dx_hy, dy_hx);
                    mE[r][0] = live ? ex : 0.f;
                    mE[r][1] = live ? ey : 0.f;
                    mE[r][2] = live ? ez : 0.f;
                }
                // ---- E sources (uniform plane test against the hoisted source
                // planes: no scalar memory load on a plane without a source)
#pragma unroll
                for (int q = 0; q < FD_MAXSRC; q++) {
                    if (k == skq[q]) {
                        const float am = sAmp[q][s - 1];
                        const int comp = Kp->g.scomp[q];
#pragma unroll
                        for (int r = 0; r < R; r++) {
                            const bool hit = incol[r] && kin &&
                                             (Kp->g.skind[q] == 1 || (x == Kp->g.si[q] && ys[r] == Kp->g.sj[q]));
                            // one select per component, no component-indexed
                            // array (which the compiler would place in scratch);
                            // a held component takes no source
                            mE[r][0] = (hit && comp == 0 && mex[r] * mk != 0.f) ? mE[r][0] + am : mE[r][0];
                            mE[r][1] = (hit && comp == 1 && mey[r] * mk != 0.f) ? mE[r][1] + am : mE[r][1];
                            mE[r][2] = (hit && comp == 2 && mez[r] != 0.f) ? mE[r][2] + am : mE[r][2];
                        }
                    }
                }
                // ---- detector flux planes (uniform plane test)
                if (planes && k >= z0 && k < z1 && k >= A.D.kmin && k <= A.D.kmax) {
                    for (int m = 0; m < A.D.ndet; m++) {
                        // an energy detector also takes Ez of the layer below its plane
                        const bool at = k == A.D.k[m], below = A.D.energy[m] && k == A.D.k[m] - 1;
                        if (!at && !below) continue;
                        if (A.D.interp[m]) {
                            // co-located flux: the raw components over the window
                            // extended by one cell in x and y (E^{n+1} of plane k,
                            // H^{n+1/2} of layers k-1 and k), combined after the sweep;
                            // energy adds Ez, Hz of plane k and Ez of layer k-1
                            const int wx = A.D.i1[m] - A.D.i0[m] + 1;
                            const long long L = (long long)wx * (A.D.j1[m] - A.D.j0[m] + 1);
#pragma unroll
                            for (int r = 0; r < R; r++) {
                                const int yy = ys[r];
                                if (own[r] && x >= A.D.i0[m] && x <= A.D.i1[m] && yy >= A.D.j0[m] && yy <= A.D.j1[m]) {
                                    float *rw = raw_n0 + (long long)(s - 1) * A.D.raw_per_step + A.D.roff[m] +
                                                (long long)(yy - A.D.j0[m]) * wx + (x - A.D.i0[m]);
                                    if (at) {
                                        rw[0] = mE[r][0];
                                        rw[L] = mE[r][1];
                                        rw[2 * L] = Ho[s][r][0];
                                        rw[3 * L] = Ho[s][r][1];
                                        rw[4 * L] = mH[r][0];
                                        rw[5 * L] = mH[r][1];
                                        if (A.D.energy[m]) {
                                            rw[6 * L] = mE[r][2];
                                            rw[7 * L] = mH[r][2];
                                        }
                                    } else {
                                        rw[8 * L] = mE[r][2];
                                    }
                                }
                            }
                            continue;
                        }
                        if (!at) continue;
#pragma unroll
                        for (int r = 0; r < R; r++) {
                            const int yy = ys[r];
                            if (own[r] && x >= A.D.i0[m] && x < A.D.i1[m] && yy >= A.D.j0[m] && yy < A.D.j1[m]) {
                                const long long e = A.D.off[m] + (long long)(yy - A.D.j0[m]) * (A.D.i1[m] - A.D.i0[m]) +
                                                    (x - A.D.i0[m]);
                                planes[(long long)(s - 1) * A.D.per_step + e] =
                                    flux_density(mE[r][0], mE[r][1], mH[r][0], mH[r][1]);
                            }
                        }
                    }
                }
                // ---- interface record (section 2.2)
                if (rec_n0 && k >= z0 && k < z1 && k >= p - 1 && k <= nz - p) {
                    float *rs = rec_n0 + (long long)(s - 1) * A.R.per_step;
                    const bool wz = k >= p && k < nz - p;
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        if (!own[r]) continue;
                        const int yy = ys[r];
                        const bool wx = x >= p && x < nx - p, wy = yy >= p && yy < ny - p;
                        // z faces: u = x, v = y
                        if (wx && wy && (k == p - 1 || k == nz - p)) {
                            const int side = k == p - 1 ? 0 : 1;
                            const long long fs = (long long)A.R.Lu[2] * A.R.Lv[2];
                            const long long e = A.R.off[4 + side] + (long long)(yy - p) * A.R.Lu[2] + (x - p);
                            rs[e] = side ? mE[r][0] : mH[r][0];
                            rs[e + fs] = side ? mE[r][1] : mH[r][1];
                        }
                        // x faces: u = y, v = z; comps (y, z)
                        if (wy && wz && (x == p - 1 || x == nx - p)) {
                            const int side = x == p - 1 ? 0 : 1;
                            const long long fs = (long long)A.R.Lu[0] * A.R.Lv[0];
                            const long long e = A.R.off[0 + side] + (long long)(k - p) * A.R.Lu[0] + (yy - p);
                            rs[e] = side ? mE[r][1] : mH[r][1];
                            rs[e + fs] = side ? mE[r][2] : mH[r][2];
                        }
                        // y faces: u = x, v = z; comps (z, x)
                        if (wx && wz && (yy == p - 1 || yy == ny - p)) {
                            const int side = yy == p - 1 ? 0 : 1;
                            const long long fs = (long long)A.R.Lu[1] * A.R.Lv[1];
                            const long long e = A.R.off[2 + side] + (long long)(k - p) * A.R.Lu[1] + (x - p);
                            rs[e] = side ? mE[r][2] : mH[r][2];
                            rs[e + fs] = side ? mE[r][0] : mH[r][0];
                        }
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; r++) {
#pragma unroll
                    for (int q = 0; q < 3; q++) { mE[r][q] = 0.f; mH[r][q] = 0.f; }
                    psi_zero<XP, YP>(mP[r]);
                }
            }
            // rotate level s-1: its new plane becomes the one level s reads next
#pragma unroll
            for (int r = 0; r < R; r++) {
#pragma unroll
                for (int q = 0; q < 3; q++) Eo[s - 1][r][q] = nE[r][q];
                Ho[s - 1][r][0] = nH[r][0];
                Ho[s - 1][r][1] = nH[r][1];
                Hc[s - 1][r] = nH[r][2];
#pragma unroll
                for (int q = 0; q < 3; q++) { nE[r][q] = mE[r][q]; nH[r][q] = mH[r][q]; }
                Po[s - 1][r] = nP[r];
                nP[r] = mP[r];
            }
        }

        // ---------------------------------------------------- level K: store
        const int kK = t - K;
#pragma unroll
        for (int r = 0; r < R; r++) {
            Ho[K][r][0] = nH[r][0];
            Ho[K][r][1] = nH[r][1];
        }
        if (kK >= z0 && kK < z1) {
            if constexpr (WIDE) {
                const size_t pb = (size_t)kK * (size_t)Kp->g.nxy;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (!own[r]) continue;
                    const unsigned c = off[r] * 4u;
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        sto(Kp->fld[ic ^ 1][q] + pb, c, nE[r][q]);
                        sto(Kp->fld[ic ^ 1][3 + q] + pb, c, nH[r][q]);
                    }
                }
            } else {
                const unsigned base = (unsigned)kK * nxy;
                float *__restrict__ oF = A.fld[ic ^ 1][0];
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (!own[r]) continue;
                    const unsigned c = (base + off[r]) * 4u;
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        sto(oF, c + q * fs, nE[r][q]);
                        sto(oF, c + (3 + q) * fs, nH[r][q]);
                    }
                }
            }
            if (p > 0) {
                const int szo = slab_coord(kK, nz, p);
                if (szo >= 0) {
                    const unsigned zb = (unsigned)szo * nxy;
                    const unsigned ps = A.pstride[2];
#pragma unroll
                    for (int r = 0; r < R; r++)
                        if (own[r]) {
                            const unsigned o = (zb + off[r]) * 4u;
#pragma unroll
                            for (int q = 0; q < 4; q++) sto(A.psi[ic ^ 1][2], o + q * ps, nP[r].z[q]);
                        }
                }
                if constexpr (XP) {
                    if (sx >= 0) {
                        const unsigned xb = (unsigned)kK * (unsigned)ny * (unsigned)(2 * p);
                        const unsigned ps = A.pstride[0];
#pragma unroll
                        for (int r = 0; r < R; r++)
                            if (own[r]) {
                                const unsigned o = (xb + soff_x[r]) * 4u;
#pragma unroll
                                for (int q = 0; q < 4; q++) sto(A.psi[ic ^ 1][0], o + q * ps, nP[r].x[q]);
                            }
                    }
                }
                if constexpr (YP) {
                    const unsigned yb = (unsigned)kK * (unsigned)(2 * p) * (unsigned)nx;
                    const unsigned ps = A.pstride[1];
#pragma unroll
                    for (int r = 0; r < R; r++)
                        if (own[r] && sy[r] >= 0) {
                            const unsigned o = (yb + soff_y[r]) * 4u;
#pragma unroll
                            for (int q = 0; q < 4; q++) sto(A.psi[ic ^ 1][1], o + q * ps, nP[r].y[q]);
                        }
                }
            }
        }
    };

    // ring of PD planes in flight
    Plane<R, XP, YP> ring[PD];
#pragma unroll
    for (int u = 0; u < PD; u++) load_plane(zlo + u, ring[u]);
    for (int t0 = zlo; t0 < zend; t0 += PD) {
#pragma unroll
        for (int u = 0; u < PD; u++) {
            const int t = t0 + u;
            if (t < zend) {
                const Plane<R, XP, YP> cur = ring[u];
                load_plane(t + PD, ring[u]);
                asm volatile("" : "+s"(Kp));
                body(t, cur);
            }
        }
    }
}

// The kernel: block b (XCD-remapped) finds its request and tile; the tile's
// class picks the march instance.
template <int K, int PD, int W, int R, int TX, bool WIDE, bool LOSSY>
__global__ __launch_bounds__(64 * W, 4) void k_tb_forward(TbLaunch)
{
    constexpr int EY = (64 * W / TX) * R;
    // (one spare row for the threads beyond the last full row when TX does
    // not divide the workgroup: they compute on it and write nothing)
    __shared__ float sE[3][EY + 1][TX];
    __shared__ float sH[3][EY + 1][TX];
    // z grading of the 2p slab planes (E b, a, 1/k, H b, a, 1/k) and the
    // source amplitudes of the K steps of this sweep, staged once so the
    // march never waits on a vector load other than its own plane fetches
    __shared__ float sGz[2 * TB_MAXP][6];
    __shared__ float sAmp[FD_MAXSRC][K];
    // (the launch block is the kernel's only parameter, at offset 0 of the
    // kernel-argument segment)
    KLaunch *Lp = (KLaunch *)__builtin_amdgcn_kernarg_segment_ptr();
    int b = blockIdx.x;
    if (Lp->xcd_remap) b = remap_xcd(b, gridDim.x);
    int r = 0;
    while (r + 1 < Lp->nreq && b >= Lp->r[r + 1].first) r++;
    KReq *Rq = &Lp->r[r];
    // Arguments used only now and then are read through a copy of this
    // pointer that is made opaque on every plane, so they are fetched where
    // they are used instead of being held in scalar registers for the whole
    // march: the source arguments, and the component bases of the WIDE
    // instance.
    KArgs *Ap = (KArgs *)Rq->args;
    const int4 *tt = Rq->tiles + 2 * (b - Rq->first);
    const int4 tl = tt[0], tz = tt[1];
    switch (tz.z) {
    case 0: tb_march<K, false, false, PD, W, R, TX, WIDE, LOSSY>(*Ap, Ap, Rq, tl, tz, sE, sH, sGz, sAmp); break;
    case 1: tb_march<K, true, false, PD, W, R, TX, WIDE, LOSSY>(*Ap, Ap, Rq, tl, tz, sE, sH, sGz, sAmp); break;
    case 2: tb_march<K, false, true, PD, W, R, TX, WIDE, LOSSY>(*Ap, Ap, Rq, tl, tz, sE, sH, sGz, sAmp); break;
    default: tb_march<K, true, true, PD, W, R, TX, WIDE, LOSSY>(*Ap, Ap, Rq, tl, tz, sE, sH, sGz, sAmp); break;
    }
}

template <int K, int W, int R, int PD, int TX, bool WIDE = false, bool LOSSY = false>
hipError_t launch_kwrp(const TbLaunch &L, hipStream_t s)
{
    constexpr int threads = 64 * W;
    if (L.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_tb_forward<K, PD, W, R, TX, WIDE, LOSSY>), dim3(L.nblocks), dim3(threads), 0, s, L);
    return hipGetLastError();
}

// workgroup shapes (one row per thread):
//   0: 16 waves of 64-lane rows, a 64 x 16 tile, one workgroup per CU
//   1: 8 waves of 32-lane rows, a 32 x 16 tile, two workgroups per CU
//   2: 16 waves as rows of 32 + 2K lanes (28 rows at K = 2): the owned part
//      of each row is one whole 128-byte line, line aligned, so no two
//      workgroups write parts of the same line
//   3: as 2 with 8 waves (two workgroups per CU)
// (two rows per thread with 8 waves, 24 owned rows at K = 2, needs about 170
// to 220 registers, so 2-3 waves per SIMD and one workgroup per CU: measured
// 2.8 times slower than shape 3, not kept)
// (12 waves, 21 rows with 17 owned at K = 2, three waves per SIMD with up
// to 168 registers and no spills, one workgroup per CU: bitwise equal, but
// 0.395 against 0.378 ms per sweep on 256^3 and 7.94 against 7.14 s for the
// 640x640x400 forward with the record; not kept)
constexpr int NSHAPE = 4;
constexpr int SHAPE_W[NSHAPE] = {16, 8, 16, 8};
constexpr int SHAPE_R[NSHAPE] = {1, 1, 1, 1};
constexpr int ALIGN_X = 32;   // floats per 128-byte line
__host__ __device__ constexpr int shape_tx(int sh, int K) { return sh == 0 ? 64 : sh == 1 ? 32 : ALIGN_X + 2 * K; }

template <int K>
hipError_t launch_k(const TbLaunch &L, int shape, bool wide, hipStream_t s)
{
    // the 64-bit-base instance exists for the default shape only
    if (wide) return shape == 3 ? launch_kwrp<K, 8, 1, 1, ALIGN_X + 2 * K, true>(L, s) : hipErrorInvalidValue;
    switch (shape) {
    case 0: return launch_kwrp<K, 16, 1, 1, 64>(L, s);
    case 2: return launch_kwrp<K, 16, 1, 1, ALIGN_X + 2 * K>(L, s);
    case 3: return launch_kwrp<K, 8, 1, 1, ALIGN_X + 2 * K>(L, s);
    default: return launch_kwrp<K, 8, 1, 1, 32>(L, s);
    }
}

int shape_index(int shape) { return shape >= 0 && shape < NSHAPE ? shape : 1; }

}  // namespace

int tb_tile_x(int K, int shape) { return shape_tx(shape_index(shape), K) - 2 * K; }
int tb_max_pml() { return TB_MAXP; }
int tb_tile_y(int K, int shape)
{
    const int sh = shape_index(shape);
    return (64 * SHAPE_W[sh] / shape_tx(sh, K)) * SHAPE_R[sh] - 2 * K;
}
bool tb_tile_aligned(int shape) { return shape_index(shape) >= 2; }
bool tb_wide_shape(int shape) { return shape_index(shape) == 3; }
int tb_wg_per_cu(int shape) { return SHAPE_W[shape_index(shape)] <= 8 ? 2 : 1; }

bool tb_lossy_ok(int K, int shape, bool wide) { return !wide && shape_index(shape) == 3 && (K == 1 || K == 2); }

hipError_t launch_tb_forward(const TbLaunch &L, int K, int shape, bool wide, bool lossy, hipStream_t s)
{
    shape = shape_index(shape);
    if (lossy) {
        // conducting cells: the default shape, 32-bit offsets, K = 1 or 2
        if (!tb_lossy_ok(K, shape, wide)) return hipErrorInvalidValue;
        return K == 1 ? launch_kwrp<1, 8, 1, 1, ALIGN_X + 2, false, true>(L, s)
                      : launch_kwrp<2, 8, 1, 1, ALIGN_X + 4, false, true>(L, s);
    }
    switch (K) {
    case 1: return launch_k<1>(L, shape, wide, s);
    case 2: return launch_k<2>(L, shape, wide, s);
    case 3: return launch_k<3>(L, shape, wide, s);
    case 4: return launch_k<4>(L, shape, wide, s);
    default: return hipErrorInvalidValue;
    }
}
