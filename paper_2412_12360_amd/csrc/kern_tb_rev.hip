// Fused reverse step as a z-march: the inverse update of the interior (arXiv
// 2412.12360, section 2.2) together with the hand-written adjoint of the
// forward step, the detector adjoint source and the replay of the interface
// record, in one pass over the grid per reverse step.
//
// Reverse step n maps the forward state s_{n+1} = (E^{n+1}, H^{n+1/2}) to s_n
// on the interior I = [p, n-p)^3 and the adjoint of s_{n+1} to the adjoint of
// s_n.  Per cell it is the same arithmetic, in the same order, as the
// per-cell phases k_bwd_a / k_bwd_b (and bitwise equal to them):
//   phase A: dJ/dd += Ebar' . curl H^{n+1/2};  E^n = E^{n+1} - srcE_n - S/eps curl H^{n+1/2};
//            Hbar += C(S/eps Ebar') with the transposed CPML (coefficients Q)
//   phase B: psibar_E <- b (psibar_E + w);  H^{n-1/2} = H^{n+1/2} - srcH_n + S curl E^n;
//            Ebar -= S C^T Hbar with the transposed CPML (coefficients R);
//            psibar_H <- b (psibar_H + w)
// Phase A at a cell reads H at -1 and Q at +1; phase B reads E^n at +1 and R
// at -1, so a workgroup marches up in z with phase A one plane behind the
// fetch and phase B two planes behind.  An owned cell's outputs need E^n of
// the cell above it in x and y (phase A there reads only owned H) and R of
// the cell below it (from Hbar of that cell, whose phase A reads Q of the
// owned cell): raw inputs one cell beyond the tile on each side suffice, so
// the halo is one cell in x and y.  In z the march starts at the tile's
// first plane (with the plane below it preloaded) and ends two planes past
// the last.
// The four x/y exchanges of a plane (H, Q, E^n, R) share one LDS round.
// Record values replace the fields on the PML-side layers (H on the low
// faces from step n, E^n on the high faces from step n-1) as they are read.
// All state is read from one buffer set and written to the other.
#include "fdtd_internal.h"

namespace {

// Workgroup: W waves as rows of EX = 32 + 2*HALO lanes; the owned part of
// a row is one whole 128-byte line, line aligned (x tiles are cut into whole
// lines), so no two workgroups write parts of the same line.  The threads
// beyond the last full row (512 - 15*34 = 2) work on a spare LDS row and
// write nothing.  8 waves and at most 128 registers, so that two workgroups
// share a CU (measured 2% faster than one 16-wave workgroup per CU at a
// two-cell halo).  With the one-cell halo 13 of 15 rows are owned.
constexpr int HALO = 1;
constexpr int EX = 32 + 2 * HALO;
// (rows_of(W) rows of a W-wave workgroup)
constexpr int rows_of(int W) { return 64 * W / EX; }

// every pointer here addresses device global memory; saying so keeps the
// loads and stores on global (not flat) instructions
#define GLOBAL __attribute__((address_space(1)))
#define LDSP __attribute__((address_space(3)))
__device__ __forceinline__ float gld(const float *p) { return *(const GLOBAL float *)p; }

// Workgroup barrier for the LDS exchanges: waits for this wave's LDS
// operations only.  (__syncthreads would also wait for every vector memory
// operation in flight, which includes the loads of the next plane that go
// straight to LDS and are meant to stay in flight across the barrier; no
// wave of a workgroup reads another's global writes.)  The memory clobber
// keeps the compiler from moving memory operations across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// main inputs of a plane staged through LDS per thread
constexpr int RV_NST = 13;
// word 3 of a raw buffer resource (32-bit data format, no swizzle; the
// range is the full 32-bit offset space)
constexpr int BUF_WORD3 = 0x00020000;

__device__ __forceinline__ int remap_xcd_r(int b, int nb)
{
    const int q = nb / 8, rem = nb % 8;
    const int xcd = b % 8, slot = b / 8;
    return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

template <bool XP, bool YP> struct PsiB {
    float z[4];
    float x[XP ? 4 : 1];
    float y[YP ? 4 : 1];
};

// one plane of inputs of a column
template <bool XP, bool YP> struct RPlane {
    float e[3], h[3], ce, ae[3], ah[3];
    PsiB<XP, YP> pb;
};

// The few values of a march iteration that come from elsewhere than the
// plane's field sets: record H of plane t on the low faces (case hc, 0 for
// none), record E^n of plane t-1 on the high faces (case ec), the dJ/dd
// accumulator of plane t-1 (gin), a conducting cell's E^n and sigma at
// plane t-1 and its ca at plane t-2.  They are loaded before the next
// plane's loads are issued, so waiting for them does not wait for those.
struct Side {
    float h0 = 0.f, h1 = 0.f, e0 = 0.f, e1 = 0.f, acc = 0.f;
    float len[3] = {0.f, 0.f, 0.f}, lsg = 0.f, lca = 0.f;
    int hc = 0, ec = 0;
    bool gin = false, lossy = false, cin = false;
};

// WIDE: field and adjoint sets of 4 GiB or more, addressed per plane from a
// 64-bit base per component (read through Kp) plus the 32-bit offset of the
// column within the plane; otherwise one base per set with 32-bit offsets.
// The handle's fixed arguments and the launch's per-request arguments, read
// with scalar loads from constant memory.
typedef const __attribute__((address_space(4))) RevArgs KArgs;
typedef const __attribute__((address_space(4))) RevReq KReq;
typedef const __attribute__((address_space(4))) RevLaunch KLaunch;
typedef const __attribute__((address_space(4))) Grid KGrid;

// LDS of the kernel, one set whatever the tile class
template <int W> struct RevLds {
    static constexpr int EY = rows_of(W);
    float sH[3][EY + 1][EX];
    float sQ[4][EY + 1][EX];
    float sEn[3][EY + 1][EX];
    float sR[4][EY + 1][EX];
    float sGz[2 * 64][6];
    float sAmp[FD_MAXSRC];   // source amplitudes of step n
};

// One tile's reverse march.
// LOSSY: the instance for handles with conducting cells (a lossy box):
// there E^n is not un-updated but read from the record of step n, dJ/dd
// takes -sigma E^n beside curl H, and the adjoint E passes ca Ebar' on.
template <bool XP, bool YP, bool WIDE, int W, bool LOSSY>
__device__ __forceinline__ void rev_march(KArgs &A, KArgs *Kp, KReq *Rq, const int4 tl, const int4 tz,
                                          RevLds<W> &L_, float (&sSt)[RV_NST][64 * W])
{
    constexpr int EY = rows_of(W);
    auto &sH = L_.sH;
    auto &sQ = L_.sQ;
    auto &sEn = L_.sEn;
    auto &sR = L_.sR;
    auto &sGz = L_.sGz;
    auto &sAmp = L_.sAmp;
    const int n = Rq->n;
    const unsigned fl = Rq->flags;
    const bool do_inv = (fl & RV_INV) != 0, do_adj = (fl & RV_ADJ) != 0, with_det = (fl & RV_DET) != 0;
    const int ic = (fl & RV_CUR) ? 1 : 0, ia = (fl & RV_ACUR) ? 1 : 0, ip = (fl & RV_APAR) ? 1 : 0;
    // forward state s_{n+1} in and s_n out, adjoint in and out (without the
    // adjoint the march still issues its adjoint loads, from the forward
    // input set, and drops them), psi-bar in and out
    const float *const fin0 = Rq->fin ? Rq->fin : A.fld[ic][0];
    float *const fout0 = A.fld[ic ^ 1][0];
    const float *const ain0 = do_adj ? A.adj[ia][0] : A.fld[ic][0];
    float *const aout0 = A.adj[ia ^ 1][0];
    const bool has_rec_h = Rq->rec_h != nullptr, has_rec_e = Rq->rec_e != nullptr;
    const bool has_gacc = Rq->gacc != nullptr;

    KGrid &g = A.g;
    const int nx = g.nx, ny = g.ny, nz = g.nz, p = g.p;
    const unsigned nxy = (unsigned)g.nxy;
    const float S = g.S;
    for (int e = threadIdx.x; e < 2 * p; e += blockDim.x) {
        const int kk = e < p ? e : nz - 2 * p + e;
        const float4 gE = A.profv[2][2 * kk], gH = A.profv[2][2 * kk + 1];
        sGz[e][0] = gE.x; sGz[e][1] = gE.y; sGz[e][2] = gE.z;
        sGz[e][3] = gH.x; sGz[e][4] = gH.y; sGz[e][5] = gH.z;
    }
    if ((int)threadIdx.x < FD_MAXSRC) sAmp[threadIdx.x] = (int)threadIdx.x < g.nsrc ? g.samp[threadIdx.x][n] : 0.f;
    lds_barrier();
    // source and detector planes (uniform; -2^31 when absent), hoisted so the
    // per-plane tests issue no scalar memory load
    constexpr int NONE = -2147483647 - 1;
    int skq[FD_MAXSRC], dkq[FD_MAXDET];
#pragma unroll
    for (int q = 0; q < FD_MAXSRC; q++) skq[q] = q < g.nsrc ? g.sk[q] : NONE;
#pragma unroll
    for (int m = 0; m < FD_MAXDET; m++) dkq[m] = (do_adj && with_det && m < A.D.ndet) ? A.D.k[m] : NONE;
    // Arguments used only on rare planes (record layers, detector, source)
    // are read through a copy of the argument pointer that is made opaque on
    // every plane, so they are fetched where used instead of being held in
    // scalar registers for the whole march.
    // (the argument block is the kernel's only parameter, at offset 0 of the
    // kernel-argument segment)
    // The same holds for the per-request record and accumulator pointers.
    KReq *Rk = Rq;
    const int x0 = tl.x, x1 = tl.y, y0 = tl.z, y1 = tl.w, z0 = tz.x, z1 = tz.y;
    const bool active = (int)threadIdx.x < EX * EY;
    const int lane = active ? (int)threadIdx.x % EX : 0;
    const int row = active ? (int)threadIdx.x / EX : EY;
    const int x = x0 - HALO + lane;
    const int y = y0 - HALO + row;
    const bool incol = active && x >= 0 && x < nx && y >= 0 && y < ny;
    const bool own = x >= x0 && x < x1 && y >= y0 && y < y1;
    const int xc = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
    const int yc = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
    const unsigned off = (unsigned)yc * (unsigned)nx + (unsigned)xc;
    // No owned cell reads E^n of the left halo column or the bottom halo row,
    // nor R (from the adjoint H) of the right column or the top row: those
    // lanes load E, or the adjoint H, from the neighbouring cell inside the
    // tile instead, whose line the tile fetches anyway, so the load costs no
    // memory traffic of its own and the loads stay the same instructions on
    // every lane.  (Except on detector planes, where the adjoint source of
    // the adjoint H reads E of the same cell.)
    // (one signed offset: > 0 moves the E loads, < 0 the adjoint-H loads; a
    // corner lane moves only its E loads)
    const int dsh = lane == 0 ? (xc + 1 < nx ? 1 : 0)
                  : row == 0 ? (yc + 1 < ny ? nx : 0)
                  : lane == EX - 1 ? (xc > 0 ? -1 : 0)
                  : row == EY - 1 ? (yc > 0 ? -nx : 0) : 0;
    const bool icol = p == 0 ? incol : (active && x >= p && x < nx - p && y >= p && y < ny - p);
    const bool wx = x >= p && x < nx - p, wy = y >= p && y < ny - p;
    const int sx = (XP && incol) ? slab_coord(x, nx, p) : -1;
    const int sy = (YP && incol) ? slab_coord(y, ny, p) : -1;
    const unsigned soff_x = sx >= 0 ? (unsigned)yc * (unsigned)(2 * p) + (unsigned)sx : 0u;
    const unsigned soff_y = sy >= 0 ? (unsigned)sy * (unsigned)nx + (unsigned)xc : 0u;
    float4 gxE = make_float4(1.f, 0.f, 1.f, 0.f), gxH = gxE, gyE = gxE, gyH = gxE;
    if constexpr (XP) {
        if (sx >= 0) { gxE = A.profv[0][2 * x]; gxH = A.profv[0][2 * x + 1]; }
    }
    if constexpr (YP) {
        if (sy >= 0) { gyE = A.profv[1][2 * y]; gyH = A.profv[1][2 * y + 1]; }
    }
    const unsigned fs = A.fstride;   // bytes between the components of a field or adjoint set
    const bool in_design_xy = x >= A.dlo.x && x < A.dhi.x && y >= A.dlo.y && y < A.dhi.y;
    // dJ/dd index of this column within a design plane, and the plane size
    const int dxy = in_design_xy ? (y - A.dlo.y) * (A.dhi.x - A.dlo.x) + (x - A.dlo.x) : 0;
    const int dplane = (A.dhi.x - A.dlo.x) * (A.dhi.y - A.dlo.y);

    // ---------------------------------------------------------- plane fetch
    // stage issues the loads of plane t (one iteration ahead, so the fetch
    // overlaps a whole plane of work); finish zeroes what lies outside the
    // grid, replays the record and adds the detector adjoint source.
    // fetch(t, f) hands f (component c, base, byte offset) for each of the
    // 13 main inputs of plane t: E 0-2, H 3-5, S/eps 6, adjoint E 7-9,
    // adjoint H 10-12.
    auto fetch = [&](int t, auto &&f) __attribute__((always_inline)) {
        const bool tin = t >= 0 && t < nz;
        bool detp = false;
#pragma unroll
        for (int m = 0; m < FD_MAXDET; m++) detp = detp || t == dkq[m];
        const unsigned oe = detp ? off : off + (unsigned)max(dsh, 0);
        const unsigned off_ah = off + (unsigned)min(dsh, 0);
        if constexpr (WIDE) {
            const size_t pb = (size_t)(tin ? t : 0) * (size_t)Kp->g.nxy;
            const unsigned c = off * 4u, ce_ = oe * 4u, ca_ = off_ah * 4u;
#pragma unroll
            for (int q = 0; q < 3; q++) {
                f(q, Kp->fld[ic][q] + pb, ce_);
                f(3 + q, Kp->fld[ic][3 + q] + pb, c);
            }
            f(6, Kp->g.ce + pb, c);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                f(7 + q, (do_adj ? Kp->adj[ia][q] : Kp->fld[ic][q]) + pb, c);
                f(10 + q, (do_adj ? Kp->adj[ia][3 + q] : Kp->fld[ic][3 + q]) + pb, ca_);
            }
        } else {
            const unsigned pl = (unsigned)(tin ? t : 0) * nxy;
            const unsigned c = (pl + off) * 4u, ce_ = (pl + oe) * 4u, ca_ = (pl + off_ah) * 4u;
#pragma unroll
            for (int q = 0; q < 3; q++) {
                f(q, fin0, ce_ + q * fs);
                f(3 + q, fin0, c + (3 + q) * fs);
            }
            f(6, g.ce, c);
            // (issued on every path, so the compiler's wait counts stay exact;
            // without an adjoint, ain points at a readable set and finish drops it)
#pragma unroll
            for (int q = 0; q < 3; q++) {
                f(7 + q, ain0, c + q * fs);
                f(10 + q, ain0, ca_ + (3 + q) * fs);
            }
        }
    };
    auto slot = [](RPlane<XP, YP> &P, int c) -> float & {
        return c < 3 ? P.e[c] : c < 6 ? P.h[c - 3] : c == 6 ? P.ce : c < 10 ? P.ae[c - 7] : P.ah[c - 10];
    };
    // psi-bar of plane t (slab cells; zero elsewhere)
    auto load_psi = [&](int t, RPlane<XP, YP> &P) __attribute__((always_inline)) {
        const bool tin = t >= 0 && t < nz;
        auto ld = [&](const float *base, unsigned o) { return *(const GLOBAL float *)((const GLOBAL char *)base + o); };
#pragma unroll
        for (int q = 0; q < 4; q++) P.pb.z[q] = 0.f;
        if constexpr (XP) {
#pragma unroll
            for (int q = 0; q < 4; q++) P.pb.x[q] = 0.f;
        }
        if constexpr (YP) {
#pragma unroll
            for (int q = 0; q < 4; q++) P.pb.y[q] = 0.f;
        }
        if (do_adj && p > 0 && tin) {
            const int szt = slab_coord(t, nz, p);
            if (szt >= 0) {
                const unsigned zi = (unsigned)szt * nxy + off;
#pragma unroll
                for (int q = 0; q < 4; q++) P.pb.z[q] = ld(A.pb[ip][2], zi * 4u + q * A.pstride[2]);
            }
            if constexpr (XP) {
                const unsigned xi = (unsigned)t * (unsigned)ny * (unsigned)(2 * p) + soff_x;
#pragma unroll
                for (int q = 0; q < 4; q++) P.pb.x[q] = ld(A.pb[ip][0], xi * 4u + q * A.pstride[0]);
            }
            if constexpr (YP) {
                const unsigned yi = (unsigned)t * (unsigned)(2 * p) * (unsigned)nx + soff_y;
#pragma unroll
                for (int q = 0; q < 4; q++) P.pb.y[q] = ld(A.pb[ip][1], yi * 4u + q * A.pstride[1]);
            }
        }
    };
    // a plane with plain loads into registers
    auto load_raw = [&](int t, RPlane<XP, YP> &P) __attribute__((always_inline)) {
        fetch(t, [&](int c, const float *base, unsigned o) __attribute__((always_inline)) {
            slot(P, c) = *(const GLOBAL float *)((const GLOBAL char *)base + o);
        });
        load_psi(t, P);
    };
    // the 13 main inputs of plane t straight into the LDS staging buffer
    // (thread i's value of component c lands at sSt[c][i]: the loads' LDS
    // address is the wave's base plus 4 bytes per lane), so the plane in
    // flight holds no registers
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    // (buffer loads: the global_load_lds form would make the compiler treat
    // every later wait for a plain load as a wait for all of them)
    auto stage = [&](int t) __attribute__((always_inline)) {
        fetch(t, [&](int c, const float *base, unsigned o) __attribute__((always_inline)) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, -1, BUF_WORD3);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LDSP void *)&sSt[c][wv * 64], 4, o, 0, 0, 0);
        });
    };
    auto unstage = [&](RPlane<XP, YP> &P) __attribute__((always_inline)) {
#pragma unroll
        for (int c = 0; c < RV_NST; c++) slot(P, c) = sSt[c][threadIdx.x];
    };
    // record H of plane t on the low-face layers (finish puts it in place)
    auto load_rech = [&](int t, Side &Sd) __attribute__((always_inline)) {
        const bool v = t >= 0 && t < nz && incol;
        if (has_rec_h && v && t >= p - 1 && t < nz - p) {
            const bool wz = t >= p;
            long long e = 0, fsr = 0;
            if (t == p - 1 && wx && wy) {
                Sd.hc = 1;
                e = Kp->R.off[4] + (long long)(y - p) * Kp->R.Lu[2] + (x - p);
                fsr = (long long)Kp->R.Lu[2] * Kp->R.Lv[2];
            } else if (wz && x == p - 1 && wy) {
                Sd.hc = 2;
                e = Kp->R.off[0] + (long long)(t - p) * Kp->R.Lu[0] + (y - p);
                fsr = (long long)Kp->R.Lu[0] * Kp->R.Lv[0];
            } else if (wz && y == p - 1 && wx) {
                Sd.hc = 3;
                e = Kp->R.off[2] + (long long)(t - p) * Kp->R.Lu[1] + (x - p);
                fsr = (long long)Kp->R.Lu[1] * Kp->R.Lv[1];
            }
            if (Sd.hc != 0) {
                Sd.h0 = gld(Rk->rec_h + e);
                Sd.h1 = gld(Rk->rec_h + e + fsr);
            }
        }
    };
    // everything else of iteration t: phase A's plane a = t-1, phase B's b = t-2
    auto side_load = [&](int t, Side &Sd) __attribute__((always_inline)) {
        load_rech(t, Sd);
        const int a = t - 1, bpl = t - 2;
        const bool kin = a >= 0 && a < nz;
        const bool interior = icol && kin && (p == 0 || (a >= p && a < nz - p));
        if constexpr (LOSSY) {
            if (interior && has_rec_h && a >= Kp->g.llo[2] && a < Kp->g.lhi[2] && x >= Kp->g.llo[0] &&
                x < Kp->g.lhi[0] && y >= Kp->g.llo[1] && y < Kp->g.lhi[1]) {
                const int bx = Kp->g.lhi[0] - Kp->g.llo[0], by = Kp->g.lhi[1] - Kp->g.llo[1];
                const long long li = ((long long)(a - Kp->g.llo[2]) * by + (y - Kp->g.llo[1])) * bx +
                                     (x - Kp->g.llo[0]);
                const long long nb = (long long)bx * by * (Kp->g.lhi[2] - Kp->g.llo[2]);
                const float *lr = Rk->rec_h + Kp->R.loff + li;
                Sd.len[0] = gld(lr); Sd.len[1] = gld(lr + nb); Sd.len[2] = gld(lr + 2 * nb);
                Sd.lsg = gld(Kp->g.lsig + li);
                Sd.lossy = true;
            }
        }
        Sd.gin = interior && do_adj && has_gacc && own && a >= z0 && a < z1 && in_design_xy && a >= A.dlo.z &&
                 a < A.dhi.z;
        if (Sd.gin) Sd.acc = gld(Rk->gacc + ((long long)(a - A.dlo.z) * dplane + dxy));
        if (do_inv && !interior && p > 0 && incol && kin) {
            const bool wz = a >= p && a < nz - p;
            long long e = 0, fsr = 0;
            if (a == nz - p && wx && wy) {
                Sd.ec = 1;
                e = Kp->R.off[5] + (long long)(y - p) * Kp->R.Lu[2] + (x - p);
                fsr = (long long)Kp->R.Lu[2] * Kp->R.Lv[2];
            } else if (wz && x == nx - p && wy) {
                Sd.ec = 2;
                e = Kp->R.off[1] + (long long)(a - p) * Kp->R.Lu[0] + (y - p);
                fsr = (long long)Kp->R.Lu[0] * Kp->R.Lv[0];
            } else if (wz && y == ny - p && wx) {
                Sd.ec = 3;
                e = Kp->R.off[3] + (long long)(a - p) * Kp->R.Lu[1] + (x - p);
                fsr = (long long)Kp->R.Lu[1] * Kp->R.Lv[1];
            }
            if (Sd.ec != 0 && has_rec_e) {
                Sd.e0 = gld(Rk->rec_e + e);
                Sd.e1 = gld(Rk->rec_e + e + fsr);
            }
        }
        if constexpr (LOSSY) {
            const bool kb = bpl >= 0 && bpl < nz;
            const bool ib = icol && kb && (p == 0 || (bpl >= p && bpl < nz - p));
            if (do_adj && own && bpl >= z0 && bpl < z1 && ib && bpl >= Kp->g.llo[2] && bpl < Kp->g.lhi[2] &&
                x >= Kp->g.llo[0] && x < Kp->g.lhi[0] && y >= Kp->g.llo[1] && y < Kp->g.lhi[1]) {
                const int bx = Kp->g.lhi[0] - Kp->g.llo[0], by = Kp->g.lhi[1] - Kp->g.llo[1];
                const long long li = ((long long)(bpl - Kp->g.llo[2]) * by + (y - Kp->g.llo[1])) * bx +
                                     (x - Kp->g.llo[0]);
                Sd.lca = gld(Kp->g.lca + li);
                Sd.cin = true;
            }
        }
    };
    auto finish = [&](int t, const RPlane<XP, YP> &R, RPlane<XP, YP> &P, const Side &Sd) __attribute__((always_inline)) {
        const bool tin = t >= 0 && t < nz;
        const bool v = tin && incol;
        const bool va = v && do_adj;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            P.e[q] = v ? R.e[q] : 0.f;
            P.h[q] = v ? R.h[q] : 0.f;
            P.ae[q] = va ? R.ae[q] : 0.f;
            P.ah[q] = va ? R.ah[q] : 0.f;
        }
        P.ce = v ? R.ce : 0.f;
        P.pb = R.pb;
        // H^{n+1/2} on the low-face layers comes from the record of step n
        // (loaded by side_load)
        if (Sd.hc == 1) { P.h[0] = Sd.h0; P.h[1] = Sd.h1; }
        if (Sd.hc == 2) { P.h[1] = Sd.h0; P.h[2] = Sd.h1; }
        if (Sd.hc == 3) { P.h[2] = Sd.h0; P.h[0] = Sd.h1; }
        // detector adjoint source: dJ/dE^{n+1}, dJ/dH^{n+1/2} (uniform plane
        // test against the hoisted detector planes)
#pragma unroll
        for (int m = 0; m < FD_MAXDET; m++) {
            if (t == dkq[m]) {
                if (v && x >= Kp->D.i0[m] && x < Kp->D.i1[m] && y >= Kp->D.j0[m] && y < Kp->D.j1[m]) {
                    const float sw = Kp->wS[m];
                    P.ae[0] = fmaf(sw, P.h[1], P.ae[0]);
                    P.ae[1] = fmaf(-sw, P.h[0], P.ae[1]);
                    P.ah[1] = fmaf(sw, P.e[0], P.ah[1]);
                    P.ah[0] = fmaf(-sw, P.e[1], P.ah[0]);
                }
            }
        }
    };

    // adjoint coefficients of the six E pairs of a column at plane k:
    // 0: Ey along z (+), 1: Ez along y (-), 2: Ex along z (-), 3: Ez along x (+),
    // 4: Ex along y (+), 5: Ey along x (-)
    auto qcoef = [&](const RPlane<XP, YP> &P, int k, float Q[6]) {
        const bool live = incol && k >= 0 && k < nz;
        const bool hex = y == 0 || k == 0, hey = x == 0 || k == 0, hez = x == 0 || y == 0;
        const float cex = P.ce * P.ae[0], cey = P.ce * P.ae[1], cez = P.ce * P.ae[2];
        float q0 = 1.f * cey, q1 = -1.f * cez, q2 = -1.f * cex, q3 = 1.f * cez, q4 = 1.f * cex, q5 = -1.f * cey;
        const int sz = (p > 0 && k >= 0 && k < nz) ? slab_coord(k, nz, p) : -1;
        if (sz >= 0) {
            const float a = sGz[sz][1], kv = sGz[sz][2];
            q0 = cpml_adj_coef(q0, P.pb.z[1], a, kv);
            q2 = cpml_adj_coef(q2, P.pb.z[0], a, kv);
        }
        if constexpr (XP) {
            if (sx >= 0) {
                q3 = cpml_adj_coef(q3, P.pb.x[1], gxE.y, gxE.z);
                q5 = cpml_adj_coef(q5, P.pb.x[0], gxE.y, gxE.z);
            }
        }
        if constexpr (YP) {
            if (sy >= 0) {
                q1 = cpml_adj_coef(q1, P.pb.y[0], gyE.y, gyE.z);
                q4 = cpml_adj_coef(q4, P.pb.y[1], gyE.y, gyE.z);
            }
        }
        Q[0] = (live && !hey) ? q0 : 0.f;
        Q[1] = (live && !hez) ? q1 : 0.f;
        Q[2] = (live && !hex) ? q2 : 0.f;
        Q[3] = (live && !hez) ? q3 : 0.f;
        Q[4] = (live && !hex) ? q4 : 0.f;
        Q[5] = (live && !hey) ? q5 : 0.f;
    };

    // adjoint coefficients of the six H pairs: 0: Hy along z (-S), 1: Hz along y (+S),
    // 2: Hz along x (-S), 3: Hx along z (+S), 4: Hx along y (-S), 5: Hy along x (+S)
    auto rcoef = [&](const float ah[3], const PsiB<XP, YP> &pb, int k, float Rr[6]) {
        const bool live = incol && k >= 0 && k < nz;
        const float sx_ = S * ah[0], sy_ = S * ah[1], sz_ = S * ah[2];
        float r0 = -1.f * sy_, r1 = 1.f * sz_, r2 = -1.f * sz_, r3 = 1.f * sx_, r4 = -1.f * sx_, r5 = 1.f * sy_;
        const int sz = (p > 0 && k >= 0 && k < nz) ? slab_coord(k, nz, p) : -1;
        if (sz >= 0) {
            const float a = sGz[sz][4], kv = sGz[sz][5];
            r0 = cpml_adj_coef(r0, pb.z[3], a, kv);
            r3 = cpml_adj_coef(r3, pb.z[2], a, kv);
        }
        if constexpr (XP) {
            if (sx >= 0) {
                r2 = cpml_adj_coef(r2, pb.x[3], gxH.y, gxH.z);
                r5 = cpml_adj_coef(r5, pb.x[2], gxH.y, gxH.z);
            }
        }
        if constexpr (YP) {
            if (sy >= 0) {
                r1 = cpml_adj_coef(r1, pb.y[2], gyH.y, gyH.z);
                r4 = cpml_adj_coef(r4, pb.y[3], gyH.y, gyH.z);
            }
        }
        Rr[0] = live ? r0 : 0.f; Rr[1] = live ? r1 : 0.f; Rr[2] = live ? r2 : 0.f;
        Rr[3] = live ? r3 : 0.f; Rr[4] = live ? r4 : 0.f; Rr[5] = live ? r5 : 0.f;
    };

    // ------------------------------------------------------------ pipeline
    // Pa: inputs of plane a = t-1; b*: plane b = t-2 (E^n, H^{n+1/2}, Ebar',
    // Hbar_new, S/eps, psibar); Rz: R of plane b-1 (z pairs); Hm: H^{n+1/2}
    // x,y of plane a-1.  Q of plane a and R of plane b are recomputed from
    // these rather than carried, which keeps the march within 128 VGPRs.
    RPlane<XP, YP> Pa;
    float bEn[3] = {0.f, 0.f, 0.f}, bH[3] = {0.f, 0.f, 0.f}, bAe[3] = {0.f, 0.f, 0.f}, bAh[3] = {0.f, 0.f, 0.f};
    float bCe = 0.f;
    PsiB<XP, YP> bPb;
#pragma unroll
    for (int q = 0; q < 4; q++) bPb.z[q] = 0.f;
    if constexpr (XP) {
#pragma unroll
        for (int q = 0; q < 4; q++) bPb.x[q] = 0.f;
    }
    if constexpr (YP) {
#pragma unroll
        for (int q = 0; q < 4; q++) bPb.y[q] = 0.f;
    }
    float Rz0 = 0.f, Rz3 = 0.f;     // R of plane b-1: Hy along z, Hx along z
    float Hm0 = 0.f, Hm1 = 0.f;     // Hx, Hy of plane a-1

    // body(t) runs phase A at t-1 and phase B at t-2: t = z0 .. z1+1
    const int zs = z0, ze = z1 + 2;
    {
        RPlane<XP, YP> R;
        Side S0;
        load_raw(zs - 1, R);        // plane a = zs - 1 (zero unless in the grid)
        load_rech(zs - 1, S0);
        finish(zs - 1, R, Pa, S0);
    }
    // one step of the march; L = the finished plane t
    auto body = [&](const int t, const RPlane<XP, YP> &L, const Side &Sd) __attribute__((always_inline)) {
        const int a = t - 1, bpl = t - 2;
        float Qa[6], bR[6];
        qcoef(Pa, a, Qa);
        rcoef(bAh, bPb, bpl, bR);

        // ---- one LDS round: H(a), Q(a), E^n(b), R(b)
#pragma unroll
        for (int q = 0; q < 3; q++) sH[q][row][lane] = Pa.h[q];
        sQ[0][row][lane] = Qa[1];   // Ez along y
        sQ[1][row][lane] = Qa[3];   // Ez along x
        sQ[2][row][lane] = Qa[4];   // Ex along y
        sQ[3][row][lane] = Qa[5];   // Ey along x
#pragma unroll
        for (int q = 0; q < 3; q++) sEn[q][row][lane] = bEn[q];
        sR[0][row][lane] = bR[1];   // Hz along y
        sR[1][row][lane] = bR[2];   // Hz along x
        sR[2][row][lane] = bR[4];   // Hx along y
        sR[3][row][lane] = bR[5];   // Hy along x
        lds_barrier();
        const int ru = row + 1 < EY ? row + 1 : row, rd = row > 0 ? row - 1 : row;
        const int lr = lane + 1 < EX ? lane + 1 : lane, ll = lane > 0 ? lane - 1 : lane;

        // ---------------------------------------------------- phase A at plane a
        float aEn[3], aAh[3];
        {
            const bool kin = a >= 0 && a < nz;
            const bool interior = icol && kin && (p == 0 || (a >= p && a < nz - p));
            const float hx = Pa.h[0], hy = Pa.h[1], hz = Pa.h[2];
            const float hz_y = sH[2][rd][lane], hx_y = sH[0][rd][lane];
            const float hz_x = sH[2][row][ll], hy_x = sH[1][row][ll];
            const float dy_hz = hz - hz_y, dz_hy = hy - Hm1;
            const float dz_hx = hx - Hm0, dx_hz = hz - hz_x;
            const float dx_hy = hy - hy_x, dy_hx = hx - hx_y;
            const bool hex = y == 0 || a == 0, hey = x == 0 || a == 0, hez = x == 0 || y == 0;
            // a conducting cell: E^n from the record of step n, and sigma
            const bool lossy = LOSSY && Sd.lossy;
            const float len[3] = {Sd.len[0], Sd.len[1], Sd.len[2]}, lsg = Sd.lsg;
            // dJ/dd += Ebar' . curl H^{n+1/2} (also in the adjoint-only mode,
            // where the forward state comes from storage instead of the inverse);
            // a conducting cell's term is Ebar' . (curl H - sigma E^n)
            if (Sd.gin) {
                float acc = Sd.acc;
                if (!lossy) {
                    if (!hex) acc = fmaf(Pa.ae[0], dy_hz - dz_hy, acc);
                    if (!hey) acc = fmaf(Pa.ae[1], dz_hx - dx_hz, acc);
                    if (!hez) acc = fmaf(Pa.ae[2], dx_hy - dy_hx, acc);
                } else {
                    if (!hex) acc = fmaf(Pa.ae[0], fmaf(-lsg, len[0], dy_hz - dz_hy), acc);
                    if (!hey) acc = fmaf(Pa.ae[1], fmaf(-lsg, len[1], dz_hx - dx_hz), acc);
                    if (!hez) acc = fmaf(Pa.ae[2], fmaf(-lsg, len[2], dx_hy - dy_hx), acc);
                }
                *(GLOBAL float *)(Rk->gacc + ((long long)(a - A.dlo.z) * dplane + dxy)) = acc;
            }
            if (do_inv && interior) {
                float ex = Pa.e[0], ey = Pa.e[1], ez = Pa.e[2];
                // sources, in order (uniform plane test against the hoisted
                // source planes; one select per component)
#pragma unroll
                for (int q = 0; q < FD_MAXSRC; q++) {
                    if (a == skq[q]) {
                        const bool hit = Kp->g.skind[q] != 0 || (x == Kp->g.si[q] && y == Kp->g.sj[q]);
                        const float Am = sAmp[q];
                        const int comp = Kp->g.scomp[q];
                        ex = (hit && comp == 0 && !hex) ? ex - Am : ex;
                        ey = (hit && comp == 1 && !hey) ? ey - Am : ey;
                        ez = (hit && comp == 2 && !hez) ? ez - Am : ez;
                    }
                }
                const float ce = Pa.ce;
                if (!hex) ex = e_unupdate(ex, ce, dy_hz, dz_hy);
                if (!hey) ey = e_unupdate(ey, ce, dz_hx, dx_hz);
                if (!hez) ez = e_unupdate(ez, ce, dx_hy, dy_hx);
                if (lossy) { ex = len[0]; ey = len[1]; ez = len[2]; }
                aEn[0] = ex; aEn[1] = ey; aEn[2] = ez;
            } else {
                aEn[0] = Pa.e[0]; aEn[1] = Pa.e[1]; aEn[2] = Pa.e[2];
                // E^n on the high-face layers from the record of step n-1 (E^0 = 0;
                // loaded by side_load)
                if (do_inv) {
                    if (Sd.ec == 1) { aEn[0] = Sd.e0; aEn[1] = Sd.e1; }
                    if (Sd.ec == 2) { aEn[1] = Sd.e0; aEn[2] = Sd.e1; }
                    if (Sd.ec == 3) { aEn[2] = Sd.e0; aEn[0] = Sd.e1; }
                }
            }
            if (!(incol && kin)) { aEn[0] = aEn[1] = aEn[2] = 0.f; }
            if (do_adj) {
                float Qt[6];
                qcoef(L, t, Qt);
                const float qa = Qa[0] - Qt[0];
                const float qb = Qa[1] - sQ[0][ru][lane];
                const float qc = Qa[2] - Qt[2];
                const float qd = Qa[3] - sQ[1][row][lr];
                const float qe = Qa[4] - sQ[2][ru][lane];
                const float qf = Qa[5] - sQ[3][row][lr];
                aAh[0] = Pa.ah[0] + (qa + qb);
                aAh[1] = Pa.ah[1] + (qc + qd);
                aAh[2] = Pa.ah[2] + (qe + qf);
            } else {
                aAh[0] = aAh[1] = aAh[2] = 0.f;
            }
        }

        // ---------------------------------------------------- phase B at plane b
        {
            const bool kin = bpl >= 0 && bpl < nz;
            const bool interior = icol && kin && (p == 0 || (bpl >= p && bpl < nz - p));
            const bool hex = y == 0 || bpl == 0, hey = x == 0 || bpl == 0, hez = x == 0 || y == 0;
            const bool store = own && bpl >= z0 && bpl < z1;
            if (store) {
                const unsigned c = WIDE ? off * 4u : ((unsigned)bpl * nxy + off) * 4u;
                auto st = [&](float *base, unsigned o, float v) { *(GLOBAL float *)((GLOBAL char *)base + o) = v; };
                // component q of the forward (stf) and adjoint (sta) output sets at plane bpl
                auto stf = [&](int q, float v) {
                    if constexpr (WIDE) st(Kp->fld[ic ^ 1][q] + (size_t)bpl * (size_t)Kp->g.nxy, c, v);
                    else st(fout0, c + q * fs, v);
                };
                auto sta = [&](int q, float v) {
                    if constexpr (WIDE) st(Kp->adj[ia ^ 1][q] + (size_t)bpl * (size_t)Kp->g.nxy, c, v);
                    else st(aout0, c + q * fs, v);
                };
                if (do_inv && interior) {
                    const float ex = bEn[0], ey = bEn[1], ez = bEn[2];
                    const float ey_x = sEn[1][row][lr], ez_x = sEn[2][row][lr];
                    const float ex_y = sEn[0][ru][lane], ez_y = sEn[2][ru][lane];
                    const float ex_z = aEn[0], ey_z = aEn[1];
#pragma unroll
                    for (int q = 0; q < 3; q++) stf(q, bEn[q]);
                    // H sources of step n, in order, before the un-update
                    float hx = bH[0], hy = bH[1], hz = bH[2];
#pragma unroll
                    for (int q = 0; q < FD_MAXSRC; q++) {
                        if (bpl == skq[q]) {
                            const bool hit = Kp->g.skind[q] != 0 || (x == Kp->g.si[q] && y == Kp->g.sj[q]);
                            const float Am = sAmp[q];
                            const int comp = Kp->g.scomp[q];
                            hx = (hit && comp == 3) ? hx - Am : hx;
                            hy = (hit && comp == 4) ? hy - Am : hy;
                            hz = (hit && comp == 5) ? hz - Am : hz;
                        }
                    }
                    stf(3, h_unupdate(hx, S, ez_y - ez, ey_z - ey));
                    stf(4, h_unupdate(hy, S, ex_z - ex, ez_x - ez));
                    stf(5, h_unupdate(hz, S, ey_x - ey, ex_y - ex));
                }
                if (do_adj) {
                    // adjoint E with the transposed H pairs (a conducting cell
                    // passes ca Ebar' on)
                    float ex = bAe[0], ey = bAe[1], ez = bAe[2];
                    if constexpr (LOSSY) {
                        if (Sd.cin) {
                            const float ca = Sd.lca;
                            if (!hex) ex = ca * ex;
                            if (!hey) ey = ca * ey;
                            if (!hez) ez = ca * ez;
                        }
                    }
                    if (!hex) {
                        const float ra = Rz0 - bR[0];
                        const float rb = sR[0][rd][lane] - bR[1];
                        ex = ex + (ra + rb);
                    }
                    if (!hey) {
                        const float ra = sR[1][row][ll] - bR[2];
                        const float rb = Rz3 - bR[3];
                        ey = ey + (ra + rb);
                    }
                    if (!hez) {
                        const float ra = sR[2][rd][lane] - bR[4];
                        const float rb = sR[3][row][ll] - bR[5];
                        ez = ez + (ra + rb);
                    }
                    sta(0, ex); sta(1, ey); sta(2, ez);
#pragma unroll
                    for (int q = 0; q < 3; q++) sta(3 + q, bAh[q]);
                    // psibar updates of the slab cells
                    if (p > 0) {
                        const float ce = bCe;
                        const int szb = slab_coord(bpl, nz, p);
                        if (szb >= 0) {
                            const unsigned zi = (unsigned)szb * nxy + off;
                            const float bE = sGz[szb][0], bHh = sGz[szb][3];
                            // z idx 0: Ex (-), idx 1: Ey (+); idx 2: Hx (+S), idx 3: Hy (-S)
                            const float w0 = -1.f * (ce * bAe[0]), w1 = 1.f * (ce * bAe[1]);
                            st(A.pb[ip ^ 1][2], zi * 4u + 0 * A.pstride[2], hex ? bPb.z[0] : bE * (bPb.z[0] + w0));
                            st(A.pb[ip ^ 1][2], zi * 4u + 1 * A.pstride[2], hey ? bPb.z[1] : bE * (bPb.z[1] + w1));
                            st(A.pb[ip ^ 1][2], zi * 4u + 2 * A.pstride[2], bHh * (bPb.z[2] + 1.f * (S * bAh[0])));
                            st(A.pb[ip ^ 1][2], zi * 4u + 3 * A.pstride[2], bHh * (bPb.z[3] + -1.f * (S * bAh[1])));
                        }
                        if constexpr (XP) {
                            if (sx >= 0) {
                                const unsigned xi = (unsigned)bpl * (unsigned)ny * (unsigned)(2 * p) + soff_x;
                                // x idx 0: Ey (-), idx 1: Ez (+); idx 2: Hy (+S), idx 3: Hz (-S)
                                const float w0 = -1.f * (ce * bAe[1]), w1 = 1.f * (ce * bAe[2]);
                                st(A.pb[ip ^ 1][0], xi * 4u + 0 * A.pstride[0], hey ? bPb.x[0] : gxE.x * (bPb.x[0] + w0));
                                st(A.pb[ip ^ 1][0], xi * 4u + 1 * A.pstride[0], hez ? bPb.x[1] : gxE.x * (bPb.x[1] + w1));
                                st(A.pb[ip ^ 1][0], xi * 4u + 2 * A.pstride[0], gxH.x * (bPb.x[2] + 1.f * (S * bAh[1])));
                                st(A.pb[ip ^ 1][0], xi * 4u + 3 * A.pstride[0], gxH.x * (bPb.x[3] + -1.f * (S * bAh[2])));
                            }
                        }
                        if constexpr (YP) {
                            if (sy >= 0) {
                                const unsigned yi = (unsigned)bpl * (unsigned)(2 * p) * (unsigned)nx + soff_y;
                                // y idx 0: Ez (-), idx 1: Ex (+); idx 2: Hz (+S), idx 3: Hx (-S)
                                const float w0 = -1.f * (ce * bAe[2]), w1 = 1.f * (ce * bAe[0]);
                                st(A.pb[ip ^ 1][1], yi * 4u + 0 * A.pstride[1], hez ? bPb.y[0] : gyE.x * (bPb.y[0] + w0));
                                st(A.pb[ip ^ 1][1], yi * 4u + 1 * A.pstride[1], hex ? bPb.y[1] : gyE.x * (bPb.y[1] + w1));
                                st(A.pb[ip ^ 1][1], yi * 4u + 2 * A.pstride[1], gyH.x * (bPb.y[2] + 1.f * (S * bAh[2])));
                                st(A.pb[ip ^ 1][1], yi * 4u + 3 * A.pstride[1], gyH.x * (bPb.y[3] + -1.f * (S * bAh[0])));
                            }
                        }
                    }
                }
            }
        }
        lds_barrier();

        // ------------------------------------------------------------ rotate
        Rz0 = bR[0];
        Rz3 = bR[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            bEn[q] = aEn[q];
            bH[q] = Pa.h[q];
            bAe[q] = Pa.ae[q];
            bAh[q] = aAh[q];
        }
        bCe = Pa.ce;
        bPb = Pa.pb;
        Hm0 = Pa.h[0];
        Hm1 = Pa.h[1];
        Pa = L;
    };
    // Plane t+1 is in flight (in the LDS staging buffer) while plane t is
    // worked on.  The psi-bar and side loads of an iteration are issued
    // before the next plane's, so waiting for them does not wait for the
    // next plane (vector memory operations complete in order); the stage
    // reads are complete before the next plane's loads write over them.
    stage(zs);
    for (int t = zs; t < ze; t++) {
        asm volatile("" : "+s"(Kp), "+s"(Rk));
        RPlane<XP, YP> R, L;
        Side Sd;
        // (the compiler's own waits for loads that write LDS are not relied on)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        unstage(R);
        load_psi(t, R);
        side_load(t, Sd);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        // (issued on every iteration, so the compiler's wait counts for the
        // side loads stay exact; the last one fetches plane t again, from L2)
        stage(t + 1 < ze ? t + 1 : t);
        finish(t, R, L, Sd);
        body(t, L, Sd);
    }
    // nothing may still be writing the workgroup's LDS when it ends
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// The kernel: block b (XCD-remapped) finds its request and tile; the tile's
// class picks the march instance.
template <bool WIDE, int W, bool LOSSY>
__global__ __launch_bounds__(64 * W, 4) void k_tb_reverse(RevLaunch)
{
    __shared__ RevLds<W> lds;
    // (a variable of its own, so the compiler sees that the LDS exchanges do
    // not touch the staging buffer and does not wait for its loads there)
    __shared__ float sSt[RV_NST][64 * W];
    // (the launch block is the kernel's only parameter, at offset 0 of the
    // kernel-argument segment)
    KLaunch *Lp = (KLaunch *)__builtin_amdgcn_kernarg_segment_ptr();
    int b = blockIdx.x;
    if (Lp->xcd_remap) b = remap_xcd_r(b, gridDim.x);
    int r = 0;
    while (r + 1 < Lp->nreq && b >= Lp->r[r + 1].first) r++;
    KReq *Rq = &Lp->r[r];
    // Arguments used only on rare planes (record layers, detector, source)
    // are read through a copy of this pointer that is made opaque on every
    // plane, so they are fetched where used instead of being held in scalar
    // registers for the whole march.
    KArgs *Ap = (KArgs *)Rq->args;
    const int4 *tt = Rq->tiles + 2 * (b - Rq->first);
    const int4 tl = tt[0], tz = tt[1];
    switch (tz.z) {
    case 0: rev_march<false, false, WIDE, W, LOSSY>(*Ap, Ap, Rq, tl, tz, lds, sSt); break;
    case 1: rev_march<true, false, WIDE, W, LOSSY>(*Ap, Ap, Rq, tl, tz, lds, sSt); break;
    case 2: rev_march<false, true, WIDE, W, LOSSY>(*Ap, Ap, Rq, tl, tz, lds, sSt); break;
    default: rev_march<true, true, WIDE, W, LOSSY>(*Ap, Ap, Rq, tl, tz, lds, sSt); break;
    }
}

}  // namespace

int rev_halo() { return HALO; }
int rev_tile_x() { return EX - 2 * HALO; }
// waves per workgroup of the reverse march: 8, two workgroups per CU.
// (12 waves, three per SIMD with up to 168 registers and no spills, 20 of 22
// rows owned, one workgroup per CU: bitwise equal, but 0.370 against 0.361
// ms per step on 200^3 and 21.2 against 19.8 s for the 640x640x400 reverse)
constexpr int REV_W = 8;
int rev_tile_y() { return rows_of(REV_W) - 2 * HALO; }
int rev_wg_per_cu() { return 2; }

hipError_t launch_tb_reverse(const RevLaunch &L, bool wide, bool lossy, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    if (lossy) {
        // conducting cells: 32-bit offsets only
        if (wide) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_tb_reverse<false, REV_W, true>), dim3(L.nblocks), dim3(64 * REV_W), 0, s, L);
    } else if (wide) {
        hipLaunchKernelGGL((k_tb_reverse<true, REV_W, false>), dim3(L.nblocks), dim3(64 * REV_W), 0, s, L);
    } else {
        hipLaunchKernelGGL((k_tb_reverse<false, REV_W, false>), dim3(L.nblocks), dim3(64 * REV_W), 0, s, L);
    }
    return hipGetLastError();
}
