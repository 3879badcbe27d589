// Host side of libfdtd: validation, workspace planning, CPML grading tables,
// launch sequencing and the extern "C" entry points declared in fdtd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdtd.h"
#include "fdtd_internal.h"

namespace {

thread_local char g_err[512] = "";

// ------------------------------------------------------------ bump planner
// The same sequence of take() calls sizes the workspace (base == nullptr) and
// carves it at create time, so footprint and layout can never disagree.
struct Bump {
    char *base;
    size_t off = 0;
    explicit Bump(void *b) : base((char *)b) {}
    float *take(size_t floats)
    {
        off = (off + 255) & ~(size_t)255;
        float *p = base ? (float *)(base + off) : nullptr;
        off += floats * sizeof(float);
        return p;
    }
    template <class T> T *take_as(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct Geometry {
    int nx, ny, nz, p;
    long long N, slab_n[3];
    RecGeom R;
    Detectors D;
    long long design_cells;
    long long lossy_cells;          // cells of the lossy box (0: none)
};

}  // namespace

struct fdtd_ctx {
    fdtd_desc desc;
    fdtd_source src[FDTD_MAX_SOURCES];
    fdtd_flux_detector det[FDTD_MAX_DETECTORS];
    int nsrc = 0, ndet = 0;
    hipStream_t stream = nullptr;
    int device = 0;                        // HIP device current at create
    char err[512] = "";
    int t = 0;
    int T = 0;
    int K = 1;
    Geometry geo;
    Grid g;
    // forward state, ping-pong
    float *fld[2][6];
    float *psi[2][3][4];
    int cur = 0;
    bool in_grad = false;                  // between fdtd_grad_begin and fdtd_grad_end
    int grad_np = 0;                       // partial sums of the interior norm at t = T
    // adjoint state: fields, psi-bar E-type (in place), psi-bar H-type (ping-pong)
    float *adj[2][6];
    float *pb[2][3][4];
    int acur = 0, apar = 0;
    float *ce = nullptr, *inv_eps = nullptr, *d_design = nullptr;
    float *lsig = nullptr, *lca = nullptr;  // conducting cells: sigma and ca per lossy-box cell
    float *prof[2][3][3];
    float *amps[FDTD_MAX_SOURCES];         // per internal source (see expand_sources)
    // total-field/scattered-field planes: their waveforms and the incident line
    int ntfsf = 0;
    int tfsf_pub[FD_MAXSRC / 2];           // public source index of each plane
    int tfsf_slot[FD_MAXSRC / 2][2];       // internal E and H source slots
    float *twave[FD_MAXSRC / 2];
    float *tline = nullptr;
    float *raw = nullptr, *eprev = nullptr;  // interpolated detectors: K raw plane sets, E^n planes
    float *red = nullptr;
    float *trace = nullptr, *planes = nullptr, *wdev = nullptr, *rec = nullptr, *gacc = nullptr;
    // detector planes of up to pcap steps are summed into the trace together:
    // pfill steps from step pbase are waiting
    int pcap = 1, pfill = 0, pbase = 0;
    float *parts[2] = {nullptr, nullptr};
    int nparts_cap = 0;
    int4 *tiles = nullptr;                 // tile tables: the reverse march, then every K' <= K
    int tb_off[5], tb_n[5];                // per table: first tile, tiles (all classes, spatial order)
    int tb_cnt[5][4];                      // per table and class: tiles
    TbArgs *targs = nullptr;               // the z-marches' fixed arguments, in the workspace
    RevArgs *rargs = nullptr;
    TbArgs host_targs;                     // (host copies, kept for the uploads)
    RevArgs host_rargs;
    unsigned fstride, pstride[3];   // z-march addressing: bytes between arrays of one set
    float4 *profv[3];
    bool naive = false;                    // per-cell kernels instead of the z-march
    bool wide = false;                     // forward z-march with 64-bit component bases
    int shape = 0;                         // z-march workgroup shape
    float wS[FDTD_MAX_DETECTORS];
    float wS_plain[FDTD_MAX_DETECTORS];   // wS with the interpolated detectors' entries zero
    float *drec = nullptr, *drec_e0 = nullptr;  // interpolated detectors' planes of every step (gradients)
    std::vector<float> host_tables;        // kept alive for async uploads
    std::vector<int4> host_tiles;
};

namespace {

fdtd_status fail(fdtd_ctx *h, fdtd_status st, const char *fmt, ...)
{
    char *dst = h ? h->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return st;
}

#define HIPCHK(h, expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((h), FDTD_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

int dim_of(const fdtd_desc *d, int a) { return a == 0 ? d->nx : a == 1 ? d->ny : d->nz; }

// The kernels see plain additive sources only (kind 0 point, kind 1 z-plane,
// components 0..5).  A total-field/scattered-field plane (public kind 2) is
// two of them: its E correction on plane k (component = polarisation) and its
// H correction on layer k-1 (Hy for Ex, Hx for Ey), both fed by the incident
// line.  Returns the number of internal sources (may exceed FD_MAXSRC).
struct IntSrc {
    int kind, comp, i, j, k;
    int pub;       // public source index
    int role;      // 0: the caller's amplitude, 1: TFSF E correction, 2: TFSF H correction
};
int expand_sources(const fdtd_source *src, int nsrc, IntSrc *out, int cap)
{
    int n = 0;
    auto put = [&](IntSrc v) { if (n < cap) out[n] = v; n++; };
    for (int s = 0; s < nsrc; s++) {
        const fdtd_source &q = src[s];
        if (q.kind != 2) {
            put({q.kind, q.comp, q.i, q.j, q.k, s, 0});
        } else {
            put({1, q.comp, 0, 0, q.k, s, 1});
            put({1, q.comp == 0 ? 4 : 3, 0, 0, q.k - 1, s, 2});
        }
    }
    return n;
}

fdtd_status validate(fdtd_ctx *h, const fdtd_desc *d, const fdtd_source *src, int nsrc,
                     const fdtd_flux_detector *det, int ndet)
{
    if (!d) return fail(h, FDTD_E_INVALID, "desc is NULL");
    for (int a = 0; a < 3; a++)
        if (dim_of(d, a) < 4 || dim_of(d, a) > (1 << 20))
            return fail(h, FDTD_E_INVALID, "grid size %d on axis %d out of range [4, 2^20]", dim_of(d, a), a);
    if ((double)d->nx * d->ny * d->nz > 4.0e10) return fail(h, FDTD_E_INVALID, "grid too large");
    if (!(d->courant > 0.f) || !((double)d->courant < 1.0 / std::sqrt(3.0)))
        return fail(h, FDTD_E_INVALID, "courant %g outside (0, 1/sqrt(3))", (double)d->courant);
    const int p = d->pml_cells;
    if (p < 0) return fail(h, FDTD_E_INVALID, "pml_cells < 0");
    for (int a = 0; a < 3; a++)
        if (p > 0 && dim_of(d, a) < 2 * p + 2)
            return fail(h, FDTD_E_INVALID, "axis %d too small for %d PML cells", a, p);
    if (!d->inv_eps) return fail(h, FDTD_E_INVALID, "inv_eps is NULL");
    if (d->n_steps < 1) return fail(h, FDTD_E_INVALID, "n_steps < 1");
    if (d->time_block < 0 || d->time_block > 4) return fail(h, FDTD_E_INVALID, "time_block outside [0,4]");
    if (d->record != 0 && d->record != 1) return fail(h, FDTD_E_INVALID, "record must be 0 or 1");
    if (nsrc < 0 || nsrc > FDTD_MAX_SOURCES) return fail(h, FDTD_E_INVALID, "nsrc outside [0,%d]", FDTD_MAX_SOURCES);
    if (ndet < 0 || ndet > FDTD_MAX_DETECTORS) return fail(h, FDTD_E_INVALID, "ndet outside [0,%d]", FDTD_MAX_DETECTORS);
    if (nsrc > 0 && !src) return fail(h, FDTD_E_INVALID, "sources NULL");
    if (ndet > 0 && !det) return fail(h, FDTD_E_INVALID, "detectors NULL");
    for (int s = 0; s < nsrc; s++) {
        const fdtd_source &q = src[s];
        if (q.kind < 0 || q.kind > 2) return fail(h, FDTD_E_INVALID, "source %d: kind must be 0, 1 or 2", s);
        if (q.kind != 2 && (q.comp < 0 || q.comp > 5)) return fail(h, FDTD_E_INVALID, "source %d: comp must be 0..5", s);
        if (q.kind == 2 && q.comp != 0 && q.comp != 1)
            return fail(h, FDTD_E_INVALID, "source %d: TFSF polarisation must be 0 (Ex) or 1 (Ey)", s);
        if (q.k < 0 || q.k >= d->nz) return fail(h, FDTD_E_INVALID, "source %d: k out of range", s);
        if (q.kind == 0 && (q.i < 0 || q.i >= d->nx || q.j < 0 || q.j >= d->ny))
            return fail(h, FDTD_E_INVALID, "source %d: (i,j) out of range", s);
        if (q.kind == 2) {
            // both layers in the z interior, and outside the design box's z range
            // (the incident line takes the plane's material as given)
            if (q.k < p + 1 || q.k >= d->nz - p)
                return fail(h, FDTD_E_INVALID, "source %d: TFSF plane k must lie in [p+1, nz-p)", s);
            if (q.k - 1 < d->design_hi[2] && d->design_lo[2] <= q.k)
                return fail(h, FDTD_E_INVALID, "source %d: TFSF layers k-1, k meet the design box", s);
        }
        if (!q.amp) return fail(h, FDTD_E_INVALID, "source %d: amp is NULL", s);
    }
    {
        IntSrc tmp[2 * FDTD_MAX_SOURCES];
        if (expand_sources(src, nsrc, tmp, 2 * FDTD_MAX_SOURCES) > FD_MAXSRC)
            return fail(h, FDTD_E_INVALID, "sources need more than %d slots (a TFSF plane takes two)", FD_MAXSRC);
    }
    const bool rec = d->record == 1;
    auto inside = [&](int lo, int hi, int a) {
        const int n = dim_of(d, a);
        const int L = rec ? p : 0, H = rec ? n - p : n;
        return lo >= L && hi <= H && lo < hi;
    };
    for (int m = 0; m < ndet; m++) {
        const fdtd_flux_detector &q = det[m];
        if (q.k < 0 || q.k >= d->nz || !inside(q.i0, q.i1, 0) || !inside(q.j0, q.j1, 1) ||
            (rec && (q.k < p || q.k >= d->nz - p)))
            return fail(h, FDTD_E_INVALID, "detector %d outside the %s", m, rec ? "interior" : "grid");
        if (!std::isfinite(q.weight)) return fail(h, FDTD_E_INVALID, "detector %d: weight not finite", m);
        if (q.interpolate != 0 && q.interpolate != 1)
            return fail(h, FDTD_E_INVALID, "detector %d: interpolate must be 0 or 1", m);
        if (q.quantity != 0 && q.quantity != 1)
            return fail(h, FDTD_E_INVALID, "detector %d: quantity must be 0 (flux) or 1 (energy)", m);
        if (q.quantity == 1 && !q.interpolate)
            return fail(h, FDTD_E_INVALID, "detector %d: the energy detector needs interpolate = 1", m);
        // the co-located flux reads layer k-1 and the cells at i1, j1
        if (q.interpolate && (q.k < 1 || q.i1 > d->nx - 1 || q.j1 > d->ny - 1))
            return fail(h, FDTD_E_INVALID, "detector %d: interpolation needs k >= 1, i1 < nx, j1 < ny", m);
    }
    for (int a = 0; a < 3; a++)
        if (!inside(d->design_lo[a], d->design_hi[a], a))
            return fail(h, FDTD_E_INVALID, "design box axis %d outside the %s or empty", a, rec ? "interior" : "grid");
    if (d->sigma) {
        // conducting cells: a box in the interior, off the layers of any TFSF plane
        for (int a = 0; a < 3; a++) {
            const int lo = d->lossy_lo[a], hi = d->lossy_hi[a];
            if (!(lo >= p && hi <= dim_of(d, a) - p && lo < hi))
                return fail(h, FDTD_E_INVALID, "lossy box axis %d outside the interior or empty", a);
        }
        for (int s = 0; s < nsrc; s++)
            if (src[s].kind == 2 && src[s].k - 1 < d->lossy_hi[2] && d->lossy_lo[2] <= src[s].k)
                return fail(h, FDTD_E_INVALID, "source %d: TFSF layers k-1, k meet the lossy box", s);
    }
    return FDTD_OK;
}

void geometry(const fdtd_desc *d, const fdtd_flux_detector *det, int ndet, Geometry &G)
{
    G.nx = d->nx; G.ny = d->ny; G.nz = d->nz; G.p = d->pml_cells;
    G.N = (long long)d->nx * d->ny * d->nz;
    const int n[3] = {d->nx, d->ny, d->nz};
    for (int a = 0; a < 3; a++) G.slab_n[a] = G.p > 0 ? 2LL * G.p * (G.N / n[a]) : 0;
    long long off = 0;
    for (int a = 0; a < 3; a++) {
        const int ua = a == 0 ? 1 : 0, va = a == 2 ? 1 : 2;
        G.R.Lu[a] = G.p > 0 ? n[ua] - 2 * G.p : 0;
        G.R.Lv[a] = G.p > 0 ? n[va] - 2 * G.p : 0;
        for (int side = 0; side < 2; side++) {
            G.R.off[2 * a + side] = off;
            off += 2LL * G.R.Lu[a] * G.R.Lv[a];
        }
    }
    // the record of step n ends with E^n of the lossy box (three components)
    G.lossy_cells = 0;
    if (d->sigma) {
        G.lossy_cells = 1;
        for (int a = 0; a < 3; a++) G.lossy_cells *= (d->lossy_hi[a] - d->lossy_lo[a]);
    }
    G.R.loff = off;
    G.R.per_step = off + 3 * G.lossy_cells;
    G.D.ndet = ndet;
    long long doff = 0, roff = 0, eoff = 0;
    for (int m = 0; m < FDTD_MAX_DETECTORS; m++) {
        G.D.roff[m] = roff;
        G.D.eoff[m] = eoff;
        if (m < ndet) {
            G.D.k[m] = det[m].k; G.D.i0[m] = det[m].i0; G.D.i1[m] = det[m].i1;
            G.D.j0[m] = det[m].j0; G.D.j1[m] = det[m].j1;
            G.D.off[m] = doff;
            doff += (long long)(det[m].i1 - det[m].i0) * (det[m].j1 - det[m].j0);
            G.D.interp[m] = det[m].interpolate ? 1 : 0;
            G.D.energy[m] = det[m].quantity == 1 ? 1 : 0;
            if (G.D.interp[m]) {
                const long long L = (long long)(det[m].i1 - det[m].i0 + 1) * (det[m].j1 - det[m].j0 + 1);
                roff += (G.D.energy[m] ? 9 : 6) * L;
                eoff += (G.D.energy[m] ? 4 : 2) * L;
            }
        } else {
            G.D.k[m] = G.D.i0[m] = G.D.i1[m] = G.D.j0[m] = G.D.j1[m] = 0;
            G.D.off[m] = doff;
            G.D.interp[m] = 0;
            G.D.energy[m] = 0;
        }
    }
    G.D.per_step = doff;
    G.D.raw_per_step = roff;
    G.D.eprev_floats = eoff;
    G.D.kmin = 1 << 30;
    G.D.kmax = -1;
    for (int m = 0; m < ndet; m++) {
        G.D.kmin = std::min(G.D.kmin, det[m].k - (det[m].quantity == 1 ? 1 : 0));
        G.D.kmax = std::max(G.D.kmax, det[m].k);
    }
    G.design_cells = 1;
    for (int a = 0; a < 3; a++) G.design_cells *= (d->design_hi[a] - d->design_lo[a]);
}

// ------------------------------------------------------------- tile planner
// (the workgroup shape, time block, tiles and march lengths: together with
// the z-march kernel they decide the sweep's memory traffic)

// forward z-march workgroup shape: 0: 16 waves of 64-lane rows (64 x 16
// tile), 1: 8 waves of 32-lane rows (32 x 16 tile, two workgroups per CU),
// 2 / 3: rows of 32 + 2K lanes whose owned part is one aligned 128-byte line,
// 16 / 8 waves.  3 measured fastest on the 256^3 benchmark grid.
int tb_shape()
{
    if (const char *e = getenv("FDTD_TB_SHAPE")) return atoi(e);
    return 3;
}

int choose_K(const fdtd_desc *d)
{
    if (d->time_block > 0) return d->time_block;
    return 2;
}

// Split [0, n) into tiles of at most `w` cells: one full tile at each end,
// the middle evenly.  With w - K >= p the middle tiles' halos stay clear of
// the CPML slabs.
std::vector<std::pair<int, int>> split_axis(int n, int w)
{
    std::vector<std::pair<int, int>> v;
    if (n <= w) { v.push_back({0, n}); return v; }
    if (n <= 2 * w) { v.push_back({0, n / 2}); v.push_back({n / 2, n}); return v; }
    v.push_back({0, w});
    const int mid = n - 2 * w;
    const int m = (mid + w - 1) / w;
    for (int i = 0; i < m; i++) v.push_back({w + (int)((long long)mid * i / m), w + (int)((long long)mid * (i + 1) / m)});
    v.push_back({n - w, n});
    return v;
}

// Split [0, n) into consecutive tiles of w cells (the last one shorter).
std::vector<std::pair<int, int>> split_uniform(int n, int w)
{
    std::vector<std::pair<int, int>> v;
    for (int a = 0; a < n; a += w) v.push_back({a, std::min(n, a + w)});
    return v;
}

// z extent of one workgroup's march.  Marches are split evenly: nz planes in
// ceil(nz / zc) chunks of equal length (up to one plane), never longer than
// zc.
int even_chunk(int nz, int zc)
{
    const int nc = (nz + zc - 1) / zc;
    return (nz + nc - 1) / nc;
}

int zchunk(const Geometry &G, int K, bool reverse)
{
    const char *e = getenv(reverse ? "FDTD_REV_ZC" : "FDTD_TB_ZC");
    if (e && atoi(e) > 0) return std::min(atoi(e), G.nz);
    if (reverse) {
        // The reverse march is kept short: the longest of at most 20 planes that
        // still gives four workgroups per slot and leaves no last chunk shorter
        // than half a march (which would hold a march of a few planes and its
        // whole z halo), else 8.  One launch holds every tile class, so many
        // short marches balance the slab classes' longer ones.  Measured on
        // 200^3: 10 planes 0.346 ms per step (11 with a 2-plane last chunk
        // 0.361, 8: 0.354, 13: 0.371, 15: 0.364, 20: 0.376).  Planes of 2M
        // cells or more take even marches of up to 60 planes while those leave
        // eight workgroups per slot: 58 x 7 on 640x640x400, 50 x 3 on
        // 2400x1600x150 (18.0 against 20.0-21.0 ms per step at 19).
        const long long tx = (long long)split_uniform(G.nx, rev_tile_x()).size();
        const long long ty = (long long)split_axis(G.ny, rev_tile_y()).size();
        const long long slots = (long long)rev_wg_per_cu() * 256;
        if ((long long)G.nx * G.ny >= (2LL << 20) && tx * ty * ((G.nz + 59) / 60) >= 8 * slots)
            return even_chunk(G.nz, std::min(60, G.nz));
        for (int zc = std::min(20, G.nz); zc > 8; zc--)
            if (tx * ty * ((G.nz + zc - 1) / zc) >= 4 * slots && (G.nz % zc == 0 || 2 * (G.nz % zc) >= zc))
                return zc;
        return even_chunk(G.nz, std::min(8, G.nz));
    }
    // The forward march: a longer one fetches its 2K-plane z halo less often
    // but leaves fewer workgroups, and the last round of workgroups may fill
    // the chip only in part.  Over even splits into 16..80-plane marches that
    // leave at least two workgroups per slot, take the least
    // rounds x (planes + 2K).  Measured on 256^3: 37 planes 86.3 Gcell/s
    // (against 81.4 at 24, 82.2 at 20, 81.9 at 43, 72.5 at 64); 640x640x400:
    // 67-80 planes 104-105 (100.5 at 134); 2400x1600x150: 75.
    const int shape = tb_shape();
    const long long fslots = (long long)tb_wg_per_cu(shape) * 256;
    const long long tx = (long long)(tb_tile_aligned(shape) ? split_uniform(G.nx, tb_tile_x(K, shape))
                                                             : split_axis(G.nx, tb_tile_x(K, shape))).size();
    const long long ty = (long long)split_axis(G.ny, tb_tile_y(K, shape)).size();
    long long best = -1;
    int bz = 0;
    for (int nc = 1; nc <= G.nz; nc++) {
        const int z = (G.nz + nc - 1) / nc;
        if (z > 80) continue;
        if (z < 16) break;
        const long long nwg = tx * ty * nc;
        if (nwg < 2 * fslots) continue;
        const long long cost = (nwg + fslots - 1) / fslots * (z + 2 * K);
        if (best < 0 || cost < best) { best = cost; bz = z; }
    }
    return bz > 0 ? bz : even_chunk(G.nz, std::min(16, G.nz));
}

// The kernels hand the XCDs contiguous runs of the table (the first nb % 8
// runs one tile longer), and each XCD starts its run's tiles in order.
// Within each run, tiles that own under three quarters of the run's largest
// tile (the last, partial x or y tile of a row or column) go last, so the
// run ends on short marches rather than on a full one started late; the
// order is otherwise kept (neighbouring tiles, which share halo lines in
// the XCD's L2, stay together).
void lpt_per_xcd(std::vector<int4> &out, int off, int n)
{
    if (n <= 0) return;
    const int q = n / 8, rem = n % 8;
    auto cells = [](const std::pair<int4, int4> &u) {
        return (long long)(u.first.y - u.first.x) * (u.first.w - u.first.z) * (u.second.y - u.second.x);
    };
    int a = 0;
    for (int x = 0; x < 8; x++) {
        const int len = q + (x < rem ? 1 : 0);
        std::vector<std::pair<int4, int4>> run(len);
        long long big = 0;
        for (int i = 0; i < len; i++) {
            run[i] = {out[2 * (off + a + i)], out[2 * (off + a + i) + 1]};
            big = std::max(big, cells(run[i]));
        }
        std::stable_partition(run.begin(), run.end(),
                              [&](const std::pair<int4, int4> &u) { return 4 * cells(u) >= 3 * big; });
        for (int i = 0; i < len; i++) {
            out[2 * (off + a + i)] = run[i].first;
            out[2 * (off + a + i) + 1] = run[i].second;
        }
        a += len;
    }
}

// Tile tables of the z-march kernels: slot 0 for the fused reverse march,
// slot K' for a forward sweep of K' = 1..K steps.  Each table lists every
// tile in spatial order (x fastest, then y, then z chunks) with its class
// (bit 0 = an x CPML slab inside the halo-extended footprint, bit 1 = a y
// slab), so that consecutive tiles -- one XCD's share after the remap --
// are neighbours with the grid's mix of classes.
void build_tiles(const Geometry &G, int K, std::vector<int4> &out, int off[5], int n[5], int cnt[5][4])
{
    out.clear();
    for (int kk = 0; kk < 5; kk++) {
        off[kk] = n[kk] = 0;
        for (int c = 0; c < 4; c++) cnt[kk][c] = 0;
    }
    // slot 0: the reverse march (halo rev_halo()); slots 1..K: forward, halo kk
    for (int kk = 0; kk <= K; kk++) {
        const int halo = kk == 0 ? rev_halo() : kk;
        const int ZC = zchunk(G, halo, kk == 0);
        const int tx = kk == 0 ? rev_tile_x() : tb_tile_x(kk, tb_shape());
        const int ty = kk == 0 ? rev_tile_y() : tb_tile_y(kk, tb_shape());
        // line-aligned shapes (and the reverse march) cut x into whole lines
        // from x = 0
        const auto xs = (kk == 0 || tb_tile_aligned(tb_shape())) ? split_uniform(G.nx, tx) : split_axis(G.nx, tx);
        const auto ys = split_axis(G.ny, ty);
        off[kk] = (int)out.size() / 2;
        for (int z0 = 0; z0 < G.nz; z0 += ZC)
            for (const auto &yt : ys)
                for (const auto &xt : xs) {
                    const int z1 = std::min(z0 + ZC, G.nz);
                    int c = 0;
                    if (G.p > 0) {
                        if (xt.first - halo < G.p || xt.second + halo > G.nx - G.p) c |= 1;
                        if (yt.first - halo < G.p || yt.second + halo > G.ny - G.p) c |= 2;
                    }
                    out.push_back(make_int4(xt.first, xt.second, yt.first, yt.second));
                    out.push_back(make_int4(z0, z1, c, 0));
                    cnt[kk][c]++;
                }
        n[kk] = (int)out.size() / 2 - off[kk];
        // (forward sweeps only: measured on 200^3, the forward with the record
        // 214.1 against 217.9 ms for 1500 steps, the reverse 546 against 520 ms)
        if (kk > 0) lpt_per_xcd(out, off[kk], n[kk]);
    }
}

// ------------------------------------------------------ end of tile planner

long long interior_cells(const Geometry &G)
{
    return (long long)(G.nx - 2 * G.p) * (G.ny - 2 * G.p) * (G.nz - 2 * G.p);
}

// Carve (or size) the workspace.  Every pointer of h is set when base != nullptr.
size_t plan(fdtd_ctx *h, const fdtd_desc *d, const Geometry &G, int K, void *base)
{
    Bump B(base);
    const int n[3] = {d->nx, d->ny, d->nz};
    const long long N = G.N;
    for (int b = 0; b < 2; b++)
        for (int q = 0; q < 6; q++) h->fld[b][q] = B.take(N);
    for (int b = 0; b < 2; b++)
        for (int a = 0; a < 3; a++)
            for (int q = 0; q < 4; q++) h->psi[b][a][q] = G.p > 0 ? B.take(G.slab_n[a]) : nullptr;
    h->ce = B.take(N);
    h->d_design = B.take(G.design_cells);
    h->lsig = G.lossy_cells > 0 ? B.take(G.lossy_cells) : nullptr;
    h->lca = G.lossy_cells > 0 ? B.take(G.lossy_cells) : nullptr;
    for (int t = 0; t < 2; t++)
        for (int a = 0; a < 3; a++)
            for (int f = 0; f < 3; f++) h->prof[t][a][f] = B.take(n[a]);
    for (int s = 0; s < FDTD_MAX_SOURCES; s++) h->amps[s] = B.take(d->n_steps);
    for (int t = 0; t < FD_MAXSRC / 2; t++) h->twave[t] = t < h->ntfsf ? B.take(d->n_steps) : nullptr;
    h->tline = h->ntfsf > 0 ? B.take(2 * (size_t)tfsf_line_nodes(d->n_steps)) : nullptr;
    h->trace = B.take((size_t)d->n_steps * std::max(1, G.D.ndet));
    // the z-march's flux planes of up to pcap steps (a multiple of K, at most
    // 64, within 256 MB) wait for one fixed-order sum launch
    {
        const int k1 = std::max(1, K);
        const long long ps = std::max<long long>(1, G.D.per_step);
        const long long fit = std::max<long long>(1, (256LL << 20) / (4 * ps));
        h->pcap = k1 * (int)std::max<long long>(1, std::min<long long>(64 / k1, fit / k1));
    }
    h->planes = B.take((size_t)h->pcap * std::max<long long>(1, G.D.per_step));
    h->raw = G.D.raw_per_step > 0 ? B.take((size_t)std::max(1, K) * G.D.raw_per_step) : nullptr;
    h->eprev = G.D.eprev_floats > 0 ? B.take(G.D.eprev_floats) : nullptr;
    // with the adjoint state, the interpolated detectors' planes of every step
    // (their adjoint source reads steps n-1, n, n+1) and of step 0
    const bool keep = d->record && G.D.raw_per_step > 0;
    h->drec = keep ? B.take((size_t)d->n_steps * G.D.raw_per_step) : nullptr;
    h->drec_e0 = keep ? B.take(G.D.eprev_floats) : nullptr;
    h->wdev = B.take(FDTD_MAX_DETECTORS);
    {
        long long rs = 1;
        for (int m = 0; m < G.D.ndet; m++)
            rs = std::max(rs, reduce_scratch_floats((long long)(G.D.i1[m] - G.D.i0[m]) * (G.D.j1[m] - G.D.j0[m]),
                                                    h->pcap));
        h->red = B.take(rs);
    }
    build_tiles(G, K, h->host_tiles, h->tb_off, h->tb_n, h->tb_cnt);
    h->tiles = B.take_as<int4>(std::max<size_t>(1, h->host_tiles.size()));
    h->targs = B.take_as<TbArgs>(1);
    h->rargs = B.take_as<RevArgs>(1);
    for (int ax = 0; ax < 3; ax++) h->profv[ax] = B.take_as<float4>(2 * (size_t)n[ax]);
    const long long nparts = (interior_cells(G) + 255) / 256;
    h->nparts_cap = (int)nparts;
    h->parts[0] = B.take(nparts);
    h->parts[1] = B.take(nparts);
    if (d->record) {
        h->rec = B.take((size_t)d->n_steps * G.R.per_step);
        for (int b = 0; b < 2; b++)
            for (int q = 0; q < 6; q++) h->adj[b][q] = B.take(N);
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 3; a++)
                for (int q = 0; q < 4; q++) h->pb[b][a][q] = G.p > 0 ? B.take(G.slab_n[a]) : nullptr;
        h->gacc = B.take(G.design_cells);
    } else {
        h->rec = nullptr;
        h->gacc = nullptr;
        for (int b = 0; b < 2; b++) {
            for (int q = 0; q < 6; q++) h->adj[b][q] = nullptr;
            for (int a = 0; a < 3; a++)
                for (int q = 0; q < 4; q++) h->pb[b][a][q] = nullptr;
        }
    }
    return B.off + 256;
}

// CFS-CPML grading (Roden-Gedney form) at the staggered coordinate u of an
// axis with n cells and p PML cells.
void grade(int n, int p, double u, double m, double smax, double kmax, double amax, float out[3])
{
    double delta = 0.0;
    if (p > 0) delta = std::max(std::max(p - u, u - (n - p)), 0.0) / p;
    if (delta <= 0.0) { out[0] = 1.f; out[1] = 0.f; out[2] = 1.f; return; }
    const double dm = std::pow(delta, m);
    const double sig = smax * dm;
    const double kap = 1.0 + (kmax - 1.0) * dm;
    const double alp = amax * (1.0 - delta);
    const double b = std::exp(-(sig / kap + alp));
    const double a = sig > 0.0 ? sig / (sig * kap + kap * kap * alp) * (b - 1.0) : 0.0;
    out[0] = (float)b; out[1] = (float)a; out[2] = (float)(1.0 / kap);
}

Fields fields_of(fdtd_ctx *h, int b)
{
    Fields F;
    for (int q = 0; q < 6; q++) F.c[q] = h->fld[b][q];
    return F;
}

Psi psi_of(fdtd_ctx *h, int b)
{
    Psi P;
    for (int a = 0; a < 3; a++)
        for (int q = 0; q < 4; q++) P.a[a][q] = h->psi[b][a][q];
    return P;
}

Psi psibar_of(fdtd_ctx *h, int par)
{
    Psi P;
    for (int a = 0; a < 3; a++)
        for (int q = 0; q < 4; q++) P.a[a][q] = h->pb[par][a][q];
    return P;
}

Fields adj_of(fdtd_ctx *h, int buf)
{
    Fields A;
    for (int q = 0; q < 6; q++) A.c[q] = h->adj[buf][q];
    return A;
}

fdtd_status zero_forward(fdtd_ctx *h)
{
    const Geometry &G = h->geo;
    for (int b = 0; b < 2; b++) {
        for (int q = 0; q < 6; q++) HIPCHK(h, launch_fill(h->fld[b][q], G.N, 0.f, h->stream));
        for (int a = 0; a < 3; a++)
            for (int q = 0; q < 4; q++)
                if (h->psi[b][a][q]) HIPCHK(h, launch_fill(h->psi[b][a][q], G.slab_n[a], 0.f, h->stream));
    }
    h->cur = 0;
    return FDTD_OK;
}

fdtd_status zero_adjoint(fdtd_ctx *h)
{
    if (!h->desc.record) return FDTD_OK;
    const Geometry &G = h->geo;
    for (int b = 0; b < 2; b++) {
        for (int q = 0; q < 6; q++) HIPCHK(h, launch_fill(h->adj[b][q], G.N, 0.f, h->stream));
        for (int a = 0; a < 3; a++)
            for (int q = 0; q < 4; q++)
                if (h->pb[b][a][q]) HIPCHK(h, launch_fill(h->pb[b][a][q], G.slab_n[a], 0.f, h->stream));
    }
    h->acur = 0;
    h->apar = 0;
    return FDTD_OK;
}

// one forward step n with the per-cell kernels (in place on buffer cur)
fdtd_status step_naive(fdtd_ctx *h, int n, int with_src, int with_rec, int with_det)
{
    Fields F = fields_of(h, h->cur);
    Psi P = psi_of(h, h->cur);
    const Geometry &G = h->geo;
    const bool interp = with_det && h->raw;
    float *rawt = h->drec ? h->drec + (size_t)n * G.D.raw_per_step : h->raw;
    if (interp) HIPCHK(h, launch_det_eprev(h->g, F, G.D, h->eprev, h->stream));
    if (interp && h->drec && n == 0) HIPCHK(h, launch_det_eprev(h->g, F, G.D, h->drec_e0, h->stream));
    HIPCHK(h, launch_h_naive(h->g, F, P, n, with_src, h->stream));
    const bool iface = with_rec && h->rec && G.p > 0;
    if (iface) HIPCHK(h, launch_record(h->g, F, G.R, h->rec + (size_t)n * G.R.per_step, 0, 0, h->stream));
    float *lrec = (with_rec && h->rec && G.lossy_cells > 0) ? h->rec + (size_t)n * G.R.per_step + G.R.loff : nullptr;
    HIPCHK(h, launch_e_naive(h->g, F, P, n, with_src, lrec, h->stream));
    if (iface) HIPCHK(h, launch_record(h->g, F, G.R, h->rec + (size_t)n * G.R.per_step, 1, 0, h->stream));
    if (with_det && G.D.ndet > 0) {
        HIPCHK(h, launch_det_planes(h->g, F, G.D, h->planes, h->stream));
        if (interp) {
            HIPCHK(h, launch_det_raw(h->g, F, G.D, rawt, h->stream));
            HIPCHK(h, launch_det_interp(h->g, G.D, rawt, h->eprev, 1, h->planes, h->stream));
        }
        for (int m = 0; m < G.D.ndet; m++) {
            const long long L = (long long)(G.D.i1[m] - G.D.i0[m]) * (G.D.j1[m] - G.D.j0[m]);
            HIPCHK(h, launch_reduce_rows2(h->planes + G.D.off[m], L, 1, G.D.per_step,
                                          h->trace + (size_t)n * G.D.ndet + m, G.D.ndet, h->red, h->stream));
        }
    }
    return FDTD_OK;
}

// The launch entry of handle h for a forward sweep of kk steps from n0
// (buffer cur -> cur^1); first = its first block in the launch.
TbReq tb_request(fdtd_ctx *h, int n0, int kk, int with_src, int with_rec, int with_det, int first)
{
    const Geometry &G = h->geo;
    TbReq q;
    q.args = (unsigned long long)(uintptr_t)h->targs;
    q.tiles = h->tiles + 2 * (size_t)h->tb_off[kk];
    q.rec = (with_rec && h->rec && G.R.per_step > 0) ? h->rec + (size_t)n0 * G.R.per_step : nullptr;
    q.planes = (with_det && G.D.ndet > 0) ? h->planes + (size_t)h->pfill * G.D.per_step : nullptr;
    q.raw = h->drec ? h->drec + (size_t)n0 * G.D.raw_per_step : h->raw;
    q.n0 = n0;
    q.first = first;
    q.flags = (h->cur ? TB_CUR : 0u) | (with_src ? TB_SRC : 0u);
    q.pad = 0;
    return q;
}

// what a forward sweep launches before its march (interpolated detectors'
// E^n gather, which reads buffer cur while the march writes the other one)
fdtd_status tb_prologue(fdtd_ctx *h, int n0, int with_det)
{
    const Geometry &G = h->geo;
    const bool planes = with_det && G.D.ndet > 0;
    if (planes && h->raw) HIPCHK(h, launch_det_eprev(h->g, fields_of(h, h->cur), G.D, h->eprev, h->stream));
    if (planes && h->drec && n0 == 0)
        HIPCHK(h, launch_det_eprev(h->g, fields_of(h, h->cur), G.D, h->drec_e0, h->stream));
    return FDTD_OK;
}

// the fixed-order sums of the waiting steps' detector planes into the trace
// (each step's sum is the same whichever steps share the launch)
fdtd_status flush_planes(fdtd_ctx *h)
{
    const Geometry &G = h->geo;
    if (h->pfill <= 0) return FDTD_OK;
    for (int m = 0; m < G.D.ndet; m++) {
        const long long L = (long long)(G.D.i1[m] - G.D.i0[m]) * (G.D.j1[m] - G.D.j0[m]);
        HIPCHK(h, launch_reduce_rows2(h->planes + G.D.off[m], L, h->pfill, G.D.per_step,
                                      h->trace + (size_t)h->pbase * G.D.ndet + m, G.D.ndet, h->red, h->stream));
    }
    h->pfill = 0;
    return FDTD_OK;
}

// what follows a forward sweep of kk steps from n0: swap the buffers, the
// detectors' densities; their sums into the trace once the planes of the
// next sweep would not fit (and at the end of every forward call)
fdtd_status tb_epilogue(fdtd_ctx *h, int n0, int kk, int with_det)
{
    const Geometry &G = h->geo;
    h->cur ^= 1;
    if (!(with_det && G.D.ndet > 0)) return FDTD_OK;
    float *raw = h->drec ? h->drec + (size_t)n0 * G.D.raw_per_step : h->raw;
    float *pl = h->planes + (size_t)h->pfill * G.D.per_step;
    if (h->raw) HIPCHK(h, launch_det_interp(h->g, G.D, raw, h->eprev, kk, pl, h->stream));
    if (h->pfill == 0) h->pbase = n0;
    h->pfill += kk;
    if (h->pfill + h->K > h->pcap) return flush_planes(h);
    return FDTD_OK;
}

// K' steps from n0 with the z-march kernel (buffer cur -> cur^1): one launch
// over the tiles of every class
fdtd_status steps_tb(fdtd_ctx *h, int n0, int kk, int with_src, int with_rec, int with_det)
{
    fdtd_status st = tb_prologue(h, n0, with_det);
    if (st != FDTD_OK) return st;
    TbLaunch L;
    L.nreq = 1;
    L.nblocks = h->tb_n[kk];
    L.xcd_remap = 1;
    L.pad = 0;
    L.r[0] = tb_request(h, n0, kk, with_src, with_rec, with_det, 0);
    HIPCHK(h, launch_tb_forward(L, kk, h->shape, h->wide, h->g.lca != nullptr, h->stream));
    return tb_epilogue(h, n0, kk, with_det);
}

fdtd_status advance(fdtd_ctx *h, int t0, int n, int with_src, int with_rec, int with_det)
{
    if (h->naive) {
        for (int s = t0; s < t0 + n; s++) {
            fdtd_status st = step_naive(h, s, with_src, with_rec, with_det);
            if (st != FDTD_OK) return st;
        }
        return FDTD_OK;
    }
    for (int s = t0; s < t0 + n;) {
        const int kk = std::min(h->K, t0 + n - s);
        fdtd_status st = steps_tb(h, s, kk, with_src, with_rec, with_det);
        if (st != FDTD_OK) return st;
        s += kk;
    }
    return flush_planes(h);
}

// one reverse step n: restore the interface layers, then the two phases
fdtd_status reverse_step(fdtd_ctx *h, int n, int do_adj)
{
    const Geometry &G = h->geo;
    Fields F = fields_of(h, h->cur);
    if (G.p > 0) {
        HIPCHK(h, launch_record(h->g, F, G.R, h->rec + (size_t)n * G.R.per_step, 0, 1, h->stream));
        if (n > 0)
            HIPCHK(h, launch_record(h->g, F, G.R, h->rec + (size_t)(n - 1) * G.R.per_step, 1, 1, h->stream));
        else
            HIPCHK(h, launch_record_zero_e(h->g, F, G.R, h->stream));
    }
    Fields A = do_adj ? adj_of(h, h->acur) : Fields{};
    if (do_adj && G.D.ndet > 0) HIPCHK(h, launch_det_adjoint(h->g, F, A, G.D, h->wS_plain, h->stream));
    Psi Pc = psibar_of(h, h->apar), Pn = psibar_of(h, h->apar ^ 1);
    const float *lrec = G.lossy_cells > 0 ? h->rec + (size_t)n * G.R.per_step + G.R.loff : nullptr;
    HIPCHK(h, launch_bwd_a(h->g, F, A, Pc, n, 1, do_adj, do_adj ? h->gacc : nullptr, h->desc.design_lo,
                           h->desc.design_hi, lrec, h->stream));
    HIPCHK(h, launch_bwd_b(h->g, F, A, Pc, Pn, n, 1, do_adj, h->stream));
    if (do_adj) h->apar ^= 1;
    return FDTD_OK;
}

// The launch entry of handle h for reverse step n with the fused z-march
// (all state ping-pong); do_inv = 0 applies only the adjoint of the
// source-free step map; fin: the forward state s_{n+1} read instead of the
// current buffer (adjoint-only mode), or nullptr.
RevReq rev_request(fdtd_ctx *h, int n, int do_inv, int do_adj, int with_det, float *gacc, const float *fin,
                   int first)
{
    const Geometry &G = h->geo;
    RevReq q;
    q.args = (unsigned long long)(uintptr_t)h->rargs;
    q.tiles = h->tiles + 2 * (size_t)h->tb_off[0];
    // (the record of step n: its interface layers, and E^n of the lossy box)
    q.rec_h = (do_inv && (G.p > 0 || G.lossy_cells > 0)) ? h->rec + (size_t)n * G.R.per_step : nullptr;
    q.rec_e = (do_inv && G.p > 0 && n > 0) ? h->rec + (size_t)(n - 1) * G.R.per_step : nullptr;
    q.gacc = gacc;
    q.fin = fin;
    q.n = n;
    q.first = first;
    q.flags = (h->cur ? RV_CUR : 0u) | (h->acur ? RV_ACUR : 0u) | (h->apar ? RV_APAR : 0u) |
              (do_inv ? RV_INV : 0u) | (do_adj ? RV_ADJ : 0u) | ((with_det && G.D.ndet > 0) ? RV_DET : 0u);
    q.pad = 0;
    return q;
}

// the buffer swaps after a reverse step
void rev_epilogue(fdtd_ctx *h, int do_inv, int do_adj)
{
    if (do_inv) h->cur ^= 1;
    if (do_adj) {
        h->acur ^= 1;
        h->apar ^= 1;
    }
}

fdtd_status reverse_fused(fdtd_ctx *h, int n, int do_inv, int do_adj, int with_det, float *gacc,
                          const Fields *fin = nullptr)
{
    RevLaunch L;
    L.nreq = 1;
    L.nblocks = h->tb_n[0];
    L.xcd_remap = 1;
    L.pad = 0;
    L.r[0] = rev_request(h, n, do_inv, do_adj, with_det, gacc, fin ? fin->c[0] : nullptr, 0);
    HIPCHK(h, launch_tb_reverse(L, h->wide, h->g.lca != nullptr, h->stream));
    rev_epilogue(h, do_inv, do_adj);
    return FDTD_OK;
}

// the z-marches' fixed arguments of handle h (host copies)
void fill_static_args(fdtd_ctx *h)
{
    const Geometry &G = h->geo;
    TbArgs &t = h->host_targs;
    memset(&t, 0, sizeof t);
    t.g = h->g;
    for (int b = 0; b < 2; b++) {
        for (int q = 0; q < 6; q++) t.fld[b][q] = h->fld[b][q];
        for (int a = 0; a < 3; a++) t.psi[b][a] = h->psi[b][a][0];
    }
    t.R = G.R;
    t.D = G.D;
    for (int a = 0; a < 3; a++) t.profv[a] = h->profv[a];
    t.fstride = h->fstride;
    for (int a = 0; a < 3; a++) t.pstride[a] = h->pstride[a];
    RevArgs &r = h->host_rargs;
    memset(&r, 0, sizeof r);
    r.g = h->g;
    for (int b = 0; b < 2; b++) {
        for (int q = 0; q < 6; q++) {
            r.fld[b][q] = h->fld[b][q];
            r.adj[b][q] = h->adj[b][q];
        }
        for (int a = 0; a < 3; a++) r.pb[b][a] = h->pb[b][a][0];
    }
    r.R = G.R;
    r.D = G.D;
    for (int m = 0; m < FD_MAXDET; m++) r.wS[m] = h->wS_plain[m];
    r.dlo = make_int3(h->desc.design_lo[0], h->desc.design_lo[1], h->desc.design_lo[2]);
    r.dhi = make_int3(h->desc.design_hi[0], h->desc.design_hi[1], h->desc.design_hi[2]);
    for (int a = 0; a < 3; a++) r.profv[a] = h->profv[a];
    r.fstride = h->fstride;
    for (int a = 0; a < 3; a++) r.pstride[a] = h->pstride[a];
}

fdtd_status upload_materials(fdtd_ctx *h, const float *inv_eps)
{
    const Geometry &G = h->geo;
    HIPCHK(h, launch_scale_ce(inv_eps, h->desc.courant, h->ce, G.N, h->stream));
    HIPCHK(h, launch_lossy_coef(h->g, inv_eps, h->ce, h->lca, h->stream));
    HIPCHK(h, launch_gather_box(inv_eps, h->g, h->desc.design_lo, h->desc.design_hi, h->d_design, h->stream));
    // incident line of each TFSF plane, with S/eps_r of the plane's centre cell
    for (int t = 0; t < h->ntfsf; t++) {
        const fdtd_source &q = h->src[h->tfsf_pub[t]];
        const float *ce_at = h->ce + ((long long)q.k * G.ny + G.ny / 2) * G.nx + G.nx / 2;
        HIPCHK(h, launch_tfsf_line(h->twave[t], h->T, h->desc.courant, ce_at, q.comp == 0 ? 1.f : -1.f, h->tline,
                                   h->amps[h->tfsf_slot[t][0]], h->amps[h->tfsf_slot[t][1]], h->stream));
    }
    return FDTD_OK;
}

// number of TFSF planes among the public sources
int count_tfsf(const fdtd_source *src, int nsrc)
{
    int c = 0;
    for (int s = 0; s < nsrc; s++) c += src[s].kind == 2;
    return c;
}

}  // namespace

// ==================================================================== C ABI

extern "C" {

fdtd_status fdtd_footprint(const fdtd_desc *desc, const fdtd_source *src, int32_t nsrc,
                           const fdtd_flux_detector *det, int32_t ndet, size_t *bytes)
{
    if (!bytes) return fail(nullptr, FDTD_E_INVALID, "bytes is NULL");
    fdtd_status st = validate(nullptr, desc, src, nsrc, det, ndet);
    if (st != FDTD_OK) return st;
    fdtd_ctx *tmp = new (std::nothrow) fdtd_ctx();
    if (!tmp) return fail(nullptr, FDTD_E_NOMEM, "host allocation failed");
    Geometry G;
    geometry(desc, det, ndet, G);
    tmp->ntfsf = count_tfsf(src, nsrc);
    *bytes = plan(tmp, desc, G, choose_K(desc), nullptr);
    delete tmp;
    return FDTD_OK;
}

fdtd_status fdtd_create(const fdtd_desc *desc, const fdtd_source *src, int32_t nsrc,
                        const fdtd_flux_detector *det, int32_t ndet, void *workspace, size_t workspace_bytes,
                        void *stream, fdtd_handle *out)
{
    if (!out) return fail(nullptr, FDTD_E_INVALID, "out is NULL");
    *out = nullptr;
    fdtd_status st = validate(nullptr, desc, src, nsrc, det, ndet);
    if (st != FDTD_OK) return st;
    if (!workspace) return fail(nullptr, FDTD_E_INVALID, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(nullptr, FDTD_E_INVALID, "workspace not 256-byte aligned");
    fdtd_ctx *h = new (std::nothrow) fdtd_ctx();
    if (!h) return fail(nullptr, FDTD_E_NOMEM, "host allocation failed");
    h->desc = *desc;
    h->nsrc = nsrc;
    h->ndet = ndet;
    for (int s = 0; s < nsrc; s++) h->src[s] = src[s];
    IntSrc isrc[FD_MAXSRC];
    const int nint = expand_sources(src, nsrc, isrc, FD_MAXSRC);
    h->ntfsf = 0;
    for (int q = 0; q < nint; q++) {
        if (isrc[q].role == 1) {
            h->tfsf_pub[h->ntfsf] = isrc[q].pub;
            h->tfsf_slot[h->ntfsf][0] = q;
            h->tfsf_slot[h->ntfsf][1] = q + 1;   // the H correction follows its E correction
            h->ntfsf++;
        }
    }
    for (int m = 0; m < ndet; m++) h->det[m] = det[m];
    h->stream = (hipStream_t)stream;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
    h->T = desc->n_steps;
    h->K = choose_K(desc);
    h->naive = false;
    if (const char *e = getenv("FDTD_NAIVE")) h->naive = atoi(e) != 0;
    // the z-march stages at most tb_max_pml() CPML planes per side
    if (desc->pml_cells > tb_max_pml()) h->naive = true;
    h->shape = tb_shape();
    geometry(desc, det, ndet, h->geo);
    const size_t need = plan(h, desc, h->geo, h->K, nullptr);
    if (workspace_bytes < need) {
        delete h;
        return fail(nullptr, FDTD_E_NOMEM, "workspace %zu bytes < footprint %zu", workspace_bytes, need);
    }
    plan(h, desc, h->geo, h->K, workspace);
    // the z-march kernel addresses a field set, and the four auxiliaries of a
    // slab axis, from one base with 32-bit byte offsets
    {
        auto stride_of = [](float *const *v, int n, unsigned &st) {
            const uintptr_t d = (uintptr_t)v[1] - (uintptr_t)v[0];
            for (int q = 1; q < n; q++)
                if ((uintptr_t)v[q] - (uintptr_t)v[q - 1] != d) return false;
            if ((unsigned long long)d * (unsigned long long)n >= (1ull << 32)) return false;
            st = (unsigned)d;
            return true;
        };
        // (the adjoint sets, when present, must have the same spacing: the
        // fused reverse march addresses them the same way)
        unsigned f0 = 0, f1 = 0;
        bool fok = stride_of(h->fld[0], 6, f0) && stride_of(h->fld[1], 6, f1) && f0 == f1;
        if (desc->record) {
            unsigned a0 = 0, a1 = 0;
            fok = fok && stride_of(h->adj[0], 6, a0) && stride_of(h->adj[1], 6, a1) && a0 == f0 && a1 == f0;
        }
        h->fstride = f0;
        bool ok = true;
        for (int a = 0; a < 3; a++) {
            h->pstride[a] = 0;
            if (h->geo.p > 0) {
                unsigned p0 = 0, p1 = 0;
                ok = ok && stride_of(h->psi[0][a], 4, p0) && stride_of(h->psi[1][a], 4, p1) && p0 == p1;
                if (desc->record) {
                    unsigned b0 = 0, b1 = 0;
                    ok = ok && stride_of(h->pb[0][a], 4, b0) && stride_of(h->pb[1][a], 4, b1) && b0 == p0 && b1 == p0;
                }
                h->pstride[a] = p0;
            }
        }
        // A field set of 4 GiB or more (above about 179M cells) runs the
        // forward and the fused reverse march with a 64-bit base per
        // component and plane, offsets within one plane still 32-bit; any
        // other addressing misfit takes the per-cell kernels.
        const bool wide_ok = tb_wide_shape(h->shape) &&
                             (unsigned long long)h->geo.nx * (unsigned long long)h->geo.ny * 4ull < (1ull << 32);
        const char *ew = getenv("FDTD_TB_WIDE");   // tests: the wide instance on any size
        const bool force_wide = ew && atoi(ew) != 0 && wide_ok;
        if (!ok || (!fok && !wide_ok)) h->naive = true;
        else if (!fok || force_wide) h->wide = true;
        // conducting cells: the z-march's lossy instances (default shape,
        // 32-bit offsets, K = 1 or 2), else the per-cell kernels
        if (desc->sigma && !tb_lossy_ok(h->K, h->shape, h->wide)) h->naive = true;
        if (h->naive) h->wide = false;
    }

    // device problem description
    const Geometry &G = h->geo;
    Grid &g = h->g;
    g.nx = G.nx; g.ny = G.ny; g.nz = G.nz; g.p = G.p;
    g.N = G.N; g.nxy = (long long)G.nx * G.ny;
    g.S = desc->courant;
    g.ce = h->ce;
    for (int t = 0; t < 2; t++)
        for (int a = 0; a < 3; a++)
            for (int f = 0; f < 3; f++) g.prof[t][a][f] = h->prof[t][a][f];
    for (int a = 0; a < 3; a++) g.slab_n[a] = G.slab_n[a];
    g.nsrc = nint;
    for (int s = 0; s < FD_MAXSRC; s++) {
        const bool on = s < nint;
        g.skind[s] = on ? isrc[s].kind : 0; g.scomp[s] = on ? isrc[s].comp : 0;
        g.si[s] = on ? isrc[s].i : 0; g.sj[s] = on ? isrc[s].j : 0; g.sk[s] = on ? isrc[s].k : -1;
        g.samp[s] = h->amps[s];
    }
    for (int a = 0; a < 3; a++) {
        g.llo[a] = G.lossy_cells > 0 ? desc->lossy_lo[a] : 0;
        g.lhi[a] = G.lossy_cells > 0 ? desc->lossy_hi[a] : 0;
    }
    g.lca = h->lca;
    g.lsig = h->lsig;

    // CPML grading tables (double precision on the host, stored as float)
    const double m = desc->pml_order >= 0.f ? desc->pml_order : 3.0;
    const double ebg = desc->pml_eps_bg > 0.f ? desc->pml_eps_bg : 1.0;
    const double smax = desc->pml_sigma_max >= 0.f ? desc->pml_sigma_max
                                                   : 0.8 * (m + 1.0) * desc->courant / std::sqrt(ebg);
    const double kmax = desc->pml_kappa_max >= 0.f ? desc->pml_kappa_max : 1.0;
    const double amax = desc->pml_alpha_max >= 0.f ? desc->pml_alpha_max : 0.01;
    const int n[3] = {G.nx, G.ny, G.nz};
    h->host_tables.clear();
    std::vector<size_t> starts;
    for (int t = 0; t < 2; t++)
        for (int a = 0; a < 3; a++) {
            std::vector<float> b(n[a]), aa(n[a]), kv(n[a]);
            for (int i = 0; i < n[a]; i++) {
                float o[3];
                grade(n[a], G.p, t == 0 ? (double)i : i + 0.5, m, smax, kmax, amax, o);
                b[i] = o[0]; aa[i] = o[1]; kv[i] = o[2];
            }
            starts.push_back(h->host_tables.size());
            h->host_tables.insert(h->host_tables.end(), b.begin(), b.end());
            h->host_tables.insert(h->host_tables.end(), aa.begin(), aa.end());
            h->host_tables.insert(h->host_tables.end(), kv.begin(), kv.end());
        }
    std::vector<size_t> vstarts;
    for (int a2 = 0; a2 < 3; a2++) {
        vstarts.push_back(h->host_tables.size());
        for (int i = 0; i < n[a2]; i++)
            for (int t = 0; t < 2; t++) {
                float o[3];
                grade(n[a2], G.p, t == 0 ? (double)i : i + 0.5, m, smax, kmax, amax, o);
                h->host_tables.push_back(o[0]); h->host_tables.push_back(o[1]);
                h->host_tables.push_back(o[2]); h->host_tables.push_back(0.f);
            }
    }
    for (int m2 = 0; m2 < FDTD_MAX_DETECTORS; m2++) {
        const float w = m2 < ndet ? det[m2].weight : 0.f;
        h->wS[m2] = desc->courant * w;
        h->wS_plain[m2] = (m2 < ndet && det[m2].interpolate) ? 0.f : h->wS[m2];
        h->host_tables.push_back(w);
    }
    {
        size_t si = 0;
        for (int t = 0; t < 2; t++)
            for (int a = 0; a < 3; a++, si++)
                for (int f = 0; f < 3; f++) {
                    hipError_t e = hipMemcpyAsync(h->prof[t][a][f], h->host_tables.data() + starts[si] + (size_t)f * n[a],
                                                  sizeof(float) * n[a], hipMemcpyHostToDevice, h->stream);
                    if (e != hipSuccess) { fdtd_status r = fail(nullptr, FDTD_E_DEVICE, "upload: %s", hipGetErrorString(e)); delete h; return r; }
                }
        for (int a2 = 0; a2 < 3; a2++) {
            hipError_t e2 = hipMemcpyAsync(h->profv[a2], h->host_tables.data() + vstarts[a2], sizeof(float) * 8 * n[a2],
                                           hipMemcpyHostToDevice, h->stream);
            if (e2 != hipSuccess) { fdtd_status r = fail(nullptr, FDTD_E_DEVICE, "upload: %s", hipGetErrorString(e2)); delete h; return r; }
        }
        hipError_t e = hipMemcpyAsync(h->wdev, h->host_tables.data() + h->host_tables.size() - FDTD_MAX_DETECTORS,
                                      sizeof(float) * FDTD_MAX_DETECTORS, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) { fdtd_status r = fail(nullptr, FDTD_E_DEVICE, "upload: %s", hipGetErrorString(e)); delete h; return r; }
    }
    if (!h->host_tiles.empty()) {
        hipError_t e = hipMemcpyAsync(h->tiles, h->host_tiles.data(), sizeof(int4) * h->host_tiles.size(),
                                      hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) { fdtd_status r = fail(nullptr, FDTD_E_DEVICE, "tiles: %s", hipGetErrorString(e)); delete h; return r; }
    }
    // the z-marches' fixed arguments
    fill_static_args(h);
    {
        hipError_t e = hipMemcpyAsync(h->targs, &h->host_targs, sizeof(TbArgs), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->rargs, &h->host_rargs, sizeof(RevArgs), hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) { fdtd_status r = fail(nullptr, FDTD_E_DEVICE, "args: %s", hipGetErrorString(e)); delete h; return r; }
    }
    // the caller's amplitudes: plain sources into their slots, TFSF waveforms
    // into the workspace (upload_materials runs their incident lines)
    for (int q = 0; q < nint; q++) {
        if (isrc[q].role == 2) continue;
        float *dst = h->amps[q];
        if (isrc[q].role == 1)
            for (int t = 0; t < h->ntfsf; t++)
                if (h->tfsf_slot[t][0] == q) dst = h->twave[t];
        hipError_t e = hipMemcpyAsync(dst, src[isrc[q].pub].amp, sizeof(float) * desc->n_steps,
                                      hipMemcpyDeviceToDevice, h->stream);
        if (e != hipSuccess) { fdtd_status r = fail(nullptr, FDTD_E_DEVICE, "amp copy: %s", hipGetErrorString(e)); delete h; return r; }
    }
    if (G.lossy_cells > 0) {
        hipError_t e = hipMemcpyAsync(h->lsig, desc->sigma, sizeof(float) * G.lossy_cells, hipMemcpyDeviceToDevice,
                                      h->stream);
        if (e != hipSuccess) { fdtd_status r = fail(nullptr, FDTD_E_DEVICE, "sigma copy: %s", hipGetErrorString(e)); delete h; return r; }
    }
    st = upload_materials(h, desc->inv_eps);
    if (st == FDTD_OK) st = zero_forward(h);
    if (st == FDTD_OK) st = zero_adjoint(h);
    if (st == FDTD_OK) {
        hipError_t e = launch_fill(h->trace, (long long)desc->n_steps * std::max(1, ndet), 0.f, h->stream);
        if (e != hipSuccess) st = fail(h, FDTD_E_DEVICE, "fill: %s", hipGetErrorString(e));
    }
    if (st != FDTD_OK) {
        snprintf(g_err, sizeof g_err, "%s", h->err);
        delete h;
        return st;
    }
    // the host tables must outlive the asynchronous uploads
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        fail(nullptr, FDTD_E_DEVICE, "create sync: %s", hipGetErrorString(e));
        delete h;
        return FDTD_E_DEVICE;
    }
    h->t = 0;
    *out = h;
    return FDTD_OK;
}

fdtd_status fdtd_forward(fdtd_handle h, int32_t n_steps, float *trace, float *J)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (n_steps < 0) return fail(h, FDTD_E_INVALID, "n_steps < 0");
    if (h->in_grad) return fail(h, FDTD_E_STATE, "a gradient is running on this handle");
    if (h->t + n_steps > h->T)
        return fail(h, FDTD_E_STATE, "t + n_steps = %d exceeds n_steps of the descriptor (%d)", h->t + n_steps, h->T);
    const int t0 = h->t;
    fdtd_status st = advance(h, t0, n_steps, 1, 1, 1);
    if (st != FDTD_OK) return st;
    h->t = t0 + n_steps;
    const Geometry &G = h->geo;
    if (trace && G.D.ndet > 0 && n_steps > 0)
        HIPCHK(h, launch_copy(trace, h->trace + (size_t)t0 * G.D.ndet, (long long)n_steps * G.D.ndet, h->stream));
    if (J) {
        if (G.D.ndet > 0)
            HIPCHK(h, launch_objective(h->trace, h->t, G.D.ndet, h->wdev, h->desc.courant, J, h->stream));
        else
            HIPCHK(h, launch_fill(J, 1, 0.f, h->stream));
    }
    return FDTD_OK;
}

fdtd_status fdtd_inverse(fdtd_handle h, int32_t n_steps)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (h->in_grad) return fail(h, FDTD_E_STATE, "a gradient is running on this handle");
    if (n_steps < 0 || n_steps > h->t) return fail(h, FDTD_E_STATE, "cannot undo %d steps at t = %d", n_steps, h->t);
    if (h->geo.p > 0 && !h->desc.record) return fail(h, FDTD_E_STATE, "inverse with a PML needs record = 1");
    if (h->geo.lossy_cells > 0 && !h->desc.record)
        return fail(h, FDTD_E_STATE, "inverse with conducting cells needs record = 1");
    for (int s = 0; s < n_steps; s++) {
        fdtd_status st = h->naive ? reverse_step(h, h->t - 1, 0) : reverse_fused(h, h->t - 1, 1, 0, 0, nullptr);
        if (st != FDTD_OK) return st;
        h->t -= 1;
    }
    return FDTD_OK;
}

// a weighted energy detector on a plane of the design box: the energy reads
// eps_r there, a term the adjoint does not carry
static bool energy_in_design(const fdtd_ctx *h)
{
    for (int m = 0; m < h->ndet; m++)
        if (h->det[m].quantity == 1 && h->det[m].weight != 0.f && h->det[m].k >= h->desc.design_lo[2] &&
            h->det[m].k < h->desc.design_hi[2])
            return true;
    return false;
}

namespace {

fdtd_status grad_begin_check(fdtd_ctx *h)
{
    if (!h->desc.record) return fail(h, FDTD_E_STATE, "the gradient needs record = 1");
    if (energy_in_design(h))
        return fail(h, FDTD_E_UNSUPPORTED, "a weighted energy detector must lie outside the design box in z");
    if (h->in_grad) return fail(h, FDTD_E_STATE, "a gradient is already running on this handle");
    if (h->t != h->T) return fail(h, FDTD_E_STATE, "the gradient needs t = T (t = %d, T = %d)", h->t, h->T);
    return FDTD_OK;
}

fdtd_status grad_begin_impl(fdtd_ctx *h)
{
    fdtd_status st0 = grad_begin_check(h);
    if (st0 != FDTD_OK) return st0;
    const Geometry &G = h->geo;
    HIPCHK(h, launch_interior_sumsq(h->g, fields_of(h, h->cur), h->parts[0], &h->grad_np, h->stream));
    fdtd_status st = zero_adjoint(h);
    if (st != FDTD_OK) return st;
    HIPCHK(h, launch_fill(h->gacc, G.design_cells, 0.f, h->stream));
    h->in_grad = true;
    return FDTD_OK;
}

// what precedes reverse step n: the interpolated detectors' adjoint source
fdtd_status grad_pre_step(fdtd_ctx *h, int n)
{
    if (h->drec)
        HIPCHK(h, launch_det_interp_adjoint(h->g, h->geo.D, h->drec, h->drec_e0, n, h->T, h->wS, adj_of(h, h->acur),
                                            h->stream));
    return FDTD_OK;
}

// one reverse step of a running gradient, on its own
fdtd_status grad_step_single(fdtd_ctx *h)
{
    const int n = h->t - 1;
    fdtd_status st = grad_pre_step(h, n);
    if (st == FDTD_OK) st = h->naive ? reverse_step(h, n, 1) : reverse_fused(h, n, 1, 1, 1, h->gacc);
    if (st == FDTD_OK) h->t = n;
    return st;
}

fdtd_status grad_end_impl(fdtd_ctx *h, float *dJ_deps, float *recon_err)
{
    const Geometry &G = h->geo;
    int np = 0;
    HIPCHK(h, launch_interior_sumsq(h->g, fields_of(h, h->cur), h->parts[1], &np, h->stream));
    if (recon_err) HIPCHK(h, launch_recon(h->parts[0], h->parts[1], np, recon_err, h->stream));
    HIPCHK(h, launch_deps(h->gacc, h->d_design, G.design_cells, h->desc.courant, dJ_deps, h->stream));
    HIPCHK(h, launch_deps_lossy(h->g, h->gacc, h->d_design, h->desc.design_lo, h->desc.design_hi, dJ_deps, h->stream));
    fdtd_status st = zero_forward(h);
    if (st != FDTD_OK) return st;
    HIPCHK(h, launch_fill(h->trace, (long long)h->T * std::max(1, G.D.ndet), 0.f, h->stream));
    h->t = 0;
    h->in_grad = false;
    return FDTD_OK;
}

}  // namespace

fdtd_status fdtd_grad(fdtd_handle h, float *dJ_deps, float *recon_err)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    fdtd_status st = grad_begin_check(h);
    if (st != FDTD_OK) return st;
    if (!dJ_deps) return fail(h, FDTD_E_INVALID, "dJ_deps is NULL");
    st = grad_begin_impl(h);
    while (st == FDTD_OK && h->t > 0) st = grad_step_single(h);
    if (st == FDTD_OK) st = grad_end_impl(h, dJ_deps, recon_err);
    if (st != FDTD_OK) h->in_grad = false;
    return st;
}

fdtd_status fdtd_grad_begin(fdtd_handle h)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    return grad_begin_impl(h);
}

fdtd_status fdtd_grad_steps(fdtd_handle h, int32_t n_steps)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (!h->in_grad) return fail(h, FDTD_E_STATE, "fdtd_grad_steps needs fdtd_grad_begin first");
    if (n_steps < 0 || n_steps > h->t) return fail(h, FDTD_E_STATE, "cannot reverse %d steps at t = %d", n_steps, h->t);
    for (int s = 0; s < n_steps; s++) {
        fdtd_status st = grad_step_single(h);
        if (st != FDTD_OK) return st;
    }
    return FDTD_OK;
}

fdtd_status fdtd_grad_end(fdtd_handle h, float *dJ_deps, float *recon_err)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (!h->in_grad) return fail(h, FDTD_E_STATE, "fdtd_grad_end needs fdtd_grad_begin first");
    if (h->t != 0) return fail(h, FDTD_E_STATE, "fdtd_grad_end needs t = 0 (t = %d)", h->t);
    if (!dJ_deps) return fail(h, FDTD_E_INVALID, "dJ_deps is NULL");
    return grad_end_impl(h, dJ_deps, recon_err);
}

// ----------------------------------------------------------------------
// Batches of handles (serving): one z-march launch per sweep spans the tiles
// of every handle in the batch.
namespace {

// common checks of a batch; the stream of the first handle is the batch's
fdtd_status batch_check(const fdtd_handle *hs, int32_t nh, const int32_t *n_steps)
{
    if (nh < 0 || (nh > 0 && (!hs || !n_steps))) return fail(nullptr, FDTD_E_INVALID, "bad batch arguments");
    for (int i = 0; i < nh; i++) {
        if (!hs[i]) return fail(nullptr, FDTD_E_INVALID, "batch handle %d is NULL", i);
        if (hs[i]->stream != hs[0]->stream)
            return fail(nullptr, FDTD_E_INVALID, "batch handle %d was created on another stream", i);
        if (n_steps[i] < 0) return fail(nullptr, FDTD_E_INVALID, "n_steps[%d] < 0", i);
        for (int j = 0; j < i; j++)
            if (hs[j] == hs[i]) return fail(nullptr, FDTD_E_INVALID, "handle %d appears twice in the batch", i);
    }
    return FDTD_OK;
}

// a batch launch failed: the message goes to every handle of the launch
fdtd_status batch_fail(fdtd_ctx *const *g, int n, hipError_t e)
{
    for (int i = 0; i < n; i++) fail(g[i], FDTD_E_DEVICE, "batched z-march launch: %s", hipGetErrorString(e));
    return fail(nullptr, FDTD_E_DEVICE, "batched z-march launch: %s", hipGetErrorString(e));
}

}  // namespace

fdtd_status fdtd_forward_batch(const fdtd_handle *hs, int32_t nh, const int32_t *n_steps, float *const *traces,
                               float *const *Js)
{
    fdtd_status st = batch_check(hs, nh, n_steps);
    if (st != FDTD_OK) return st;
    for (int i = 0; i < nh; i++) {
        if (hs[i]->in_grad) return fail(hs[i], FDTD_E_STATE, "a gradient is running on batch handle %d", i);
        if (hs[i]->t + n_steps[i] > hs[i]->T)
            return fail(hs[i], FDTD_E_STATE, "t + n_steps = %d exceeds n_steps of the descriptor (%d)",
                        hs[i]->t + n_steps[i], hs[i]->T);
    }
    std::vector<int> t0(nh), pos(nh);
    for (int i = 0; i < nh; i++) t0[i] = pos[i] = hs[i]->t;
    // handles on the per-cell kernels advance on their own
    for (int i = 0; i < nh; i++)
        if (hs[i]->naive) {
            st = advance(hs[i], pos[i], n_steps[i], 1, 1, 1);
            if (st != FDTD_OK) return st;
            pos[i] += n_steps[i];
        }
    // every round: one launch per (sweep length, instance) group of handles
    for (;;) {
        bool any = false;
        for (int kk = 1; kk <= 4; kk++)
            for (int wide = 0; wide < 2; wide++)
                for (int shape = 0; shape < 4; shape++)
                for (int lossy = 0; lossy < 2; lossy++) {
                    std::vector<fdtd_ctx *> grp;
                    std::vector<int> idx;
                    for (int i = 0; i < nh; i++) {
                        fdtd_ctx *h = hs[i];
                        const int rem = t0[i] + n_steps[i] - pos[i];
                        if (h->naive || rem <= 0 || std::min(h->K, rem) != kk || (int)h->wide != wide ||
                            h->shape != shape || (int)(h->g.lca != nullptr) != lossy)
                            continue;
                        grp.push_back(h);
                        idx.push_back(i);
                    }
                    for (size_t a = 0; a < grp.size(); a += ZM_MAXREQ) {
                        const int cnt = (int)std::min<size_t>(ZM_MAXREQ, grp.size() - a);
                        TbLaunch L;
                        L.nreq = cnt;
                        L.nblocks = 0;
                        L.xcd_remap = 1;
                        L.pad = 0;
                        for (int j = 0; j < cnt; j++) {
                            fdtd_ctx *h = grp[a + j];
                            const int i = idx[a + j];
                            st = tb_prologue(h, pos[i], 1);
                            if (st != FDTD_OK) return st;
                            L.r[j] = tb_request(h, pos[i], kk, 1, 1, 1, L.nblocks);
                            L.nblocks += h->tb_n[kk];
                        }
                        const hipError_t e = launch_tb_forward(L, kk, shape, wide != 0, lossy != 0, grp[a]->stream);
                        if (e != hipSuccess) return batch_fail(grp.data() + a, cnt, e);
                        for (int j = 0; j < cnt; j++) {
                            fdtd_ctx *h = grp[a + j];
                            const int i = idx[a + j];
                            st = tb_epilogue(h, pos[i], kk, 1);
                            if (st != FDTD_OK) return st;
                            pos[i] += kk;
                        }
                        any = true;
                    }
                }
        if (!any) break;
    }
    // outputs, as fdtd_forward gives them
    for (int i = 0; i < nh; i++) {
        fdtd_ctx *h = hs[i];
        const Geometry &G = h->geo;
        st = flush_planes(h);
        if (st != FDTD_OK) return st;
        h->t = t0[i] + n_steps[i];
        float *trace = traces ? traces[i] : nullptr;
        float *J = Js ? Js[i] : nullptr;
        if (trace && G.D.ndet > 0 && n_steps[i] > 0)
            HIPCHK(h, launch_copy(trace, h->trace + (size_t)t0[i] * G.D.ndet, (long long)n_steps[i] * G.D.ndet,
                                  h->stream));
        if (J) {
            if (G.D.ndet > 0)
                HIPCHK(h, launch_objective(h->trace, h->t, G.D.ndet, h->wdev, h->desc.courant, J, h->stream));
            else
                HIPCHK(h, launch_fill(J, 1, 0.f, h->stream));
        }
    }
    return FDTD_OK;
}

fdtd_status fdtd_grad_steps_batch(const fdtd_handle *hs, int32_t nh, const int32_t *n_steps)
{
    fdtd_status st = batch_check(hs, nh, n_steps);
    if (st != FDTD_OK) return st;
    for (int i = 0; i < nh; i++) {
        if (!hs[i]->in_grad) return fail(hs[i], FDTD_E_STATE, "batch handle %d has no running gradient", i);
        if (n_steps[i] > hs[i]->t)
            return fail(hs[i], FDTD_E_STATE, "cannot reverse %d steps at t = %d", n_steps[i], hs[i]->t);
    }
    std::vector<int> left(n_steps, n_steps + nh);
    for (int i = 0; i < nh; i++)
        if (hs[i]->naive)
            for (; left[i] > 0; left[i]--) {
                st = grad_step_single(hs[i]);
                if (st != FDTD_OK) return st;
            }
    // every round: one reverse step of every handle that has steps left, one
    // launch per instance
    for (;;) {
        bool any = false;
        for (int wide = 0; wide < 2; wide++)
        for (int lossy = 0; lossy < 2; lossy++) {
            std::vector<fdtd_ctx *> grp;
            std::vector<int> idx;
            for (int i = 0; i < nh; i++)
                if (!hs[i]->naive && left[i] > 0 && (int)hs[i]->wide == wide &&
                    (int)(hs[i]->g.lca != nullptr) == lossy) {
                    grp.push_back(hs[i]);
                    idx.push_back(i);
                }
            for (size_t a = 0; a < grp.size(); a += ZM_MAXREQ) {
                const int cnt = (int)std::min<size_t>(ZM_MAXREQ, grp.size() - a);
                RevLaunch L;
                L.nreq = cnt;
                L.nblocks = 0;
                L.xcd_remap = 1;
                L.pad = 0;
                for (int j = 0; j < cnt; j++) {
                    fdtd_ctx *h = grp[a + j];
                    st = grad_pre_step(h, h->t - 1);
                    if (st != FDTD_OK) return st;
                    L.r[j] = rev_request(h, h->t - 1, 1, 1, 1, h->gacc, nullptr, L.nblocks);
                    L.nblocks += h->tb_n[0];
                }
                const hipError_t e = launch_tb_reverse(L, wide != 0, lossy != 0, grp[a]->stream);
                if (e != hipSuccess) return batch_fail(grp.data() + a, cnt, e);
                for (int j = 0; j < cnt; j++) {
                    fdtd_ctx *h = grp[a + j];
                    rev_epilogue(h, 1, 1);
                    h->t -= 1;
                    left[idx[a + j]]--;
                }
                any = true;
            }
        }
        if (!any) break;
    }
    return FDTD_OK;
}

// ----------------------------------------------------------------------
// Checkpointed gradient (a comparator for the time-reversal gradient): the
// store holds nseg complete forward states (fields and CPML auxiliaries,
// one per segment start) followed by the fields after each step of one
// segment.
namespace {

struct CkptPlan {
    int C, nseg;
    size_t snap_bytes, step_bytes, total;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

CkptPlan ckpt_plan(const fdtd_ctx *h, int C)
{
    CkptPlan P;
    P.C = C;
    P.nseg = (h->T + C - 1) / C;
    const Geometry &G = h->geo;
    P.step_bytes = 6 * align256((size_t)G.N * 4);
    P.snap_bytes = P.step_bytes;
    if (G.p > 0)
        for (int a = 0; a < 3; a++) P.snap_bytes += 4 * align256((size_t)G.slab_n[a] * 4);
    P.total = (size_t)P.nseg * P.snap_bytes + (size_t)C * P.step_bytes;
    return P;
}

// the 6 field arrays and (if snap) the 12 auxiliaries of one stored state
void ckpt_arrays(const fdtd_ctx *h, char *base, float *fld[6], float *psi[3][4])
{
    const Geometry &G = h->geo;
    size_t off = 0;
    for (int q = 0; q < 6; q++) {
        fld[q] = (float *)(base + off);
        off += align256((size_t)G.N * 4);
    }
    if (psi)
        for (int a = 0; a < 3; a++)
            for (int q = 0; q < 4; q++) {
                psi[a][q] = G.p > 0 ? (float *)(base + off) : nullptr;
                if (G.p > 0) off += align256((size_t)G.slab_n[a] * 4);
            }
}

fdtd_status copy_state(fdtd_ctx *h, float *const dfld[6], float *const dpsi[3][4], float *const sfld[6],
                       float *const spsi[3][4])
{
    const Geometry &G = h->geo;
    for (int q = 0; q < 6; q++) HIPCHK(h, launch_copy(dfld[q], sfld[q], G.N, h->stream));
    if (dpsi && spsi && G.p > 0)
        for (int a = 0; a < 3; a++)
            for (int q = 0; q < 4; q++) HIPCHK(h, launch_copy(dpsi[a][q], spsi[a][q], G.slab_n[a], h->stream));
    return FDTD_OK;
}

}  // namespace

fdtd_status fdtd_checkpoint_bytes(fdtd_handle h, int32_t segment, size_t *bytes)
{
    if (!h || !bytes) return fail(h, FDTD_E_INVALID, "NULL argument");
    if (segment < 1 || segment > h->T) return fail(h, FDTD_E_INVALID, "segment %d not in [1, T]", segment);
    *bytes = ckpt_plan(h, segment).total;
    return FDTD_OK;
}

namespace {
fdtd_status grad_checkpointed_impl(fdtd_handle h, int32_t segment, void *store, size_t store_bytes,
                                   float *dJ_deps, float *J)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (!h->desc.record) return fail(h, FDTD_E_STATE, "the checkpointed gradient needs the adjoint state (record = 1)");
    if (energy_in_design(h))
        return fail(h, FDTD_E_UNSUPPORTED, "a weighted energy detector must lie outside the design box in z");
    if (h->geo.lossy_cells > 0) return fail(h, FDTD_E_UNSUPPORTED, "the checkpointed gradients take no conducting cells");
    if (h->naive) return fail(h, FDTD_E_UNSUPPORTED, "the checkpointed gradient runs on the z-march path only");
    if (h->in_grad) return fail(h, FDTD_E_STATE, "a gradient is running on this handle");
    if (h->wide) return fail(h, FDTD_E_UNSUPPORTED, "the checkpointed gradient needs field sets under 4 GiB");
    if (segment < 1 || segment > h->T) return fail(h, FDTD_E_INVALID, "segment %d not in [1, T]", segment);
    if (!store || !dJ_deps) return fail(h, FDTD_E_INVALID, "store or dJ_deps is NULL");
    if (((uintptr_t)store & 255) != 0) return fail(h, FDTD_E_INVALID, "store not 256-byte aligned");
    const CkptPlan P = ckpt_plan(h, segment);
    if (store_bytes < P.total) return fail(h, FDTD_E_NOMEM, "store %zu bytes < %zu", store_bytes, P.total);
    // the reverse march addresses a kept field set from its first array at
    // the workspace's component spacing: the store must use the same one
    if ((size_t)h->fstride != align256((size_t)h->geo.N * 4))
        return fail(h, FDTD_E_UNSUPPORTED, "field spacing %u differs from the store's", h->fstride);
    const Geometry &G = h->geo;
    char *base = (char *)store;
    auto snap = [&](int sidx, float *fld[6], float *psi[3][4]) { ckpt_arrays(h, base + (size_t)sidx * P.snap_bytes, fld, psi); };
    auto kept = [&](int j, float *fld[6]) { ckpt_arrays(h, base + (size_t)P.nseg * P.snap_bytes + (size_t)j * P.step_bytes, fld, nullptr); };

    // forward from zero fields, keeping the state at every segment start
    fdtd_status st = zero_forward(h);
    if (st != FDTD_OK) return st;
    HIPCHK(h, launch_fill(h->trace, (long long)h->T * std::max(1, G.D.ndet), 0.f, h->stream));
    for (int sidx = 0; sidx < P.nseg; sidx++) {
        float *sf[6], *sp[3][4];
        snap(sidx, sf, sp);
        st = copy_state(h, sf, sp, h->fld[h->cur], h->psi[h->cur]);
        if (st != FDTD_OK) return st;
        const int n0 = sidx * P.C, cnt = std::min(P.C, h->T - n0);
        st = advance(h, n0, cnt, 1, 0, 1);
        if (st != FDTD_OK) return st;
    }
    if (J) {
        if (G.D.ndet > 0)
            HIPCHK(h, launch_objective(h->trace, h->T, G.D.ndet, h->wdev, h->desc.courant, J, h->stream));
        else
            HIPCHK(h, launch_fill(J, 1, 0.f, h->stream));
    }

    // backwards over the segments: restore, recompute keeping every step's
    // fields, then the adjoint steps (no inverse) on the kept states
    st = zero_adjoint(h);
    if (st != FDTD_OK) return st;
    HIPCHK(h, launch_fill(h->gacc, G.design_cells, 0.f, h->stream));
    for (int sidx = P.nseg - 1; sidx >= 0; sidx--) {
        const int n0 = sidx * P.C, n1 = std::min(h->T, n0 + P.C);
        float *sf[6], *sp[3][4];
        snap(sidx, sf, sp);
        st = copy_state(h, h->fld[h->cur], h->psi[h->cur], sf, sp);
        if (st != FDTD_OK) return st;
        for (int n = n0; n < n1; n++) {
            st = advance(h, n, 1, 1, 0, 0);
            if (st != FDTD_OK) return st;
            float *kf[6];
            kept(n - n0, kf);
            st = copy_state(h, kf, nullptr, h->fld[h->cur], nullptr);
            if (st != FDTD_OK) return st;
        }
        for (int n = n1 - 1; n >= n0; n--) {
            float *kf[6];
            kept(n - n0, kf);
            Fields F;
            for (int q = 0; q < 6; q++) F.c[q] = kf[q];
            if (h->drec)
                HIPCHK(h, launch_det_interp_adjoint(h->g, G.D, h->drec, h->drec_e0, n, h->T, h->wS,
                                                    adj_of(h, h->acur), h->stream));
            st = reverse_fused(h, n, 0, 1, 1, h->gacc, &F);
            if (st != FDTD_OK) return st;
        }
    }
    HIPCHK(h, launch_deps(h->gacc, h->d_design, G.design_cells, h->desc.courant, dJ_deps, h->stream));
    st = zero_forward(h);
    if (st != FDTD_OK) return st;
    HIPCHK(h, launch_fill(h->trace, (long long)h->T * std::max(1, G.D.ndet), 0.f, h->stream));
    h->t = 0;
    return FDTD_OK;
}
}  // namespace

fdtd_status fdtd_grad_checkpointed(fdtd_handle h, int32_t segment, void *store, size_t store_bytes,
                                   float *dJ_deps, float *J)
{
    return grad_checkpointed_impl(h, segment, store, store_bytes, dJ_deps, J);
}

// ----------------------------------------------------------------------
// Allocation-free variant: the checkpoint store is a fixed device array of
// the library instead of caller memory.  Each GPU holds its own copy until
// the process ends; host code must use its address from hipGetSymbolAddress
// (the array's name on the host is only a stand-in), taken once per device
// with that device current.
namespace {

constexpr size_t NOALLOC_STORE_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_STORE_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of this device's store (taken once per device, with that
// device current, and kept)
fdtd_status scratch_address(fdtd_ctx *h, void **out)
{
    *out = nullptr;
    if (h->device < 0 || h->device >= NOALLOC_MAX_DEVICES)
        return fail(h, FDTD_E_UNSUPPORTED, "device %d beyond the %d the store table holds", h->device,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[h->device]) {
        int prev = 0;
        HIPCHK(h, hipGetDevice(&prev));
        if (prev != h->device) HIPCHK(h, hipSetDevice(h->device));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != h->device) HIPCHK(h, hipSetDevice(prev));
        if (e != hipSuccess || !ptr)
            return fail(h, FDTD_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[h->device] = ptr;
    }
    *out = g_scratch_ptr[h->device];
    return FDTD_OK;
}

}  // namespace

fdtd_status fdtd_grad_checkpointed_noalloc(fdtd_handle h, int32_t segment, float *dJ_deps, float *J)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (segment < 1 || segment > h->T) return fail(h, FDTD_E_INVALID, "segment %d not in [1, T]", segment);
    const size_t need = ckpt_plan(h, segment).total;
    if (need > NOALLOC_STORE_BYTES)
        return fail(h, FDTD_E_NOMEM, "checkpoint store of %zu bytes exceeds the library's fixed %zu-byte store",
                    need, NOALLOC_STORE_BYTES);
    void *store = nullptr;
    const fdtd_status st = scratch_address(h, &store);
    if (st != FDTD_OK) return st;
    return grad_checkpointed_impl(h, segment, store, NOALLOC_STORE_BYTES, dJ_deps, J);
}

size_t fdtd_noalloc_store_bytes(void) { return NOALLOC_STORE_BYTES; }

// ----------------------------------------------------------------------
// Checkpoint schedules of section 2.2 for the gradient without time
// reversal: recursive halving (the states at the midpoints of ever smaller
// halves are kept) and treeverse (with a fixed number k of kept states, the
// split points that need the fewest forward steps, by dynamic programming).
// A schedule is a list of actions on one forward state (the handle's
// current buffer) and k snapshot slots:
//   restore slot a (a = -1: the zero state s_0), advance b steps from step
//   a, save to slot a, adjoint of step a (on the current state s_{a+1}).
namespace {

enum { RV_RESTORE = 0, RV_ADVANCE = 1, RV_SAVE = 2, RV_ADJOINT = 3 };
struct RevAct {
    int op, a, b;
};

struct RevPlanner {
    int T = 0, sched = 0, k = 0;
    // treeverse: best[l][j] = fewest forward steps to reverse l steps with j
    // free slots (the first state already kept), split[l][j] = its first split
    std::vector<long long> best;
    std::vector<int> split;
    std::vector<RevAct> acts;
    long long fwd = 0;
    int peak = 0;

    long long &B(int l, int j) { return best[(size_t)l * (k + 1) + j]; }
    int &P(int l, int j) { return split[(size_t)l * (k + 1) + j]; }

    void table()
    {
        best.assign((size_t)(T + 1) * (k + 1), 0);
        split.assign((size_t)(T + 1) * (k + 1), 0);
        for (int j = 0; j <= k; j++) B(1, j) = 1;
        for (int l = 2; l <= T; l++) {
            B(l, 0) = (long long)l * (l + 1) / 2;
            for (int j = 1; j <= k; j++) {
                long long bv = -1;
                int bm = 1;
                // advance m steps, keep that state, reverse the right part
                // with one slot fewer, then the left part with all of them
                for (int m = 1; m < l; m++) {
                    const long long c = m + B(l - m, j - 1) + B(m, j);
                    if (bv < 0 || c < bv) { bv = c; bm = m; }
                }
                B(l, j) = bv;
                P(l, j) = bm;
            }
        }
    }

    // reverse steps [s, e) with state s in slot `slot` (-1: s_0), j free slots
    void rec(int s, int e, int slot, int j, int used)
    {
        peak = std::max(peak, used);
        const int l = e - s;
        if (l <= 0) return;
        if (l == 1) {
            acts.push_back({RV_RESTORE, slot, 0});
            acts.push_back({RV_ADVANCE, s, 1});
            acts.push_back({RV_ADJOINT, s, 0});
            fwd += 1;
            return;
        }
        if (j == 0) {
            for (int n = e - 1; n >= s; n--) {
                acts.push_back({RV_RESTORE, slot, 0});
                acts.push_back({RV_ADVANCE, s, n + 1 - s});
                acts.push_back({RV_ADJOINT, n, 0});
                fwd += n + 1 - s;
            }
            return;
        }
        const int m = sched == 0 ? l / 2 : P(l, j);
        acts.push_back({RV_RESTORE, slot, 0});
        acts.push_back({RV_ADVANCE, s, m});
        acts.push_back({RV_SAVE, used, 0});
        fwd += m;
        rec(s + m, e, used, j - 1, used + 1);
        rec(s, s + m, slot, j, used);
    }

    // sched 0: recursive halving (k is set to the depth it needs);
    // sched 1: treeverse with k slots
    void build(int T_, int sched_, int k_)
    {
        T = T_;
        sched = sched_;
        k = k_;
        if (sched == 0) {
            k = 0;
            while ((1LL << k) < T) k++;
        } else {
            table();
        }
        acts.clear();
        fwd = 0;
        peak = 0;
        rec(0, T, -1, k, 0);
    }
};

fdtd_status revolve_check(int T, int schedule, int snapshots)
{
    if (T < 1) return fail(nullptr, FDTD_E_INVALID, "T = %d < 1", T);
    if (schedule != 0 && schedule != 1) return fail(nullptr, FDTD_E_INVALID, "schedule %d not 0 or 1", schedule);
    if (schedule == 1 && (snapshots < 0 || snapshots > 64))
        return fail(nullptr, FDTD_E_INVALID, "snapshots %d not in [0, 64]", snapshots);
    if (schedule == 1 && (long long)T * (snapshots + 1) > (1LL << 26))
        return fail(nullptr, FDTD_E_UNSUPPORTED, "treeverse table of %d x %d too large", T, snapshots + 1);
    return FDTD_OK;
}

}  // namespace

fdtd_status fdtd_revolve_plan(int32_t T, int32_t schedule, int32_t snapshots, int64_t *forward_steps,
                              int32_t *peak_snapshots, int32_t *actions, int32_t cap, int32_t *n_actions)
{
    fdtd_status st = revolve_check(T, schedule, snapshots);
    if (st != FDTD_OK) return st;
    RevPlanner P;
    P.build(T, schedule, snapshots);
    if (forward_steps) *forward_steps = P.fwd;
    if (peak_snapshots) *peak_snapshots = P.peak;
    if (n_actions) *n_actions = (int32_t)P.acts.size();
    if (actions) {
        if (cap < (int32_t)P.acts.size()) return fail(nullptr, FDTD_E_INVALID, "cap %d < %zu actions", cap, P.acts.size());
        for (size_t i = 0; i < P.acts.size(); i++) {
            actions[3 * i] = P.acts[i].op;
            actions[3 * i + 1] = P.acts[i].a;
            actions[3 * i + 2] = P.acts[i].b;
        }
    }
    return FDTD_OK;
}

fdtd_status fdtd_revolve_bytes(fdtd_handle h, int32_t schedule, int32_t snapshots, size_t *bytes)
{
    if (!h || !bytes) return fail(h, FDTD_E_INVALID, "NULL argument");
    fdtd_status st = revolve_check(h->T, schedule, snapshots);
    if (st != FDTD_OK) return fail(h, st, "%s", g_err);
    RevPlanner P;
    P.build(h->T, schedule, snapshots);
    *bytes = (size_t)std::max(1, P.peak) * ckpt_plan(h, 1).snap_bytes;
    return FDTD_OK;
}

fdtd_status fdtd_grad_revolve(fdtd_handle h, int32_t schedule, int32_t snapshots, void *store, size_t store_bytes,
                              float *dJ_deps, float *J)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (!h->desc.record) return fail(h, FDTD_E_STATE, "the checkpointed gradient needs the adjoint state (record = 1)");
    if (energy_in_design(h))
        return fail(h, FDTD_E_UNSUPPORTED, "a weighted energy detector must lie outside the design box in z");
    if (h->geo.lossy_cells > 0) return fail(h, FDTD_E_UNSUPPORTED, "the checkpointed gradients take no conducting cells");
    if (h->naive) return fail(h, FDTD_E_UNSUPPORTED, "the checkpointed gradient runs on the z-march path only");
    if (h->in_grad) return fail(h, FDTD_E_STATE, "a gradient is running on this handle");
    fdtd_status st = revolve_check(h->T, schedule, snapshots);
    if (st != FDTD_OK) return fail(h, st, "%s", g_err);
    if (!store || !dJ_deps) return fail(h, FDTD_E_INVALID, "store or dJ_deps is NULL");
    if (((uintptr_t)store & 255) != 0) return fail(h, FDTD_E_INVALID, "store not 256-byte aligned");
    RevPlanner P;
    P.build(h->T, schedule, snapshots);
    const size_t snap = ckpt_plan(h, 1).snap_bytes;
    if (store_bytes < (size_t)std::max(1, P.peak) * snap)
        return fail(h, FDTD_E_NOMEM, "store %zu bytes < %zu", store_bytes, (size_t)std::max(1, P.peak) * snap);
    const Geometry &G = h->geo;
    char *base = (char *)store;
    st = zero_forward(h);
    if (st == FDTD_OK) st = zero_adjoint(h);
    if (st != FDTD_OK) return st;
    HIPCHK(h, launch_fill(h->trace, (long long)h->T * std::max(1, G.D.ndet), 0.f, h->stream));
    HIPCHK(h, launch_fill(h->gacc, G.design_cells, 0.f, h->stream));
    int at = 0;      // step of the state in the current buffer
    int high = 0;    // steps below this one have run once (their detector output is in the trace)
    std::vector<int> slot_step(std::max(1, P.peak), -1);
    for (const RevAct &a : P.acts) {
        if (a.op == RV_RESTORE) {
            // the forward step is deterministic: a buffer at step s holds the
            // bits of any kept state of step s, so a restore to the current
            // step is skipped
            const int want = a.a < 0 ? 0 : slot_step[a.a];
            if (want != at) {
                if (a.a < 0) {
                    st = zero_forward(h);
                } else {
                    float *sf[6], *sp[3][4];
                    ckpt_arrays(h, base + (size_t)a.a * snap, sf, sp);
                    st = copy_state(h, h->fld[h->cur], h->psi[h->cur], sf, sp);
                }
                if (st != FDTD_OK) return st;
                at = want;
            }
        } else if (a.op == RV_ADVANCE) {
            const int s0 = a.a, s1 = a.a + a.b;
            const int old_end = std::min(s1, std::max(s0, high));
            if (old_end > s0) {
                st = advance(h, s0, old_end - s0, 1, 0, 0);
                if (st != FDTD_OK) return st;
            }
            if (s1 > old_end) {
                st = advance(h, old_end, s1 - old_end, 1, 0, 1);
                if (st != FDTD_OK) return st;
                high = s1;
            }
            at = s1;
        } else if (a.op == RV_SAVE) {
            float *sf[6], *sp[3][4];
            ckpt_arrays(h, base + (size_t)a.a * snap, sf, sp);
            st = copy_state(h, sf, sp, h->fld[h->cur], h->psi[h->cur]);
            if (st != FDTD_OK) return st;
            slot_step[a.a] = at;
        } else {
            st = grad_pre_step(h, a.a);
            if (st == FDTD_OK) st = reverse_fused(h, a.a, 0, 1, 1, h->gacc);
            if (st != FDTD_OK) return st;
        }
    }
    if (J) {
        if (G.D.ndet > 0)
            HIPCHK(h, launch_objective(h->trace, h->T, G.D.ndet, h->wdev, h->desc.courant, J, h->stream));
        else
            HIPCHK(h, launch_fill(J, 1, 0.f, h->stream));
    }
    HIPCHK(h, launch_deps(h->gacc, h->d_design, G.design_cells, h->desc.courant, dJ_deps, h->stream));
    st = zero_forward(h);
    if (st != FDTD_OK) return st;
    HIPCHK(h, launch_fill(h->trace, (long long)h->T * std::max(1, G.D.ndet), 0.f, h->stream));
    h->t = 0;
    return FDTD_OK;
}

fdtd_status fdtd_set_inv_eps(fdtd_handle h, const float *inv_eps)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (!inv_eps) return fail(h, FDTD_E_INVALID, "inv_eps is NULL");
    if (h->t != 0) return fail(h, FDTD_E_STATE, "materials can change only at t = 0");
    return upload_materials(h, inv_eps);
}

fdtd_status fdtd_reset(fdtd_handle h)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    fdtd_status st = zero_forward(h);
    if (st == FDTD_OK) st = zero_adjoint(h);
    if (st != FDTD_OK) return st;
    HIPCHK(h, launch_fill(h->trace, (long long)h->T * std::max(1, h->geo.D.ndet), 0.f, h->stream));
    h->t = 0;
    h->in_grad = false;
    return FDTD_OK;
}

fdtd_status fdtd_set_stream(fdtd_handle h, void *stream)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (h->in_grad) return fail(h, FDTD_E_STATE, "a gradient is running on this handle");
    h->stream = (hipStream_t)stream;
    return FDTD_OK;
}

fdtd_status fdtd_destroy(fdtd_handle h)
{
    if (!h) return FDTD_OK;
    // the handle owns host state only
    delete h;
    return FDTD_OK;
}

fdtd_status fdtd_time(fdtd_handle h, int32_t *t)
{
    if (!h || !t) return fail(h, FDTD_E_INVALID, "NULL argument");
    *t = h->t;
    return FDTD_OK;
}

const char *fdtd_last_error(fdtd_handle h) { return h ? h->err : g_err; }

fdtd_status fdtd_field_ptr(fdtd_handle h, int32_t which, int32_t comp, float **dev)
{
    if (!h || !dev) return fail(h, FDTD_E_INVALID, "NULL argument");
    if (comp < 0 || comp > 5) return fail(h, FDTD_E_INVALID, "comp outside 0..5");
    if (which == 0) { *dev = h->fld[h->cur][comp]; return FDTD_OK; }
    if (which == 1) {
        if (!h->desc.record) return fail(h, FDTD_E_STATE, "no adjoint state without record = 1");
        *dev = h->adj[h->acur][comp];
        return FDTD_OK;
    }
    return fail(h, FDTD_E_INVALID, "which must be 0 or 1");
}

fdtd_status fdtd_state_arrays(fdtd_handle h, int32_t which, float **ptrs, size_t *counts, int32_t cap, int32_t *n)
{
    if (!h || !ptrs || !counts || !n) return fail(h, FDTD_E_INVALID, "NULL argument");
    if (which == 1 && !h->desc.record) return fail(h, FDTD_E_STATE, "no adjoint state without record = 1");
    if (which != 0 && which != 1) return fail(h, FDTD_E_INVALID, "which must be 0 or 1");
    std::vector<std::pair<float *, size_t>> v;
    const Geometry &G = h->geo;
    for (int q = 0; q < 6; q++) v.push_back({which == 0 ? h->fld[h->cur][q] : h->adj[h->acur][q], (size_t)G.N});
    if (G.p > 0)
        for (int a = 0; a < 3; a++)
            for (int q = 0; q < 4; q++) {
                float *p = which == 0 ? h->psi[h->cur][a][q] : h->pb[h->apar][a][q];
                v.push_back({p, (size_t)G.slab_n[a]});
            }
    if ((int)v.size() > cap) return fail(h, FDTD_E_INVALID, "capacity %d < %zu arrays", cap, v.size());
    for (size_t i = 0; i < v.size(); i++) { ptrs[i] = v[i].first; counts[i] = v[i].second; }
    *n = (int32_t)v.size();
    return FDTD_OK;
}

fdtd_status fdtd_linear_steps(fdtd_handle h, int32_t n, int32_t adjoint)
{
    if (!h) return fail(nullptr, FDTD_E_INVALID, "handle is NULL");
    if (n < 0) return fail(h, FDTD_E_INVALID, "n < 0");
    if (adjoint && !h->desc.record) return fail(h, FDTD_E_STATE, "no adjoint state without record = 1");
    if (!adjoint) return advance(h, 0, n, 0, 0, 0);
    for (int s = 0; s < n; s++) {
        fdtd_status st;
        if (!h->naive) {
            st = reverse_fused(h, 0, 0, 1, 0, nullptr);
        } else {
            Fields F = fields_of(h, h->cur), A = adj_of(h, h->acur);
            Psi Pc = psibar_of(h, h->apar), Pn = psibar_of(h, h->apar ^ 1);
            HIPCHK(h, launch_bwd_a(h->g, F, A, Pc, 0, 0, 1, nullptr, h->desc.design_lo, h->desc.design_hi, nullptr,
                                   h->stream));
            HIPCHK(h, launch_bwd_b(h->g, F, A, Pc, Pn, 0, 0, 1, h->stream));
            h->apar ^= 1;
            st = FDTD_OK;
        }
        if (st != FDTD_OK) return st;
    }
    return FDTD_OK;
}

fdtd_status fdtd_record_ptr(fdtd_handle h, int32_t n, float **dev, size_t *floats_per_step)
{
    if (!h || !dev || !floats_per_step) return fail(h, FDTD_E_INVALID, "NULL argument");
    if (!h->desc.record) return fail(h, FDTD_E_STATE, "record = 0");
    if (n < 0 || n >= h->T) return fail(h, FDTD_E_INVALID, "step outside [0, T)");
    *dev = h->rec + (size_t)n * h->geo.R.per_step;
    *floats_per_step = (size_t)h->geo.R.per_step;
    return FDTD_OK;
}

fdtd_status fdtd_time_block(fdtd_handle h, int32_t *K)
{
    if (!h || !K) return fail(h, FDTD_E_INVALID, "NULL argument");
    *K = h->K;
    return FDTD_OK;
}

fdtd_status fdtd_kernel_path(fdtd_handle h, int32_t *path)
{
    if (!h || !path) return fail(h, FDTD_E_INVALID, "NULL argument");
    *path = h->naive ? 0 : h->wide ? 2 : 1;
    return FDTD_OK;
}

fdtd_status fdtd_tile_classes(fdtd_handle h, int32_t march, int32_t counts[4])
{
    if (!h || !counts) return fail(h, FDTD_E_INVALID, "NULL argument");
    if (march < 0 || march > h->K) return fail(h, FDTD_E_INVALID, "march %d outside [0, K = %d]", march, h->K);
    for (int c = 0; c < 4; c++) counts[c] = h->naive ? 0 : h->tb_cnt[march][c];
    return FDTD_OK;
}

}  // extern "C"
