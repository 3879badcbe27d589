// Internal declarations of libfdtd: device-side problem description, the
// canonical float32 update expressions every kernel shares, and launchers.
//
// Update expressions (the Yee leapfrog of arXiv 2412.12360, section 2.1, with
// the convolutional PML the paper cites).  For a difference d along axis a of a
// component inside that axis' PML slab:
//     psi' = fma(b, psi, a*d)          T = fma(d, 1/kappa, psi')
// and outside any slab T = d.  With b = 1, a = 0, 1/kappa = 1 both forms give
// the same bits.  Then
//     H' = fma(-S, T1 - T2, H)         E' = fma(S/eps_r, T1 - T2, E)
// and the inverse step (section 2.2) evaluates the identical increment:
//     E  = fma(-S/eps_r, T1 - T2, E')  H  = fma(S, T1 - T2, H')
// Every kernel, at any time-block size, uses exactly these expressions, so the
// naive and the temporally blocked paths agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define FD_MAXSRC 4
#define FD_MAXDET 4

// CPML auxiliary arrays per slab axis a (cells with coordinate a in [0,p) or
// [n_a-p, n_a), the other two coordinates full range):
//   0: E comp (a+1)%3   1: E comp (a+2)%3   2: H comp (a+1)%3   3: H comp (a+2)%3
// Slab storage replaces coordinate a by s in [0,2p) (s = c for c < p,
// s = c - (n_a - 2p) for c >= n_a - p) and keeps [z][y][x] order.
struct Grid {
    int nx, ny, nz, p;
    long long N;
    long long nxy;
    float S;
    const float *ce;               // S/eps_r per cell
    const float *prof[2][3][3];    // [E=0/H=1][axis][b=0, a=1, 1/kappa=2] -> n_a values
    long long slab_n[3];           // cells per slab axis
    // sources
    int nsrc;
    int skind[FD_MAXSRC], scomp[FD_MAXSRC], si[FD_MAXSRC], sj[FD_MAXSRC], sk[FD_MAXSRC];
    const float *samp[FD_MAXSRC];
    // conducting cells: the box [llo, lhi) and per box cell ([z][y][x] over
    // the box) ca = (1-u)/(1+u) and sigma; ce holds cb = S/eps/(1+u) there.
    // lca == nullptr: none.
    int llo[3], lhi[3];
    const float *lca, *lsig;
};

// index of cell (i,j,k) in a lossy-box array, or -1 outside the box
__device__ __forceinline__ long long lossy_index(const Grid &g, int i, int j, int k)
{
    if (!g.lca || i < g.llo[0] || i >= g.lhi[0] || j < g.llo[1] || j >= g.lhi[1] || k < g.llo[2] || k >= g.lhi[2])
        return -1;
    return ((long long)(k - g.llo[2]) * (g.lhi[1] - g.llo[1]) + (j - g.llo[1])) * (g.lhi[0] - g.llo[0]) +
           (i - g.llo[0]);
}

struct Fields {
    float *c[6];                   // Ex, Ey, Ez, Hx, Hy, Hz
};

struct Psi {
    float *a[3][4];                // per slab axis, the four arrays above (nullptr if p == 0)
};

// interface record geometry (section 2.2): per face f = 2a + side, two
// tangential components over the interior window of the two other axes.
struct RecGeom {
    int Lu[3], Lv[3];              // window sizes per face axis
    long long off[6];              // float offset of face f within one step
    long long loff;                // float offset of the lossy box's E^n (3 x box cells) within one step
    long long per_step;            // floats per step
};

struct Detectors {
    int ndet;
    int k[FD_MAXDET], i0[FD_MAXDET], i1[FD_MAXDET], j0[FD_MAXDET], j1[FD_MAXDET];
    long long off[FD_MAXDET];      // offset of the detector's window in a flux plane set
    long long per_step;            // floats of all windows for one step
    // interpolated (co-located) detectors: per step the six raw planes Ex, Ey
    // (E^{n+1}, plane k), Hx, Hy (H^{n+1/2}, layer k-1), Hx, Hy (layer k) over
    // the window extended by one cell in x and y; and E^n of plane k (Ex, Ey)
    int interp[FD_MAXDET];
    int energy[FD_MAXDET];         // co-located energy instead of flux: three more raw planes
                                   // (Ez, Hz of plane k, Ez of layer k-1), E^n of Ez on k and k-1
    long long roff[FD_MAXDET];     // offset of the detector's raw planes in a raw set
    long long raw_per_step;        // floats of all raw planes for one step
    long long eoff[FD_MAXDET];     // offset of the detector's two E^n planes
    long long eprev_floats;
    int kmin, kmax;                // planes on which any detector emits (kmin > kmax: none)
};

// ------------------------------------------------------------ device helpers

__device__ __forceinline__ int slab_coord(int c, int n, int p)
{
    return c < p ? c : (c >= n - p ? c - (n - 2 * p) : -1);
}

__device__ __forceinline__ long long slab_index(const Grid &g, int axis, int s, int i, int j, int k)
{
    const int w = 2 * g.p;
    if (axis == 0) return ((long long)k * g.ny + j) * w + s;
    if (axis == 1) return ((long long)k * w + s) * g.nx + i;
    return ((long long)s * g.ny + j) * g.nx + i;
}

__device__ __forceinline__ float cpml_term(float d, float &psi, float b, float a, float kinv)
{
    psi = fmaf(b, psi, a * d);
    return fmaf(d, kinv, psi);
}

__device__ __forceinline__ float h_update(float h, float S, float t1, float t2) { return fmaf(-S, t1 - t2, h); }
__device__ __forceinline__ float e_update(float e, float ce, float t1, float t2) { return fmaf(ce, t1 - t2, e); }
__device__ __forceinline__ float e_unupdate(float e, float ce, float t1, float t2) { return fmaf(-ce, t1 - t2, e); }
__device__ __forceinline__ float h_unupdate(float h, float S, float t1, float t2) { return fmaf(S, t1 - t2, h); }

// adjoint of one CPML-wrapped difference: with weight w on T, the coefficient
// of the difference is w/kappa + a*(psibar + w) and psibar becomes b*(psibar + w).
__device__ __forceinline__ float cpml_adj_coef(float w, float psibar, float a, float kinv)
{
    return fmaf(w, kinv, a * (psibar + w));
}

// non-interpolated flux density Ex*Hy - Ey*Hx
__device__ __forceinline__ float flux_density(float ex, float ey, float hx, float hy)
{
    return fmaf(ex, hy, -(ey * hx));
}

// tangential E on the index-0 planes is held at zero
__device__ __forceinline__ bool held_ex(int i, int j, int k) { (void)i; return j == 0 || k == 0; }
__device__ __forceinline__ bool held_ey(int i, int j, int k) { (void)j; return i == 0 || k == 0; }
__device__ __forceinline__ bool held_ez(int i, int j, int k) { (void)k; return i == 0 || j == 0; }

// ------------------------------------------------------------------ launchers
// All return hipSuccess or the launch error.

hipError_t launch_h_naive(const Grid &g, const Fields &F, const Psi &P, int n, int with_src, hipStream_t s);
// lrec: E^n of the lossy box into the record of step n (or nullptr)
hipError_t launch_e_naive(const Grid &g, const Fields &F, const Psi &P, int n, int with_src, float *lrec,
                          hipStream_t s);

// phase A of a reverse step: inverse E (interior), dJ/dd accumulation, adjoint H;
// lrec: E^n of the lossy box from the record of step n (or nullptr)
hipError_t launch_bwd_a(const Grid &g, const Fields &F, const Fields &A, const Psi &Pb, int n,
                        int do_inv, int do_adj, float *gacc, const int *dlo, const int *dhi,
                        const float *lrec, hipStream_t s);
// phase B: inverse H (interior), adjoint E, psi-bar updates (H-type ping-pong)
hipError_t launch_bwd_b(const Grid &g, const Fields &F, const Fields &A, const Psi &Pb_cur,
                        const Psi &Pb_next, int n, int do_inv, int do_adj, hipStream_t s);

// incident-field line of a TFSF plane: nodes for T steps (scratch 2*nodes - 1
// floats), and the launch writing the E and H correction series (T each)
int tfsf_line_nodes(int T);
hipError_t launch_tfsf_line(const float *amp, int T, float S, const float *ce_at, float hsign, float *line,
                            float *outE, float *outH, hipStream_t s);

// interpolated detectors: E^n of their planes before a sweep (or step); the
// raw planes of one step from the fields (per-cell path); the co-located flux
// density of `levels` steps from the raw planes into the flux planes
hipError_t launch_det_eprev(const Grid &g, const Fields &F, const Detectors &D, float *eprev, hipStream_t s);
hipError_t launch_det_raw(const Grid &g, const Fields &F, const Detectors &D, float *raw, hipStream_t s);
hipError_t launch_det_interp(const Grid &g, const Detectors &D, const float *raw, const float *eprev, int levels,
                             float *planes, hipStream_t s);
// their adjoint source before reverse step n (drec: raw planes of every step,
// e0: E planes of step 0; wS[m] = S * weight, zero weights skipped)
hipError_t launch_det_interp_adjoint(const Grid &g, const Detectors &D, const float *drec, const float *e0, int n,
                                    int T, const float *wS, const Fields &A, hipStream_t s);

hipError_t launch_record(const Grid &g, const Fields &F, const RecGeom &R, float *rec_step,
                         int side, int restore, hipStream_t s);
hipError_t launch_record_zero_e(const Grid &g, const Fields &F, const RecGeom &R, hipStream_t s);
hipError_t launch_det_planes(const Grid &g, const Fields &F, const Detectors &D, float *planes,
                             hipStream_t s);
hipError_t launch_det_adjoint(const Grid &g, const Fields &F, const Fields &A, const Detectors &D,
                              const float *weights_S, hipStream_t s);
hipError_t launch_reduce_rows(const float *in, long long len, int rows, long long row_stride,
                              float *out, int out_stride, hipStream_t s);
// two-level fixed-order row sums for long rows (scratch: reduce_scratch_floats)
hipError_t launch_reduce_rows2(const float *in, long long len, int rows, long long row_stride,
                               float *out, int out_stride, float *scratch, hipStream_t s);
long long reduce_scratch_floats(long long len, int rows);
hipError_t launch_objective(const float *trace, int steps, int ndet, const float *w, float S,
                            float *J, hipStream_t s);
hipError_t launch_interior_sumsq(const Grid &g, const Fields &F, float *partials, int *nparts,
                                 hipStream_t s);
hipError_t launch_recon(const float *part_T, const float *part_0, int nparts, float *out,
                        hipStream_t s);
hipError_t launch_deps(const float *gacc, const float *d_design, long long D, float S, float *out,
                       hipStream_t s);
// dJ/deps of the design cells that conduct: -d^2 S/(1+u)^2 g (overwrites launch_deps' values there)
hipError_t launch_deps_lossy(const Grid &g, const float *gacc, const float *d_design, const int *dlo, const int *dhi,
                             float *out, hipStream_t s);
// ca and cb = S/eps/(1+u) of the lossy box from 1/eps and sigma
hipError_t launch_lossy_coef(const Grid &g, const float *inv_eps, float *ce, float *lca, hipStream_t s);
hipError_t launch_fill(float *p, long long n, float v, hipStream_t s);
hipError_t launch_copy(float *dst, const float *src, long long n, hipStream_t s);
hipError_t launch_scale_ce(const float *inv_eps, float S, float *ce, long long n, hipStream_t s);
hipError_t launch_gather_box(const float *src, const Grid &g, const int *lo, const int *hi,
                             float *dst, hipStream_t s);

// ---------------------------------------------------------------- z-marches
// A z-march launch covers the tiles of every class of one or more handles
// (a batch of requests): block b finds its request r by the prefix counts
// first[], its tile in that request's table, and the tile's class picks the
// kernel body (bit 0: an x CPML slab in the halo-extended footprint, bit 1:
// a y slab).  What stays fixed over a handle's life (grid, both buffer sets,
// geometry of records and detectors) lives in device memory, one struct per
// handle, written at create; what changes per launch (step index, which
// buffer is current, per-step pointers) travels in the launch arguments.
constexpr int ZM_MAXREQ = 32;

// forward pass over K steps (fields and psi ping-pong)
struct TbArgs {
    Grid g;
    float *fld[2][6];       // the two field sets: component q of set b
    float *psi[2][3];       // the two CPML auxiliary sets: auxiliary 0 of slab axis a
    RecGeom R;
    Detectors D;
    const float4 *profv[3]; // per axis, per index: (b, a, 1/kappa) at E then H positions
    unsigned fstride;       // bytes from component q to q+1 of a field set (both sets alike)
    unsigned pstride[3];    // bytes from CPML auxiliary q to q+1 of axis a (both sets alike)
};
enum { TB_CUR = 1, TB_SRC = 2 };
struct TbReq {
    unsigned long long args;   // device address of the handle's TbArgs
    const int4 *tiles;      // per tile two int4: (x0, x1, y0, y1), (z0, z1, class, 0) owned box
    float *rec;             // record of step n0 (or nullptr); step n0+s at rec + s*per_step
    float *planes;          // detector flux planes of step n0 (or nullptr); + s*D.per_step
    float *raw;             // raw planes of the interpolated detectors, step n0; + s*D.raw_per_step
    int n0;                 // first step index of this block of K steps
    int first;              // first block of this request in the launch
    unsigned flags;         // TB_CUR: set 1 is the input; TB_SRC: apply sources
    int pad;
};
struct TbLaunch {
    int nreq, nblocks, xcd_remap, pad;
    TbReq r[ZM_MAXREQ];
};
// one sweep of K steps over every tile of the launch (wide: the instance
// with a 64-bit base per component and plane, for field sets of 4 GiB or
// more; fstride is unused there)
// lossy: the instance for handles with conducting cells (default shape,
// 32-bit offsets, K = 1 or 2: tb_lossy_ok)
hipError_t launch_tb_forward(const TbLaunch &L, int K, int shape, bool wide, bool lossy, hipStream_t s);
bool tb_lossy_ok(int K, int shape, bool wide);
int tb_tile_x(int K, int shape);
int tb_tile_y(int K, int shape);
bool tb_tile_aligned(int shape);   // x tiles start on 128-byte lines (uniform split)
bool tb_wide_shape(int shape);     // the wide instance exists for this shape
int tb_wg_per_cu(int shape);       // workgroups of this shape that share a CU
int tb_max_pml();

// fused reverse step (inverse + adjoint) as a z-march, tile halo rev_halo()
struct RevArgs {
    Grid g;
    float *fld[2][6];        // the two forward field sets
    float *adj[2][6];        // the two adjoint field sets
    float *pb[2][3];         // the two psi-bar sets: auxiliary 0 of slab axis a
    RecGeom R;
    Detectors D;
    float wS[FD_MAXDET];     // S * detector weight (interpolated detectors 0)
    int3 dlo, dhi;           // design box
    const float4 *profv[3];
    unsigned fstride;        // bytes from component q to q+1 of a field or adjoint set
    unsigned pstride[3];     // bytes from auxiliary q to q+1 of axis a (both sets alike)
};
// RV_CUR: forward set 1 is s_{n+1}; RV_ACUR: adjoint set 1 is the input;
// RV_APAR: psi-bar set 1 is the input
enum { RV_CUR = 1, RV_ACUR = 2, RV_APAR = 4, RV_INV = 8, RV_ADJ = 16, RV_DET = 32 };
struct RevReq {
    unsigned long long args;  // device address of the handle's RevArgs
    const int4 *tiles;
    const float *rec_h;      // record of step n (H on the low faces) or nullptr
    const float *rec_e;      // record of step n-1 (E on the high faces) or nullptr (E^0 = 0)
    float *gacc;             // dJ/dd accumulator over the design box (or nullptr)
    const float *fin;        // forward state read instead of set RV_CUR (or nullptr)
    int n;                   // forward step being reversed
    int first;
    unsigned flags;
    int pad;
};
struct RevLaunch {
    int nreq, nblocks, xcd_remap, pad;
    RevReq r[ZM_MAXREQ];
};
// lossy: the instance for handles with conducting cells (32-bit offsets only)
hipError_t launch_tb_reverse(const RevLaunch &L, bool wide, bool lossy, hipStream_t s);
int rev_halo();
int rev_tile_x();
int rev_tile_y();
int rev_wg_per_cu();
