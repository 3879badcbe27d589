/*
 * fdtd.h -- C ABI of the MI355X reversible 3D FDTD library (libfdtd.so).
 *
 * The library advances Maxwell's curl equations on a Yee grid (arXiv
 * 2412.12360, section 2.1, eqs. 1-2) in normalised units: cell size 1,
 * c = eps0 = mu0 = 1, time step dt = S (the Courant number).  One step is
 *     H^{n+1/2} = H^{n-1/2} - S * curl E^n           (forward differences)
 *     E^{n+1}   = E^n + S/eps_r * curl H^{n+1/2}      (backward differences)
 * with a convolutional PML on all six faces (section 2.1), a perfectly
 * conducting box behind it, additive E sources and non-interpolated
 * Poynting-flux detectors (section 2.1).  The gradient of the detector
 * objective with respect to eps_r is computed by the paper's time-reversal
 * method (section 2.2): the interior is rebuilt step by step by the exact
 * inverse update, the PML-interface layers are replayed from a per-step
 * record, and a hand-written adjoint runs alongside.
 *
 * Conventions
 *  - Every array is float32, [nz][ny][nx] with x fastest, in device memory
 *    unless stated otherwise.  Component ids: 0..2 = Ex,Ey,Ez, 3..5 = Hx,Hy,Hz.
 *    Component positions (cell (i,j,k)): Ex(i+1/2,j,k), Ey(i,j+1/2,k),
 *    Ez(i,j,k+1/2), Hx(i,j+1/2,k+1/2), Hy(i+1/2,j,k+1/2), Hz(i+1/2,j+1/2,k).
 *  - The box is perfectly conducting: tangential E on the index-0 planes is
 *    held at zero; reads at index n_a are zero.
 *  - Ownership: the caller owns every device buffer (workspace, inputs,
 *    outputs).  The library copies inv_eps and source amplitudes into the
 *    workspace at create time; the workspace must outlive the handle.  The
 *    library allocates no device memory.
 *  - Streams: every call enqueues work on the stream given at create time (a
 *    hipStream_t passed as void*; NULL = the default stream) and returns
 *    without synchronising.  Outputs are valid once that stream has drained.
 *    One handle must not be used by two host threads at once.
 *  - Errors: arguments are validated before any work is enqueued; on error
 *    nothing is enqueued and fdtd_last_error() describes the cause.  No
 *    exception or abort crosses the ABI.
 *  - Determinism: no atomics; every reduction has a fixed order, so results
 *    are bitwise reproducible and independent of the time-block size.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_ctx *fdtd_handle;

typedef enum {
    FDTD_OK = 0,
    FDTD_E_INVALID = 1,      /* an argument is out of range or inconsistent   */
    FDTD_E_NOMEM = 2,        /* workspace smaller than fdtd_footprint()        */
    FDTD_E_DEVICE = 3,       /* a HIP call or kernel launch failed             */
    FDTD_E_STATE = 4,        /* call not allowed in the handle's current state */
    FDTD_E_UNSUPPORTED = 5   /* valid request this library does not implement  */
} fdtd_status;

enum { FDTD_EX = 0, FDTD_EY, FDTD_EZ, FDTD_HX, FDTD_HY, FDTD_HZ };

/* Grid, materials and run length (section 2.1: Yee grid, eps per cell, CPML). */
typedef struct {
    int32_t nx, ny, nz;          /* cells per axis, each >= 4                          */
    float courant;               /* S = c dt / dx, 0 < S < 1/sqrt(3)                   */
    int32_t pml_cells;           /* p >= 0 CPML cells on every face (0 = bare PEC box) */
    /* CFS-CPML grading in per-step units.  A negative value selects the default:
     * order 3, sigma_max = 0.8 (order+1) S / sqrt(pml_eps_bg), kappa_max 1,
     * alpha_max 0.01.  pml_eps_bg <= 0 means 1.                                    */
    float pml_order, pml_sigma_max, pml_kappa_max, pml_alpha_max, pml_eps_bg;
    const float *inv_eps;        /* device, N values of 1/eps_r (> 0); copied      */
    int32_t design_lo[3];        /* half-open design box (x,y,z); gradient target  */
    int32_t design_hi[3];
    int32_t n_steps;             /* T: length of the source amplitudes and trace,  */
                                 /* and the number of steps fdtd_grad reverses     */
    int32_t record;              /* 1: keep the per-step interface record (needed  */
                                 /* by fdtd_grad and by fdtd_inverse with a PML)   */
    int32_t time_block;          /* K steps fused per pass over the grid (0 = auto,*/
                                 /* 1..4); results are bitwise independent of K    */
    /* Conducting (lossy) cells.  Section 2.2 bases the time reversal on
     * lossless media: a conducting cell damps E by a factor below one per
     * step, so its update is not inverted.  As for the PML, the record keeps
     * what the inverse cannot rebuild: E^n of every cell of the lossy box,
     * each step (12 B per box cell per step).  In a box cell the E update is
     *     E^{n+1} = ca E^n + cb curl H^{n+1/2},  u = sigma S / (2 eps_r),
     *     ca = (1 - u) / (1 + u),  cb = S / (eps_r (1 + u))
     * (eps dE/dt = curl H - sigma E with E averaged over the two time levels),
     * and the gradient carries ca and cb and their derivatives in eps_r.
     * sigma: device, one value >= 0 per cell of the half-open box
     * [lossy_lo, lossy_hi) (x, y, z), [z][y][x] over the box, or NULL for
     * none; copied at create.  The box lies in the interior [p, n-p) and
     * outside the z layers of any TFSF plane.  A handle with conducting
     * cells runs lossy instances of the z-marches (time_block 0, 1 or 2 and
     * 32-bit offsets; bitwise equal to the per-cell kernels), else the
     * per-cell kernels; the checkpointed gradients refuse it
     * (FDTD_E_UNSUPPORTED).                                               */
    const float *sigma;
    int32_t lossy_lo[3];
    int32_t lossy_hi[3];
} fdtd_desc;

/* Sources (section 2.1).
 * kind 0 / 1, additive ("soft"): after the half step of step n that updates
 *   component comp (0..5 = Ex, Ey, Ez, Hx, Hy, Hz), that component gains amp[n]
 *   at the cell (i, j, k) (kind 0) or on every cell of the z-normal plane k
 *   (kind 1).  Held PEC cells of E components are skipped.
 * kind 2, one-sided total-field/scattered-field plane wave along +z (the
 *   source type section 2.1 names): comp = polarisation (0 = Ex, 1 = Ey);
 *   k = the first total-field E plane, p+1 <= k < nz-p, with the layers k-1
 *   and k outside the design box's z range; amp = the incident waveform,
 *   imposed on a 1D incident line one cell below the plane.  The library runs
 *   that line (the grid's S, eps_r of the plane's centre cell) at create and
 *   at fdtd_set_inv_eps, and adds its two corrections every step: S/eps H_inc
 *   to the polarisation component on plane k, +-S E_inc to Hy (Ex) or Hx (Ey)
 *   on layer k-1.  For normal incidence the line is exact, so below the plane
 *   the grid holds only the field scattered back.  Takes two of the
 *   FDTD_MAX_SOURCES slots; i, j are ignored.
 * amp: device, n_steps floats (copied at create). */
typedef struct {
    int32_t kind, comp, i, j, k;
    const float *amp;
} fdtd_source;

/* Poynting flux through the z-normal plane k over the window [i0,i1) x [j0,j1)
 * (section 2.1), and the objective J = S * sum_n weight * P[n].
 * interpolate = 0 (the default of the paper's optimisation runs): the
 *     components as they lie on the Yee grid,
 *         P[n] = sum Ex*Hy - Ey*Hx   with E^{n+1} and H^{n+1/2} at index (i,j,k).
 * interpolate = 1 (the paper's evaluation mode): every component averaged
 *     onto the point (i+1/2, j+1/2, k) at time n+1/2 -- Ex over j, j+1 and the
 *     steps n, n+1; Ey over i, i+1 and the two steps; Hx over i, i+1 and the
 *     layers k-1, k; Hy over j, j+1 and the two layers -- then the same sum.
 *     Needs k >= 1, i1 < nx, j1 < ny.  With record = 1 the library keeps the
 *     six planes such a detector reads (E^{n+1} of plane k, H^{n+1/2} of
 *     layers k-1 and k; 24 B per cell of the window extended by one cell in
 *     x and y, per step) so that the gradients can apply its adjoint source. */
/* quantity = 1 (with interpolate = 1): instead of the flux, the co-located
 * energy density sum of 1/2 (eps_r |E|^2 + |H|^2) at the same points and
 * time, eps_r of cell (i,j,k): Ez averaged over i, i+1, j, j+1, the layers
 * k-1, k and the two steps; Hz lies at the point already.  The gradients
 * apply its adjoint source; they return FDTD_E_UNSUPPORTED when a weighted
 * energy detector's plane lies in the design box's z range (the energy reads
 * eps_r there). */
typedef struct {
    int32_t k, i0, i1, j0, j1;
    float weight;
    int32_t interpolate;
    int32_t quantity;            /* 0 = Poynting flux, 1 = energy density */
} fdtd_flux_detector;

#define FDTD_MAX_SOURCES 4
#define FDTD_MAX_DETECTORS 4

/* Bytes of workspace the problem needs (fields, material, PML state, record,
 * adjoint state, scratch).  No device work.  bytes: host. */
fdtd_status fdtd_footprint(const fdtd_desc *desc, const fdtd_source *src, int32_t nsrc,
                           const fdtd_flux_detector *det, int32_t ndet, size_t *bytes);

/* Validate the problem, carve the caller's workspace and enqueue its
 * initialisation (fields zero, t = 0) on `stream`.  Checks: sizes, S, indices,
 * nsrc/ndet limits, design box and detector windows inside the interior
 * [p, n-p) when record = 1, inv_eps > 0 is the caller's duty.  Returns
 * FDTD_E_NOMEM if workspace_bytes < fdtd_footprint().  out: host. */
fdtd_status fdtd_create(const fdtd_desc *desc, const fdtd_source *src, int32_t nsrc,
                        const fdtd_flux_detector *det, int32_t ndet,
                        void *workspace, size_t workspace_bytes, void *stream,
                        fdtd_handle *out);

/* Advance n_steps time steps (section 2.1).  Requires t + n_steps <= n_steps of
 * the descriptor.  trace (device, may be NULL): receives [n_steps][ndet] fluxes
 * of these steps.  J (device, may be NULL): receives the objective accumulated
 * from t = 0 to the new t.  With record = 1 each step also writes its interface
 * record (section 2.2). */
fdtd_status fdtd_forward(fdtd_handle h, int32_t n_steps, float *trace, float *J);

/* Undo n_steps steps by the inverse update (section 2.2): E then H un-updated.
 * On a bare PEC box (p = 0) the whole grid is rebuilt; with a PML only the
 * interior [p, n-p)^3 is, using the record (record = 1 required). */
fdtd_status fdtd_inverse(fdtd_handle h, int32_t n_steps);

/* Gradient of J with respect to eps_r over the design box (section 2.2): runs
 * all T steps backwards, each an adjoint step fused with the inverse step.
 * Requires record = 1 and t = T reached from a reset.  Leaves t = 0.
 * dJ_deps: device, design-box cells, x fastest.  recon_err (device, may be
 * NULL): RMS of the rebuilt interior fields at t = 0 (exactly zero in exact
 * arithmetic) over the RMS of the interior fields at t = T. */
fdtd_status fdtd_grad(fdtd_handle h, float *dJ_deps, float *recon_err);

/* The same gradient in chunks (section 2.2), so that a caller can interleave
 * the reverse steps of several solves:
 *   fdtd_grad_begin  requires what fdtd_grad requires (record = 1, t = T from
 *                    a reset); zeroes the adjoint state and the accumulator.
 *   fdtd_grad_steps  runs n_steps reverse steps (n_steps <= t); t decreases.
 *   fdtd_grad_end    at t = 0: writes dJ_deps (and recon_err), as fdtd_grad.
 * begin, steps of any sizes summing to T, then end give the bits of
 * fdtd_grad.  Between begin and end, fdtd_forward, fdtd_inverse and the
 * checkpointed gradient return FDTD_E_STATE; fdtd_reset abandons the
 * gradient. */
fdtd_status fdtd_grad_begin(fdtd_handle h);
fdtd_status fdtd_grad_steps(fdtd_handle h, int32_t n_steps);
fdtd_status fdtd_grad_end(fdtd_handle h, float *dJ_deps, float *recon_err);

/* Batches of handles, for a serving loop that advances many solves at once
 * (continuous batching; the forward step of section 2.1 and the reverse
 * step of section 2.2 on several grids).  hs[0..nh) are distinct handles
 * created on one stream (the batch's); each keeps its own grid, state and
 * outputs.  Every sweep of the forward z-march, and every reverse step, is
 * one kernel launch whose tiles span all handles that take a sweep of that
 * length (handles on the per-cell kernels advance on their own).  The bits
 * of every handle's results are those of the single-handle calls.
 *   fdtd_forward_batch:    hs[i] as fdtd_forward(hs[i], n_steps[i],
 *                          traces ? traces[i] : NULL, Js ? Js[i] : NULL).
 *   fdtd_grad_steps_batch: hs[i] as fdtd_grad_steps(hs[i], n_steps[i]).
 * Host arrays: hs, n_steps, traces, Js (traces[i], Js[i]: device or NULL).
 * Errors: FDTD_E_INVALID for NULL or repeated handles, handles on different
 * streams or negative counts (fdtd_last_error(NULL)); FDTD_E_STATE as the
 * single-handle calls (that handle's message); nothing is enqueued on a
 * validation error.  A launch error is reported on every handle of the
 * launch and on fdtd_last_error(NULL). */
fdtd_status fdtd_forward_batch(const fdtd_handle *hs, int32_t nh, const int32_t *n_steps, float *const *traces,
                               float *const *Js);
fdtd_status fdtd_grad_steps_batch(const fdtd_handle *hs, int32_t nh, const int32_t *n_steps);

/* Gradient by checkpointing, the baseline the time-reversal gradient is
 * measured against (section 2.2 compares the two): runs the forward pass from
 * zero fields, keeping the complete state (fields and CPML auxiliaries) at
 * the start of every segment of `segment` steps, then walks the segments
 * backwards: restores the segment's first state, recomputes the segment one
 * step at a time keeping the fields after each step, and applies the adjoint
 * steps (no inverse) to the kept states.  Same dJ/deps as fdtd_grad up to the
 * rounding of the time reversal.
 *   store: caller-owned device memory, 256-byte aligned, of at least
 *          fdtd_checkpoint_bytes(h, segment) bytes (ceil(T/segment) full
 *          states + segment field states); the library does not allocate.
 *   dJ_deps: device, design cells; J: device [1] or NULL (the objective).
 * Needs a handle created with record = 1 (for the adjoint state; the record
 * itself is not used) on the z-march path.  Any t on entry; t = 0 on return
 * with zeroed fields.  Errors: E_STATE without record, E_UNSUPPORTED on the
 * per-cell fallback or on field sets of 4 GiB or more (the 64-bit-base path),
 * E_INVALID for a segment outside [1, T] or NULL/unaligned
 * pointers, E_NOMEM when store_bytes is too small. */
fdtd_status fdtd_checkpoint_bytes(fdtd_handle h, int32_t segment, size_t *bytes);
fdtd_status fdtd_grad_checkpointed(fdtd_handle h, int32_t segment, void *store, size_t store_bytes,
                                   float *dJ_deps, float *J);

/* Gradient by the checkpoint schedules section 2.2 contrasts with time
 * reversal, for measuring memory against time:
 *   schedule 0, recursive halving: the state at the middle of the span still
 *     to be reversed is kept, recursively, so ceil(log2 T) states at most are
 *     held; for T a power of two it costs T/2 log2 T forward steps beyond the
 *     T a stored history needs (the count the paper gives).
 *   schedule 1, treeverse: at most `snapshots` kept states, placed where the
 *     fewest forward steps result (dynamic programming over span length and
 *     free slots); 0 recomputes every step from s_0.
 * Each kept state is a complete forward state (fields and CPML auxiliaries).
 * The adjoint steps are those of fdtd_grad_checkpointed, applied in order
 * T-1 .. 0 to recomputed states, so dJ_deps and J equal its results bit for
 * bit.
 *   fdtd_revolve_plan (host only, no handle): for T steps, the forward steps
 *     the schedule runs, the most states it keeps at once, and (when actions
 *     is not NULL, capacity cap triples) its actions as (op, a, b) triples:
 *     op 0 restore kept state a (a = -1: the zero state s_0), op 1 advance b
 *     steps from step a, op 2 keep the current state as state a, op 3 the
 *     adjoint of step a on the current state (which is then s_{a+1}).
 *     n_actions receives the count.  E_INVALID for T < 1, a schedule other
 *     than 0 or 1, snapshots outside [0, 64], or cap too small;
 *     E_UNSUPPORTED when T x (snapshots + 1) exceeds 2^26.
 *   fdtd_revolve_bytes: device bytes of the store for handle h.
 *   fdtd_grad_revolve: runs the forward pass itself from zero fields and the
 *     whole gradient; store: caller-owned device memory, 256-byte aligned, of
 *     at least fdtd_revolve_bytes bytes.  Requirements and errors as
 *     fdtd_grad_checkpointed; t = 0 on return. */
fdtd_status fdtd_revolve_plan(int32_t T, int32_t schedule, int32_t snapshots, int64_t *forward_steps,
                              int32_t *peak_snapshots, int32_t *actions, int32_t cap, int32_t *n_actions);
fdtd_status fdtd_revolve_bytes(fdtd_handle h, int32_t schedule, int32_t snapshots, size_t *bytes);
fdtd_status fdtd_grad_revolve(fdtd_handle h, int32_t schedule, int32_t snapshots, void *store, size_t store_bytes,
                              float *dJ_deps, float *J);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the same
 * computation as fdtd_grad_checkpointed, with the checkpoint store taken from
 * a fixed device array inside the library instead of caller memory.  The
 * array holds fdtd_noalloc_store_bytes() bytes (256 MiB) on every GPU the
 * library runs this call on, from the first call on that GPU until the
 * process ends; the call allocates nothing.  Every call on one GPU uses the
 * same array (each call writes every store byte it later reads), so calls
 * that overlap on one GPU -- from two handles, threads or streams -- race and
 * must be serialised by the caller.  Errors: as fdtd_grad_checkpointed, and
 * FDTD_E_NOMEM when fdtd_checkpoint_bytes(h, segment) exceeds the array. */
fdtd_status fdtd_grad_checkpointed_noalloc(fdtd_handle h, int32_t segment, float *dJ_deps, float *J);
size_t fdtd_noalloc_store_bytes(void);

/* Replace 1/eps_r (device, N values) and the per-cell update coefficients;
 * allowed when t = 0. */
fdtd_status fdtd_set_inv_eps(fdtd_handle h, const float *inv_eps);

/* Zero the fields, PML state and adjoint state; t = 0. */
fdtd_status fdtd_reset(fdtd_handle h);

/* Move the handle to another stream (a hipStream_t as void*; NULL = the
 * default stream): later calls enqueue their work there.  The caller orders
 * the new stream after the work already enqueued on the old one (fdtd_create
 * returns with its own work finished).  A serving loop creates each handle on
 * a stream of its own, so that the creation does not wait for other
 * requests' queued work, and then moves it to the stream of its batches.
 * Not allowed while a chunked gradient runs (FDTD_E_STATE). */
fdtd_status fdtd_set_stream(fdtd_handle h, void *stream);

/* Release host-side state.  The workspace is the caller's to free.  The
 * handle is gone even when a HIP teardown call fails; that failure is
 * reported as FDTD_E_DEVICE with the message in fdtd_last_error(NULL). */
fdtd_status fdtd_destroy(fdtd_handle h);

/* Current time step t (host). */
fdtd_status fdtd_time(fdtd_handle h, int32_t *t);

/* Message of the last failed call on this handle (or of the last failed
 * handle-less call on this thread when h is NULL). */
const char *fdtd_last_error(fdtd_handle h);

/* ---- test and diagnostic hooks ------------------------------------------ */

/* Device pointer of the current buffer of field component comp (0..5) of the
 * forward state (which = 0) or the adjoint state (which = 1). */
fdtd_status fdtd_field_ptr(fdtd_handle h, int32_t which, int32_t comp, float **dev);

/* All device arrays that make up the forward (which = 0) or adjoint (which = 1)
 * state: the six fields and every CPML auxiliary array.  ptrs/counts are host
 * arrays of capacity `cap`; *n receives the number of arrays.  Inner products
 * over these arrays are layout independent. */
fdtd_status fdtd_state_arrays(fdtd_handle h, int32_t which, float **ptrs, size_t *counts,
                              int32_t cap, int32_t *n);

/* Apply the source-free step map M n times to the forward state (adjoint = 0),
 * or its exact transpose M^T n times to the adjoint state (adjoint = 1), with
 * the same kernels and launch configuration as fdtd_forward / fdtd_grad.
 * Does not change t. */
fdtd_status fdtd_linear_steps(fdtd_handle h, int32_t n, int32_t adjoint);

/* Device pointer to the interface record of step n: layout per step is, for
 * faces f = 2a + side (a = axis, side 0 = low face: H on layer p-1, side 1 =
 * high face: E on layer n_a - p), components (a+1)%3 then (a+2)%3, each over
 * the interior window of the two other axes u < v as [v][u]. */
fdtd_status fdtd_record_ptr(fdtd_handle h, int32_t n, float **dev, size_t *floats_per_step);

/* Time-block size K actually used (host). */
fdtd_status fdtd_time_block(fdtd_handle h, int32_t *K);

/* Kernels the forward and reverse steps run on (host): 0 = per-cell kernels
 * (a CPML thicker than the z-march stages, or FDTD_NAIVE); 1 = the forward
 * and reverse z-marches with 32-bit offsets from one base per field set;
 * 2 = the same marches with a 64-bit base per component and plane (a field
 * set of 4 GiB or more; fdtd_grad_checkpointed then returns
 * FDTD_E_UNSUPPORTED).  All three give the same bits. */
fdtd_status fdtd_kernel_path(fdtd_handle h, int32_t *path);

/* Tiles of each z-march class (host): counts[c] for class c = bit 0 (an x
 * CPML slab within the tile's halo-extended footprint) | bit 1 (a y slab);
 * class 0 tiles run the instance without x/y auxiliaries.  march = 0: the
 * fused reverse march; march = K' in 1..K: a forward sweep of K' steps.
 * All zero on the per-cell path.  Lets tests confirm which kernel instances
 * a problem exercises. */
fdtd_status fdtd_tile_classes(fdtd_handle h, int32_t march, int32_t counts[4]);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_H */
