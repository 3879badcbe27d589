/* Host-side paths of libfdtd's C ABI that need no GPU -- descriptor
 * validation and workspace sizing (fdtd_footprint), argument checks of
 * fdtd_create, the checkpoint-schedule planner (fdtd_revolve_plan) and the
 * error messages -- for a build of fdtd_api.hip with AddressSanitizer and
 * UBSan on its host code.  Test infrastructure: built and run by
 * tests/test_sanitizers.py. */
#include <stdio.h>
#include <string.h>
#include "fdtd.h"
int main() {
    fdtd_desc d; memset(&d, 0, sizeof d);
    d.nx = 40; d.ny = 36; d.nz = 44; d.courant = 0.57f; d.pml_cells = 6;
    d.pml_order = -1; d.pml_sigma_max = -1; d.pml_kappa_max = -1; d.pml_alpha_max = -1; d.pml_eps_bg = 2.25f;
    d.inv_eps = (const float *)16; for (int a = 0; a < 3; a++) { d.design_lo[a] = 14; d.design_hi[a] = 22; }
    d.n_steps = 50; d.record = 1;
    fdtd_source s; memset(&s, 0, sizeof s); s.kind = 1; s.comp = 0; s.k = 8; s.amp = (const float *)16;
    fdtd_flux_detector det; memset(&det, 0, sizeof det); det.k = 35; det.i0 = 6; det.i1 = 34; det.j0 = 6; det.j1 = 30; det.weight = 1;
    size_t b = 0;
    printf("ok %d %zu\n", fdtd_footprint(&d, &s, 1, &det, 1, &b), b);
    d.sigma = (const float *)16; for (int a = 0; a < 3; a++) { d.lossy_lo[a] = 10; d.lossy_hi[a] = 20; }
    printf("lossy %d\n", fdtd_footprint(&d, &s, 1, &det, 1, &b));
    d.lossy_lo[0] = 2; printf("bad lossy %d %s\n", fdtd_footprint(&d, &s, 1, &det, 1, &b), fdtd_last_error(0));
    d.sigma = 0; d.nx = 2; printf("bad nx %d %s\n", fdtd_footprint(&d, &s, 1, &det, 1, &b), fdtd_last_error(0));
    fdtd_handle h = 0;
    printf("create null ws %d %s\n", fdtd_create(&d, &s, 1, &det, 1, 0, 0, 0, &h), fdtd_last_error(0));
    int64_t f; int32_t pk, n;
    printf("revolve %d\n", fdtd_revolve_plan(1000, 1, 5, &f, &pk, 0, 0, &n));
    int32_t acts[3 * 4000];
    printf("revolve acts %d %d %lld\n", fdtd_revolve_plan(200, 0, 0, &f, &pk, acts, 4000, &n), n, (long long)f);
    d.nx = 40;
    for (int v = 0; v < 12; v++) {          /* one invalid field at a time */
        fdtd_desc e = d;
        e.sigma = 0;
        switch (v) {
        case 0: e.courant = 0.7f; break;
        case 1: e.pml_cells = 30; break;
        case 2: e.time_block = 9; break;
        case 3: e.n_steps = 0; break;
        case 4: e.record = 3; break;
        case 5: e.design_hi[2] = 60; break;
        case 6: e.inv_eps = 0; break;
        case 7: e.design_lo[0] = e.design_hi[0]; break;
        default: break;
        }
        fdtd_source s2 = s; fdtd_flux_detector d2 = det;
        if (v == 8) s2.kind = 2, s2.k = 1;
        if (v == 9) d2.interpolate = 1, d2.i1 = 40;
        if (v == 10) d2.quantity = 1;
        if (v == 11) s2.amp = 0;
        int st = fdtd_footprint(&e, &s2, 1, &d2, 1, &b);
        printf("case %d -> %d %s\n", v, st, st ? fdtd_last_error(0) : "");
        if (st == 0) return 1;
    }
    return 0;
}
