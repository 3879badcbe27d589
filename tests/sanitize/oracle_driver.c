/* Runs the FP64 oracle's entry points on tiny problems so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer checks their memory
 * accesses: forward with the record, inverse, linear step and its transpose,
 * both gradients, with a CPML, a TFSF-like pair of plane sources, an
 * interpolated and an energy detector, and a lossy box.  Test infrastructure:
 * built and run by tests/test_sanitizers.py. */
#include <stdio.h>
#include <stdlib.h>
#include "../../oracle/fdtd_oracle.c"

static double frand(unsigned *s) { *s = *s * 1103515245u + 12345u; return ((*s >> 8) & 0xffff) / 65536.0; }

static int run(int p, int lossy)
{
    or_problem P;
    memset(&P, 0, sizeof P);
    P.nx = 13; P.ny = 11; P.nz = 12; P.S = 0.57; P.p = p;
    P.m = 3; P.sigma_max = p ? 1.2 : 0; P.kappa_max = 2; P.alpha_max = 0.01;
    size_t N = (size_t)P.nx * P.ny * P.nz;
    int T = 9;
    double *d = malloc(sizeof(double) * N), *sig = calloc(N, sizeof(double));
    unsigned s = 7;
    for (size_t c = 0; c < N; c++) d[c] = 1.0 / (1.0 + 10.0 * frand(&s));
    double *amp = malloc(sizeof(double) * T), *amp2 = malloc(sizeof(double) * T);
    for (int n = 0; n < T; n++) { amp[n] = frand(&s); amp2[n] = frand(&s); }
    P.d = d;
    P.nsrc = 2;
    P.src_kind[0] = 1; P.src_comp[0] = 0; P.src_k[0] = p + 2; P.src_amp[0] = amp;
    P.src_kind[1] = 0; P.src_comp[1] = 4; P.src_i[1] = 6; P.src_j[1] = 5; P.src_k[1] = 6; P.src_amp[1] = amp2;
    P.ndet = 3;
    int lo = p > 0 ? p : 1;
    for (int m = 0; m < 3; m++) {
        P.det_k[m] = P.nz - lo - 2 + (m == 2 ? 0 : 0);
        P.det_i0[m] = lo; P.det_i1[m] = P.nx - lo - 1; P.det_j0[m] = lo; P.det_j1[m] = P.ny - lo - 1;
        P.det_w[m] = 1.0 + m;
    }
    P.det_interp[1] = 1;
    P.det_interp[2] = 1; P.det_energy[2] = 1;
    P.dlo[0] = 4; P.dlo[1] = 4; P.dlo[2] = 4; P.dhi[0] = 8; P.dhi[1] = 7; P.dhi[2] = 7;
    if (lossy) {
        P.sig = sig;
        P.llo[0] = 3; P.llo[1] = 3; P.llo[2] = 4; P.lhi[0] = 9; P.lhi[1] = 8; P.lhi[2] = 6;
        for (int k = P.llo[2]; k < P.lhi[2]; k++)
            for (int j = P.llo[1]; j < P.lhi[1]; j++)
                for (int i = P.llo[0]; i < P.lhi[0]; i++) sig[((size_t)k * P.ny + j) * P.nx + i] = frand(&s);
    }
    size_t SZ = OR_NSLOT * N, rf = or_record_floats(&P);
    double *st = calloc(SZ, sizeof(double)), *tr = calloc((size_t)T * 3, sizeof(double));
    double *rec = calloc((size_t)T * (rf ? rf : 1), sizeof(double));
    double J = or_forward(&P, st, 0, T, tr, rec);
    or_inverse(&P, st, 0, T, rec);
    or_step_linear(&P, st, 2);
    or_adjoint_linear(&P, st, 2);
    double *g = calloc(N, sizeof(double)), *g2 = calloc(N, sizeof(double)), recon = 0;
    double J1 = or_grad_history(&P, T, 3, g, tr);
    double J2 = or_grad_reversed(&P, T, g2, tr, &recon);
    double out3[3];
    or_grade(&P, 0, 1.5, out3);
    printf("p=%d lossy=%d J=%.6e J1=%.6e J2=%.6e recon=%.2e\n", p, lossy, J, J1, J2, recon);
    free(d); free(sig); free(amp); free(amp2); free(st); free(tr); free(rec); free(g); free(g2);
    return 0;
}

int main(void)
{
    return run(0, 0) | run(3, 0) | run(0, 1) | run(3, 1);
}
