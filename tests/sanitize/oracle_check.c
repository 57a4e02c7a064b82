/*
 * oracle_check.c -- runs the FP64 oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every entry point on periodic and walled
 * lattices, both force couplings, a body force, lattices of one row and one
 * column, and the invalid-argument paths.  Checks that results are finite
 * and that mass is conserved; any sanitizer report aborts the program.
 * Prints "ok" and exits 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sclbm_oracle.h"

#define FAIL(...)                                \
    do {                                         \
        fprintf(stderr, "oracle_check: ");       \
        fprintf(stderr, __VA_ARGS__);            \
        fprintf(stderr, "\n");                   \
        exit(1);                                 \
    } while (0)

static double urand(unsigned* s)
{
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

static void run_case(int nx, int ny, int walls, int forcing, double body)
{
    oracle_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.walls = walls;
    p.forcing = forcing;
    p.tau[0] = 0.9;
    p.tau[1] = 1.2;
    p.Ga[0] = -12.55;
    p.Ga[1] = -11.80;
    p.Gr[0] = 11.70;
    p.Gr[1] = 10.95;
    p.Gx = 0.58;
    p.rho0 = 0.7;
    p.psi_amp = 0.7;
    p.wall_u[1] = walls ? 0.05 : 0.0;
    p.body_F0 = body;
    const size_t N = (size_t)nx * ny;
    double* rho = malloc(sizeof(double) * 2 * N);
    double* f = malloc(sizeof(double) * 18 * N);
    double* out = malloc(sizeof(double) * 2 * N);
    double* ux = malloc(sizeof(double) * N);
    double* uy = malloc(sizeof(double) * N);
    double* row_u = malloc(sizeof(double) * ny);
    double* row_s = malloc(sizeof(double) * ny);
    double* psi = malloc(sizeof(double) * 2 * N);
    double* F = malloc(sizeof(double) * 4 * N);
    if (!rho || !f || !out || !ux || !uy || !row_u || !row_s || !psi || !F) FAIL("malloc");
    unsigned seed = 12345u + (unsigned)(nx * 31 + ny);
    for (size_t k = 0; k < 2 * N; ++k) rho[k] = 0.7 * (1.0 + 0.05 * (2.0 * urand(&seed) - 1.0));
    if (oracle_init(&p, rho, NULL, NULL, f)) FAIL("init %dx%d", nx, ny);
    double t0[6], t1[6], wm[4] = {0, 0, 0, 0}, sf[2];
    if (oracle_totals(&p, f, t0)) FAIL("totals");
    if (oracle_run(&p, f, 30, wm)) FAIL("run");
    if (oracle_totals(&p, f, t1)) FAIL("totals");
    if (oracle_moments(&p, f, out, ux, uy)) FAIL("moments");
    if (oracle_row_profiles(&p, f, row_u, row_s)) FAIL("row profiles");
    if (oracle_shear_flow(&p, f, sf)) FAIL("shear flow");
    for (size_t k = 0; k < 2 * N; ++k) psi[k] = oracle_psi(&p, out[k]);
    if (oracle_forces(&p, psi, out, F)) FAIL("forces");
    for (size_t k = 0; k < 2 * N; ++k)
        if (!isfinite(out[k])) FAIL("non-finite density %dx%d", nx, ny);
    for (int s = 0; s < 2; ++s)
        if (fabs(t1[s] - t0[s]) > 1e-12 * t0[s]) FAIL("mass %dx%d species %d", nx, ny, s);
    if (!isfinite(sf[0]) || !isfinite(sf[1]) || !isfinite(wm[2])) FAIL("observables");
    free(rho); free(f); free(out); free(ux); free(uy); free(row_u); free(row_s);
    free(psi); free(F);
}

int main(void)
{
    run_case(17, 13, 0, 0, 0.0);
    run_case(16, 9, 1, 0, 0.0);
    run_case(12, 20, 0, 1, 1e-5);
    run_case(11, 8, 1, 1, 0.0);
    run_case(1, 7, 0, 0, 0.0);
    run_case(9, 1, 0, 0, 0.0);
    run_case(5, 2, 1, 0, 0.0);
    /* invalid arguments are refused */
    oracle_params bad;
    memset(&bad, 0, sizeof bad);
    double dummy[18];
    if (oracle_run(&bad, dummy, 1, NULL) == 0) FAIL("invalid params accepted");
    bad.nx = bad.ny = 1;
    bad.tau[0] = bad.tau[1] = 0.4;
    bad.rho0 = 0.7;
    if (oracle_init(&bad, dummy, NULL, NULL, dummy) == 0) FAIL("tau <= 1/2 accepted");
    oracle_set_threads(2);
    run_case(10, 10, 1, 0, 0.0);
    printf("ok\n");
    return 0;
}
