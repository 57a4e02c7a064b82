/*
 * sclbm_oracle.c -- plain FP64 CPU oracle of one time step of the two-species
 * multi-range Shan-Chen lattice Boltzmann model (Benzi, Chibbaro & Succi,
 * arXiv:0807.4471).
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by tests/, bench.py (cpu_baseline) and
 * __graft_entry__.smoke(), never by the product path.  Shares nothing with
 * the HIP library.  Built with gcc -O2 -ffp-contract=off: every product and
 * sum below is rounded exactly where it is written.
 *
 * What follows the paper, and where:
 *   - lattice kinetic equation: stream + BGK relaxation + force, Eq. (1);
 *   - forces F^a (first belt, weights w), F^r (both belts, weights p_1, p_2)
 *     and F^X (first belt, uses the other species' density), the FORCE
 *     equations, with a leading minus sign so that positive couplings repel
 *     as the text after the FORCE equations states;
 *   - normalisation of w and p and 8th-order isotropy of p, the constraints
 *     listed after the FORCE equations and the remark on the 24-speed
 *     lattice near the end of the letter;
 *   - pseudo-potential Psi[rho] = A (1 - exp(-rho/rho0)), given right after
 *     the weight constraints (the paper uses A = sqrt(rho0); A is a
 *     parameter here).
 * Readings where the paper is silent:
 *   - force-to-population coupling: Shan-Chen equilibrium-velocity shift with
 *     the common velocity u' = sum_s(j_s/tau_s) / sum_s(rho_s/tau_s) and
 *     u_eq,s = u' + tau_s F_s / rho_s (the SC method the letter builds on);
 *     or, as a variant, Guo's source term with the barycentric velocity
 *     (j + F/2) / rho (exactly momentum-conserving for equal tau_s);
 *   - local equilibrium: second-order D2Q9 polynomial;
 *   - physical velocity: (sum_s j_s + F_s/2) / sum_s rho_s;
 *   - walls: half-way bounce-back with the moving-wall correction
 *     -2 w_i rho_s (c_i . u_w)/c_s^2, mirrored Psi/rho ghost rows.
 *
 * Parity pins (tests/test_oracle_*.py): weight tables solved from the paper's
 * constraints in exact rationals; 12/7 factor; point-source force pattern;
 * long-wave force expansion with the effective couplings G_s1, G_s2;
 * 8th-order isotropy of the repulsion stencil; zero net force; mass and
 * momentum conservation; uniform state; shear-wave viscosity
 * c_s^2 (tau - 1/2); exact Couette profile between walls; Galilean advection;
 * Stokes' first problem (wall stress rho U sqrt(nu / (pi t)) and the erfc
 * layer); a 90-degree rotation of the lattice rotating the result; Laplace
 * law dP ~ 1/R; the sign of the surface tension from whether a rippled flat
 * interface relaxes; 1 and N OpenMP threads bitwise equal.  Every function
 * below is pinned by at least one of these; the long-run physics built on
 * them (arrest, ageing curves, the sigma(rho0) curve) has no pin in the
 * paper beyond figures: parity unpinned there.  The read-outs (physical velocity with the half
 * force, sigma_xy, totals, row profiles, u_bar, I_AB) are checked with forces
 * and a body force on against a whole-array brute-force evaluation of their
 * definitions on tiny lattices, periodic and with walls.  Those definitions
 * are readings (the paper gives neither); the G = 0 textbook cases (exact
 * Couette velocity and stress) confirm them physically.
 */
#include "sclbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0)

/* D2Q9: rest, 4 axis speeds, 4 diagonal speeds (first belt). */
static const int32_t CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int32_t CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int32_t OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* First-belt weights w_i (Sum w = 1, Sum w c_x^2 = 1/3, fourth-order
 * isotropic): 4/9 at rest, 1/9 on the axes, 1/36 on the diagonals. */
static double w_of(int i)
{
    if (i == 0) return 4.0 / 9.0;
    if (i <= 4) return 1.0 / 9.0;
    return 1.0 / 36.0;
}

/* Repulsion weights p by shell |e|^2 = 1, 2 (first belt) and 4, 5, 8 (second
 * belt): the unique solution of Sum p = 1, Sum p c_x^2 = 1/3 and isotropy of
 * the lattice tensors up to 8th order. */
static double p_of_shell(int e2)
{
    switch (e2) {
    case 1: return 4.0 / 63.0;
    case 2: return 4.0 / 135.0;
    case 4: return 1.0 / 180.0;
    case 5: return 2.0 / 945.0;
    case 8: return 1.0 / 15120.0;
    default: return 0.0;
    }
}

/* Second-belt offsets (16 of them): |e|^2 = 4, 5, 8. */
static const int32_t B2X[16] = {2, 0, -2, 0, 2, 1, -1, -2, -2, -1, 1, 2, 2, -2, -2, 2};
static const int32_t B2Y[16] = {0, 2, 0, -2, 1, 2, 2, 1, -1, -2, -2, -1, 2, 2, -2, -2};

void oracle_d2q9(int32_t cx[9], int32_t cy[9], double w[9])
{
    for (int i = 0; i < 9; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        w[i] = w_of(i);
    }
}

void oracle_stencil(int32_t ex[24], int32_t ey[24], double wa[24], double wr[24],
                    double* w0, double* p0)
{
    for (int i = 1; i <= 8; ++i) {
        ex[i - 1] = CX[i];
        ey[i - 1] = CY[i];
        wa[i - 1] = w_of(i);
        wr[i - 1] = p_of_shell(CX[i] * CX[i] + CY[i] * CY[i]);
    }
    for (int k = 0; k < 16; ++k) {
        ex[8 + k] = B2X[k];
        ey[8 + k] = B2Y[k];
        wa[8 + k] = 0.0;
        wr[8 + k] = p_of_shell(B2X[k] * B2X[k] + B2Y[k] * B2Y[k]);
    }
    if (w0) *w0 = w_of(0);
    if (p0) *p0 = 247.0 / 420.0;
}

int32_t oracle_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n < 1) n = omp_get_num_procs();
    omp_set_num_threads(n);
    return n;
#else
    (void)n;
    return 1;
#endif
}

int32_t oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

double oracle_psi(const oracle_params* p, double rho)
{
    return p->psi_amp * (1.0 - exp(-rho / p->rho0));
}

void oracle_feq(double rho, double ux, double uy, double feq[9])
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        feq[i] = w_of(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

static int valid(const oracle_params* p)
{
    if (!p || p->nx < 1 || p->ny < 1) return 0;
    if (p->walls && p->ny < 2) return 0;
    if (!(p->tau[0] > 0.5) || !(p->tau[1] > 0.5) || !(p->rho0 > 0.0)) return 0;
    if (p->forcing != 0 && p->forcing != 1) return 0;
    return 1;
}

static int wrapx(const oracle_params* p, int x)
{
    x %= p->nx;
    return x < 0 ? x + p->nx : x;
}

/* Row of the neighbour at y + dy for the force stencil: periodic wrap, or
 * mirror images about the wall planes y = -1/2 and y = ny - 1/2. */
static int nbr_row(const oracle_params* p, int y, int dy)
{
    int yy = y + dy;
    if (!p->walls) {
        yy %= p->ny;
        return yy < 0 ? yy + p->ny : yy;
    }
    if (yy < 0) yy = -1 - yy;
    if (yy > p->ny - 1) yy = 2 * p->ny - 1 - yy;
    return yy;
}

int32_t oracle_forces(const oracle_params* p, const double* psi, const double* rho, double* F)
{
    if (!valid(p)) return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    for (int s = 0; s < 2; ++s) {
        const int so = 1 - s;
        const double* ps = psi + s * N;
        const double* rs = rho + s * N;
        const double* ro = rho + so * N;
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                const size_t n = (size_t)y * nx + x;
                /* F^a: first belt, weights w_i, on Psi_s. */
                double ax = 0.0, ay = 0.0;
                /* F^r: first belt with p_1i plus second belt with p_2i, on Psi_s. */
                double rx = 0.0, ry = 0.0;
                /* F^X: first belt, weights w_i, on rho of the other species. */
                double xx = 0.0, xy = 0.0;
                for (int i = 1; i <= 8; ++i) {
                    const size_t m = (size_t)nbr_row(p, y, CY[i]) * nx + wrapx(p, x + CX[i]);
                    const double wi = w_of(i);
                    const double pi = p_of_shell(CX[i] * CX[i] + CY[i] * CY[i]);
                    ax += wi * ps[m] * CX[i];
                    ay += wi * ps[m] * CY[i];
                    rx += pi * ps[m] * CX[i];
                    ry += pi * ps[m] * CY[i];
                    xx += wi * ro[m] * CX[i];
                    xy += wi * ro[m] * CY[i];
                }
                for (int k = 0; k < 16; ++k) {
                    const size_t m = (size_t)nbr_row(p, y, B2Y[k]) * nx + wrapx(p, x + B2X[k]);
                    const double pk = p_of_shell(B2X[k] * B2X[k] + B2Y[k] * B2Y[k]);
                    rx += pk * ps[m] * B2X[k];
                    ry += pk * ps[m] * B2Y[k];
                }
                const double gx = p->Gx / p->rho0;
                F[(s * 2 + 0) * N + n] = -p->Ga[s] * ps[n] * ax - p->Gr[s] * ps[n] * rx
                                         - gx * rs[n] * xx;
                F[(s * 2 + 1) * N + n] = -p->Ga[s] * ps[n] * ay - p->Gr[s] * ps[n] * ry
                                         - gx * rs[n] * xy;
            }
        }
    }
    return 0;
}

int32_t oracle_init(const oracle_params* p, const double* rho, const double* ux,
                    const double* uy, double* f)
{
    if (!valid(p)) return -1;
    const size_t N = (size_t)p->nx * p->ny;
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < N; ++n) {
            double feq[9];
            oracle_feq(rho[s * N + n], ux ? ux[n] : 0.0, uy ? uy[n] : 0.0, feq);
            for (int i = 0; i < 9; ++i) f[(s * 9 + i) * N + n] = feq[i];
        }
    return 0;
}

/* Densities, momenta, Psi and total force (interaction + body force) at
 * time t.  Work arrays are [2][N] (rho, jx, jy, psi) and [2][2][N] (F). */
static void fields(const oracle_params* p, const double* f, double* rho, double* jx,
                   double* jy, double* psi, double* F)
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    for (int s = 0; s < 2; ++s)
#pragma omp parallel for schedule(static)
        for (size_t n = 0; n < N; ++n) {
            double r = 0.0, mx = 0.0, my = 0.0;
            for (int i = 0; i < 9; ++i) {
                const double v = f[(s * 9 + i) * N + n];
                r += v;
                mx += v * CX[i];
                my += v * CY[i];
            }
            rho[s * N + n] = r;
            jx[s * N + n] = mx;
            jy[s * N + n] = my;
            psi[s * N + n] = oracle_psi(p, r);
        }
    oracle_forces(p, psi, rho, F);
    if (p->body_F0 != 0.0) {
        const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            const double sy = sin(two_pi * (double)y / (double)ny);
            for (int x = 0; x < nx; ++x) {
                const size_t n = (size_t)y * nx + x;
                for (int s = 0; s < 2; ++s)
                    F[(s * 2 + 0) * N + n] += rho[s * N + n] * p->body_F0 * sy;
            }
        }
    }
}

int32_t oracle_run(const oracle_params* p, double* f, int64_t nsteps, double* wall_mom)
{
    if (!valid(p) || nsteps < 0) return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    double* rho = malloc(sizeof(double) * 2 * N);
    double* jx = malloc(sizeof(double) * 2 * N);
    double* jy = malloc(sizeof(double) * 2 * N);
    double* psi = malloc(sizeof(double) * 2 * N);
    double* F = malloc(sizeof(double) * 4 * N);
    double* fn = malloc(sizeof(double) * 18 * N);
    if (!rho || !jx || !jy || !psi || !F || !fn) {
        free(rho); free(jx); free(jy); free(psi); free(F); free(fn);
        return -2;
    }
    for (int64_t t = 0; t < nsteps; ++t) {
        fields(p, f, rho, jx, jy, psi, F);
        /* Rows run in parallel: every site writes its own streamed
         * destinations, and only row 0 (bottom wall) and row ny - 1 (top
         * wall) add into wall_mom, each into its own entries in site order,
         * so the result is the same for any number of threads. */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = (size_t)y * nx + x;
                double feq[9];
                double upx = 0.0, upy = 0.0;
                if (p->forcing == 0) {
                    /* Common velocity u' weighted by rho_s / tau_s. */
                    double num_x = 0.0, num_y = 0.0, den = 0.0;
                    for (int s = 0; s < 2; ++s) {
                        num_x += jx[s * N + n] / p->tau[s];
                        num_y += jy[s * N + n] / p->tau[s];
                        den += rho[s * N + n] / p->tau[s];
                    }
                    if (den > 0.0) {
                        upx = num_x / den;
                        upy = num_y / den;
                    }
                } else {
                    /* Guo: barycentric velocity with half the force. */
                    double mx = 0.0, my = 0.0, rt = 0.0;
                    for (int s = 0; s < 2; ++s) {
                        mx += jx[s * N + n] + 0.5 * F[(s * 2 + 0) * N + n];
                        my += jy[s * N + n] + 0.5 * F[(s * 2 + 1) * N + n];
                        rt += rho[s * N + n];
                    }
                    if (rt > 0.0) {
                        upx = mx / rt;
                        upy = my / rt;
                    }
                }
                for (int s = 0; s < 2; ++s) {
                    const double r = rho[s * N + n];
                    const double Fx = F[(s * 2 + 0) * N + n], Fy = F[(s * 2 + 1) * N + n];
                    double uex = upx, uey = upy;
                    if (p->forcing == 0 && r > 0.0) {
                        uex = upx + p->tau[s] * Fx / r;
                        uey = upy + p->tau[s] * Fy / r;
                    }
                    oracle_feq(r, uex, uey, feq);
                    for (int i = 0; i < 9; ++i) {
                        const double fi = f[(s * 9 + i) * N + n];
                        /* BGK relaxation of Eq. (1), then free streaming. */
                        double fs = fi - (fi - feq[i]) / p->tau[s];
                        if (p->forcing == 1) {
                            const double cu = CX[i] * upx + CY[i] * upy;
                            const double cf = CX[i] * Fx + CY[i] * Fy;
                            const double uf = upx * Fx + upy * Fy;
                            fs += (1.0 - 0.5 / p->tau[s]) * w_of(i) *
                                  (3.0 * (cf - uf) + 9.0 * cu * cf);
                        }
                        const int yd = y + CY[i];
                        if (p->walls && (yd < 0 || yd >= ny)) {
                            const int top = yd >= ny;
                            const double uw = p->wall_u[top];
                            const double back = fs - 2.0 * w_of(i) * r * (CX[i] * uw) / CS2;
                            fn[(s * 9 + OPP[i]) * N + n] = back;
                            if (wall_mom) {
                                wall_mom[top * 2 + 0] += CX[i] * (fs + back);
                                wall_mom[top * 2 + 1] += CY[i] * (fs + back);
                            }
                        } else {
                            const int yy = ((yd % ny) + ny) % ny;
                            const size_t m = (size_t)yy * nx + wrapx(p, x + CX[i]);
                            fn[(s * 9 + i) * N + m] = fs;
                        }
                    }
                }
            }
        memcpy(f, fn, sizeof(double) * 18 * N);
    }
    free(rho); free(jx); free(jy); free(psi); free(F); free(fn);
    return 0;
}

/* Physical velocity and deviatoric shear stress at every site. */
static int observe(const oracle_params* p, const double* f, double* rho, double* ux,
                   double* uy, double* sxy, double* mom)
{
    const size_t N = (size_t)p->nx * p->ny;
    double* r = malloc(sizeof(double) * 2 * N);
    double* jx = malloc(sizeof(double) * 2 * N);
    double* jy = malloc(sizeof(double) * 2 * N);
    double* psi = malloc(sizeof(double) * 2 * N);
    double* F = malloc(sizeof(double) * 4 * N);
    if (!r || !jx || !jy || !psi || !F) {
        free(r); free(jx); free(jy); free(psi); free(F);
        return -2;
    }
    fields(p, f, r, jx, jy, psi, F);
#pragma omp parallel for schedule(static)
    for (size_t n = 0; n < N; ++n) {
        double feq[9];
        double mx = 0.0, my = 0.0, rt = 0.0;
        for (int s = 0; s < 2; ++s) {
            mx += jx[s * N + n] + 0.5 * F[(s * 2 + 0) * N + n];
            my += jy[s * N + n] + 0.5 * F[(s * 2 + 1) * N + n];
            rt += r[s * N + n];
        }
        const double vx = rt > 0.0 ? mx / rt : 0.0;
        const double vy = rt > 0.0 ? my / rt : 0.0;
        if (rho) {
            rho[n] = r[n];
            rho[N + n] = r[N + n];
        }
        if (ux) ux[n] = vx;
        if (uy) uy[n] = vy;
        if (mom) {
            mom[2 * n] = mx;
            mom[2 * n + 1] = my;
        }
        if (sxy) {
            double acc = 0.0;
            for (int s = 0; s < 2; ++s) {
                oracle_feq(r[s * N + n], vx, vy, feq);
                double q = 0.0;
                for (int i = 0; i < 9; ++i)
                    q += CX[i] * CY[i] * (f[(s * 9 + i) * N + n] - feq[i]);
                acc += -(1.0 - 0.5 / p->tau[s]) * q;
            }
            sxy[n] = acc;
        }
    }
    free(r); free(jx); free(jy); free(psi); free(F);
    return 0;
}

int32_t oracle_moments(const oracle_params* p, const double* f, double* rho, double* ux,
                       double* uy)
{
    if (!valid(p)) return -1;
    return observe(p, f, rho, ux, uy, NULL, NULL);
}

int32_t oracle_totals(const oracle_params* p, const double* f, double out[6])
{
    if (!valid(p)) return -1;
    const size_t N = (size_t)p->nx * p->ny;
    double* rho = malloc(sizeof(double) * 2 * N);
    double* sxy = malloc(sizeof(double) * N);
    double* mom = malloc(sizeof(double) * 2 * N);
    if (!rho || !sxy || !mom) {
        free(rho); free(sxy); free(mom);
        return -2;
    }
    int rc = observe(p, f, rho, NULL, NULL, sxy, mom);
    if (rc == 0) {
        double ma = 0.0, mb = 0.0, px = 0.0, py = 0.0, sx = 0.0, bad = 0.0;
        for (size_t n = 0; n < N; ++n) {
            ma += rho[n];
            mb += rho[N + n];
            px += mom[2 * n];
            py += mom[2 * n + 1];
            sx += sxy[n];
            if (!(rho[n] > 0.0) || !(rho[N + n] > 0.0) || !isfinite(rho[n]) ||
                !isfinite(rho[N + n]))
                bad += 1.0;
        }
        out[0] = ma; out[1] = mb; out[2] = px; out[3] = py; out[4] = sx; out[5] = bad;
    }
    free(rho); free(sxy); free(mom);
    return rc;
}

int32_t oracle_row_profiles(const oracle_params* p, const double* f, double* ux_row,
                            double* sxy_row)
{
    if (!valid(p)) return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    double* ux = malloc(sizeof(double) * N);
    double* sxy = malloc(sizeof(double) * N);
    if (!ux || !sxy) {
        free(ux); free(sxy);
        return -2;
    }
    int rc = observe(p, f, NULL, ux, NULL, sxy, NULL);
    if (rc == 0)
        for (int y = 0; y < ny; ++y) {
            double a = 0.0, b = 0.0;
            for (int x = 0; x < nx; ++x) {
                a += ux[(size_t)y * nx + x];
                b += sxy[(size_t)y * nx + x];
            }
            if (ux_row) ux_row[y] = a / nx;
            if (sxy_row) sxy_row[y] = b / nx;
        }
    free(ux); free(sxy);
    return rc;
}

int32_t oracle_shear_flow(const oracle_params* p, const double* f, double out[2])
{
    if (!valid(p)) return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    double* rho = malloc(sizeof(double) * 2 * N);
    double* ux = malloc(sizeof(double) * N);
    if (!rho || !ux) {
        free(rho); free(ux);
        return -2;
    }
    int rc = observe(p, f, rho, ux, NULL, NULL, NULL);
    if (rc == 0) {
        const double two_pi = 6.283185307179586476925286766559;
        double proj = 0.0, iab = 0.0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = (size_t)y * nx + x;
                proj += ux[n] * sin(two_pi * (double)y / (double)ny);
                double g[2][2] = {{0.0, 0.0}, {0.0, 0.0}};  /* [species][component] */
                for (int i = 1; i < 9; ++i) {
                    const size_t m = (size_t)nbr_row(p, y, CY[i]) * nx + wrapx(p, x + CX[i]);
                    for (int s = 0; s < 2; ++s) {
                        g[s][0] += 3.0 * w_of(i) * CX[i] * rho[s * N + m];
                        g[s][1] += 3.0 * w_of(i) * CY[i] * rho[s * N + m];
                    }
                }
                iab += g[0][0] * g[1][0] + g[0][1] * g[1][1];
            }
        out[0] = 2.0 * proj / (double)N;
        out[1] = iab;
    }
    free(rho); free(ux);
    return rc;
}
