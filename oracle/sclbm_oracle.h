/*
 * sclbm_oracle.h -- plain FP64 CPU oracle for the two-species, multi-range
 * Shan-Chen lattice Boltzmann model of Benzi, Chibbaro & Succi,
 * "Mesoscopic lattice Boltzmann modeling of flowing soft systems"
 * (arXiv:0807.4471).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, bench.py's cpu_baseline leg and
 * __graft_entry__.smoke() may load this library.  It shares no code, header,
 * table or helper with the HIP library in paper_0807_4471_amd/: it is the
 * independent definition the GPU path is checked against.
 *
 * Conventions (all fields are FP64, row-major, x fastest):
 *   site index        n = y*nx + x
 *   populations       f[((s*9 + i)*ny + y)*nx + x]     s = 0 (A), 1 (B)
 *   scalar fields     a[s*N + n]                       N = nx*ny
 *   force fields      F[(s*2 + c)*N + n]               c = 0 (x), 1 (y)
 * The state is the post-streaming, pre-collision population set f_is(r,t)
 * of Eq. (1): time t is the number of completed steps.
 *
 * The pins of each function, and what is parity unpinned, are listed at the
 * top of sclbm_oracle.c.
 */
#ifndef SCLBM_ORACLE_H
#define SCLBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny;      /* lattice size; nx >= 1, ny >= 1 (ny >= 2 with walls) */
    int32_t walls;       /* 0: periodic in y; 1: half-way bounce-back walls at
                            y = -1/2 (bottom) and y = ny - 1/2 (top)          */
    int32_t forcing;     /* how the force enters Eq. (1):
                            0: Shan-Chen shift of the equilibrium velocity,
                               u_eq,s = u' + tau_s F_s / rho_s;
                            1: Guo source term: both species relax towards
                               f^eq(rho_s, u), u = (sum_s j_s + F_s/2) / sum_s rho_s,
                               and gain (1 - 1/(2 tau_s)) w_i [3 (c_i - u).F_s
                               + 9 (c_i.u)(c_i.F_s)]                          */
    double tau[2];       /* BGK relaxation times tau_s (> 1/2), Eq. (1)        */
    double Ga[2];        /* like-species attraction G^a_s, first belt          */
    double Gr[2];        /* like-species repulsion  G^r_s, both belts          */
    double Gx;           /* cross-species repulsion G_AB                       */
    double rho0;         /* reference density of the pseudo-potential (> 0)    */
    double psi_amp;      /* amplitude A of Psi = A (1 - exp(-rho/rho0))        */
    double wall_u[2];    /* x-velocity of the bottom and top wall (walls = 1)  */
    double body_F0;      /* Kolmogorov body force amplitude: g_s,x =
                            rho_s * body_F0 * sin(2 pi y / ny); 0 = off        */
} oracle_params;

/* D2Q9 set used for streaming: velocities and weights w_i (first belt). */
void oracle_d2q9(int32_t cx[9], int32_t cy[9], double w[9]);

/* The 24 force offsets e (first belt: 8, second belt: 16) with their
 * attraction weight (w_i on the first belt, 0 on the second) and their
 * repulsion weight (p_1i or p_2i).  Also returns the rest weights w_0, p_0. */
void oracle_stencil(int32_t ex[24], int32_t ey[24], double wa[24], double wr[24],
                    double* w0, double* p0);

/* Psi_s[rho] = A (1 - exp(-rho/rho0)). */
double oracle_psi(const oracle_params* p, double rho);

/* Second-order D2Q9 equilibrium for density rho and velocity (ux, uy). */
void oracle_feq(double rho, double ux, double uy, double feq[9]);

/* Interaction forces F_s = F^a_s + F^r_s + F^X_s from supplied Psi and rho
 * fields (each [2][N]); writes F[2 species][2 comps][N].  Returns 0 or <0. */
int32_t oracle_forces(const oracle_params* p, const double* psi, const double* rho,
                      double* F);

/* f_is(r, 0) = f^eq_i(rho_s(r), u(r)); rho is [2][N], ux/uy are [N]. */
int32_t oracle_init(const oracle_params* p, const double* rho, const double* ux,
                    const double* uy, double* f);

/* Advance f by nsteps steps in place.  If wall_mom is not NULL, the momentum
 * received by the walls is ADDED to wall_mom[wall*2 + comp] (wall 0 bottom,
 * 1 top).  Returns 0, or <0 on invalid parameters / allocation failure. */
int32_t oracle_run(const oracle_params* p, double* f, int64_t nsteps, double* wall_mom);

/* Observables at time t: rho [2][N], physical velocity
 * u = (sum_s j_s + F_s/2) / sum_s rho_s into ux, uy [N] (any may be NULL). */
int32_t oracle_moments(const oracle_params* p, const double* f, double* rho,
                       double* ux, double* uy);

/* Lattice totals at time t:
 *   out[0], out[1]  mass of A and B
 *   out[2], out[3]  momentum  sum_r (sum_s j_s + F_s/2)
 *   out[4]          sum over sites of the deviatoric shear stress sigma_xy
 *   out[5]          number of sites with a non-finite or non-positive density */
int32_t oracle_totals(const oracle_params* p, const double* f, double out[6]);

/* Row profiles at time t for shear observables, each [ny]:
 *   ux_row[y]  row mean of the physical x-velocity
 *   sxy_row[y] row mean of the deviatoric shear stress sigma_xy             */
int32_t oracle_row_profiles(const oracle_params* p, const double* f, double* ux_row,
                            double* sxy_row);

/* Observables of the shear-flow experiment (the rheology part of the paper,
 * with the figure of R and I_AB) at time t:
 *   out[0]  U_bar = (2 / (nx ny)) sum_r u_x(r) sin(2 pi y / ny), the
 *           amplitude of the physical x-velocity on the forcing mode (the
 *           paper's plain row sum of U would vanish for a sine profile);
 *           R = U_bar / U0
 *   out[1]  I_AB = sum_r grad rho_A . grad rho_B, each gradient the
 *           isotropic D2Q9 difference 3 sum_i w_i c_i rho(r + c_i)
 *           (neighbours wrapped, or mirrored at walls)                      */
int32_t oracle_shear_flow(const oracle_params* p, const double* f, double out[2]);

/* Threads of the oracle's parallel loops (OpenMP over lattice rows; the
 * arithmetic, and so every result, is the same for any number of threads).
 * n < 1 selects all processors.  Returns the number set (1 without OpenMP). */
int32_t oracle_set_threads(int32_t n);
/* Threads the next parallel loop will use. */
int32_t oracle_threads(void);

#ifdef __cplusplus
}
#endif
#endif
