// sclbm_internal.h -- shared between the HIP kernels and the host runtime of
// libsclbm.so (not part of the public ABI).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sclbm {

// Slots of the FP64 diagnostics record.
enum {
    D_MASS_A = 0,
    D_MASS_B = 1,
    D_MOM_X = 2,
    D_MOM_Y = 3,
    D_SXY = 4,
    D_BAD = 5,
    D_UPROJ = 6,  // sum_r u_x sin(2 pi y / ny)
    D_IAB = 7,    // sum_r grad rho_A . grad rho_B
    NDIAG = 8
};

// Kernel modes: a full step, a step that also reduces diagnostics of the
// state it starts from, a read-out of moments, a diagnostics-only pass.
// M_PHI: the order parameter phi = rho_A - rho_B of the state, written to
// out[0] if set, with FP64 sums of phi * out[1] (a reference field, if set)
// and phi^2 in diagnostics slots 0 and 1.
enum { M_STEP = 0, M_STEP_DIAG = 1, M_READ = 2, M_DIAG = 3, M_PHI = 4 };

// Population storage in HBM: f[s][i][row][x], s-major then direction, rows of
// `pitch` elements, `plane` elements between consecutive (s, i) planes.  With
// walls there are two ghost rows (row 0 below the channel, row ny + 1 above);
// real row y sits at row y + walls.  The 9 planes of a species span < 2^31
// bytes (they are addressed through one buffer resource with 32-bit
// offsets).  What is stored is the post-collision
// set f*(t-1); a step pulls f_i(x, t) = f*_i(x - c_i, t-1).
struct Geo {
    int32_t nx, ny, walls, rows, pitch;
    int32_t pad_;
    int64_t plane;
};

// Per-instance constants in the arithmetic type A of the kernel.
//   Force on species s (pair form of the FORCE equations, offsets e and -e
//   combined):  F_s = -Psi_s(x) * S_s - rho_s(x) * X_s, with shell
//   coefficients K(|e|^2) = G^a_s w(|e|^2) + G^r_s p(|e|^2) folded into
//   K1, K2, K4x2 = 2 K(4), K5, K8x2 = 2 K(8), and X1 = (G_AB/rho0) w(1),
//   X2 = (G_AB/rho0) w(2).
template <class A>
struct Coef {
    A K1[2], K2[2], K4x2[2], K5[2], K8x2[2];
    A X1, X2;
    A tau[2], omega[2], hs[2];  // hs = 1 - 1/(2 tau): stress prefactor
    A psi_amp, neg_inv_rho0;
    A wall6u[2];                // 6 u_w (bottom, top): 2 (c_i.u_w)/c_s^2 = 6 c_ix u_w
    A rho_base[2];              // FP16 deviation storage: rho_ref_s (0 otherwise)
    int32_t tau1[2];            // 1 if tau_s == 1 exactly (BGK lands on f^eq)
    int32_t guo, pad_;          // 1: Guo source term instead of the velocity shift
    double body_F0;             // Kolmogorov amplitude (0 = off)
    double two_pi_over_ny;
};

// Everything one instance's tile sweep needs.
template <class S, class A>
struct Inst {
    const S* fin;
    S* fout;
    Geo g;
    Coef<A> c;
    int32_t W, H;               // interior columns per strip, rows per chunk
    int32_t nstrips, nchunks;
    int32_t throttle;           // wait for the previous row's stores each iteration
    int32_t pad2_;
    int64_t t;                  // time at the start of this step (FP16 rounding key)
    double* partials;           // [nblocks][NDIAG] (diagnostic modes)
    double* wall_acc;           // [2 walls][2 comps][nx], accumulated every step
    double* out[5];             // READ mode: rhoA, rhoB, ux, uy, sxy (any NULL);
                                // PHI mode: phi out, phi reference (either NULL)
};

// One instance inside a persistent batch launch.  `I` describes the
// instance's first step of the launch (fin/fout, time); later steps swap the
// population copies and advance the time.
template <class S, class A>
struct BatchInst {
    Inst<S, A> I;
    int64_t steps;    // steps of this instance in this launch
    int32_t stacked;  // 1: stacked 4-wave tiles, 0: 4-wave-wide sweep strips
    int32_t pad_;
};

struct BatchItem {
    int32_t inst, tile;  // tile = strip * nchunks + chunk of that instance
};

// Grid-barrier state of a batch launch (zeroed before each launch).
struct BatchCtl {
    uint32_t count, gen, err, pad_;
};

// Row of the lattice whose values a (ring) row index r stands for.
// Periodic: r mod ny.  Walls: the mirror images about the wall planes
// y = -1/2 and y = ny - 1/2 repeat with period 2 ny (even extension), so any
// r (tile rows may reach y0 + RW + 1 >= 2 ny on very short lattices) folds
// into [0, ny).
__host__ __device__ inline int fold_row(int r, int ny, bool walls)
{
    if (!walls) {
        r %= ny;
        return r < 0 ? r + ny : r;
    }
    const int p = 2 * ny;
    r %= p;
    if (r < 0) r += p;
    return r < ny ? r : p - 1 - r;
}

// Host-side launchers, dispatching on the storage type (sclbm_dispatch.cpp).
// cw > 0: sweep strips cw waves wide; cw < 0: stacked tiles of -cw waves,
// with write-through population stores if wt.
hipError_t launch_sweep(int storage, int cw, int wt, int mode, const void* inst, int nblocks,
                        hipStream_t st);
hipError_t launch_reduce(const double* partials, int nblocks, double* out, hipStream_t st);
// Tile paths a batch kernel holds: stacked tiles, sweep strips, or both.
enum { B_STACKED = 0, B_SWEEP = 1, B_MIXED = 2 };

// Largest co-resident grid of the batch kernel of this storage and kind, 0 on
// error.
int batch_grid(int storage, int kind);
// Persistent batch launch: max_steps steps in one cooperative launch; a
// workgroup gives up at a grid barrier after spin_limit sleeps.
hipError_t launch_batch(int storage, int kind, const void* insts, const BatchItem* items,
                        int nitems, int64_t max_steps, BatchCtl* ctl, uint32_t spin_limit,
                        int grid, hipStream_t st);
// Step s of every instance with steps > s: one ordinary launch of nitems
// workgroups (one per item).
hipError_t launch_batch_step(int storage, int kind, const void* insts, const BatchItem* items,
                             int nitems, int64_t s, hipStream_t st);
hipError_t launch_init(int storage, const void* inst, const double* rhoA, const double* rhoB,
                       const double* ux, const double* uy, int random, uint64_t seed,
                       double meanA, double meanB, double amp, hipStream_t st);

// The kernels of one storage type, from the unit built with -DSCLBM_STORAGE=k
// (sclbm_kernels.hip is compiled once per storage type).
#define SCLBM_CAT2_(a, b) a##b
#define SCLBM_CAT_(a, b) SCLBM_CAT2_(a, b)
#define SCLBM_SFX(name) SCLBM_CAT_(name, SCLBM_CAT_(_s, SCLBM_STORAGE))
#define SCLBM_DECLARE_STORAGE_UNIT(k)                                                       \
    hipError_t launch_sweep_s##k(int cw, int wt, int walls, int mode, const void* inst,   \
                                 int nb, hipStream_t st);                                 \
    int batch_grid_s##k(int kind);                                                        \
    hipError_t launch_batch_s##k(int kind, const void* insts, const BatchItem* items,     \
                                 int nitems, int64_t max_steps, BatchCtl* ctl,             \
                                 uint32_t spin_limit, int grid, hipStream_t st);          \
    hipError_t launch_batch_step_s##k(int kind, const void* insts, const BatchItem* items, \
                                      int nitems, int64_t s, hipStream_t st);             \
    hipError_t launch_init_s##k(const void* inst, const double* rA, const double* rB,     \
                                const double* ux, const double* uy, int random,           \
                                uint64_t seed, double mA, double mB, double amp,          \
                                hipStream_t st);
SCLBM_DECLARE_STORAGE_UNIT(0)
SCLBM_DECLARE_STORAGE_UNIT(1)
SCLBM_DECLARE_STORAGE_UNIT(2)
SCLBM_DECLARE_STORAGE_UNIT(3)

}  // namespace sclbm
