/*
 * sclbm.h -- C ABI of the MI355X (gfx950) two-species multi-range Shan-Chen
 * lattice Boltzmann library (libsclbm.so).
 *
 * Method: Benzi, Chibbaro & Succi, "Mesoscopic lattice Boltzmann modeling of
 * flowing soft systems" (arXiv:0807.4471).  One time step is the lattice
 * kinetic equation, Eq. (1): free streaming plus BGK relaxation towards the
 * local equilibrium with time scale tau_s, plus the pseudo-potential body
 * force of the FORCE equations: like-species attraction G^a_s on the first
 * belt (D2Q9 weights w_i), like-species repulsion G^r_s on both belts (24
 * neighbours, weights p_1i and p_2i, 8th-order isotropic) and cross-species
 * repulsion G_AB on the first belt, built from Psi_s[rho] = A(1-exp(-rho/rho0))
 * and from the densities.  The force enters through the Shan-Chen shift of
 * the equilibrium velocity or, per instance, through Guo's source term
 * (sclbm_desc.forcing).
 *
 * Conventions
 *   - Every function returns an int32_t status (sclbm_status); nothing aborts
 *     or throws.  Detail for the last failure on the calling thread is in
 *     sclbm_last_error().  Invalid arguments are reported before any launch.
 *   - "device pointer" arguments are HIP device addresses on the current
 *     device; "host pointer" arguments are ordinary host memory.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  Functions marked
 *     "async" only enqueue work on that stream; functions marked "syncs"
 *     return after the stream has drained.
 *   - The library never allocates or frees device memory.  The caller owns
 *     every device buffer and must keep it alive while a handle refers to it.
 *     The library owns only the small opaque host handles.
 *   - Scalar fields exchanged with the caller are FP64, ny*nx, row-major,
 *     x fastest: element (x, y) at index y*nx + x.
 *   - Time t is the number of completed steps.  Moments are those of the
 *     post-streaming populations f_is(r, t) of Eq. (1).
 *   - One handle must not be used from two host threads at once; different
 *     handles may share a stream.
 */
#ifndef SCLBM_H
#define SCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCLBM_ABI_VERSION 2

typedef enum {
    SCLBM_OK = 0,
    SCLBM_EINVAL = -1,        /* invalid argument or descriptor             */
    SCLBM_ESIZE = -2,         /* buffer too small / size out of range        */
    SCLBM_EDEVICE = -3,       /* a HIP call failed (detail in last_error)    */
    SCLBM_ENONFINITE = -4,    /* diagnostics found a non-finite or
                                 non-positive density                        */
    SCLBM_EUNSUPPORTED = -5,  /* valid request the library does not support  */
    SCLBM_ESTATE = -6         /* handle not initialised / wrong state        */
} sclbm_status;

enum { SCLBM_PERIODIC = 0, SCLBM_WALLS_Y = 1 };
enum { SCLBM_F64 = 0, SCLBM_F32 = 1, SCLBM_F16DEV = 2, SCLBM_F16DEV_SR = 3 };
enum { SCLBM_FORCING_SHIFT = 0, SCLBM_FORCING_GUO = 1 };

/* Lattice, couplings, relaxation times and pseudo-potential of one instance.
 * Copied at bind; the caller may free it afterwards. */
typedef struct {
    int32_t nx, ny;        /* lattice size: 1 <= nx, ny <= 65536 (ny >= 2 with walls);
                              the 9 population planes of a species must span
                              < 2 GiB (about 59M sites in FP32, 30M in FP64,
                              119M in FP16), else SCLBM_EUNSUPPORTED           */
    int32_t boundary;      /* SCLBM_PERIODIC, or SCLBM_WALLS_Y: periodic in x,
                              half-way bounce-back walls at y = -1/2, ny - 1/2      */
    int32_t storage;       /* SCLBM_F64: FP64 populations, FP64 arithmetic;
                              SCLBM_F32: FP32 populations, FP32 arithmetic;
                              SCLBM_F16DEV: binary16 deviations f - w_i rho_ref_s,
                              FP32 arithmetic, the rest population rounded
                              stochastically, the others to nearest;
                              SCLBM_F16DEV_SR: the same with every population
                              rounded stochastically (no rounding bias where
                              populations are nearly steady, e.g. at sheared
                              walls; slower on DRAM-resident lattices)          */
    double tau[2];         /* BGK relaxation times tau_A, tau_B of Eq. (1), > 1/2  */
    double G_a[2];         /* bare like-species attraction G^a_s (first belt)      */
    double G_r[2];         /* bare like-species repulsion G^r_s (both belts)       */
    double G_x;            /* cross-species coupling G_AB (first belt, on rho)     */
    double rho0;           /* reference density of Psi, > 0                       */
    double psi_amp;        /* amplitude A of Psi = A (1 - exp(-rho / rho0)), > 0   */
    double rho_ref[2];     /* SCLBM_F16DEV(_SR) only: reference densities of the
                              deviation storage (ignored otherwise)               */
    double wall_u[2];      /* SCLBM_WALLS_Y only: x-velocity of bottom, top wall    */
    double body_F0;        /* Kolmogorov body force: species s feels
                              g_s,x = rho_s * body_F0 * sin(2 pi y / ny); 0 = off */
    int32_t diag_every;    /* K > 0: fused FP64 diagnostics at every step t with
                              t % K == 0 (read with sclbm_fused_diagnostics);
                              0: off                                               */
    int32_t forcing;       /* how the force enters Eq. (1), which the paper leaves
                              open: SCLBM_FORCING_SHIFT (0): Shan-Chen shift of
                              the equilibrium velocity, u_eq,s = u' + tau_s F_s /
                              rho_s with u' = sum_s(j_s/tau_s) / sum_s(rho_s/tau_s);
                              SCLBM_FORCING_GUO (1): both species relax towards
                              f^eq(rho_s, u), u = sum_s(j_s + F_s/2) / sum_s rho_s,
                              and gain Guo's source (1 - 1/(2 tau_s)) w_i
                              [3 (c_i - u).F_s + 9 (c_i.u)(c_i.F_s)] (momentum
                              exactly conserved for equal tau_s)                 */
} sclbm_desc;

/* FP64 totals over the lattice at time `step`. */
typedef struct {
    double mass[2];        /* sum_r rho_s                                          */
    double mom[2];         /* sum_r (sum_s j_s + F_s / 2), x and y                 */
    double sxy;            /* sum_r of the deviatoric shear stress
                              sigma_xy = -sum_s (1 - 1/(2 tau_s))
                                          sum_i c_ix c_iy (f_is - f^eq_i(rho_s, u)) */
    double wall_mom[2][2]; /* [wall: 0 bottom, 1 top][x, y] momentum received by
                              the walls, summed over wall_steps steps             */
    int64_t wall_steps;    /* steps accumulated in wall_mom since the last reset  */
    int64_t step;          /* time t of the totals                                 */
    int64_t bad_sites;     /* sites with a non-finite or non-positive density      */
    double u_bar;          /* (2 / (nx ny)) sum_r u_x sin(2 pi y / ny): amplitude
                              of the physical x-velocity on the Kolmogorov
                              forcing mode; the response of the rheology
                              experiment is R = u_bar / U0                         */
    double i_ab;           /* interface indicator sum_r grad rho_A . grad rho_B,
                              gradients 3 sum_i w_i c_i rho(r + c_i) (neighbours
                              wrapped, or mirrored at walls)                      */
} sclbm_diag;

/* Tile shape of the fused step.
 * stacked = 0 (sweep): a workgroup of 64*waves lanes (waves in {1, 2, 4})
 *   owns a strip of tile_x columns (lane <-> column, 2 halo columns each
 *   side, so tile_x <= 64*waves - 4) and sweeps it upward over a chunk of
 *   tile_y >= min(4, ny) rows, one row per iteration.
 * stacked = 1 (tile, for small lattices): waves in {4, 8} stacked along y,
 *   one row each; tile_y == waves, tile_x <= 60.
 * throttle = 1 makes each sweep iteration wait until the previous row's
 *   stores have completed before it stages the next row (fewer memory
 *   requests in flight, which suits DRAM-resident lattices); 0 lets stores
 *   overlap the following rows.
 * write_through = 1 (stacked tiles only) writes the populations through the
 *   L2 (system-coherent stores) instead of leaving them dirty there until
 *   the end of the step: faster when the state stays in the Infinity Cache
 *   (small lattices), slower when it streams from HBM.  0 otherwise.
 * Always tile_x >= min(32, nx).  The result of a step does not depend on
 * the tiling (bit for bit). */
typedef struct {
    int32_t tile_x, tile_y, waves, stacked;
    int32_t throttle, write_through;
} sclbm_tiling;

typedef struct sclbm_inst sclbm_inst;     /* opaque host handle: one lattice  */
typedef struct sclbm_batch sclbm_batch;   /* opaque host handle: a batch plan */

/* Version of this ABI (SCLBM_ABI_VERSION of the compiled library). */
int32_t sclbm_abi_version(void);

/* Host-only self-check of the lattice index helpers the kernels use (row
 * folding for periodic and wall boundaries): 0 if consistent.  No device
 * work; usable without a GPU. */
int32_t sclbm_selftest(void);

/* Static description of a status code.  Never NULL. */
const char* sclbm_strerror(int32_t status);

/* Detail of the last failure on the calling thread ("" if none).  The string
 * is owned by the library and valid until the next call on that thread. */
const char* sclbm_last_error(void);

/* Device bytes the state of one instance needs (two population copies,
 * ghost rows, diagnostics partials, wall accumulators), or 0 if *desc is
 * invalid.  Layout and alignment are internal. */
size_t sclbm_state_bytes(const sclbm_desc* desc);

/* Create a handle for an instance whose state lives in the caller's device
 * buffer dev_buf (>= sclbm_state_bytes(desc) bytes, 256-byte aligned).  The
 * handle is uninitialised (time undefined) until sclbm_init_*.  No device
 * work is done.  Errors: EINVAL (bad desc / NULL), ESIZE (bytes too small). */
int32_t sclbm_bind(const sclbm_desc* desc, void* dev_buf, size_t bytes, sclbm_inst** out);

/* Initial state t = 0 with f_is = f^eq_i(rho_s, 0): rho_s(r) =
 * mean[s] * (1 + amp * U), U in [-1, 1) from the SplitMix64 output number
 * s*nx*ny + y*nx + x of the stream seeded with `seed` (counter-based; the
 * same recipe as the Python input generator).  Async.  Also clears the
 * diagnostics and wall accumulators. */
int32_t sclbm_init_random(sclbm_inst* inst, uint64_t seed, const double mean[2], double amp,
                          void* hip_stream);

/* Initial state t = 0 with f_is = f^eq_i(rho_s, u) from caller fields:
 * rhoA, rhoB, ux, uy are device pointers to ny*nx FP64 arrays (ux, uy may be
 * NULL for zero velocity).  Async: the caller keeps them alive until the
 * stream has passed this call. */
int32_t sclbm_init_fields(sclbm_inst* inst, const double* rhoA, const double* rhoB,
                          const double* ux, const double* uy, void* hip_stream);

/* Advance n >= 0 time steps of Eq. (1): one fused stream + moments + Psi +
 * forces + velocity shift (or Guo source) + BGK pass per step.  Async. */
int32_t sclbm_step(sclbm_inst* inst, int64_t n, void* hip_stream);

/* Choose the tiling of sclbm_step for this instance (the library starts
 * from a size-based default; the Python autotuner measures and sets it).
 * No device work.  Errors: EINVAL if the tiling violates the limits above. */
int32_t sclbm_set_tiling(sclbm_inst* inst, const sclbm_tiling* tiling);

/* Current tiling of sclbm_step for this instance. */
int32_t sclbm_get_tiling(const sclbm_inst* inst, sclbm_tiling* out);

/* Time t of the instance (host-side counter; no device work). */
int32_t sclbm_time(const sclbm_inst* inst, int64_t* t);

/* Moments at the current time into caller device arrays (ny*nx FP64 each,
 * any may be NULL): densities rho_A, rho_B; physical velocity
 * u = (sum_s j_s + F_s/2) / sum_s rho_s; deviatoric shear stress sigma_xy.
 * Async. */
int32_t sclbm_read_moments(sclbm_inst* inst, double* rhoA, double* rhoB, double* ux,
                           double* uy, double* sxy, void* hip_stream);

/* Order parameter phi = rho_A - rho_B of the state at time t, for the ageing
 * overlap of the paper's Eq. (CORRE): C(t_w, tau) = <sum_r phi(r, t_w)
 * phi(r, t_w + tau)> / <sum_r phi(r, t_w)^2>, brackets an ensemble average.
 * phi_out: device array [ny][nx] (row-major, FP64) that receives phi, or
 * NULL; phi_ref: device array [ny][nx] of a reference phi (e.g. taken at
 * t_w), or NULL.  out[0] = sum_r phi(r) phi_ref(r) (0 without phi_ref),
 * out[1] = sum_r phi(r)^2, both FP64 in a fixed order.  phi_ref and
 * phi_out may not alias.  Syncs hip_stream. */
int32_t sclbm_order_parameter(sclbm_inst* inst, const double* phi_ref, double* phi_out,
                              double out[2], void* hip_stream);

/* FP64 totals of the current state into *out (host).  Runs one read-only
 * pass, then syncs.  Returns ENONFINITE (with *out filled) if any density is
 * non-finite or non-positive. */
int32_t sclbm_diagnostics(sclbm_inst* inst, sclbm_diag* out, void* hip_stream);

/* The most recent fused diagnostics (desc.diag_every > 0) into *out (host);
 * out->step tells which time they describe (-1 if none yet).  Syncs.
 * Returns ENONFINITE as sclbm_diagnostics does. */
int32_t sclbm_fused_diagnostics(sclbm_inst* inst, sclbm_diag* out, void* hip_stream);

/* Zero the wall-momentum accumulators (async). */
int32_t sclbm_reset_wall_accum(sclbm_inst* inst, void* hip_stream);

/* Bytes of a checkpoint of this instance. */
size_t sclbm_checkpoint_bytes(const sclbm_inst* inst);

/* Copy the state at the current time (raw storage, plus time) into the host
 * buffer host_buf (>= sclbm_checkpoint_bytes).  Syncs. */
int32_t sclbm_checkpoint(sclbm_inst* inst, void* host_buf, size_t bytes, void* hip_stream);

/* Load a checkpoint written by sclbm_checkpoint of an instance with the same
 * nx, ny, boundary and storage.  Syncs.  Errors: EINVAL (mismatch). */
int32_t sclbm_restore(sclbm_inst* inst, const void* host_buf, size_t bytes, void* hip_stream);

/* Free the handle (never the caller's device buffer).  NULL is a no-op. */
int32_t sclbm_release(sclbm_inst* inst);

/* ---------------- batching: many instances advanced together ------------ */

/* Device bytes the plan of `n` instances with the given tilings needs
 * (per-instance parameter table, tile table, grid-barrier state), 0 if the
 * arguments are invalid (reason in sclbm_last_error). */
size_t sclbm_batch_bytes(sclbm_inst* const* insts, int32_t n, const sclbm_tiling* tiling);

/* Build a batch over n >= 1 initialised instances, all with the same
 * storage and diag_every == 0, any sizes and boundaries.  tiling[k] applies
 * to insts[k] and must have waves == 4: a sweep strip (stacked = 0,
 * tile_x <= 252) or a stacked tile (stacked = 1, tile_x <= 60, tile_y = 4).
 * The tile table goes into the caller's device workspace (>=
 * sclbm_batch_bytes, 256-byte aligned), which must stay alive, unchanged,
 * until sclbm_batch_release.  Syncs hip_stream once (table upload).  The
 * instance handles must outlive the batch. */
int32_t sclbm_batch_plan(sclbm_inst* const* insts, int32_t n, const sclbm_tiling* tiling,
                         void* dev_workspace, size_t bytes, void* hip_stream,
                         sclbm_batch** out);

/* Advance instance k of the batch by steps[k] >= 0 steps: in PERSISTENT mode
 * in ONE cooperative launch (all workgroups co-resident, a grid barrier
 * after each step), in STEPWISE mode in max_k steps[k] ordinary launches;
 * instances with fewer steps drop out early.  Per site the arithmetic is
 * that of sclbm_step, so each instance's result is bitwise equal to running
 * it alone.  Async; the instances' times advance.  A failed barrier (never
 * expected) is reported by sclbm_batch_status. */
int32_t sclbm_batch_step(sclbm_batch* batch, const int64_t* steps, void* hip_stream);

/* Syncs hip_stream; EDEVICE if a grid barrier of the last launch timed out
 * (results of that launch are then invalid), else OK. */
int32_t sclbm_batch_status(sclbm_batch* batch, void* hip_stream);

/* Execution mode of a batch (sclbm_batch_set_mode).
 * PERSISTENT (default): each sclbm_batch_step is ONE cooperative launch whose
 *   co-resident workgroups walk the tile table step after step, meeting at a
 *   grid barrier after every step.
 * STEPWISE: each sclbm_batch_step enqueues one ordinary launch per step,
 *   one workgroup per tile of every instance that still has steps; the
 *   kernel boundaries order the steps (no grid barrier, full occupancy).
 * Both give every instance the bits of running it alone. */
enum { SCLBM_BATCH_PERSISTENT = 0, SCLBM_BATCH_STEPWISE = 1 };

/* Select the execution mode of later sclbm_batch_step calls.  Host only;
 * EINVAL for an unknown mode. */
int32_t sclbm_batch_set_mode(sclbm_batch* batch, int32_t mode);

/* Bound the wait at each grid barrier of later PERSISTENT launches: a
 * workgroup that has slept `sleeps` times (each ~60 ns plus one coherent
 * poll) without seeing the barrier complete marks the launch failed and
 * leaves the kernel, and every other workgroup leaves at its current or
 * next barrier; sclbm_batch_status then returns EDEVICE and the launch's
 * results are invalid.  0 restores the default (2^26 sleeps, seconds: far
 * beyond any real wait).  Small values exist to test the failure path
 * without a fault or a hang.  Host only; EINVAL for a NULL batch. */
int32_t sclbm_batch_set_barrier_limit(sclbm_batch* batch, uint32_t sleeps);

/* Launch shape of a planned batch: out[0] = workgroups of this kernel kind
 * that are co-resident on the device (occupancy x compute units), out[1] =
 * tiles per step, out[2] = kernel kind (0: all stacked tiles, 1: all sweep
 * strips, 2: both).  The persistent grid is min(out[0], out[1]) workgroups.
 * Tile-shape tuners size their tiles from out[0].  Host only. */
int32_t sclbm_batch_info(const sclbm_batch* batch, int32_t out[3]);

/* Free the batch handle (not the workspace or the instances). */
int32_t sclbm_batch_release(sclbm_batch* batch);

/* Bytes of the static device array behind sclbm_batch_step_static. */
#define SCLBM_STATIC_SCRATCH_BYTES (4u << 20)

/* For callers that cannot allocate device memory (tight serving loops,
 * hosts that forbid hipMalloc): plan and run
 * a batch in one call, as sclbm_batch_plan + sclbm_batch_step in STEPWISE
 * mode would, with the batch tables (per-instance parameters and tile
 * table) in a static device array of SCLBM_STATIC_SCRATCH_BYTES instead of
 * a caller workspace.  The library holds that array on every GPU it runs
 * this call on until the process ends; its address on the current device is
 * looked up once per device.  Arguments as for sclbm_batch_plan (insts,
 * n >= 1, tiling) and sclbm_batch_step (steps[k] >= 0).  ESIZE, before any
 * device work, if the tables exceed SCLBM_STATIC_SCRATCH_BYTES (each
 * instance takes a parameter record of a few hundred bytes, each tile 8
 * bytes: e.g. 64 instances of up to 500 000 tiles in all).
 * Calls no allocation routine: the tables are built in a static host array,
 * copied by one upload, and hip_stream (which must belong to the current
 * device) is synced once after that upload; the step launches are then
 * enqueued asynchronously.  Because of that one sync the call cannot itself
 * be recorded into a HIP graph.  Every call on a GPU shares that GPU's array and
 * overwrites it, so calls whose work overlaps on one GPU (other streams,
 * other host threads) race; host calls are serialised by a lock.  Results
 * are bitwise those of sclbm_batch_step. */
int32_t sclbm_batch_step_static(sclbm_inst* const* insts, int32_t n, const sclbm_tiling* tiling,
                                const int64_t* steps, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
