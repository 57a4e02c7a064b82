// sclbm_kernels.hip -- gfx950 kernels of the two-species multi-range
// Shan-Chen lattice Boltzmann step (Benzi, Chibbaro & Succi, arXiv:0807.4471).
//
// One fused, HBM-bound pass per time step (Eq. (1) plus the FORCE equations):
//   pull-stream f_i(x,t) = f*_i(x - c_i, t-1) -> moments rho_s, j_s ->
//   Psi_s = A (1 - exp(-rho_s/rho0)) -> Psi/rho halo in LDS -> forces
//   (24-neighbour like-species stencil, 8-neighbour cross term) ->
//   Shan-Chen velocity shift -> BGK -> store f*(t).  Per instance, Guo's
//   forcing can replace the shift: BGK towards the equilibrium at the
//   barycentric velocity (half the force included), plus Guo's source term.
//
// Work decomposition.  A workgroup of 64*CW lanes owns a strip of W <=
// 64*CW - 4 columns (lane <-> column, two halo columns on each side) and
// sweeps it upward over a chunk of H rows.  Each sweep iteration pulls ONE
// new row (18 coalesced loads per lane), writes that row's (Psi_A, Psi_B)
// and (rho_A, rho_B) into a 6-row LDS ring, and finishes the row two below:
// its forces read the 5x5 Psi neighbourhood and the 3x3 rho neighbourhood
// from LDS, its populations were pulled two iterations earlier and kept in
// registers.  So every population is read from HBM once per sweep (plus 4
// halo rows per chunk and 4 halo columns per strip, served by L2/MALL) and
// written once.  One barrier per row; the 6-slot ring makes a single
// barrier sufficient (the slot a lane writes in iteration y+1 is not read in
// iteration y).
//
// Tiles are numbered row-major (all strips of one chunk row, then the next
// chunk row), and since workgroups are dispatched round-robin over the 8
// XCDs, blocks are remapped so that each XCD gets a contiguous range of
// tiles: horizontally adjacent strips, whose edges share cache lines, and
// most vertically adjacent chunks, which share halo rows, run under one L2.
// (Strip-major numbering fetched ~12% more than the algorithmic bytes on
// DRAM-resident lattices and was 5-16% slower.)
//
// Other kernels in this file: stacked tiles for small lattices (RW waves
// along y, one row each, same per-site code); the batch kernels (many
// instances per launch: one persistent cooperative launch with a grid
// barrier per step, or one ordinary launch per step); read-out passes of
// the sweep (moments, FP64 diagnostics, the order parameter); the fixed-order
// reduction of per-block FP64 partials; the initialiser.
#include <algorithm>
#include <type_traits>

#include "sclbm_internal.h"

namespace sclbm {

// Storage traits: population type S in HBM, arithmetic type A; DEV: S holds
// deviations from w_i rho_ref; SR: every population (not only the rest one)
// is rounded to binary16 stochastically.
struct TF64 {
    using S = double;
    using A = double;
    using A2 = double2;
    static constexpr bool DEV = false, SR = false;
};
struct TF32 {
    using S = float;
    using A = float;
    using A2 = float2;
    static constexpr bool DEV = false, SR = false;
};
struct TF16 {
    using S = _Float16;
    using A = float;
    using A2 = float2;
    static constexpr bool DEV = true, SR = false;
};
struct TF16SR {
    using S = _Float16;
    using A = float;
    using A2 = float2;
    static constexpr bool DEV = true, SR = true;
};

// D2Q9: i = 0 rest, 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1),
// 7 (-1,-1), 8 (1,-1); weights 4/9, 1/9, 1/36.
#define W0 (4.0 / 9.0)
#define W1 (1.0 / 9.0)
#define W2 (1.0 / 36.0)
constexpr int CX_[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY_[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP_[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Key of the FP16 stochastic rounding in the step that starts at time t: a
// fixed function of t (SplitMix64 output function), so results are
// reproducible and independent of how steps are launched or batched.
__device__ __forceinline__ uint32_t step_seed(int64_t t)
{
    uint64_t z = (uint64_t)t * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)(z ^ (z >> 31));
}

// 32-bit integer finaliser "lowbias32" (C. Wellons, hash-prospector): the
// random bits of the stochastic rounding, keyed by step seed, site, species.
__device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Populations are loaded and stored through one raw buffer resource per
// species (its 9 planes, < 2^31 bytes) with a 32-bit per-lane byte offset:
// column (per lane) + row and plane (uniform).  A lane that owns no site
// stores with offset DROP + uniform part >= 2^31, outside the resource, and
// the hardware range check discards the write; so every lane executes the
// store instruction (no divergent branch) and nothing is written for it.
constexpr uint32_t DROP = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t species_rsrc(const char* base, int nrec)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, nrec, 0x00020000);
}

// Cache-policy bits of buffer loads and stores (gfx950: 1 sc0, 2 nt, 16 sc1).
// Population stores either stay in L2 until the end of the kernel (0) or
// write through it with system coherence (CPOL_WT).
constexpr int CPOL_WT = 16;

// voff: the per-lane part of the byte offset (a column); soff: the part
// that is uniform across the wave (row and plane), passed in a scalar
// register so that no per-load vector add is needed.  A lane whose voff is
// DROP is out of range whatever soff is (both are < 2^31).
template <class S>
__device__ __forceinline__ S bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(S) == 8)
        return __builtin_bit_cast(
            S, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else if constexpr (sizeof(S) == 4)
        return __builtin_bit_cast(
            S, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else
        return __builtin_bit_cast(
            S, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}

template <class S, int CP = 0>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                       S v)
{
    if constexpr (sizeof(S) == 8) {
        typedef unsigned u2 __attribute__((__vector_size__(2 * sizeof(unsigned))));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff,
                                              CP);
    } else if constexpr (sizeof(S) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff,
                                              CP);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff,
                                              CP);
    }
}

template <class T>
__device__ __forceinline__ typename T::A rcp(typename T::A v)
{
    if constexpr (std::is_same<typename T::A, double>::value)
        return 1.0 / v;
    else
        return __builtin_amdgcn_rcpf(v);
}

// exp of the pseudo-potential: ocml exp in FP64; in FP32 the hardware
// base-2 exponential (v_exp_f32) of v log2(e), whose error (about one ulp
// for the arguments here, -rho/rho0 in [-10, 0]) is far below the FP32
// storage rounding of a step.
template <class T>
__device__ __forceinline__ typename T::A expo(typename T::A v)
{
    if constexpr (std::is_same<typename T::A, double>::value)
        return exp(v);
    else
        return __builtin_amdgcn_exp2f(v * 1.4426950408889634f);
}

// Register representation of the populations.  FP64 / FP32 storage: v_i =
// f_i.  FP16 deviation storage: v_i = h_i = f_i - w_i rho_ref (the deviation
// from the exact reference populations), and all arithmetic stays in that
// form: rho = rho_ref + sum_i h_i, j = sum_i c_i h_i (the reference carries
// no momentum), f^eq_i - w_i rho_ref = w_i ((rho - rho_ref) + rho P_i).  Sums
// of binary16 values are exact in FP32, so the mass bookkeeping is exact.
template <class T, int CW, bool WALLS, int MODE, int NS = 6, int SCP = 0>
struct Sweep {
    using S = typename T::S;
    using A = typename T::A;
    using A2 = typename T::A2;
    static constexpr bool DEV = T::DEV;
    // Rows are prefetched one iteration ahead (loads in flight while the
    // previous row is finished) except in FP64, where three resident rows of
    // doubles leave no registers for a fourth.
    static constexpr bool PF = !std::is_same<A, double>::value;
    // The uniform (row and plane) part of population offsets goes in the
    // buffer instructions' scalar offset for FP64 and FP32 storage, which
    // saves a vector add per access; FP16 keeps the whole offset per lane,
    // which measured faster for its 2-byte accesses.
    static constexpr bool SOFF = !DEV;
    static constexpr int NC = 64 * CW;

    const Inst<S, A>& I;
    A2 (*lpsi)[NC];
    A2 (*lrho)[NC];
    double* acc;
    int t, nx, ny, xw, xm, xp;
    bool own;
    uint32_t cw, cm, cp;  // column byte offsets of x, x-1, x+1
    const char* finb;
    char* foutb;
    int64_t plane_b, pitch_b;
    __amdgpu_buffer_rsrc_t rin[2], rout[2];  // per-species resources
    uint32_t sw_, sm_, sp_;                  // store column offsets, DROP if not own
    uint32_t seed;  // FP16 stochastic-rounding key of this step
    S R[18];  // raw loads of the next row

    __device__ Sweep(const Inst<S, A>& I_, int strip, A2 (*lp)[NC], A2 (*lr)[NC], double* acc_)
        : I(I_), lpsi(lp), lrho(lr), acc(acc_)
    {
        t = threadIdx.x & (NC - 1);
        nx = I.g.nx;
        ny = I.g.ny;
        const int x = strip * I.W - 2 + t;
        xw = x % nx;
        if (xw < 0) xw += nx;
        xm = xw == 0 ? nx - 1 : xw - 1;
        xp = xw == nx - 1 ? 0 : xw + 1;
        own = t >= 2 && t < I.W + 2 && x < nx;
        cw = (uint32_t)xw * sizeof(S);
        cm = (uint32_t)xm * sizeof(S);
        cp = (uint32_t)xp * sizeof(S);
        finb = reinterpret_cast<const char*>(I.fin);
        foutb = reinterpret_cast<char*>(I.fout);
        plane_b = I.g.plane * (int64_t)sizeof(S);
        pitch_b = (int64_t)I.g.pitch * (int64_t)sizeof(S);
        const int nrec = (int)(9 * plane_b);
        rin[0] = species_rsrc(finb, nrec);
        rin[1] = species_rsrc(finb + 9 * plane_b, nrec);
        rout[0] = species_rsrc(foutb, nrec);
        rout[1] = species_rsrc(foutb + 9 * plane_b, nrec);
        sw_ = own ? cw : DROP;
        sm_ = own ? cm : DROP;
        sp_ = own ? cp : DROP;
        seed = DEV ? step_seed(I.t) : 0u;
    }

    // Ring row r (may lie outside the lattice) -> real row in [0, ny).
    __device__ int real_row(int r) const { return fold_row(r, ny, WALLS); }

    // Issue the 18 loads f_i(x, t) = f*_i(x - c_i, t-1) of ring row r into R.
    // Plane and row parts of each address are uniform; each lane adds one of
    // three fixed 32-bit column byte offsets (x, x-1, x+1).  With walls the
    // rows just outside the channel are the ghost rows holding bounced-back
    // populations.
    __device__ void load(int r)
    {
        const int rr = real_row(r);
        int r0, rm, rp;
        if constexpr (WALLS) {
            r0 = rr + 1;
            rm = rr;
            rp = rr + 2;
        } else {
            r0 = rr;
            rm = rr == 0 ? ny - 1 : rr - 1;
            rp = rr == ny - 1 ? 0 : rr + 1;
        }
        const uint32_t o0 = (uint32_t)(r0 * pitch_b), om = (uint32_t)(rm * pitch_b),
                       op = (uint32_t)(rp * pitch_b);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint32_t ro = CY_[i] > 0 ? om : CY_[i] < 0 ? op : o0;
                const uint32_t co = CX_[i] > 0 ? cm : CX_[i] < 0 ? cp : cw;
                if constexpr (SOFF)
                    R[s * 9 + i] = bload<S>(rin[s], co, ro + (uint32_t)(i * plane_b));
                else
                    R[s * 9 + i] = bload<S>(rin[s], co + (ro + (uint32_t)(i * plane_b)), 0u);
            }
    }

    __device__ void convert(A* v) const
    {
#pragma unroll
        for (int k = 0; k < 18; ++k) v[k] = (A)R[k];
    }

    // FP64 / FP32: the loads land directly in a row buffer.
    __device__ void load_into(int r, A* v)
    {
        load(r);
        if constexpr (!DEV) {
#pragma unroll
            for (int k = 0; k < 18; ++k) v[k] = R[k];
        }
    }

    // rho_s - rho_base_s = sum_i v_i (fixed order)
    __device__ static A mass(const A* v)
    {
        return v[0] + v[1] + v[2] + v[3] + v[4] + v[5] + v[6] + v[7] + v[8];
    }

    // Stage a row: (Psi_A, Psi_B) and (rhod_A, rhod_B) into ring slot
    // `slot`, rhod = rho - rho_base (= rho except for FP16 deviations, where
    // it is the exact FP32 sum of the binary16 deviations).
    __device__ void stage(int slot, const A* v) const
    {
        const Coef<A>& c = I.c;
        const A da = mass(v), db = mass(v + 9);
        A ra = da, rb = db;
        if constexpr (DEV) {
            ra += c.rho_base[0];
            rb += c.rho_base[1];
        }
        const A pa = c.psi_amp * (A(1) - expo<T>(ra * c.neg_inv_rho0));
        const A pb = c.psi_amp * (A(1) - expo<T>(rb * c.neg_inv_rho0));
        lpsi[slot][t] = A2{pa, pb};
        lrho[slot][t] = A2{da, db};
    }

    // Relax species populations v towards equilibrium (in the register
    // representation); v[0] becomes the remainder rhod - sum_{i>0} v_i, so
    // the collision conserves mass to one rounding whatever the rounding of
    // the weights (in FP32 4/9 + 4/9 + 4/36 rounds to 1 + 7.4e-9).
    __device__ static void bgk(A* v, A rho, A rhod, A ux, A uy, A omega, bool tau1, bool guo,
                               A Fx, A Fy, A tau)
    {
        const A usq15 = A(1.5) * (ux * ux + uy * uy);
        const A w1r = A(W1) * rho, w2r = A(W2) * rho;
        const A w1d = A(W1) * rhod, w2d = A(W2) * rhod;
        const A up = ux + uy, um = ux - uy;
        // P_i = 3 cu + 4.5 cu^2 - 1.5 u^2 ;  veq_i = w_i (rhod + rho P_i)
        auto veq = [&](A wr, A wd, A cu) {
            const A P = cu * (A(3) + A(4.5) * cu) - usq15;
            return wr * P + wd;
        };
        A eq[9] = {A(0),           veq(w1r, w1d, ux), veq(w1r, w1d, uy),
                   veq(w1r, w1d, -ux), veq(w1r, w1d, -uy), veq(w2r, w2d, up),
                   veq(w2r, w2d, -um), veq(w2r, w2d, -up), veq(w2r, w2d, um)};
        if (guo) {
            // Guo's source (1 - 1/(2 tau)) w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)]
            // enters as (tau - 1/2) w_i [...] added to the equilibrium, since
            // omega (tau - 1/2) = 1 - 1/(2 tau).  It carries no mass.
            const A g3 = A(3) * (tau - A(0.5));
            const A uf = ux * Fx + uy * Fy;
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const A cu = A(CX_[i]) * ux + A(CY_[i]) * uy;
                const A cf = A(CX_[i]) * Fx + A(CY_[i]) * Fy;
                eq[i] += (i < 5 ? A(W1) : A(W2)) * g3 * ((cf - uf) + A(3) * cu * cf);
            }
        }
        if (tau1) {
#pragma unroll
            for (int i = 1; i < 9; ++i) v[i] = eq[i];
        } else {
#pragma unroll
            for (int i = 1; i < 9; ++i) v[i] = v[i] + omega * (eq[i] - v[i]);
        }
        v[0] = rhod - (((v[1] + v[2]) + (v[3] + v[4])) + ((v[5] + v[6]) + (v[7] + v[8])));
    }

    // Finish row y: forces from the LDS ring (slot sb holds row y-2), then
    // collision + store (step), moment read-out or diagnostics.  Every lane
    // runs it: lanes owning no site (halo lanes, columns beyond nx) read a
    // clamped LDS column and their stores are dropped by the buffer range
    // check, so the stores are not under a divergent branch and the
    // compiler's wait counts stay exact (otherwise the next row's loads
    // would also wait for these stores).
    __device__ void finish(int y, int sb, A* v)
    {
        const Coef<A>& c = I.c;
        const int tc = own ? t : 2;
        int sl[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) sl[k] = sb + k >= NS ? sb + k - NS : sb + k;
        auto Ps = [&](int dx, int dy) { return lpsi[sl[dy + 2]][tc + dx]; };
        auto Rs = [&](int dx, int dy) { return lrho[sl[dy + 2]][tc + dx]; };
        auto dif = [](A2 a, A2 b) { return A2{a.x - b.x, a.y - b.y}; };
        // Psi differences over the 12 opposite pairs (both species)
        const A2 a10 = dif(Ps(1, 0), Ps(-1, 0)), a01 = dif(Ps(0, 1), Ps(0, -1));
        const A2 a11 = dif(Ps(1, 1), Ps(-1, -1)), b11 = dif(Ps(-1, 1), Ps(1, -1));
        const A2 a20 = dif(Ps(2, 0), Ps(-2, 0)), a02 = dif(Ps(0, 2), Ps(0, -2));
        const A2 a21 = dif(Ps(2, 1), Ps(-2, -1)), a12 = dif(Ps(1, 2), Ps(-1, -2));
        const A2 b12 = dif(Ps(-1, 2), Ps(1, -2)), b21 = dif(Ps(-2, 1), Ps(2, -1));
        const A2 a22 = dif(Ps(2, 2), Ps(-2, -2)), b22 = dif(Ps(-2, 2), Ps(2, -2));
        // rho differences over the 4 first-belt pairs (cross force)
        const A2 r10 = dif(Rs(1, 0), Rs(-1, 0)), r01 = dif(Rs(0, 1), Rs(0, -1));
        const A2 r11 = dif(Rs(1, 1), Rs(-1, -1)), q11 = dif(Rs(-1, 1), Rs(1, -1));
        const A2 pc = Ps(0, 0);
        const A2 rc = Rs(0, 0);  // rhod of this row, staged two rows ago
        const A rhod[2] = {rc.x, rc.y};
        A rho[2] = {rc.x, rc.y};
        if constexpr (DEV) {
            rho[0] += c.rho_base[0];
            rho[1] += c.rho_base[1];
        }
        if constexpr (MODE == M_PHI) {  // order parameter (ageing overlap)
            if (own) {
                const int64_t n = (int64_t)y * nx + xw;
                const double ph = (double)rho[0] - (double)rho[1];
                if (I.out[0]) I.out[0][n] = ph;
                if (I.out[1]) acc[0] += ph * I.out[1][n];
                acc[1] += ph * ph;
            }
            return;
        }
        A F[2][2];
        auto force = [&](int s, A d10, A d01, A d11, A e11, A d20, A d02, A d21, A d12, A e12,
                         A e21, A d22, A e22, A psi, A rho, A o10, A o01, A o11, A p11) {
            const A Sx = c.K1[s] * d10 + c.K2[s] * (d11 - e11) + c.K4x2[s] * d20 +
                         c.K5[s] * (A(2) * d21 + d12 - e12 - A(2) * e21) + c.K8x2[s] * (d22 - e22);
            const A Sy = c.K1[s] * d01 + c.K2[s] * (d11 + e11) + c.K4x2[s] * d02 +
                         c.K5[s] * (d21 + A(2) * d12 + A(2) * e12 + e21) + c.K8x2[s] * (d22 + e22);
            const A Xx = c.X1 * o10 + c.X2 * (o11 - p11);
            const A Xy = c.X1 * o01 + c.X2 * (o11 + p11);
            F[s][0] = -psi * Sx - rho * Xx;
            F[s][1] = -psi * Sy - rho * Xy;
        };
        force(0, a10.x, a01.x, a11.x, b11.x, a20.x, a02.x, a21.x, a12.x, b12.x, b21.x, a22.x,
              b22.x, pc.x, rho[0], r10.y, r01.y, r11.y, q11.y);
        force(1, a10.y, a01.y, a11.y, b11.y, a20.y, a02.y, a21.y, a12.y, b12.y, b21.y, a22.y,
              b22.y, pc.y, rho[1], r10.x, r01.x, r11.x, q11.x);
        if (c.body_F0 != 0.0) {  // uniform branch
            const A gy = (A)c.body_F0 * (A)sin((A)c.two_pi_over_ny * (A)y);
            F[0][0] += rho[0] * gy;
            F[1][0] += rho[1] * gy;
        }

        A jx[2], jy[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const A* f = v + 9 * s;
            jx[s] = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
            jy[s] = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
        }

        if constexpr (MODE == M_STEP_DIAG || MODE == M_DIAG || MODE == M_READ) {
            const A rt = rho[0] + rho[1];
            const A mx = (jx[0] + A(0.5) * F[0][0]) + (jx[1] + A(0.5) * F[1][0]);
            const A my = (jy[0] + A(0.5) * F[0][1]) + (jy[1] + A(0.5) * F[1][1]);
            const A irt = rt > A(0) ? rcp<T>(rt) : A(0);
            const A vx = mx * irt, vy = my * irt;
            A sxy = A(0);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const A* f = v + 9 * s;
                sxy -= c.hs[s] * ((f[5] - f[6]) + (f[7] - f[8]) - rho[s] * vx * vy);
            }
            if constexpr (MODE == M_READ) {
                const int64_t n = (int64_t)y * nx + xw;
                if (!own) return;
                if (I.out[0]) I.out[0][n] = (double)rho[0];
                if (I.out[1]) I.out[1][n] = (double)rho[1];
                if (I.out[2]) I.out[2][n] = (double)vx;
                if (I.out[3]) I.out[3][n] = (double)vy;
                if (I.out[4]) I.out[4][n] = (double)sxy;
            } else if (own) {
                acc[D_MASS_A] += (double)rhod[0] + (double)c.rho_base[0] * DEV;
                acc[D_MASS_B] += (double)rhod[1] + (double)c.rho_base[1] * DEV;
                acc[D_MOM_X] += (double)mx;
                acc[D_MOM_Y] += (double)my;
                acc[D_SXY] += (double)sxy;
                const bool ok = rho[0] > A(0) && rho[1] > A(0) && rho[0] < A(1e30) &&
                                rho[1] < A(1e30);
                acc[D_BAD] += ok ? 0.0 : 1.0;
                // shear-flow observables: the forcing-mode projection of u_x,
                // and grad rho_A . grad rho_B with the isotropic D2Q9
                // gradient 3 sum_i w_i c_i rho(r + c_i) from the LDS ring
                // (rhod differs from rho by a constant)
                acc[D_UPROJ] += (double)vx * sin(c.two_pi_over_ny * (double)y);
                const A gxa = A(3) * (A(W1) * r10.x + A(W2) * (r11.x - q11.x));
                const A gya = A(3) * (A(W1) * r01.x + A(W2) * (r11.x + q11.x));
                const A gxb = A(3) * (A(W1) * r10.y + A(W2) * (r11.y - q11.y));
                const A gyb = A(3) * (A(W1) * r01.y + A(W2) * (r11.y + q11.y));
                acc[D_IAB] += (double)gxa * (double)gxb + (double)gya * (double)gyb;
            }
        }

        if constexpr (MODE == M_STEP || MODE == M_STEP_DIAG) {
            // Shan-Chen velocity shift: common velocity weighted by rho_s/tau_s,
            // species shift tau_s F_s / rho_s.  Guo forcing instead: the
            // barycentric velocity with half the force for both species, and
            // a source term after the relaxation (uniform branch).
            A upx, upy;
            if (!c.guo) {
                const A den = rho[0] * c.omega[0] + rho[1] * c.omega[1];
                const A nmx = jx[0] * c.omega[0] + jx[1] * c.omega[1];
                const A nmy = jy[0] * c.omega[0] + jy[1] * c.omega[1];
                const A iden = den > A(0) ? rcp<T>(den) : A(0);
                upx = nmx * iden;
                upy = nmy * iden;
            } else {
                const A rt = rho[0] + rho[1];
                const A irt = rt > A(0) ? rcp<T>(rt) : A(0);
                upx = ((jx[0] + jx[1]) + A(0.5) * (F[0][0] + F[1][0])) * irt;
                upy = ((jy[0] + jy[1]) + A(0.5) * (F[0][1] + F[1][1])) * irt;
            }
            const int ro = y + (WALLS ? 1 : 0);
            const uint32_t soff = (uint32_t)(ro * pitch_b);  // uniform row offsets
            // Wall rows: a population that would leave the channel returns to
            // its node reversed, minus 2 w_i rho (c_i.u_w)/c_s^2 (half-way
            // bounce-back), written to the ghost row where the next pull of
            // the reversed direction looks for it.  The outgoing value itself
            // is never read and is not stored.
            const bool bot = WALLS && y == 0, top = WALLS && y == ny - 1;  // uniform
            const A u6 = WALLS ? c.wall6u[top ? 1 : 0] : A(0);
            const uint32_t goff = (uint32_t)((top ? ny + 1 : 0) * pitch_b);
            double mxw = 0.0, myw = 0.0;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                A* f = v + 9 * s;
                A uex = upx, uey = upy;
                if (!c.guo) {
                    const A ir = rho[s] > A(0) ? c.tau[s] * rcp<T>(rho[s]) : A(0);
                    uex += F[s][0] * ir;
                    uey += F[s][1] * ir;
                }
                bgk(f, rho[s], rhod[s], uex, uey, c.omega[s], c.tau1[s] != 0, c.guo != 0,
                    F[s][0], F[s][1], c.tau[s]);
                const A corr = A(W2) * rho[s] * u6;  // diagonal Ladd term; axis term is 0
                [[maybe_unused]] A qsum = A(0);
                [[maybe_unused]] uint32_t rr = 0;
                if constexpr (T::SR)
                    rr = hash32(seed ^ (uint32_t)(((uint32_t)y * (uint32_t)nx + (uint32_t)xw) * 2u +
                                                  s) ^ 0x5bd1e995u);
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const bool out = (bot && CY_[i] < 0) || (top && CY_[i] > 0);  // uniform
                    A val = f[i];
                    int k = s * 9 + i;
                    uint32_t col = sw_, ro_off = soff;
                    if (out) {
                        val = f[i] - A(CX_[i]) * corr;
                        k = s * 9 + OPP_[i];
                        col = CX_[i] > 0 ? sp_ : CX_[i] < 0 ? sm_ : sw_;
                        ro_off = goff;
                        mxw += (double)CX_[i] * ((double)f[i] + (double)val);
                        myw += (double)CY_[i] * ((double)f[i] + (double)val);
                        if constexpr (DEV)  // the reference populations' share
                            myw += (double)CY_[i] * 2.0 * (double)c.rho_base[s] *
                                   (CX_[i] == 0 ? W1 : W2);
                    }
                    const uint32_t dsoff = ro_off + (uint32_t)((k - 9 * s) * plane_b);
                    if constexpr (DEV) {
                        _Float16 h;
                        if constexpr (T::SR) {
                            typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
                            h2_t hv = {(_Float16)0, (_Float16)0};
                            hv = __builtin_amdgcn_cvt_sr_f16_f32(hv, val, rr, false);
                            h = hv[0];
                            rr = rr * 0x9E3779B1u + 0x7F4A7C15u;  // next random word (LCG)
                        } else {
                            h = (_Float16)val;
                        }
                        bstore<_Float16, SCP>(rout[s], col + dsoff, 0u, h);
                        qsum += (float)h;  // exact: sum of binary16 values
                    } else {
                        bstore<S, SCP>(rout[s], col, dsoff, (S)val);
                    }
                }
                if constexpr (DEV) {
                    // The rest population absorbs the rounding of the other
                    // eight deviations and is itself rounded stochastically
                    // (unbiased): the site's stored mass is rho_s up to one
                    // zero-mean rounding.
                    const float h0 = rhod[s] - qsum;
                    const uint32_t r = hash32(
                        seed ^ (uint32_t)(((uint32_t)y * (uint32_t)nx + (uint32_t)xw) * 2u + s));
                    typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
                    h2_t hv = {(_Float16)0, (_Float16)0};
                    hv = __builtin_amdgcn_cvt_sr_f16_f32(hv, h0, r, false);
                    bstore<_Float16, SCP>(rout[s], sw_ + soff, 0u, hv[0]);
                } else {
                    bstore<S, SCP>(rout[s], sw_, soff, (S)f[0]);
                }
            }
            if constexpr (WALLS) {
                if ((bot || top) && own) {
                    double* wa = I.wall_acc + (top ? 2 : 0) * (int64_t)nx;
                    wa[xw] += mxw;
                    wa[nx + xw] += myw;
                }
            }
        }
    }

    // One sweep iteration: stage row y+2 (buffer PC), barrier, start the
    // loads of row y+3 (into PD, or the raw buffer R for FP16), finish row y
    // (PA).  FP64 loads row y+2 here instead (no prefetch).
    __device__ void iterate(int y, int& sb, int y1, A* PA, A* PC, A* PD)
    {
        const int snew = sb + 4 >= 6 ? sb - 2 : sb + 4;
        if constexpr (!PF) load_into(y + 2, PC);
        // optional throttle: all earlier memory operations (the previous
        // row's stores included) complete before this row is staged
        // (s_waitcnt vmcnt(0); expcnt, lgkmcnt untouched)
        if (I.throttle) __builtin_amdgcn_s_waitcnt(0x0F70);
        if constexpr (DEV) convert(PC);
        stage(snew, PC);
        __syncthreads();
        if constexpr (PF) {
            if (y + 1 < y1) {
                if constexpr (DEV)
                    load(y + 3);
                else
                    load_into(y + 3, PD);
            }
        }
        finish(y, sb, PA);
        sb = sb == 5 ? 0 : sb + 1;
    }

    __device__ void run(int chunk)
    {
        const int y0 = chunk * I.H;
        const int y1 = min(y0 + I.H, ny);
        A P0[18], P1[18], P2[18];
        // prologue: rows y0-2 .. y0+1 in slots 0..3; keep rows y0, y0+1
        auto pro = [&](int r, int slot, A* v) {
            load(r);
            convert(v);
            stage(slot, v);
        };
        pro(y0 - 2, 0, P2);
        pro(y0 - 1, 1, P2);
        pro(y0, 2, P0);
        pro(y0 + 1, 3, P1);
        int sb = 0;  // slot of row y-2
        int y = y0;
        if constexpr (PF && !DEV) {
            // four row buffers rotate (row y, y+1, y+2 resident, y+3 loading)
            A P3[18];
            load_into(y0 + 2, P2);
            for (; y + 4 <= y1; y += 4) {
                iterate(y, sb, y1, P0, P2, P3);
                iterate(y + 1, sb, y1, P1, P3, P0);
                iterate(y + 2, sb, y1, P2, P0, P1);
                iterate(y + 3, sb, y1, P3, P1, P2);
            }
            if (y < y1) iterate(y, sb, y1, P0, P2, P3);
            if (y + 1 < y1) iterate(y + 1, sb, y1, P1, P3, P0);
            if (y + 2 < y1) iterate(y + 2, sb, y1, P2, P0, P1);
        } else {
            // three row buffers (FP16: raw prefetch buffer R besides)
            if constexpr (PF) load(y0 + 2);
            for (; y + 3 <= y1; y += 3) {
                iterate(y, sb, y1, P0, P2, nullptr);
                iterate(y + 1, sb, y1, P1, P0, nullptr);
                iterate(y + 2, sb, y1, P2, P1, nullptr);
            }
            if (y < y1) iterate(y, sb, y1, P0, P2, nullptr);
            if (y + 1 < y1) iterate(y + 1, sb, y1, P1, P0, nullptr);
        }
    }
};

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8);
// give each XCD a contiguous range of logical (row-major) tiles.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int per = n / 8, rem = n % 8, xcd = b % 8, k = b / 8;
    return xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

// Debug builds (-DSCLBM_POISON_LDS=1) fill the Psi/rho ring with NaN before
// a tile stages anything, so a force that reads a ring cell its own pass
// never staged (a missed halo row or column) poisons that site and fails
// the parity tests.  Regular builds compile this away.
#ifndef SCLBM_POISON_LDS
#define SCLBM_POISON_LDS 0
#endif
template <class A2>
__device__ __forceinline__ void poison_ring(A2* psi, A2* rho, int cells)
{
    if constexpr (SCLBM_POISON_LDS) {
        using A = decltype(A2{}.x);
        const A nan = (A)__builtin_nan("");
        for (int k = threadIdx.x; k < cells; k += blockDim.x) {
            psi[k] = A2{nan, nan};
            rho[k] = A2{nan, nan};
        }
        __syncthreads();
    }
}

template <int CW>
__device__ __forceinline__ void block_reduce(double* acc, double (*red)[NDIAG], double* out)
{
#pragma unroll
    for (int j = 0; j < NDIAG; ++j) {
        double v = acc[j];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        acc[j] = v;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int j = 0; j < NDIAG; ++j) red[w][j] = acc[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < NDIAG; ++j) {
            double s = 0.0;
            for (int k = 0; k < CW; ++k) s += red[k][j];
            out[j] = s;
        }
    }
}

template <class T, int CW, bool WALLS, int MODE>
__global__ __launch_bounds__(64 * CW) void sweep_kernel(Inst<typename T::S, typename T::A> I)
{
    __shared__ typename T::A2 lpsi[6][64 * CW];
    __shared__ typename T::A2 lrho[6][64 * CW];
    __shared__ double red[CW][NDIAG];
    poison_ring(&lpsi[0][0], &lrho[0][0], 6 * 64 * CW);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = b / I.nstrips, strip = b - chunk * I.nstrips;
    double acc[NDIAG] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    Sweep<T, CW, WALLS, MODE> sw(I, strip, lpsi, lrho, acc);
    sw.run(chunk);
    if constexpr (MODE == M_STEP_DIAG || MODE == M_DIAG || MODE == M_PHI)
        block_reduce<CW>(acc, red, I.partials + (int64_t)b * NDIAG);
}

// Tile mode for lattices too small to fill the chip with sweeps: RW waves
// stacked along y, one row each.  Wave w stages its own row y0+w (and keeps
// its populations in registers); waves 0..3 also stage the four halo rows
// y0-2, y0-1, y0+RW, y0+RW+1; one barrier; every wave finishes its row.  The
// dependency chain per workgroup is one row instead of H+4 rows.
template <class T, int RW, bool WALLS, int MODE, int SCP = 0>
__device__ __forceinline__ void tile_body(const Inst<typename T::S, typename T::A>& I, int strip,
                                          int chunk, typename T::A2 (*lpsi)[64],
                                          typename T::A2 (*lrho)[64], double* acc)
{
    static_assert(RW >= 4, "four waves stage the halo rows");
    using A = typename T::A;
    Sweep<T, 1, WALLS, MODE, RW + 4, SCP> sw(I, strip, lpsi, lrho, acc);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int y0 = chunk * RW;
    A P[18];
    sw.load(y0 + w);
    sw.convert(P);
    if (w < 4) {
        A Q[18];
        const int hr = w < 2 ? y0 - 2 + w : y0 + RW + (w - 2);
        const int hs = w < 2 ? w : RW + w;
        sw.load(hr);
        sw.convert(Q);
        sw.stage(hs, Q);
    }
    sw.stage(w + 2, P);
    __syncthreads();
    if (y0 + w < sw.ny) sw.finish(y0 + w, w, P);  // wave-uniform
}

template <class T, int RW, bool WALLS, int MODE, int SCP>
__global__ __launch_bounds__(64 * RW) void tile_kernel(Inst<typename T::S, typename T::A> I)
{
    __shared__ typename T::A2 lpsi[RW + 4][64];
    __shared__ typename T::A2 lrho[RW + 4][64];
    __shared__ double red[RW][NDIAG];
    poison_ring(&lpsi[0][0], &lrho[0][0], (RW + 4) * 64);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = b / I.nstrips, strip = b - chunk * I.nstrips;
    double acc[NDIAG] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    tile_body<T, RW, WALLS, MODE, SCP>(I, strip, chunk, lpsi, lrho, acc);
    if constexpr (MODE == M_STEP_DIAG || MODE == M_DIAG)
        block_reduce<RW>(acc, red, I.partials + (int64_t)b * NDIAG);
}

#if SCLBM_STORAGE == 0
// Fixed-order FP64 reduction of per-block partials: deterministic.
__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ partials, int nb,
                                                     double* __restrict__ out)
{
    __shared__ double sh[256];
    const int t = threadIdx.x;
    for (int j = 0; j < NDIAG; ++j) {
        double s = 0.0;
        for (int b = t; b < nb; b += 256) s += partials[(int64_t)b * NDIAG + j];
        sh[t] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w) sh[t] += sh[t + w];
            __syncthreads();
        }
        if (t == 0) out[j] = sh[0];
        __syncthreads();
    }
}
#endif

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator: output
// number c of the stream seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Initial state: f_i(x, 0) = f^eq_i(rho_s, u), stored where the first pull
// looks for it, i.e. at x - c_i (ghost rows for sources outside the walls).
template <class T>
__global__ __launch_bounds__(256) void init_kernel(Inst<typename T::S, typename T::A> I,
                                                   const double* rA, const double* rB,
                                                   const double* ux, const double* uy,
                                                   int random, uint64_t seed, double mA,
                                                   double mB, double amp)
{
#pragma clang fp contract(off)
    const Geo& g = I.g;
    const int64_t N = (int64_t)g.nx * g.ny;
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % g.nx), y = (int)(n / g.nx);
    double rho[2];
    if (random) {
        for (int s = 0; s < 2; ++s) {
            const uint64_t h = splitmix64(seed, (uint64_t)s * (uint64_t)N + (uint64_t)n);
            const double U = 2.0 * ((double)(h >> 11) * 0x1.0p-53) - 1.0;
            rho[s] = (s ? mB : mA) * (1.0 + amp * U);
        }
    } else {
        rho[0] = rA[n];
        rho[1] = rB[n];
    }
    const double vx = ux ? ux[n] : 0.0, vy = uy ? uy[n] : 0.0;
    const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double w[9] = {W0, W1, W1, W1, W1, W2, W2, W2, W2};
    const double usq = vx * vx + vy * vy;
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < 9; ++i) {
            const double cu = cx[i] * vx + cy[i] * vy;
            const double feq = w[i] * rho[s] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
            int xs = x - cx[i];
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            int ys = y - cy[i];
            if (g.walls)
                ys += 1;  // ghost row 0 / ny+1 hold sources outside the channel
            else
                ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            typename T::S* dst = I.fout + (int64_t)(s * 9 + i) * g.plane + (int64_t)ys * g.pitch + xs;
            if constexpr (T::DEV)  // deviation from w_i rho_ref
                *dst = (_Float16)(float)(feq - w[i] * (double)I.c.rho_base[s]);
            else
                *dst = (typename T::S)feq;
        }
}

// ------------------------------------------------------------- batching
//
// Persistent batch: many instances (any sizes, periodic or walls, sweep or
// stacked tiling, one storage type) advance in ONE cooperative launch.  Each
// global step every workgroup walks the item table (instance, tile) with a
// grid stride and runs exactly the per-site code of the single-instance
// kernels, then all workgroups meet at a grid barrier before the next step
// (the next step reads halos written by other workgroups, and overwrites the
// copy they were reading).  Instances with fewer steps drop out early.

// Grid barrier for a cooperative (co-resident) grid.  The workgroup barrier
// orders every lane's stores before lane 0 arrives; lane 0 arrives with a
// release RMW (on gfx950 one write-back of its XCD's L2), waits with relaxed
// polls (coherent loads that do not touch the L2 state), and leaves through
// one acquire fence (one L2 invalidate); the last arriver acquires the
// others' stores before releasing the new generation.  Acquire polls or
// agent-scope fences on every lane would invalidate and write back the L2 of
// the XCD once per poll and per workgroup, which costs about 170 ns per
// workgroup per barrier (measured: 131 us at 768 workgroups, against 21 us
// this way).  The wait is bounded: after spin_limit sleeps (the host's
// choice, normally 2^26) the barrier reports failure through ctl->err, and
// every workgroup leaves the kernel at its current or next barrier.
__device__ __forceinline__ bool grid_barrier(BatchCtl* ctl, uint32_t spin_limit)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int good = 1;
        const uint32_t n = gridDim.x;
        const uint32_t g = __hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t arrived =
            __hip_atomic_fetch_add(&ctl->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == n - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > spin_limit ||
                    __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// KIND selects the tile paths compiled into the batch kernel: stacked
// 4-wave tiles only (B_STACKED), 4-wave-wide sweep strips only (B_SWEEP) or
// both (B_MIXED).  A single-path kernel needs fewer registers than the mixed
// one, so more workgroups are co-resident.  Workgroup b takes items b, b + G,
// b + 2G, ... of the (instance-major, tile-major) item table, so the
// workgroups in flight at any moment work on neighbouring tiles of few
// instances (their halo rows meet in L2, their pages in the TLB).  (Giving
// each XCD a contiguous range of the items in flight, as the single-instance
// kernels do, measured no better here.)
// One item (instance, tile) of step s of a batch launch: the instance's
// populations swap roles every step and its time advances with s.  Tiles are
// decoded strip-major, or row-major (as the single-instance kernels number
// them) if ROW.
template <class T, int KIND, bool ROW>
__device__ __forceinline__ void batch_item(const BatchInst<typename T::S, typename T::A>& bi,
                                           int tile, int64_t s, typename T::A2 (*lpsi)[256],
                                           typename T::A2 (*lrho)[256], double* acc)
{
    using S = typename T::S;
    using A = typename T::A;
    using A2 = typename T::A2;
    Inst<S, A> I = bi.I;
    if (s & 1) {
        const S* a = I.fin;
        I.fin = I.fout;
        I.fout = const_cast<S*>(a);
    }
    I.t += s;
    poison_ring(&lpsi[0][0], &lrho[0][0], (KIND == B_STACKED ? 2 : 6) * 256);
    int strip, chunk;
    if (ROW) {
        chunk = tile / I.nstrips;
        strip = tile - chunk * I.nstrips;
    } else {
        strip = tile / I.nchunks;
        chunk = tile - strip * I.nchunks;
    }
    if (KIND == B_STACKED || (KIND == B_MIXED && bi.stacked)) {
        auto lp = reinterpret_cast<A2(*)[64]>(&lpsi[0][0]);
        auto lr = reinterpret_cast<A2(*)[64]>(&lrho[0][0]);
        if (I.g.walls)
            tile_body<T, 4, true, M_STEP>(I, strip, chunk, lp, lr, acc);
        else
            tile_body<T, 4, false, M_STEP>(I, strip, chunk, lp, lr, acc);
    } else if constexpr (KIND != B_STACKED) {
        if (I.g.walls) {
            Sweep<T, 4, true, M_STEP> sw(I, strip, lpsi, lrho, acc);
            sw.run(chunk);
        } else {
            Sweep<T, 4, false, M_STEP> sw(I, strip, lpsi, lrho, acc);
            sw.run(chunk);
        }
    }
}

template <class T, int KIND>
__global__ __launch_bounds__(256) void batch_kernel(
    const BatchInst<typename T::S, typename T::A>* __restrict__ insts,
    const BatchItem* __restrict__ items, int nitems, int64_t max_steps, BatchCtl* ctl,
    uint32_t spin_limit)
{
    using A2 = typename T::A2;
    __shared__ A2 lpsi[KIND == B_STACKED ? 2 : 6][256];  // stacked tiles use 8 x 64
    __shared__ A2 lrho[KIND == B_STACKED ? 2 : 6][256];
    double acc[NDIAG] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t s = 0; s < max_steps; ++s) {
        for (int k = blockIdx.x; k < nitems; k += gridDim.x) {
            const BatchItem it = items[k];
            const auto& bi = insts[it.inst];
            if (s >= bi.steps) continue;  // uniform: this instance is done
            batch_item<T, KIND, false>(bi, it.tile, s, lpsi, lrho, acc);
            __syncthreads();  // the next item reuses the LDS ring
        }
        if (!grid_barrier(ctl, spin_limit)) return;
    }
}

// Step-wise batch: step s of every instance that still has steps, one
// ordinary launch with one workgroup per item; consecutive launches on the
// stream order the steps.  Items are remapped so each XCD gets a contiguous
// range (neighbouring tiles of few instances share its L2), and tiles are
// numbered row-major within an instance, as in the single-instance kernels.
template <class T, int KIND>
__global__ __launch_bounds__(256) void batch_step_kernel(
    const BatchInst<typename T::S, typename T::A>* __restrict__ insts,
    const BatchItem* __restrict__ items, int64_t s)
{
    using A2 = typename T::A2;
    __shared__ A2 lpsi[KIND == B_STACKED ? 2 : 6][256];
    __shared__ A2 lrho[KIND == B_STACKED ? 2 : 6][256];
    const BatchItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const auto& bi = insts[it.inst];
    if (s >= bi.steps) return;  // uniform: this instance is done
    double acc[NDIAG] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    batch_item<T, KIND, true>(bi, it.tile, s, lpsi, lrho, acc);
}

template <class T, int KIND>
static int batch_grid_t()
{
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<T, KIND>, 256, 0) !=
        hipSuccess)
        return 0;
    // Every co-resident workgroup meets at each grid barrier, whose cost
    // grows with their number: at most 2 per CU (3 per CU measured 15%
    // slower per step on the uneven batch mix).
    return std::min(per_cu, 2) * cus;
}

template <class T>
static int batch_grid_k(int kind)
{
    switch (kind) {
    case B_STACKED: return batch_grid_t<T, B_STACKED>();
    case B_SWEEP: return batch_grid_t<T, B_SWEEP>();
    case B_MIXED: return batch_grid_t<T, B_MIXED>();
    }
    return 0;
}

template <class T, int KIND>
static hipError_t batch_go(const void* insts, const BatchItem* items, int nitems,
                           int64_t max_steps, BatchCtl* ctl, uint32_t spin_limit, int grid,
                           hipStream_t st)
{
    auto bi = static_cast<const BatchInst<typename T::S, typename T::A>*>(insts);
    void* args[] = {(void*)&bi,        (void*)&items, (void*)&nitems, (void*)&max_steps,
                    (void*)&ctl,       (void*)&spin_limit};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&batch_kernel<T, KIND>),
                                      dim3(grid), dim3(256), args, 0, st);
}

template <class T>
static hipError_t batch_go_k(int kind, const void* insts, const BatchItem* items, int nitems,
                             int64_t max_steps, BatchCtl* ctl, uint32_t lim, int grid,
                             hipStream_t st)
{
    switch (kind) {
    case B_STACKED: return batch_go<T, B_STACKED>(insts, items, nitems, max_steps, ctl, lim, grid, st);
    case B_SWEEP: return batch_go<T, B_SWEEP>(insts, items, nitems, max_steps, ctl, lim, grid, st);
    case B_MIXED: return batch_go<T, B_MIXED>(insts, items, nitems, max_steps, ctl, lim, grid, st);
    }
    return hipErrorInvalidValue;
}

template <class T>
static hipError_t batch_step_go(int kind, const void* insts, const BatchItem* items, int nitems,
                                int64_t s, hipStream_t st)
{
    auto bi = static_cast<const BatchInst<typename T::S, typename T::A>*>(insts);
    switch (kind) {
    case B_STACKED:
        hipLaunchKernelGGL((batch_step_kernel<T, B_STACKED>), dim3(nitems), dim3(256), 0, st, bi,
                           items, s);
        break;
    case B_SWEEP:
        hipLaunchKernelGGL((batch_step_kernel<T, B_SWEEP>), dim3(nitems), dim3(256), 0, st, bi,
                           items, s);
        break;
    case B_MIXED:
        hipLaunchKernelGGL((batch_step_kernel<T, B_MIXED>), dim3(nitems), dim3(256), 0, st, bi,
                           items, s);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers

template <class T, int RW, bool WALLS, int MODE>
static hipError_t go_tile(int wt, const void* inst, int nb, hipStream_t st)
{
    const auto& I = *static_cast<const Inst<typename T::S, typename T::A>*>(inst);
    if (wt)
        hipLaunchKernelGGL((tile_kernel<T, RW, WALLS, MODE, CPOL_WT>), dim3(nb), dim3(64 * RW), 0,
                           st, I);
    else
        hipLaunchKernelGGL((tile_kernel<T, RW, WALLS, MODE, 0>), dim3(nb), dim3(64 * RW), 0, st,
                           I);
    return hipGetLastError();
}

template <class T, int CW, bool WALLS, int MODE>
static hipError_t go(const void* inst, int nb, hipStream_t st)
{
    const auto& I = *static_cast<const Inst<typename T::S, typename T::A>*>(inst);
    hipLaunchKernelGGL((sweep_kernel<T, CW, WALLS, MODE>), dim3(nb), dim3(64 * CW), 0, st, I);
    return hipGetLastError();
}

template <class T, int CW, bool WALLS>
static hipError_t go_mode(int mode, const void* inst, int nb, hipStream_t st)
{
    switch (mode) {
    case M_STEP: return go<T, CW, WALLS, M_STEP>(inst, nb, st);
    case M_STEP_DIAG: return go<T, CW, WALLS, M_STEP_DIAG>(inst, nb, st);
    case M_READ: return go<T, CW, WALLS, M_READ>(inst, nb, st);
    case M_DIAG: return go<T, CW, WALLS, M_DIAG>(inst, nb, st);
    case M_PHI: return go<T, CW, WALLS, M_PHI>(inst, nb, st);
    }
    return hipErrorInvalidValue;
}

template <class T, bool WALLS>
static hipError_t go_stacked(int rw, int wt, int mode, const void* inst, int nb, hipStream_t st)
{
    if (mode != M_STEP && mode != M_STEP_DIAG) return hipErrorInvalidValue;
    const bool d = mode == M_STEP_DIAG;
    switch (rw) {
    case 4: return d ? go_tile<T, 4, WALLS, M_STEP_DIAG>(wt, inst, nb, st)
                     : go_tile<T, 4, WALLS, M_STEP>(wt, inst, nb, st);
    case 8: return d ? go_tile<T, 8, WALLS, M_STEP_DIAG>(wt, inst, nb, st)
                     : go_tile<T, 8, WALLS, M_STEP>(wt, inst, nb, st);
    }
    return hipErrorInvalidValue;
}

template <class T>
static hipError_t go_cw(int cw, int wt, int walls, int mode, const void* inst, int nb,
                        hipStream_t st)
{
    if (cw < 0)  // stacked tile mode with -cw waves
        return walls ? go_stacked<T, true>(-cw, wt, mode, inst, nb, st)
                     : go_stacked<T, false>(-cw, wt, mode, inst, nb, st);
    switch (cw) {
    case 1: return walls ? go_mode<T, 1, true>(mode, inst, nb, st)
                         : go_mode<T, 1, false>(mode, inst, nb, st);
    case 2: return walls ? go_mode<T, 2, true>(mode, inst, nb, st)
                         : go_mode<T, 2, false>(mode, inst, nb, st);
    case 4: return walls ? go_mode<T, 4, true>(mode, inst, nb, st)
                         : go_mode<T, 4, false>(mode, inst, nb, st);
    }
    return hipErrorInvalidValue;
}

template <class T>
static hipError_t init_go(const void* inst, const double* rA, const double* rB,
                          const double* ux, const double* uy, int random, uint64_t seed,
                          double mA, double mB, double amp, hipStream_t st)
{
    const auto& I = *static_cast<const Inst<typename T::S, typename T::A>*>(inst);
    const int64_t N = (int64_t)I.g.nx * I.g.ny;
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL(init_kernel<T>, dim3(nb), dim3(256), 0, st, I, rA, rB, ux, uy, random,
                       seed, mA, mB, amp);
    return hipGetLastError();
}

// ------------------------------------------------- entry points of this unit
//
// The file is compiled once per storage type (-DSCLBM_STORAGE = 0 FP64, 1
// FP32, 2 FP16 deviations, 3 FP16 deviations with stochastic rounding), so
// the four sets of kernels build in parallel; the storage-dispatching
// launchers of sclbm_internal.h call the suffixed functions below.
#if SCLBM_STORAGE == 0
using TS = TF64;
#elif SCLBM_STORAGE == 1
using TS = TF32;
#elif SCLBM_STORAGE == 2
using TS = TF16;
#elif SCLBM_STORAGE == 3
using TS = TF16SR;
#else
#error "SCLBM_STORAGE must be 0, 1, 2 or 3"
#endif

hipError_t SCLBM_SFX(launch_sweep)(int cw, int wt, int walls, int mode, const void* inst, int nb,
                                   hipStream_t st)
{
    return go_cw<TS>(cw, wt, walls, mode, inst, nb, st);
}

int SCLBM_SFX(batch_grid)(int kind) { return batch_grid_k<TS>(kind); }

hipError_t SCLBM_SFX(launch_batch)(int kind, const void* insts, const BatchItem* items,
                                   int nitems, int64_t max_steps, BatchCtl* ctl,
                                   uint32_t spin_limit, int grid, hipStream_t st)
{
    return batch_go_k<TS>(kind, insts, items, nitems, max_steps, ctl, spin_limit, grid, st);
}

hipError_t SCLBM_SFX(launch_batch_step)(int kind, const void* insts, const BatchItem* items,
                                        int nitems, int64_t s, hipStream_t st)
{
    return batch_step_go<TS>(kind, insts, items, nitems, s, st);
}

hipError_t SCLBM_SFX(launch_init)(const void* inst, const double* rA, const double* rB,
                                  const double* ux, const double* uy, int random, uint64_t seed,
                                  double mA, double mB, double amp, hipStream_t st)
{
    return init_go<TS>(inst, rA, rB, ux, uy, random, seed, mA, mB, amp, st);
}

#if SCLBM_STORAGE == 0
hipError_t launch_reduce(const double* partials, int nb, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, partials, nb, out);
    return hipGetLastError();
}
#endif

}  // namespace sclbm
