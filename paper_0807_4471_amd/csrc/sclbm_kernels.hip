// sclbm_kernels.hip -- gfx950 kernels of the two-species multi-range
// Shan-Chen lattice Boltzmann step (Benzi, Chibbaro & Succi, arXiv:0807.4471).
//
// One fused, HBM-bound pass per time step (Eq. (1) plus the FORCE equations):
//   pull-stream f_i(x,t) = f*_i(x - c_i, t-1) -> moments rho_s, j_s ->
//   Psi_s = A (1 - exp(-rho_s/rho0)) -> Psi/rho halo in LDS -> forces
//   (24-neighbour like-species stencil, 8-neighbour cross term) ->
//   Shan-Chen velocity shift -> BGK -> store f*(t).
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
// Workgroups are dispatched round-robin over the 8 XCDs; blocks are remapped
// so that each XCD gets a contiguous range of (strip, chunk) tiles, keeping
// the halo rows shared by vertically adjacent chunks in one L2.
#include <type_traits>

#include "sclbm_internal.h"

namespace sclbm {

struct TF64 {
    using S = double;
    using A = double;
    using A2 = double2;
};
struct TF32 {
    using S = float;
    using A = float;
    using A2 = float2;
};
struct TF16 {
    using S = _Float16;
    using A = float;
    using A2 = float2;
};

// D2Q9: i = 0 rest, 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1),
// 7 (-1,-1), 8 (1,-1); weights 4/9, 1/9, 1/36.
#define W0 (4.0 / 9.0)
#define W1 (1.0 / 9.0)
#define W2 (1.0 / 36.0)

template <class T>
__device__ __forceinline__ typename T::A ld(const typename T::S* __restrict__ p,
                                            typename T::A base)
{
    if constexpr (std::is_same<T, TF16>::value)
        return base + (float)(*p);
    else
        return (typename T::A)(*p);
}

template <class T>
__device__ __forceinline__ void st(typename T::S* __restrict__ p, typename T::A v,
                                   typename T::A base)
{
    if constexpr (std::is_same<T, TF16>::value)
        *p = (_Float16)(v - base);
    else
        *p = (typename T::S)v;
}

template <class T>
__device__ __forceinline__ typename T::A rcp(typename T::A v)
{
    if constexpr (std::is_same<typename T::A, double>::value)
        return 1.0 / v;
    else
        return __builtin_amdgcn_rcpf(v);
}

template <class T>
__device__ __forceinline__ typename T::A expo(typename T::A v)
{
    if constexpr (std::is_same<typename T::A, double>::value)
        return exp(v);
    else
        return expf(v);
}

// Pull the 18 post-streaming populations of real row rr at column xw:
// f_i(x, t) = f*_i(x - c_i, t-1).  With walls the rows +-1 beyond the channel
// are the ghost rows holding the bounced-back populations.
template <class T, bool WALLS>
__device__ __forceinline__ void pull(const Inst<typename T::S, typename T::A>& I,
                                     const typename T::S* __restrict__ fin, int rr, int xw,
                                     int xm, int xp, typename T::A f[18])
{
    const Geo& g = I.g;
    int r0, rm, rp;
    if constexpr (WALLS) {
        r0 = rr + 1;
        rm = rr;
        rp = rr + 2;
    } else {
        r0 = rr;
        rm = rr == 0 ? g.ny - 1 : rr - 1;
        rp = rr == g.ny - 1 ? 0 : rr + 1;
    }
    const int o0 = r0 * g.pitch, om = rm * g.pitch, op = rp * g.pitch;
    const int off[9] = {o0 + xw, o0 + xm, om + xw, o0 + xp, op + xw,
                        om + xm, om + xp, op + xp, op + xm};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[s * 9 + i] = ld<T>(fin + (int64_t)(s * 9 + i) * g.plane + off[i], I.c.base[s][i]);
}

template <class A>
__device__ __forceinline__ void moments(const A* f, A& rho, A& jx, A& jy)
{
    rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
}

// One BGK relaxation towards f^eq(rho, u) (second-order D2Q9 polynomial).
template <class A>
__device__ __forceinline__ void bgk(A* f, A rho, A ux, A uy, A omega)
{
    const A usq = ux * ux + uy * uy;
    const A com = A(1) - A(1.5) * usq;
    const A r0 = A(W0) * rho, r1 = A(W1) * rho, r2 = A(W2) * rho;
    auto eq = [&](A rw, A cu) { return rw * (com + A(3) * cu + A(4.5) * cu * cu); };
    const A up = ux + uy, um = ux - uy;
    const A feq[9] = {r0 * com,     eq(r1, ux),  eq(r1, uy),  eq(r1, -ux), eq(r1, -uy),
                      eq(r2, up),   eq(r2, -um), eq(r2, -up), eq(r2, um)};
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = f[i] - omega * (f[i] - feq[i]);
}

// Sweep one (strip, chunk) tile.  MODE selects step / step+diagnostics /
// moment read-out / diagnostics only.  acc[] collects FP64 diagnostics of
// the owned sites.
template <class T, int CW, bool WALLS, int MODE>
__device__ __forceinline__ void sweep(const Inst<typename T::S, typename T::A>& I, int strip,
                                      int chunk, typename T::A2 (*lpsi)[64 * CW],
                                      typename T::A2 (*lrho)[64 * CW], double* acc)
{
    using A = typename T::A;
    using A2 = typename T::A2;
    const typename T::S* __restrict__ fin = I.fin;
    typename T::S* __restrict__ fout = I.fout;
    const Geo& g = I.g;
    const int nx = g.nx, ny = g.ny;
    const int t = threadIdx.x;
    const int x = strip * I.W - 2 + t;
    int xw = x % nx;
    if (xw < 0) xw += nx;
    const int xm = xw == 0 ? nx - 1 : xw - 1;
    const int xp = xw == nx - 1 ? 0 : xw + 1;
    const bool own = t >= 2 && t < I.W + 2 && x < nx;
    const int y0 = chunk * I.H;
    const int y1 = min(y0 + I.H, ny);
    const Coef<A>& c = I.c;

    auto real_row = [&](int r) {
        if constexpr (WALLS) {
            if (r < 0) r = -1 - r;
            if (r > ny - 1) r = 2 * ny - 1 - r;
            return r;
        } else {
            r %= ny;
            return r < 0 ? r + ny : r;
        }
    };

    A P0[18], P1[18], P2[18];

    // Pull row r into f, stage its Psi and rho in ring slot `slot`.
    auto stage = [&](int r, int slot, A* f) {
        pull<T, WALLS>(I, fin, real_row(r), xw, xm, xp, f);
        A ra, rb, jx, jy;
        moments<A>(f, ra, jx, jy);
        moments<A>(f + 9, rb, jx, jy);
        const A pa = c.psi_amp * (A(1) - expo<T>(ra * c.neg_inv_rho0));
        const A pb = c.psi_amp * (A(1) - expo<T>(rb * c.neg_inv_rho0));
        lpsi[slot][t] = A2{pa, pb};
        lrho[slot][t] = A2{ra, rb};
    };

    // Prologue: rows y0-2 .. y0+1 in slots 0..3; keep rows y0, y0+1.
    stage(y0 - 2, 0, P2);
    stage(y0 - 1, 1, P2);
    stage(y0, 2, P0);
    stage(y0 + 1, 3, P1);

    int sb = 0;  // slot of row y-2
    for (int y = y0; y < y1; ++y) {
        const int snew = sb + 4 >= 6 ? sb - 2 : sb + 4;
        stage(y + 2, snew, P2);
        __syncthreads();
        if (own) {
            int sl[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) sl[k] = (sb + k) % 6;
            auto Ps = [&](int dx, int dy) { return lpsi[sl[dy + 2]][t + dx]; };
            auto Rs = [&](int dx, int dy) { return lrho[sl[dy + 2]][t + dx]; };
            auto dif = [](A2 a, A2 b) { return A2{a.x - b.x, a.y - b.y}; };
            // Psi differences over the 12 opposite pairs (both species).
            const A2 a10 = dif(Ps(1, 0), Ps(-1, 0)), a01 = dif(Ps(0, 1), Ps(0, -1));
            const A2 a11 = dif(Ps(1, 1), Ps(-1, -1)), b11 = dif(Ps(-1, 1), Ps(1, -1));
            const A2 a20 = dif(Ps(2, 0), Ps(-2, 0)), a02 = dif(Ps(0, 2), Ps(0, -2));
            const A2 a21 = dif(Ps(2, 1), Ps(-2, -1)), a12 = dif(Ps(1, 2), Ps(-1, -2));
            const A2 b12 = dif(Ps(-1, 2), Ps(1, -2)), b21 = dif(Ps(-2, 1), Ps(2, -1));
            const A2 a22 = dif(Ps(2, 2), Ps(-2, -2)), b22 = dif(Ps(-2, 2), Ps(2, -2));
            // rho differences over the 4 first-belt pairs (cross force).
            const A2 r10 = dif(Rs(1, 0), Rs(-1, 0)), r01 = dif(Rs(0, 1), Rs(0, -1));
            const A2 r11 = dif(Rs(1, 1), Rs(-1, -1)), q11 = dif(Rs(-1, 1), Rs(1, -1));
            const A2 pc = Ps(0, 0);
            const A2 rc = Rs(0, 0);

            A F[2][2];
            auto force = [&](int s, A d10, A d01, A d11, A e11, A d20, A d02, A d21, A d12,
                             A e12, A e21, A d22, A e22, A psi, A rho, A o10, A o01, A o11,
                             A p11) {
                const A Sx = c.K1[s] * d10 + c.K2[s] * (d11 - e11) + c.K4x2[s] * d20 +
                             c.K5[s] * (A(2) * d21 + d12 - e12 - A(2) * e21) +
                             c.K8x2[s] * (d22 - e22);
                const A Sy = c.K1[s] * d01 + c.K2[s] * (d11 + e11) + c.K4x2[s] * d02 +
                             c.K5[s] * (d21 + A(2) * d12 + A(2) * e12 + e21) +
                             c.K8x2[s] * (d22 + e22);
                const A Xx = c.X1 * o10 + c.X2 * (o11 - p11);
                const A Xy = c.X1 * o01 + c.X2 * (o11 + p11);
                F[s][0] = -psi * Sx - rho * Xx;
                F[s][1] = -psi * Sy - rho * Xy;
            };
            force(0, a10.x, a01.x, a11.x, b11.x, a20.x, a02.x, a21.x, a12.x, b12.x, b21.x, a22.x,
                  b22.x, pc.x, rc.x, r10.y, r01.y, r11.y, q11.y);
            force(1, a10.y, a01.y, a11.y, b11.y, a20.y, a02.y, a21.y, a12.y, b12.y, b21.y, a22.y,
                  b22.y, pc.y, rc.y, r10.x, r01.x, r11.x, q11.x);
            if (c.body_F0 != 0.0) {
                const A gy = (A)(c.body_F0 * sin(c.two_pi_over_ny * (double)y));
                F[0][0] += rc.x * gy;
                F[1][0] += rc.y * gy;
            }

            A rho[2], jx[2], jy[2];
            moments<A>(P0, rho[0], jx[0], jy[0]);
            moments<A>(P0 + 9, rho[1], jx[1], jy[1]);

            if constexpr (MODE == M_STEP_DIAG || MODE == M_DIAG || MODE == M_READ) {
                const A rt = rho[0] + rho[1];
                const A mx = (jx[0] + A(0.5) * F[0][0]) + (jx[1] + A(0.5) * F[1][0]);
                const A my = (jy[0] + A(0.5) * F[0][1]) + (jy[1] + A(0.5) * F[1][1]);
                const A irt = rt > A(0) ? rcp<T>(rt) : A(0);
                const A vx = mx * irt, vy = my * irt;
                A sxy = A(0);
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const A* f = s ? P0 + 9 : P0;
                    sxy -= c.hs[s] * ((f[5] - f[6]) + (f[7] - f[8]) - rho[s] * vx * vy);
                }
                if constexpr (MODE == M_READ) {
                    const int64_t n = (int64_t)y * nx + xw;
                    if (I.out[0]) I.out[0][n] = (double)rho[0];
                    if (I.out[1]) I.out[1][n] = (double)rho[1];
                    if (I.out[2]) I.out[2][n] = (double)vx;
                    if (I.out[3]) I.out[3][n] = (double)vy;
                    if (I.out[4]) I.out[4][n] = (double)sxy;
                } else {
                    acc[D_MASS_A] += (double)rho[0];
                    acc[D_MASS_B] += (double)rho[1];
                    acc[D_MOM_X] += (double)mx;
                    acc[D_MOM_Y] += (double)my;
                    acc[D_SXY] += (double)sxy;
                    const bool ok = rho[0] > A(0) && rho[1] > A(0) && rho[0] < A(1e30) &&
                                    rho[1] < A(1e30);
                    acc[D_BAD] += ok ? 0.0 : 1.0;
                }
            }

            if constexpr (MODE == M_STEP || MODE == M_STEP_DIAG) {
                // Shan-Chen velocity shift: common velocity weighted by
                // rho_s/tau_s, species shift tau_s F_s / rho_s.
                const A den = rho[0] * c.omega[0] + rho[1] * c.omega[1];
                const A nmx = jx[0] * c.omega[0] + jx[1] * c.omega[1];
                const A nmy = jy[0] * c.omega[0] + jy[1] * c.omega[1];
                const A iden = den > A(0) ? rcp<T>(den) : A(0);
                const A upx = nmx * iden, upy = nmy * iden;
                const int ro = y + (WALLS ? 1 : 0);
                const int64_t site = (int64_t)ro * g.pitch + xw;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    A* f = s ? P0 + 9 : P0;
                    const A ir = rho[s] > A(0) ? c.tau[s] * rcp<T>(rho[s]) : A(0);
                    const A uex = upx + F[s][0] * ir, uey = upy + F[s][1] * ir;
                    bgk<A>(f, rho[s], uex, uey, c.omega[s]);
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        st<T>(fout + (int64_t)(s * 9 + i) * g.plane + site, f[i], c.base[s][i]);
                }
                if constexpr (WALLS) {
                    // Half-way bounce-back: a population leaving the channel
                    // returns to its node reversed, minus 2 w_i rho (c_i.u_w)/c_s^2.
                    // It is written to the ghost row where the next pull of the
                    // reversed direction looks for it.
                    if (y == 0 || y == ny - 1) {
                        const bool top = y == ny - 1;
                        const A u6 = c.wall6u[top ? 1 : 0];
                        const int grow = top ? ny + 1 : 0;
                        const int64_t gb = (int64_t)grow * g.pitch;
                        // outgoing i -> stored as j = opp(i): bottom (4->2, 7->5, 8->6),
                        // top (2->4, 5->7, 6->8); column x + c_ix.
                        const int io0 = top ? 2 : 4, io1 = top ? 5 : 7, io2 = top ? 6 : 8;
                        const int jo0 = top ? 4 : 2, jo1 = top ? 7 : 5, jo2 = top ? 8 : 6;
                        const int cx1 = top ? 1 : -1;  // c_x of io1; io2 has -cx1
                        const int col1 = top ? xp : xm, col2 = top ? xm : xp;
                        double mxw = 0.0, myw = 0.0;
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            const A* f = s ? P0 + 9 : P0;
                            const A corr = A(W2) * rho[s] * u6;
                            const A v0 = f[io0];
                            const A v1 = f[io1] - A(cx1) * corr;
                            const A v2 = f[io2] + A(cx1) * corr;
                            st<T>(fout + (int64_t)(s * 9 + jo0) * g.plane + gb + xw, v0,
                                  c.base[s][jo0]);
                            st<T>(fout + (int64_t)(s * 9 + jo1) * g.plane + gb + col1, v1,
                                  c.base[s][jo1]);
                            st<T>(fout + (int64_t)(s * 9 + jo2) * g.plane + gb + col2, v2,
                                  c.base[s][jo2]);
                            // momentum received by the wall: c_i (f*_i + reflected)
                            const double cy = top ? 1.0 : -1.0;
                            mxw += (double)cx1 * ((double)f[io1] + (double)v1) -
                                   (double)cx1 * ((double)f[io2] + (double)v2);
                            myw += cy * (((double)f[io0] + (double)v0) +
                                         ((double)f[io1] + (double)v1) +
                                         ((double)f[io2] + (double)v2));
                        }
                        double* wa = I.wall_acc + (top ? 2 : 0) * (int64_t)nx;
                        wa[xw] += mxw;
                        wa[nx + xw] += myw;
                    }
                }
            }
        }
        // rotate the register rows
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            P0[k] = P1[k];
            P1[k] = P2[k];
        }
        sb = sb == 5 ? 0 : sb + 1;
    }
}

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8);
// give each XCD a contiguous range of logical tiles.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int per = n / 8, rem = n % 8, xcd = b % 8, k = b / 8;
    return xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

template <int CW>
__device__ __forceinline__ void block_reduce(double* acc, double (*red)[NDIAG], double* out)
{
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double v = acc[j];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        acc[j] = v;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int j = 0; j < 6; ++j) red[w][j] = acc[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < CW; ++k) s += red[k][j];
            out[j] = s;
        }
        out[6] = 0.0;
        out[7] = 0.0;
    }
}

template <class T, int CW, bool WALLS, int MODE>
__global__ __launch_bounds__(64 * CW) void sweep_kernel(Inst<typename T::S, typename T::A> I)
{
    __shared__ typename T::A2 lpsi[6][64 * CW];
    __shared__ typename T::A2 lrho[6][64 * CW];
    __shared__ double red[CW][NDIAG];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int strip = b / I.nchunks, chunk = b - (b / I.nchunks) * I.nchunks;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    sweep<T, CW, WALLS, MODE>(I, strip, chunk, lpsi, lrho, acc);
    if constexpr (MODE == M_STEP_DIAG || MODE == M_DIAG)
        block_reduce<CW>(acc, red, I.partials + (int64_t)b * NDIAG);
}

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
            st<T>(I.fout + (int64_t)(s * 9 + i) * g.plane + (int64_t)ys * g.pitch + xs,
                  (typename T::A)feq, I.c.base[s][i]);
        }
}

// ---------------------------------------------------------------- launchers

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
    }
    return hipErrorInvalidValue;
}

template <class T>
static hipError_t go_cw(int cw, int walls, int mode, const void* inst, int nb, hipStream_t st)
{
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

hipError_t launch_sweep(int storage, int cw, int mode, const void* inst, int nb, hipStream_t st)
{
    // walls flag lives in the Geo at the same offset for every instantiation
    const int walls = static_cast<const Inst<float, float>*>(inst)->g.walls;
    switch (storage) {
    case 0: return go_cw<TF64>(cw, walls, mode, inst, nb, st);
    case 1: return go_cw<TF32>(cw, walls, mode, inst, nb, st);
    case 2: return go_cw<TF16>(cw, walls, mode, inst, nb, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const double* partials, int nb, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, partials, nb, out);
    return hipGetLastError();
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

hipError_t launch_init(int storage, const void* inst, const double* rA, const double* rB,
                       const double* ux, const double* uy, int random, uint64_t seed,
                       double mA, double mB, double amp, hipStream_t st)
{
    switch (storage) {
    case 0: return init_go<TF64>(inst, rA, rB, ux, uy, random, seed, mA, mB, amp, st);
    case 1: return init_go<TF32>(inst, rA, rB, ux, uy, random, seed, mA, mB, amp, st);
    case 2: return init_go<TF16>(inst, rA, rB, ux, uy, random, seed, mA, mB, amp, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace sclbm
