// sclbm_api.cpp -- host runtime of libsclbm.so: descriptor validation, state
// layout inside the caller's device buffer, kernel launches on the caller's
// stream, error mapping.  The declarations and their contracts are in
// include/sclbm.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sclbm.h"
#include "sclbm_internal.h"

using namespace sclbm;

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int32_t fail(int32_t code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int32_t hip_fail(hipError_t e, const char* what)
{
    return fail(SCLBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t ALIGN = 256;
constexpr int MIN_TILE_X = 32;  // smallest strip width a tiling may use
constexpr int MIN_TILE_Y = 4;   // smallest chunk height a tiling may use
constexpr uint64_t CKPT_MAGIC = 0x53434C424D434B31ull;  // "SCLBMCK1"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int storage) { return storage == SCLBM_F64 ? 8 : storage == SCLBM_F32 ? 4 : 2; }
bool is_dev(int storage) { return storage == SCLBM_F16DEV || storage == SCLBM_F16DEV_SR; }

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int32_t validate(const sclbm_desc* d)
{
    if (!d) return fail(SCLBM_EINVAL, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nx > 65536 || d->ny > 65536)
        return fail(SCLBM_EINVAL, "lattice %d x %d out of range [1, 65536]", d->nx, d->ny);
    if ((int64_t)d->nx * d->ny > 2147483647LL)
        return fail(SCLBM_EINVAL, "nx * ny exceeds 2^31 - 1");
    if (d->boundary != SCLBM_PERIODIC && d->boundary != SCLBM_WALLS_Y)
        return fail(SCLBM_EINVAL, "unknown boundary %d", d->boundary);
    if (d->boundary == SCLBM_WALLS_Y && d->ny < 2)
        return fail(SCLBM_EINVAL, "walls need ny >= 2");
    if (d->storage != SCLBM_F64 && d->storage != SCLBM_F32 && d->storage != SCLBM_F16DEV &&
        d->storage != SCLBM_F16DEV_SR)
        return fail(SCLBM_EINVAL, "unknown storage %d", d->storage);
    for (int s = 0; s < 2; ++s) {
        if (!(isfinite(d->tau[s]) && d->tau[s] > 0.5))
            return fail(SCLBM_EINVAL, "tau[%d] = %g must be finite and > 1/2", s, d->tau[s]);
        if (!isfinite(d->G_a[s]) || !isfinite(d->G_r[s]))
            return fail(SCLBM_EINVAL, "couplings of species %d must be finite", s);
        if (is_dev(d->storage) && !(isfinite(d->rho_ref[s]) && d->rho_ref[s] >= 0.0))
            return fail(SCLBM_EINVAL, "rho_ref[%d] must be finite and >= 0", s);
        if (d->boundary == SCLBM_WALLS_Y && !isfinite(d->wall_u[s]))
            return fail(SCLBM_EINVAL, "wall_u[%d] must be finite", s);
    }
    if (!isfinite(d->G_x)) return fail(SCLBM_EINVAL, "G_x must be finite");
    if (!finite_pos(d->rho0)) return fail(SCLBM_EINVAL, "rho0 must be finite and > 0");
    if (!finite_pos(d->psi_amp)) return fail(SCLBM_EINVAL, "psi_amp must be finite and > 0");
    if (!isfinite(d->body_F0)) return fail(SCLBM_EINVAL, "body_F0 must be finite");
    if (d->diag_every < 0) return fail(SCLBM_EINVAL, "diag_every must be >= 0");
    if (d->forcing != SCLBM_FORCING_SHIFT && d->forcing != SCLBM_FORCING_GUO)
        return fail(SCLBM_EINVAL, "unknown forcing %d", d->forcing);
    // populations are addressed through one buffer resource per species
    // with 32-bit offsets: its 9 planes must span < 2^31 bytes
    const int64_t rows = d->ny + (d->boundary == SCLBM_WALLS_Y ? 2 : 0);
    const int64_t plane_bytes = ((((int64_t)d->nx + 63) / 64 * 64) * rows + 128) *
                                (int64_t)(d->storage == SCLBM_F64 ? 8 : d->storage == SCLBM_F32 ? 4 : 2);
    if (9 * plane_bytes >= (int64_t)1 << 31)
        return fail(SCLBM_EUNSUPPORTED,
                    "the 9 population planes of a species would span %lld bytes (>= 2 GiB); "
                    "split the lattice", (long long)(9 * plane_bytes));
    return SCLBM_OK;
}

struct Layout {
    Geo g;
    size_t pop_bytes;     // one population copy
    size_t off_f[2];
    size_t off_partials;
    int max_blocks;
    size_t off_diag;
    size_t off_wall;
    size_t total;
};

Layout layout(const sclbm_desc* d)
{
    Layout L{};
    const int walls = d->boundary == SCLBM_WALLS_Y;
    L.g.nx = d->nx;
    L.g.ny = d->ny;
    L.g.walls = walls;
    L.g.rows = d->ny + 2 * walls;
    L.g.pitch = (int32_t)align_up((size_t)d->nx, 64);
    // pad each (s, i) plane by 64 elements beyond a 64-element multiple so
    // the 18 streams do not start on the same DRAM channel
    L.g.plane = (int64_t)align_up((size_t)L.g.pitch * L.g.rows, 64) + 64;
    const size_t eb = elem_bytes(d->storage);
    L.pop_bytes = align_up((size_t)L.g.plane * 18 * eb, ALIGN);
    L.off_f[0] = 0;
    L.off_f[1] = L.pop_bytes;
    L.off_partials = 2 * L.pop_bytes;
    const int64_t ms = (d->nx + MIN_TILE_X - 1) / MIN_TILE_X;
    const int64_t mc = (d->ny + MIN_TILE_Y - 1) / MIN_TILE_Y;
    L.max_blocks = (int)(ms * mc);
    L.off_diag = L.off_partials + align_up((size_t)L.max_blocks * NDIAG * 8, ALIGN);
    L.off_wall = L.off_diag + align_up(2 * NDIAG * 8, ALIGN);  // fused, on-demand
    L.total = L.off_wall + align_up((size_t)4 * d->nx * 8, ALIGN);
    return L;
}

const double W_OF_SHELL[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 0, 0, 0, 0, 0, 0};
// Repulsion weights per shell |e|^2: the unique weights with Sum p = 1,
// Sum p c_x^2 = 1/3 and lattice tensors isotropic to 8th order.
double p_of_shell(int e2)
{
    switch (e2) {
    case 1: return 4.0 / 63.0;
    case 2: return 4.0 / 135.0;
    case 4: return 1.0 / 180.0;
    case 5: return 2.0 / 945.0;
    case 8: return 1.0 / 15120.0;
    }
    return 0.0;
}

template <class A>
Coef<A> coefficients(const sclbm_desc* d)
{
    Coef<A> c{};
    for (int s = 0; s < 2; ++s) {
        auto K = [&](int e2) {
            const double w = e2 == 1 ? W_OF_SHELL[1] : e2 == 2 ? W_OF_SHELL[2] : 0.0;
            return d->G_a[s] * w + d->G_r[s] * p_of_shell(e2);
        };
        c.K1[s] = (A)K(1);
        c.K2[s] = (A)K(2);
        c.K4x2[s] = (A)(2.0 * K(4));
        c.K5[s] = (A)K(5);
        c.K8x2[s] = (A)(2.0 * K(8));
        c.tau[s] = (A)d->tau[s];
        c.omega[s] = (A)(1.0 / d->tau[s]);
        c.hs[s] = (A)(1.0 - 0.5 / d->tau[s]);
        c.wall6u[s] = (A)(6.0 * d->wall_u[s]);
        c.rho_base[s] = is_dev(d->storage) ? (A)d->rho_ref[s] : (A)0;
        c.tau1[s] = d->tau[s] == 1.0;
    }
    const double gx = d->G_x / d->rho0;
    c.X1 = (A)(gx * W_OF_SHELL[1]);
    c.X2 = (A)(gx * W_OF_SHELL[2]);
    c.psi_amp = (A)d->psi_amp;
    c.neg_inv_rho0 = (A)(-1.0 / d->rho0);
    c.guo = d->forcing == SCLBM_FORCING_GUO;
    c.pad_ = 0;
    c.body_F0 = d->body_F0;
    c.two_pi_over_ny = 6.283185307179586476925286766559 / (double)d->ny;
    return c;
}

}  // namespace

struct sclbm_inst {
    sclbm_desc d;
    char* buf;
    size_t bytes;
    Layout L;
    Coef<double> cd;
    Coef<float> cf;
    int cur;              // copy holding f*(t-1)
    int64_t t;
    bool inited;
    int64_t fused_step;
    int64_t wall_steps;
    int cw, W, H, nstrips, nchunks;
    int stacked;          // 1: tile mode, cw waves stacked along y (H == cw)
    int throttle;         // sweep iterations wait for the previous row's stores
    int wt;               // stacked tiles: write-through population stores
};

namespace {

void set_tiling(sclbm_inst* h, int cw, int W, int H, int stacked = 0, int throttle = 0,
                int wt = 0)
{
    h->stacked = stacked;
    h->throttle = throttle;
    h->wt = wt;
    h->cw = cw;
    h->W = W;
    h->H = H;
    h->nstrips = (h->d.nx + W - 1) / W;
    h->nchunks = (h->d.ny + H - 1) / H;
}

// Default tiling.  Lattices of up to 2^20 sites use stacked tiles (4 waves,
// one row each) so that enough short-lived workgroups exist; larger ones
// sweep the widest strips that fit over chunks sized for about 8 waves per
// CU on 256 CUs.  The autotuner refines this per size.
void default_tiling(sclbm_inst* h)
{
    const int nx = h->d.nx, ny = h->d.ny;
    if ((int64_t)nx * ny <= (1 << 20)) {
        const int ns = (nx + 59) / 60;
        const int W = std::max((nx + ns - 1) / ns, std::min(MIN_TILE_X, nx));
        set_tiling(h, 4, std::min(W, 60), 4, 1);
        return;
    }
    int cw = nx >= 192 ? 4 : nx >= 96 ? 2 : 1;
    if (h->d.storage == SCLBM_F64 && cw == 4) cw = 2;
    const int wmax = 64 * cw - 4;
    const int ns = (nx + wmax - 1) / wmax;
    int W = (nx + ns - 1) / ns;
    W = std::max(W, std::min(MIN_TILE_X, wmax));
    const int target_blocks = std::max(1, 2048 / cw);
    int nc = std::max(1, target_blocks / ns);
    int H = std::max(MIN_TILE_Y, (ny + nc - 1) / nc);
    set_tiling(h, cw, W, H, 0, 1);
}

template <class S, class A>
Inst<S, A> make_inst(const sclbm_inst* h, const Coef<A>& c, int from, int to, int W, int H)
{
    Inst<S, A> I{};
    I.t = h->t;
    I.fin = reinterpret_cast<const S*>(h->buf + h->L.off_f[from]);
    I.fout = reinterpret_cast<S*>(h->buf + h->L.off_f[to]);
    I.g = h->L.g;
    I.c = c;
    I.W = W;
    I.H = H;
    I.nstrips = (h->d.nx + W - 1) / W;
    I.nchunks = (h->d.ny + H - 1) / H;
    I.throttle = h->throttle;
    I.partials = reinterpret_cast<double*>(h->buf + h->L.off_partials);
    I.wall_acc = reinterpret_cast<double*>(h->buf + h->L.off_wall);
    return I;
}

// Launch one sweep in `mode` with the given tiling; for READ mode `out`
// holds the five output pointers.
int32_t sweep(sclbm_inst* h, int mode, int cw, int W, int H, int from, int to,
              double* const* out, hipStream_t st, int* nblocks, int wt = 0)
{
    hipError_t e;
    int nb = 0;
    auto run = [&](auto& I) {
        if (out)
            for (int k = 0; k < 5; ++k) I.out[k] = out[k];
        nb = I.nstrips * I.nchunks;
        return launch_sweep(h->d.storage, cw, wt, mode, &I, nb, st);
    };
    if (h->d.storage == SCLBM_F64) {
        auto I = make_inst<double, double>(h, h->cd, from, to, W, H);
        e = run(I);
    } else if (h->d.storage == SCLBM_F32) {
        auto I = make_inst<float, float>(h, h->cf, from, to, W, H);
        e = run(I);
    } else {
        auto I = make_inst<_Float16, float>(h, h->cf, from, to, W, H);
        e = run(I);
    }
    if (nblocks) *nblocks = nb;
    if (e != hipSuccess) return hip_fail(e, "sweep kernel launch");
    return SCLBM_OK;
}

// Read-only passes use one-wave strips of 60 columns and 16-row chunks.
constexpr int RO_CW = 1, RO_W = 60, RO_H = 16;

void fill_diag(const sclbm_inst* h, const double* v, const double* wall, sclbm_diag* out,
               int64_t step)
{
    memset(out, 0, sizeof *out);
    out->mass[0] = v[D_MASS_A];
    out->mass[1] = v[D_MASS_B];
    out->mom[0] = v[D_MOM_X];
    out->mom[1] = v[D_MOM_Y];
    out->sxy = v[D_SXY];
    out->bad_sites = (int64_t)v[D_BAD];
    out->u_bar = 2.0 * v[D_UPROJ] / ((double)h->d.nx * (double)h->d.ny);
    out->i_ab = v[D_IAB];
    out->step = step;
    out->wall_steps = h->wall_steps;
    if (wall) {
        const int nx = h->d.nx;
        for (int w = 0; w < 2; ++w)
            for (int c = 0; c < 2; ++c) {
                double s = 0.0;
                for (int x = 0; x < nx; ++x) s += wall[(w * 2 + c) * nx + x];
                out->wall_mom[w][c] = s;
            }
    }
}

int32_t read_wall(const sclbm_inst* h, double* host, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(host, h->buf + h->L.off_wall, sizeof(double) * 4 * h->d.nx,
                                  hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "wall accumulator copy");
    return SCLBM_OK;
}

}  // namespace

extern "C" {

int32_t sclbm_abi_version(void) { return SCLBM_ABI_VERSION; }

// Host self-check of index helpers shared with the kernels (no device work):
// every row a kernel may stage, r in [-2, ny + 9], must fold into [0, ny),
// and the folds must be the periodic wrap / the mirror images.  Returns 0 on
// success, else the first failing ny.
int32_t sclbm_selftest(void)
{
    for (int ny = 1; ny <= 40; ++ny)
        for (int walls = 0; walls < 2; ++walls) {
            if (walls && ny < 2) continue;
            for (int r = -2; r <= ny + 9; ++r) {
                const int f = fold_row(r, ny, walls != 0);
                if (f < 0 || f >= ny) return ny;
                if (!walls && f != ((r % ny) + ny) % ny) return ny;
                if (walls && r >= -ny && r < 2 * ny) {
                    const int m = r < 0 ? -1 - r : (r >= ny ? 2 * ny - 1 - r : r);
                    if (f != m) return ny;
                }
            }
        }
    return 0;
}

const char* sclbm_strerror(int32_t status)
{
    switch (status) {
    case SCLBM_OK: return "ok";
    case SCLBM_EINVAL: return "invalid argument";
    case SCLBM_ESIZE: return "buffer too small or size out of range";
    case SCLBM_EDEVICE: return "HIP device error";
    case SCLBM_ENONFINITE: return "non-finite or non-positive density";
    case SCLBM_EUNSUPPORTED: return "unsupported";
    case SCLBM_ESTATE: return "handle in the wrong state";
    }
    return "unknown status";
}

const char* sclbm_last_error(void) { return g_err.c_str(); }

size_t sclbm_state_bytes(const sclbm_desc* desc)
{
    if (validate(desc) != SCLBM_OK) return 0;
    return layout(desc).total;
}

int32_t sclbm_bind(const sclbm_desc* desc, void* dev_buf, size_t bytes, sclbm_inst** out)
{
    if (!out) return fail(SCLBM_EINVAL, "out is NULL");
    *out = nullptr;
    int32_t rc = validate(desc);
    if (rc) return rc;
    if (!dev_buf) return fail(SCLBM_EINVAL, "dev_buf is NULL");
    if ((uintptr_t)dev_buf % ALIGN) return fail(SCLBM_EINVAL, "dev_buf must be 256-byte aligned");
    Layout L = layout(desc);
    if (bytes < L.total)
        return fail(SCLBM_ESIZE, "buffer of %zu bytes < %zu needed", bytes, L.total);
    sclbm_inst* h = new (std::nothrow) sclbm_inst();
    if (!h) return fail(SCLBM_EINVAL, "out of host memory");
    h->d = *desc;
    h->buf = static_cast<char*>(dev_buf);
    h->bytes = bytes;
    h->L = L;
    h->cd = coefficients<double>(desc);
    h->cf = coefficients<float>(desc);
    h->cur = 0;
    h->t = 0;
    h->inited = false;
    h->fused_step = -1;
    h->wall_steps = 0;
    default_tiling(h);
    *out = h;
    return SCLBM_OK;
}

int32_t sclbm_release(sclbm_inst* h)
{
    delete h;
    return SCLBM_OK;
}

static int32_t init_common(sclbm_inst* h, const double* rA, const double* rB, const double* ux,
                           const double* uy, int random, uint64_t seed, const double* mean,
                           double amp, hipStream_t st)
{
    hipError_t e = hipMemsetAsync(h->buf, 0, h->L.total, st);
    if (e != hipSuccess) return hip_fail(e, "state clear");
    h->cur = 0;
    auto run = [&](auto& I) {
        return launch_init(h->d.storage, &I, rA, rB, ux, uy, random, seed,
                           mean ? mean[0] : 0.0, mean ? mean[1] : 0.0, amp, st);
    };
    if (h->d.storage == SCLBM_F64) {
        auto I = make_inst<double, double>(h, h->cd, 1, 0, h->W, h->H);
        e = run(I);
    } else if (h->d.storage == SCLBM_F32) {
        auto I = make_inst<float, float>(h, h->cf, 1, 0, h->W, h->H);
        e = run(I);
    } else {
        auto I = make_inst<_Float16, float>(h, h->cf, 1, 0, h->W, h->H);
        e = run(I);
    }
    if (e != hipSuccess) return hip_fail(e, "init kernel launch");
    h->t = 0;
    h->inited = true;
    h->fused_step = -1;
    h->wall_steps = 0;
    return SCLBM_OK;
}

int32_t sclbm_init_random(sclbm_inst* h, uint64_t seed, const double mean[2], double amp,
                          void* stream)
{
    if (!h || !mean) return fail(SCLBM_EINVAL, "NULL argument");
    if (!isfinite(mean[0]) || !isfinite(mean[1]) || !isfinite(amp))
        return fail(SCLBM_EINVAL, "mean and amp must be finite");
    return init_common(h, nullptr, nullptr, nullptr, nullptr, 1, seed, mean, amp,
                       (hipStream_t)stream);
}

int32_t sclbm_init_fields(sclbm_inst* h, const double* rhoA, const double* rhoB,
                          const double* ux, const double* uy, void* stream)
{
    if (!h || !rhoA || !rhoB) return fail(SCLBM_EINVAL, "NULL argument");
    return init_common(h, rhoA, rhoB, ux, uy, 0, 0, nullptr, 0.0, (hipStream_t)stream);
}

int32_t sclbm_step(sclbm_inst* h, int64_t n, void* stream)
{
    if (!h) return fail(SCLBM_EINVAL, "NULL handle");
    if (!h->inited) return fail(SCLBM_ESTATE, "instance not initialised");
    if (n < 0) return fail(SCLBM_EINVAL, "n must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    for (int64_t k = 0; k < n; ++k) {
        const bool diag = h->d.diag_every > 0 && h->t % h->d.diag_every == 0;
        int nb = 0;
        int32_t rc = sweep(h, diag ? M_STEP_DIAG : M_STEP, h->stacked ? -h->cw : h->cw, h->W,
                           h->H, h->cur, 1 - h->cur, nullptr, st, &nb, h->stacked ? h->wt : 0);
        if (rc) return rc;
        if (diag) {
            hipError_t e = launch_reduce(reinterpret_cast<double*>(h->buf + h->L.off_partials),
                                         nb, reinterpret_cast<double*>(h->buf + h->L.off_diag),
                                         st);
            if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
            h->fused_step = h->t;
        }
        h->cur = 1 - h->cur;
        h->t += 1;
        if (h->d.boundary == SCLBM_WALLS_Y) h->wall_steps += 1;
    }
    return SCLBM_OK;
}

int32_t sclbm_set_tiling(sclbm_inst* h, const sclbm_tiling* tl)
{
    if (!h || !tl) return fail(SCLBM_EINVAL, "NULL argument");
    const int cw = tl->waves, W = tl->tile_x, H = tl->tile_y;
    if (tl->stacked != 0 && tl->stacked != 1) return fail(SCLBM_EINVAL, "stacked must be 0 or 1");
    if (tl->throttle != 0 && tl->throttle != 1) return fail(SCLBM_EINVAL, "throttle must be 0 or 1");
    if (tl->write_through != 0 && tl->write_through != 1)
        return fail(SCLBM_EINVAL, "write_through must be 0 or 1");
    if (tl->write_through && !tl->stacked)
        return fail(SCLBM_EINVAL, "write_through needs stacked tiles");
    if (tl->stacked) {
        if (cw != 4 && cw != 8) return fail(SCLBM_EINVAL, "stacked tiles need waves 4 or 8");
        if (H != cw) return fail(SCLBM_EINVAL, "stacked tiles need tile_y == waves");
        if (W > 60) return fail(SCLBM_EINVAL, "stacked tile_x %d > 60", W);
    } else {
        if (cw != 1 && cw != 2 && cw != 4) return fail(SCLBM_EINVAL, "waves must be 1, 2 or 4");
        if (W > 64 * cw - 4) return fail(SCLBM_EINVAL, "tile_x %d > 64*waves - 4", W);
        if (H < std::min(MIN_TILE_Y, h->d.ny)) return fail(SCLBM_EINVAL, "tile_y %d too small", H);
    }
    if (W < std::min(MIN_TILE_X, h->d.nx)) return fail(SCLBM_EINVAL, "tile_x %d too small", W);
    set_tiling(h, cw, W, H, tl->stacked, tl->throttle, tl->write_through);
    return SCLBM_OK;
}

int32_t sclbm_get_tiling(const sclbm_inst* h, sclbm_tiling* out)
{
    if (!h || !out) return fail(SCLBM_EINVAL, "NULL argument");
    out->tile_x = h->W;
    out->tile_y = h->H;
    out->waves = h->cw;
    out->stacked = h->stacked;
    out->throttle = h->throttle;
    out->write_through = h->wt;
    return SCLBM_OK;
}

int32_t sclbm_time(const sclbm_inst* h, int64_t* t)
{
    if (!h || !t) return fail(SCLBM_EINVAL, "NULL argument");
    *t = h->t;
    return SCLBM_OK;
}

int32_t sclbm_read_moments(sclbm_inst* h, double* rhoA, double* rhoB, double* ux, double* uy,
                           double* sxy, void* stream)
{
    if (!h) return fail(SCLBM_EINVAL, "NULL handle");
    if (!h->inited) return fail(SCLBM_ESTATE, "instance not initialised");
    double* out[5] = {rhoA, rhoB, ux, uy, sxy};
    return sweep(h, M_READ, RO_CW, RO_W, RO_H, h->cur, h->cur, out, (hipStream_t)stream,
                 nullptr);
}

int32_t sclbm_order_parameter(sclbm_inst* h, const double* phi_ref, double* phi_out,
                              double out[2], void* stream)
{
    if (!h || !out) return fail(SCLBM_EINVAL, "NULL argument");
    if (phi_ref && phi_ref == phi_out) return fail(SCLBM_EINVAL, "phi_ref aliases phi_out");
    if (!h->inited) return fail(SCLBM_ESTATE, "instance not initialised");
    hipStream_t st = (hipStream_t)stream;
    double* io[5] = {phi_out, const_cast<double*>(phi_ref), nullptr, nullptr, nullptr};
    int nb = 0;
    int32_t rc = sweep(h, M_PHI, RO_CW, RO_W, RO_H, h->cur, h->cur, io, st, &nb);
    if (rc) return rc;
    double* rec = reinterpret_cast<double*>(h->buf + h->L.off_diag) + NDIAG;
    hipError_t e = launch_reduce(reinterpret_cast<double*>(h->buf + h->L.off_partials), nb, rec, st);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
    double v[NDIAG];
    e = hipMemcpyAsync(v, rec, sizeof v, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "order parameter copy");
    out[0] = phi_ref ? v[0] : 0.0;
    out[1] = v[1];
    return SCLBM_OK;
}

int32_t sclbm_diagnostics(sclbm_inst* h, sclbm_diag* out, void* stream)
{
    if (!h || !out) return fail(SCLBM_EINVAL, "NULL argument");
    if (!h->inited) return fail(SCLBM_ESTATE, "instance not initialised");
    hipStream_t st = (hipStream_t)stream;
    int nb = 0;
    int32_t rc = sweep(h, M_DIAG, RO_CW, RO_W, RO_H, h->cur, h->cur, nullptr, st, &nb);
    if (rc) return rc;
    // on-demand record sits after the fused one
    double* rec = reinterpret_cast<double*>(h->buf + h->L.off_diag) + NDIAG;
    hipError_t e = launch_reduce(reinterpret_cast<double*>(h->buf + h->L.off_partials), nb, rec, st);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
    double v[NDIAG];
    e = hipMemcpyAsync(v, rec, sizeof v, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "diag copy");
    double* wall = nullptr;
    double wbuf_small[4 * 64];
    double* wbuf = h->d.nx <= 64 ? wbuf_small : new (std::nothrow) double[4 * (size_t)h->d.nx];
    if (!wbuf) return fail(SCLBM_EINVAL, "out of host memory");
    rc = read_wall(h, wbuf, st);
    if (!rc) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "stream sync");
    }
    if (!rc) {
        wall = wbuf;
        fill_diag(h, v, wall, out, h->t);
    }
    if (wbuf != wbuf_small) delete[] wbuf;
    if (rc) return rc;
    if (out->bad_sites > 0)
        return fail(SCLBM_ENONFINITE, "%lld sites with non-finite or non-positive density",
                    (long long)out->bad_sites);
    return SCLBM_OK;
}

int32_t sclbm_fused_diagnostics(sclbm_inst* h, sclbm_diag* out, void* stream)
{
    if (!h || !out) return fail(SCLBM_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    if (h->fused_step < 0) {
        memset(out, 0, sizeof *out);
        out->step = -1;
        return SCLBM_OK;
    }
    double v[NDIAG];
    hipError_t e = hipMemcpyAsync(v, h->buf + h->L.off_diag, sizeof v, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "diag copy");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    fill_diag(h, v, nullptr, out, h->fused_step);
    if (out->bad_sites > 0)
        return fail(SCLBM_ENONFINITE, "%lld sites with non-finite or non-positive density",
                    (long long)out->bad_sites);
    return SCLBM_OK;
}

int32_t sclbm_reset_wall_accum(sclbm_inst* h, void* stream)
{
    if (!h) return fail(SCLBM_EINVAL, "NULL handle");
    hipError_t e = hipMemsetAsync(h->buf + h->L.off_wall, 0, sizeof(double) * 4 * h->d.nx,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "wall reset");
    h->wall_steps = 0;
    return SCLBM_OK;
}

struct CkptHeader {
    uint64_t magic;
    int32_t nx, ny, boundary, storage;
    int64_t t;
    uint64_t pop_bytes;
};

size_t sclbm_checkpoint_bytes(const sclbm_inst* h)
{
    if (!h) return 0;
    return sizeof(CkptHeader) + h->L.pop_bytes;
}

int32_t sclbm_checkpoint(sclbm_inst* h, void* host_buf, size_t bytes, void* stream)
{
    if (!h || !host_buf) return fail(SCLBM_EINVAL, "NULL argument");
    if (!h->inited) return fail(SCLBM_ESTATE, "instance not initialised");
    if (bytes < sclbm_checkpoint_bytes(h)) return fail(SCLBM_ESIZE, "checkpoint buffer too small");
    CkptHeader hd{CKPT_MAGIC, h->d.nx, h->d.ny, h->d.boundary, h->d.storage, h->t,
                  (uint64_t)h->L.pop_bytes};
    memcpy(host_buf, &hd, sizeof hd);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(static_cast<char*>(host_buf) + sizeof hd, h->buf + h->L.off_f[h->cur],
                                  h->L.pop_bytes, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    return SCLBM_OK;
}

int32_t sclbm_restore(sclbm_inst* h, const void* host_buf, size_t bytes, void* stream)
{
    if (!h || !host_buf) return fail(SCLBM_EINVAL, "NULL argument");
    if (bytes < sizeof(CkptHeader)) return fail(SCLBM_ESIZE, "checkpoint too small");
    CkptHeader hd;
    memcpy(&hd, host_buf, sizeof hd);
    if (hd.magic != CKPT_MAGIC || hd.nx != h->d.nx || hd.ny != h->d.ny ||
        hd.boundary != h->d.boundary || hd.storage != h->d.storage ||
        hd.pop_bytes != (uint64_t)h->L.pop_bytes)
        return fail(SCLBM_EINVAL, "checkpoint does not match this instance");
    if (bytes < sizeof hd + h->L.pop_bytes) return fail(SCLBM_ESIZE, "checkpoint truncated");
    hipStream_t st = (hipStream_t)stream;
    h->cur = 0;
    hipError_t e = hipMemcpyAsync(h->buf + h->L.off_f[0], static_cast<const char*>(host_buf) + sizeof hd,
                                  h->L.pop_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "restore copy");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    h->t = hd.t;
    h->inited = true;
    h->fused_step = -1;
    return SCLBM_OK;
}


}  // extern "C"

// ------------------------------------------------------------------ batching

// Sleeps a workgroup waits at one grid barrier before it reports failure:
// seconds, far beyond any real wait.
constexpr uint32_t DEFAULT_SPIN_LIMIT = 1u << 26;

struct sclbm_batch {
    int n = 0, storage = 0, nitems = 0, grid = 0, kind = 0, capacity = 0;
    int mode = SCLBM_BATCH_PERSISTENT;
    uint32_t spin_limit = DEFAULT_SPIN_LIMIT;  // sleeps before a barrier gives up
    std::vector<sclbm_inst*> insts;
    std::vector<sclbm_tiling> tl;
    char* ws = nullptr;
    size_t inst_bytes = 0, off_items = 0, off_ctl = 0, total = 0;
    std::vector<char> host_insts;  // staging of the per-launch instance table
    hipEvent_t uploaded = nullptr;  // the staging buffer may be reused after it
};

namespace {

size_t batch_inst_size(int storage)
{
    switch (storage) {
    case SCLBM_F64: return sizeof(BatchInst<double, double>);
    case SCLBM_F32: return sizeof(BatchInst<float, float>);
    default: return sizeof(BatchInst<_Float16, float>);
    }
}

int32_t check_batch_tiling(const sclbm_inst* h, const sclbm_tiling& t)
{
    if ((t.throttle != 0 && t.throttle != 1) || t.write_through != 0)
        return fail(SCLBM_EINVAL, "batch tilings: throttle 0 or 1, write_through 0");
    if (t.waves != 4) return fail(SCLBM_EINVAL, "batch tilings need waves == 4");
    if (t.stacked) {
        if (t.tile_y != 4 || t.tile_x > 60)
            return fail(SCLBM_EINVAL, "stacked batch tiles are tile_x <= 60 by 4 rows");
    } else {
        if (t.tile_x > 252) return fail(SCLBM_EINVAL, "batch strips are at most 252 wide");
        if (t.tile_y < std::min(MIN_TILE_Y, h->d.ny)) return fail(SCLBM_EINVAL, "tile_y too small");
    }
    if (t.tile_x < std::min(MIN_TILE_X, h->d.nx)) return fail(SCLBM_EINVAL, "tile_x too small");
    return SCLBM_OK;
}

int32_t batch_layout(sclbm_inst* const* insts, int32_t n, const sclbm_tiling* tl,
                     size_t* inst_bytes, size_t* off_items, size_t* off_ctl, size_t* total,
                     int* nitems)
{
    if (!insts || !tl || n < 1) return fail(SCLBM_EINVAL, "empty batch or NULL arrays");
    const int storage = insts[0] ? insts[0]->d.storage : -1;
    int64_t items = 0;
    for (int k = 0; k < n; ++k) {
        const sclbm_inst* h = insts[k];
        if (!h) return fail(SCLBM_EINVAL, "instance %d is NULL", k);
        if (h->d.storage != storage) return fail(SCLBM_EINVAL, "mixed storage types in a batch");
        if (h->d.diag_every != 0) return fail(SCLBM_EUNSUPPORTED, "fused diagnostics in a batch");
        int32_t rc = check_batch_tiling(h, tl[k]);
        if (rc) return rc;
        items += (int64_t)((h->d.nx + tl[k].tile_x - 1) / tl[k].tile_x) *
                 ((h->d.ny + tl[k].tile_y - 1) / tl[k].tile_y);
    }
    if (items > (1 << 30)) return fail(SCLBM_ESIZE, "too many tiles");
    // one state stepped twice in one launch would race, and its time and
    // ping-pong copy would be advanced twice
    std::vector<const sclbm_inst*> seen(insts, insts + n);
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
        return fail(SCLBM_EINVAL, "the same instance appears twice in a batch");
    *inst_bytes = align_up(batch_inst_size(storage) * n, ALIGN);
    *off_items = *inst_bytes;
    *off_ctl = *off_items + align_up(sizeof(BatchItem) * (size_t)items, ALIGN);
    *total = *off_ctl + align_up(sizeof(BatchCtl), ALIGN);
    *nitems = (int)items;
    return SCLBM_OK;
}

template <class S, class A>
void fill_batch_inst(const sclbm_inst* h, const Coef<A>& c, const sclbm_tiling& t, int64_t steps,
                     void* dst)
{
    BatchInst<S, A> b{};
    b.I = make_inst<S, A>(h, c, h->cur, 1 - h->cur, t.tile_x, t.tile_y);
    b.I.throttle = t.throttle;
    b.steps = steps;
    b.stacked = t.stacked;
    memcpy(dst, &b, sizeof b);
}

}  // namespace

extern "C" {

size_t sclbm_batch_bytes(sclbm_inst* const* insts, int32_t n, const sclbm_tiling* tiling)
{
    size_t ib, oi, oc, total;
    int ni;
    if (batch_layout(insts, n, tiling, &ib, &oi, &oc, &total, &ni)) return 0;
    return total;
}

int32_t sclbm_batch_plan(sclbm_inst* const* insts, int32_t n, const sclbm_tiling* tiling,
                         void* dev_workspace, size_t bytes, void* stream, sclbm_batch** out)
{
    if (!out) return fail(SCLBM_EINVAL, "out is NULL");
    *out = nullptr;
    size_t ib, oi, oc, total;
    int ni;
    int32_t rc = batch_layout(insts, n, tiling, &ib, &oi, &oc, &total, &ni);
    if (rc) return rc;
    for (int k = 0; k < n; ++k)
        if (!insts[k]->inited) return fail(SCLBM_ESTATE, "instance %d not initialised", k);
    if (!dev_workspace || (uintptr_t)dev_workspace % ALIGN)
        return fail(SCLBM_EINVAL, "workspace NULL or not 256-byte aligned");
    if (bytes < total) return fail(SCLBM_ESIZE, "workspace of %zu bytes < %zu needed", bytes, total);
    const int storage = insts[0]->d.storage;
    int nstacked = 0;
    for (int k = 0; k < n; ++k) nstacked += tiling[k].stacked != 0;
    const int kind = nstacked == n ? B_STACKED : nstacked == 0 ? B_SWEEP : B_MIXED;
    const int grid = batch_grid(storage, kind);
    if (grid <= 0) return fail(SCLBM_EDEVICE, "cannot size the cooperative grid");
    sclbm_batch* b = new (std::nothrow) sclbm_batch();
    if (!b) return fail(SCLBM_EINVAL, "out of host memory");
    b->n = n;
    b->storage = storage;
    b->kind = kind;
    b->nitems = ni;
    b->capacity = grid;
    b->grid = std::min(grid, ni);
    b->insts.assign(insts, insts + n);
    b->tl.assign(tiling, tiling + n);
    b->ws = static_cast<char*>(dev_workspace);
    b->inst_bytes = ib;
    b->off_items = oi;
    b->off_ctl = oc;
    b->total = total;
    b->host_insts.resize(ib);
    // tile table: instance-major, each instance's tiles strip-major
    std::vector<BatchItem> items;
    items.reserve(ni);
    for (int k = 0; k < n; ++k) {
        const sclbm_inst* h = insts[k];
        const int ns = (h->d.nx + tiling[k].tile_x - 1) / tiling[k].tile_x;
        const int nc = (h->d.ny + tiling[k].tile_y - 1) / tiling[k].tile_y;
        for (int tt = 0; tt < ns * nc; ++tt) items.push_back(BatchItem{k, tt});
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(b->ws + oi, items.data(), sizeof(BatchItem) * items.size(),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // `items` is a local
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch plan upload");
    }
    *out = b;
    return SCLBM_OK;
}

int32_t sclbm_batch_step(sclbm_batch* b, const int64_t* steps, void* stream)
{
    if (!b || !steps) return fail(SCLBM_EINVAL, "NULL argument");
    int64_t max_steps = 0;
    for (int k = 0; k < b->n; ++k) {
        if (steps[k] < 0) return fail(SCLBM_EINVAL, "steps[%d] < 0", k);
        if (!b->insts[k]->inited) return fail(SCLBM_ESTATE, "instance %d not initialised", k);
        max_steps = std::max(max_steps, steps[k]);
    }
    if (max_steps == 0) return SCLBM_OK;
    hipStream_t st = (hipStream_t)stream;
    // the staging buffer of the previous launch must have been consumed
    hipError_t e = hipEventSynchronize(b->uploaded);
    if (e != hipSuccess) return hip_fail(e, "batch staging wait");
    const size_t isz = batch_inst_size(b->storage);
    for (int k = 0; k < b->n; ++k) {
        const sclbm_inst* h = b->insts[k];
        void* dst = b->host_insts.data() + isz * k;
        if (b->storage == SCLBM_F64)
            fill_batch_inst<double, double>(h, h->cd, b->tl[k], steps[k], dst);
        else if (b->storage == SCLBM_F32)
            fill_batch_inst<float, float>(h, h->cf, b->tl[k], steps[k], dst);
        else
            fill_batch_inst<_Float16, float>(h, h->cf, b->tl[k], steps[k], dst);
    }
    e = hipMemcpyAsync(b->ws, b->host_insts.data(), isz * b->n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(b->uploaded, st);
    if (e == hipSuccess) e = hipMemsetAsync(b->ws + b->off_ctl, 0, sizeof(BatchCtl), st);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
    const BatchItem* items = reinterpret_cast<const BatchItem*>(b->ws + b->off_items);
    if (b->mode == SCLBM_BATCH_STEPWISE) {
        for (int64_t s = 0; s < max_steps && e == hipSuccess; ++s)
            e = launch_batch_step(b->storage, b->kind, b->ws, items, b->nitems, s, st);
    } else {
        e = launch_batch(b->storage, b->kind, b->ws, items, b->nitems, max_steps,
                         reinterpret_cast<BatchCtl*>(b->ws + b->off_ctl), b->spin_limit,
                         b->grid, st);
    }
    if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
    for (int k = 0; k < b->n; ++k) {
        sclbm_inst* h = b->insts[k];
        h->t += steps[k];
        h->cur ^= (int)(steps[k] & 1);
        if (h->d.boundary == SCLBM_WALLS_Y) h->wall_steps += steps[k];
    }
    return SCLBM_OK;
}

int32_t sclbm_batch_set_mode(sclbm_batch* b, int32_t mode)
{
    if (!b) return fail(SCLBM_EINVAL, "NULL batch");
    if (mode != SCLBM_BATCH_PERSISTENT && mode != SCLBM_BATCH_STEPWISE)
        return fail(SCLBM_EINVAL, "unknown batch mode %d", mode);
    b->mode = mode;
    return SCLBM_OK;
}

int32_t sclbm_batch_set_barrier_limit(sclbm_batch* b, uint32_t sleeps)
{
    if (!b) return fail(SCLBM_EINVAL, "NULL batch");
    b->spin_limit = sleeps ? sleeps : DEFAULT_SPIN_LIMIT;
    return SCLBM_OK;
}

int32_t sclbm_batch_info(const sclbm_batch* b, int32_t out[3])
{
    if (!b || !out) return fail(SCLBM_EINVAL, "NULL argument");
    out[0] = b->capacity;
    out[1] = b->nitems;
    out[2] = b->kind;
    return SCLBM_OK;
}

int32_t sclbm_batch_status(sclbm_batch* b, void* stream)
{
    if (!b) return fail(SCLBM_EINVAL, "NULL batch");
    BatchCtl c;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&c, b->ws + b->off_ctl, sizeof c, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "batch status");
    if (c.err) return fail(SCLBM_EDEVICE, "batch grid barrier timed out; results invalid");
    return SCLBM_OK;
}

int32_t sclbm_batch_release(sclbm_batch* b)
{
    if (b) {
        if (b->uploaded) {
            (void)hipEventSynchronize(b->uploaded);
            (void)hipEventDestroy(b->uploaded);
        }
        delete b;
    }
    return SCLBM_OK;
}

}  // extern "C"

// ----------------------------------------------- allocation-free batch step
//
// The tables of sclbm_batch_step_static live in this static device array
// (one copy per GPU, held until the process ends).  In host code `scratch`
// names a host-side stand-in, not the device array: its device address is
// looked up with hipGetSymbolAddress once per device and only that address
// is passed to kernels or copies.
static __device__ __align__(256) char scratch[SCLBM_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu;                       // guards the two arrays below
char* g_scratch_dev[MAX_DEVICES] = {};        // device address of `scratch`, per device
alignas(256) char g_stage[SCLBM_STATIC_SCRATCH_BYTES];  // host staging of the tables

// Device address of `scratch` on the current device (looked up on the
// first call on that device).  Called with g_static_mu held.
int32_t static_scratch(char** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(SCLBM_EDEVICE, "device %d out of range", dev);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "static scratch address");
        if (!p) return fail(SCLBM_EDEVICE, "static scratch has no device address");
        g_scratch_dev[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_dev[dev];
    return SCLBM_OK;
}

}  // namespace

extern "C" int32_t sclbm_batch_step_static(sclbm_inst* const* insts, int32_t n,
                                           const sclbm_tiling* tiling, const int64_t* steps,
                                           void* stream)
{
    if (!steps) return fail(SCLBM_EINVAL, "steps is NULL");
    size_t ib, oi, oc, total;
    int ni;
    int32_t rc = batch_layout(insts, n, tiling, &ib, &oi, &oc, &total, &ni);
    if (rc) return rc;
    const size_t used = oi + sizeof(BatchItem) * (size_t)ni;  // no barrier state here
    if (used > SCLBM_STATIC_SCRATCH_BYTES)
        return fail(SCLBM_ESIZE, "batch tables of %zu bytes exceed the static scratch of %u bytes",
                    used, (unsigned)SCLBM_STATIC_SCRATCH_BYTES);
    int64_t max_steps = 0;
    for (int k = 0; k < n; ++k) {
        if (!insts[k]->inited) return fail(SCLBM_ESTATE, "instance %d not initialised", k);
        if (steps[k] < 0) return fail(SCLBM_EINVAL, "steps[%d] < 0", k);
        max_steps = std::max(max_steps, steps[k]);
    }
    if (max_steps == 0) return SCLBM_OK;
    const int storage = insts[0]->d.storage;
    int nstacked = 0;
    for (int k = 0; k < n; ++k) nstacked += tiling[k].stacked != 0;
    const int kind = nstacked == n ? B_STACKED : nstacked == 0 ? B_SWEEP : B_MIXED;
    hipStream_t st = (hipStream_t)stream;

    std::lock_guard<std::mutex> lock(g_static_mu);
    char* dev = nullptr;
    rc = static_scratch(&dev);
    if (rc) return rc;
    // tables in the static host stage, laid out as in a plan's workspace
    const size_t isz = batch_inst_size(storage);
    for (int k = 0; k < n; ++k) {
        const sclbm_inst* h = insts[k];
        void* dst = g_stage + isz * k;
        if (storage == SCLBM_F64)
            fill_batch_inst<double, double>(h, h->cd, tiling[k], steps[k], dst);
        else if (storage == SCLBM_F32)
            fill_batch_inst<float, float>(h, h->cf, tiling[k], steps[k], dst);
        else
            fill_batch_inst<_Float16, float>(h, h->cf, tiling[k], steps[k], dst);
    }
    BatchItem* items = reinterpret_cast<BatchItem*>(g_stage + oi);
    int m = 0;
    for (int k = 0; k < n; ++k) {
        const sclbm_inst* h = insts[k];
        const int ns = (h->d.nx + tiling[k].tile_x - 1) / tiling[k].tile_x;
        const int nc = (h->d.ny + tiling[k].tile_y - 1) / tiling[k].tile_y;
        for (int tt = 0; tt < ns * nc; ++tt) items[m++] = BatchItem{k, tt};
    }
    // one upload; the stage may be rewritten by the next call once it is done
    hipError_t e = hipMemcpyAsync(dev, g_stage, used, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "static batch upload");
    const BatchItem* ditems = reinterpret_cast<const BatchItem*>(dev + oi);
    for (int64_t s = 0; s < max_steps && e == hipSuccess; ++s)
        e = launch_batch_step(storage, kind, dev, ditems, ni, s, st);
    if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
    for (int k = 0; k < n; ++k) {
        sclbm_inst* h = insts[k];
        h->t += steps[k];
        h->cur ^= (int)(steps[k] & 1);
        if (h->d.boundary == SCLBM_WALLS_Y) h->wall_steps += steps[k];
    }
    return SCLBM_OK;
}
