// hbm_ceiling.hip -- what HBM bandwidth the step's memory access pattern can
// reach on this GPU, with no arithmetic: a plain 16-byte-per-lane copy, and
// the 18-plane pull of one lattice step (each plane read at the site shifted
// by its D2Q9 velocity, written in place, through raw buffer loads and
// stores) with 1..8 columns per lane and chunk heights of 4..256 rows, in
// 4-byte (FP32) and 2-byte (FP16) elements.  Prints one line per
// configuration and a JSON summary of the best rate of each pattern.
//
//     hbm_ceiling [side]      (default 4096: a DRAM-resident lattice)
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>

#define CK(x)                                                                         \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            exit(1);                                                                  \
        }                                                                             \
    } while (0)

constexpr int CXv[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CYv[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

template <int B> struct Vec;
template <> struct Vec<2> { typedef unsigned short T; };
template <> struct Vec<4> { typedef unsigned T; };
template <> struct Vec<8> { typedef unsigned T __attribute__((ext_vector_type(2))); };
template <> struct Vec<16> { typedef unsigned T __attribute__((ext_vector_type(4))); };

// Cache-policy bits of the buffer instructions (gfx950): 1 sc0, 2 nt, 16 sc1.
template <int B, int CP = 0>
__device__ __forceinline__ typename Vec<B>::T load(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (B == 2) return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, CP);
    else if constexpr (B == 4) return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, CP);
    else if constexpr (B == 8) return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CP);
    else return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CP);
}
template <int B, int CP = 0>
__device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t off, typename Vec<B>::T v)
{
    if constexpr (B == 2) __builtin_amdgcn_raw_buffer_store_b16(v, r, off, 0, CP);
    else if constexpr (B == 4) __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, CP);
    else if constexpr (B == 8) __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, CP);
    else __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, CP);
}

// ES-byte elements, V per lane; rows 0..ny+1 (ghost rows 0 and ny+1),
// columns at element offset 32 + x; a workgroup of 256 lanes sweeps H rows
// of a strip of 256 V columns, loading the next row before storing this one.
// SX: planes read with their column shift (the step's pattern) or without
// (every load aligned like the stores); LP / SP: cache policy of the loads /
// stores.
template <int ES, int V, bool SX = true, int LP = 0, int SP = 0>
__global__ __launch_bounds__(256) void pull18(const char* fin, char* fout, int nx, int ny, int pitch,
                                              int plane, int H, int nstrips)
{
    constexpr int B = ES * V;
    using T = typename Vec<B>::T;
    const int strip = blockIdx.x % nstrips, chunk = blockIdx.x / nstrips;
    const int x0 = (strip * 256 + (int)threadIdx.x) * V;
    const int nrec = 18 * plane * ES;
    const auto rin = __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(fin), (short)0, nrec, 0x00020000);
    const auto rout = __builtin_amdgcn_make_buffer_rsrc(fout, (short)0, nrec, 0x00020000);
    const bool act = x0 < nx;
    const int y0 = chunk * H, y1 = min(y0 + H, ny);
    T R[18], Q[18];
    auto ld = [&](int y, T* dst) {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const int i = k % 9;
            const uint32_t off =
                (uint32_t)(((y + 1 - CYv[i]) * pitch + 32 + x0 - (SX ? CXv[i] : 0) + k * plane) * ES);
            dst[k] = load<B, LP>(rin, act ? off : 0x80000000u);
        }
    };
    auto st = [&](int y, const T* src) {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const uint32_t off = (uint32_t)(((y + 1) * pitch + 32 + x0 + k * plane) * ES);
            store<B, SP>(rout, act ? off : 0x80000000u, src[k]);
        }
    };
    if (y0 < y1) ld(y0, R);
    int y = y0;
    for (; y + 2 <= y1; y += 2) {
        ld(y + 1, Q);
        st(y, R);
        if (y + 2 < y1) ld(y + 2, R);
        st(y + 1, Q);
    }
    if (y < y1) st(y, R);
}

// The same pull with the loads of the next TWO rows in flight while a row
// is stored (prefetch depth 2; pull18 keeps one row ahead).
template <int ES, int V>
__global__ __launch_bounds__(256) void pull18d2(const char* fin, char* fout, int nx, int ny, int pitch,
                                                int plane, int H, int nstrips)
{
    constexpr int B = ES * V;
    using T = typename Vec<B>::T;
    const int strip = blockIdx.x % nstrips, chunk = blockIdx.x / nstrips;
    const int x0 = (strip * 256 + (int)threadIdx.x) * V;
    const int nrec = 18 * plane * ES;
    const auto rin = __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(fin), (short)0, nrec, 0x00020000);
    const auto rout = __builtin_amdgcn_make_buffer_rsrc(fout, (short)0, nrec, 0x00020000);
    const bool act = x0 < nx;
    const int y0 = chunk * H, y1 = min(y0 + H, ny);
    T A[18], Bq[18], C[18];
    auto ld = [&](int y, T* dst) {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const int i = k % 9;
            const uint32_t off =
                (uint32_t)(((y + 1 - CYv[i]) * pitch + 32 + x0 - CXv[i] + k * plane) * ES);
            dst[k] = load<B>(rin, act ? off : 0x80000000u);
        }
    };
    auto st = [&](int y, const T* src) {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const uint32_t off = (uint32_t)(((y + 1) * pitch + 32 + x0 + k * plane) * ES);
            store<B>(rout, act ? off : 0x80000000u, src[k]);
        }
    };
    if (y0 < y1) ld(y0, A);
    if (y0 + 1 < y1) ld(y0 + 1, Bq);
    int y = y0;
    for (; y + 3 <= y1; y += 3) {
        if (y + 2 < y1) ld(y + 2, C);
        st(y, A);
        if (y + 3 < y1) ld(y + 3, A);
        st(y + 1, Bq);
        if (y + 4 < y1) ld(y + 4, Bq);
        st(y + 2, C);
    }
    if (y < y1) st(y, A);
    if (y + 1 < y1) st(y + 1, Bq);
}

__global__ __launch_bounds__(256) void copy16(const uint4* __restrict__ a, uint4* __restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        b[i] = a[i];
}

// Copy with U 16-byte loads in flight per lane before their stores, through
// buffer instructions with cache policies LP / SP; n16 16-byte words, the
// whole buffer < 2^31 bytes.
template <int U, int LP, int SP>
__global__ __launch_bounds__(256) void copy16u(const char* a, char* b, uint32_t n16)
{
    const auto ra = __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(a), (short)0, (int)(n16 * 16u), 0x00020000);
    const auto rb = __builtin_amdgcn_make_buffer_rsrc(b, (short)0, (int)(n16 * 16u), 0x00020000);
    const uint32_t stride = gridDim.x * 256u;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n16; i += U * stride) {
        Vec<16>::T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = i + u * stride;
            v[u] = load<16, LP>(ra, j < n16 ? j * 16u : 0x80000000u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = i + u * stride;
            store<16, SP>(rb, j < n16 ? j * 16u : 0x80000000u, v[u]);
        }
    }
}

template <int ES, int V>
double time_pull_d2(char* a, char* b, int nx, int ny, int pitch, int plane, int H)
{
    const int nstrips = (nx + 256 * V - 1) / (256 * V);
    const int nb = nstrips * ((ny + H - 1) / H);
    const int reps = nx <= 1024 ? 1000 : 20;
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    for (int k = 0; k < 3; ++k)
        hipLaunchKernelGGL((pull18d2<ES, V>), dim3(nb), dim3(256), 0, 0, a, b, nx, ny, pitch, plane, H, nstrips);
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0, 0));
    for (int k = 0; k < reps; ++k)
        hipLaunchKernelGGL((pull18d2<ES, V>), dim3(nb), dim3(256), 0, 0, (k & 1) ? b : a, (k & 1) ? a : b,
                           nx, ny, pitch, plane, H, nstrips);
    CK(hipEventRecord(e1, 0));
    CK(hipEventSynchronize(e1));
    float ms;
    CK(hipEventElapsedTime(&ms, e0, e1));
    CK(hipGetLastError());
    const double us = ms / reps * 1e3;
    const double tbs = 2.0 * 18 * nx * (double)ny * ES / (us * 1e-6) / 1e12;
    printf("pull18 prefetch depth 2, %d-byte elements, %d per lane, H=%3d, %6d workgroups: %8.2f us  %.3f TB/s\n",
           ES, V, H, nb, us, tbs);
    fflush(stdout);
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    return tbs;
}

template <int U, int LP, int SP>
double time_copyu(char* a, char* b, uint32_t n16, int grid, int reps, const char* tag)
{
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    for (int k = 0; k < 3; ++k)
        hipLaunchKernelGGL((copy16u<U, LP, SP>), dim3(grid), dim3(256), 0, 0, a, b, n16);
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0, 0));
    for (int k = 0; k < reps; ++k)
        hipLaunchKernelGGL((copy16u<U, LP, SP>), dim3(grid), dim3(256), 0, 0, a, b, n16);
    CK(hipEventRecord(e1, 0));
    CK(hipEventSynchronize(e1));
    float ms;
    CK(hipEventElapsedTime(&ms, e0, e1));
    CK(hipGetLastError());
    const double us = ms / reps * 1e3;
    const double tbs = 2.0 * n16 * 16.0 / (us * 1e-6) / 1e12;
    printf("copy%s, %5d workgroups: %8.2f us  %.3f TB/s\n", tag, grid, us, tbs);
    fflush(stdout);
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    return tbs;
}

struct Best {
    double tbs = 0;
    int v = 0, h = 0;
};

template <int ES, int V, bool SX = true, int LP = 0, int SP = 0>
double time_pull(char* a, char* b, int nx, int ny, int pitch, int plane, int H,
                 const char* tag = "")
{
    const int nstrips = (nx + 256 * V - 1) / (256 * V);
    const int nb = nstrips * ((ny + H - 1) / H);
    const int reps = nx <= 1024 ? 1000 : 20;
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    for (int k = 0; k < 3; ++k)
        hipLaunchKernelGGL((pull18<ES, V, SX, LP, SP>), dim3(nb), dim3(256), 0, 0, a, b, nx, ny, pitch, plane, H, nstrips);
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0, 0));
    for (int k = 0; k < reps; ++k)
        hipLaunchKernelGGL((pull18<ES, V, SX, LP, SP>), dim3(nb), dim3(256), 0, 0, (k & 1) ? b : a, (k & 1) ? a : b,
                           nx, ny, pitch, plane, H, nstrips);
    CK(hipEventRecord(e1, 0));
    CK(hipEventSynchronize(e1));
    float ms;
    CK(hipEventElapsedTime(&ms, e0, e1));
    CK(hipGetLastError());
    const double us = ms / reps * 1e3;
    const double tbs = 2.0 * 18 * nx * (double)ny * ES / (us * 1e-6) / 1e12;
    printf("pull18%s %d-byte elements, %d per lane, H=%3d, %6d workgroups: %8.2f us  %.3f TB/s\n", tag,
           ES, V, H, nb, us, tbs);
    fflush(stdout);
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    return tbs;
}

template <int ES, int V>
void sweep(Best& best, char* a, char* b, int nx, int ny, int pitch, int plane)
{
    for (int H : {4, 8, 16, 32, 64, 128, 256}) {
        if (H > ny) break;
        const double t = time_pull<ES, V>(a, b, nx, ny, pitch, plane, H);
        if (t > best.tbs) best = Best{t, V, H};
    }
}

int main(int argc, char** argv)
{
    const int nx = argc > 1 ? atoi(argv[1]) : 4096;
    if (nx < 256 || nx > 8192 || nx % 2048 != 0 && nx != 512 && nx != 1024) {
        fprintf(stderr, "side must be 512, 1024 or a multiple of 2048 up to 8192\n");
        return 2;
    }
    const int ny = nx, pitch = nx + 64;
    const int plane = pitch * (ny + 2) + 64;
    const size_t bytes = (size_t)18 * plane * 4 + 4096;  // both element sizes fit
    if (bytes >= (size_t)1 << 31) {
        fprintf(stderr, "lattice too large for 32-bit buffer offsets\n");
        return 2;
    }
    char *a, *b;
    CK(hipMalloc(&a, bytes));
    CK(hipMalloc(&b, bytes));
    CK(hipMemset(a, 0, bytes));
    CK(hipMemset(b, 0, bytes));
    // plain copy of the FP32 lattice's bytes
    double copy_best = 0;
    {
        const size_t n = (size_t)18 * plane * 4 / 16;
        const int reps = nx <= 1024 ? 1000 : 20;
        hipEvent_t e0, e1;
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        for (int g : {512, 1024, 2048, 4096, 8192}) {
            for (int k = 0; k < 3; ++k)
                hipLaunchKernelGGL(copy16, dim3(g), dim3(256), 0, 0, (const uint4*)a, (uint4*)b, n);
            CK(hipDeviceSynchronize());
            CK(hipEventRecord(e0, 0));
            for (int k = 0; k < reps; ++k)
                hipLaunchKernelGGL(copy16, dim3(g), dim3(256), 0, 0, (const uint4*)a, (uint4*)b, n);
            CK(hipEventRecord(e1, 0));
            CK(hipEventSynchronize(e1));
            float ms;
            CK(hipEventElapsedTime(&ms, e0, e1));
            const double us = ms / reps * 1e3;
            const double tbs = 2.0 * n * 16 / (us * 1e-6) / 1e12;
            if (tbs > copy_best) copy_best = tbs;
            printf("copy 16 bytes per lane, %5d workgroups: %8.2f us  %.3f TB/s\n", g, us, tbs);
            fflush(stdout);
        }
        CK(hipEventDestroy(e0));
        CK(hipEventDestroy(e1));
    }
    Best f32, f16;
    sweep<4, 1>(f32, a, b, nx, ny, pitch, plane);
    sweep<4, 2>(f32, a, b, nx, ny, pitch, plane);
    sweep<4, 4>(f32, a, b, nx, ny, pitch, plane);
    sweep<2, 1>(f16, a, b, nx, ny, pitch, plane);
    sweep<2, 2>(f16, a, b, nx, ny, pitch, plane);
    sweep<2, 4>(f16, a, b, nx, ny, pitch, plane);
    sweep<2, 8>(f16, a, b, nx, ny, pitch, plane);
    // variants: copies with several loads in flight and cache policies; the
    // pull without column shifts (aligned loads) and with cache policies
    const int reps = nx <= 1024 ? 1000 : 20;
    const uint32_t n16 = (uint32_t)((size_t)18 * plane * 4 / 16);
    double vc[6] = {0, 0, 0, 0, 0, 0};
    for (int g : {1024, 2048, 4096}) {
        vc[0] = fmax(vc[0], time_copyu<1, 0, 0>(a, b, n16, g, reps, " buffer 1 in flight"));
        vc[1] = fmax(vc[1], time_copyu<4, 0, 0>(a, b, n16, g, reps, " buffer 4 in flight"));
        vc[2] = fmax(vc[2], time_copyu<4, 2, 2>(a, b, n16, g, reps, " buffer 4 in flight, nt loads+stores"));
        vc[3] = fmax(vc[3], time_copyu<4, 0, 2>(a, b, n16, g, reps, " buffer 4 in flight, nt stores"));
        vc[4] = fmax(vc[4], time_copyu<4, 0, 16>(a, b, n16, g, reps, " buffer 4 in flight, sc1 stores"));
        vc[5] = fmax(vc[5], time_copyu<8, 0, 0>(a, b, n16, g, reps, " buffer 8 in flight"));
    }
    double vp[10];
    vp[0] = time_pull<4, 1, false>(a, b, nx, ny, pitch, plane, 4, " aligned");
    vp[1] = time_pull<4, 1, true, 0, 2>(a, b, nx, ny, pitch, plane, 4, " nt stores");
    vp[2] = time_pull<4, 1, true, 0, 16>(a, b, nx, ny, pitch, plane, 4, " sc1 stores");
    vp[3] = time_pull<4, 1, true, 2, 2>(a, b, nx, ny, pitch, plane, 4, " nt loads+stores");
    vp[4] = time_pull<4, 1, false, 0, 2>(a, b, nx, ny, pitch, plane, 4, " aligned, nt stores");
    vp[5] = time_pull<2, 1, false>(a, b, nx, ny, pitch, plane, 4, " aligned");
    vp[6] = time_pull<2, 1, true, 0, 2>(a, b, nx, ny, pitch, plane, 4, " nt stores");
    vp[7] = time_pull<2, 1, true, 0, 16>(a, b, nx, ny, pitch, plane, 4, " sc1 stores");
    vp[8] = time_pull<2, 8, true, 0, 2>(a, b, nx, ny, pitch, plane, 4, " nt stores");
    vp[9] = time_pull<4, 1, true, 0, 0>(a, b, nx, ny, pitch, plane, 4, " (again)");
    // prefetch depth 2 at the long chunks a sweep uses (one row ahead: the
    // pull18 lines of the sweep above at the same H)
    double d2[6];
    d2[0] = time_pull_d2<4, 1>(a, b, nx, ny, pitch, plane, 64);
    d2[1] = time_pull_d2<4, 1>(a, b, nx, ny, pitch, plane, 128);
    d2[2] = time_pull_d2<4, 1>(a, b, nx, ny, pitch, plane, 256);
    d2[3] = time_pull_d2<2, 1>(a, b, nx, ny, pitch, plane, 64);
    d2[4] = time_pull_d2<2, 1>(a, b, nx, ny, pitch, plane, 128);
    d2[5] = time_pull_d2<2, 1>(a, b, nx, ny, pitch, plane, 256);
    printf("{\"side\": %d, \"copy_TBps\": %.3f, \"pull_f32_TBps\": %.3f, \"pull_f32_best\": [%d, %d], "
           "\"pull_f16_TBps\": %.3f, \"pull_f16_best\": [%d, %d], "
           "\"copy_buffer\": {\"u1\": %.3f, \"u4\": %.3f, \"u4_nt\": %.3f, \"u4_nt_store\": %.3f, "
           "\"u4_sc1_store\": %.3f, \"u8\": %.3f}, "
           "\"pull_h4\": {\"f32_aligned\": %.3f, \"f32_nt_store\": %.3f, \"f32_sc1_store\": %.3f, "
           "\"f32_nt\": %.3f, \"f32_aligned_nt_store\": %.3f, \"f16_aligned\": %.3f, "
           "\"f16_nt_store\": %.3f, \"f16_sc1_store\": %.3f, \"f16x8_nt_store\": %.3f, "
           "\"f32_again\": %.3f}, \"depth2_f32_h64_128_256\": [%.3f, %.3f, %.3f], "
           "\"depth2_f16_h64_128_256\": [%.3f, %.3f, %.3f]}\n",
           nx, copy_best, f32.tbs, f32.v, f32.h, f16.tbs, f16.v, f16.h, vc[0], vc[1], vc[2], vc[3],
           vc[4], vc[5], vp[0], vp[1], vp[2], vp[3], vp[4], vp[5], vp[6], vp[7], vp[8], vp[9],
           d2[0], d2[1], d2[2], d2[3], d2[4], d2[5]);
    CK(hipFree(a));
    CK(hipFree(b));
    return 0;
}
