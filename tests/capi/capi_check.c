/*
 * capi_check.c -- drives libsclbm.so through its C ABI alone: no Python, no
 * torch.  The caller owns the device memory (hipMalloc), binds a lattice,
 * initialises it from the seeded generator, steps it, reads the moments
 * back and checks them against the library's own FP64 totals, the time
 * counter, two error paths and a checkpoint round trip.  Prints "ok" and
 * exits 0 on success; any failure prints its reason and exits 1.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "sclbm.h"

#define FAIL(...)                             \
    do {                                      \
        fprintf(stderr, "capi_check: ");      \
        fprintf(stderr, __VA_ARGS__);         \
        fprintf(stderr, "\n");                \
        return 1;                             \
    } while (0)
#define CHECK(call)                                                                 \
    do {                                                                            \
        int32_t rc_ = (call);                                                       \
        if (rc_ != SCLBM_OK)                                                        \
            FAIL("%s: %s (%s)", #call, sclbm_strerror(rc_), sclbm_last_error());   \
    } while (0)
#define CHECK_HIP(call)                                                             \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) FAIL("%s: %s", #call, hipGetErrorString(e_));       \
    } while (0)

static int read_rho(sclbm_inst* h, double* dA, double* dB, double* hA, double* hB, size_t n)
{
    CHECK(sclbm_read_moments(h, dA, dB, NULL, NULL, NULL, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    CHECK_HIP(hipMemcpy(hA, dA, n * sizeof(double), hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(hB, dB, n * sizeof(double), hipMemcpyDeviceToHost));
    return 0;
}

int main(void)
{
    if (sclbm_abi_version() != SCLBM_ABI_VERSION) FAIL("ABI version mismatch");
    sclbm_desc d;
    memset(&d, 0, sizeof d);
    d.nx = 96;
    d.ny = 80;
    d.boundary = SCLBM_PERIODIC;
    d.storage = SCLBM_F32;
    d.tau[0] = d.tau[1] = 1.0;
    d.G_a[0] = -12.55;
    d.G_a[1] = -11.80;
    d.G_r[0] = 11.70;
    d.G_r[1] = 10.95;
    d.G_x = 0.58;
    d.rho0 = 0.70;
    d.psi_amp = 0.70;
    d.forcing = SCLBM_FORCING_SHIFT;
    const size_t n = (size_t)d.nx * d.ny;

    const size_t bytes = sclbm_state_bytes(&d);
    if (bytes == 0) FAIL("state_bytes: %s", sclbm_last_error());
    void* buf = NULL;
    double *dA = NULL, *dB = NULL;
    CHECK_HIP(hipMalloc(&buf, bytes));
    CHECK_HIP(hipMalloc((void**)&dA, n * sizeof(double)));
    CHECK_HIP(hipMalloc((void**)&dB, n * sizeof(double)));
    double* hA = malloc(n * sizeof(double));
    double* hB = malloc(n * sizeof(double));
    double* hA2 = malloc(n * sizeof(double));
    double* hB2 = malloc(n * sizeof(double));
    if (!hA || !hB || !hA2 || !hB2) FAIL("host allocation");

    sclbm_inst* h = NULL;
    CHECK(sclbm_bind(&d, buf, bytes, &h));
    sclbm_inst* h2 = NULL;
    if (sclbm_bind(&d, buf, 16, &h2) != SCLBM_ESIZE || h2) FAIL("short buffer not refused");

    const double mean[2] = {0.7, 0.7};
    CHECK(sclbm_init_random(h, 1234, mean, 0.05, NULL));
    sclbm_diag d0, d1;
    CHECK(sclbm_diagnostics(h, &d0, NULL));
    CHECK(sclbm_step(h, 200, NULL));
    if (sclbm_step(h, -1, NULL) != SCLBM_EINVAL) FAIL("negative step count not refused");
    CHECK(sclbm_diagnostics(h, &d1, NULL));
    int64_t t = -1;
    CHECK(sclbm_time(h, &t));
    if (t != 200 || d1.step != 200) FAIL("time %lld, diagnostics step %lld", (long long)t,
                                         (long long)d1.step);
    for (int s = 0; s < 2; ++s)
        if (fabs(d1.mass[s] / d0.mass[s] - 1.0) > 1e-5) FAIL("mass drift species %d", s);
    if (d1.bad_sites != 0) FAIL("bad sites");

    /* moments read back through caller device arrays match the FP64 totals */
    if (read_rho(h, dA, dB, hA, hB, n)) return 1;
    double mA = 0.0, mB = 0.0;
    for (size_t k = 0; k < n; ++k) {
        mA += hA[k];
        mB += hB[k];
    }
    if (fabs(mA / d1.mass[0] - 1.0) > 1e-12 || fabs(mB / d1.mass[1] - 1.0) > 1e-12)
        FAIL("moments and totals disagree: %.17g vs %.17g", mA, d1.mass[0]);

    /* checkpoint, step 50, restore, step 50 again: the same bits */
    const size_t cb = sclbm_checkpoint_bytes(h);
    void* cp = malloc(cb);
    if (!cp) FAIL("checkpoint allocation");
    CHECK(sclbm_checkpoint(h, cp, cb, NULL));
    CHECK(sclbm_step(h, 50, NULL));
    if (read_rho(h, dA, dB, hA, hB, n)) return 1;
    CHECK(sclbm_restore(h, cp, cb, NULL));
    CHECK(sclbm_time(h, &t));
    if (t != 200) FAIL("restored time %lld", (long long)t);
    CHECK(sclbm_step(h, 50, NULL));
    if (read_rho(h, dA, dB, hA2, hB2, n)) return 1;
    if (memcmp(hA, hA2, n * sizeof(double)) || memcmp(hB, hB2, n * sizeof(double)))
        FAIL("checkpoint round trip changed the result");

    CHECK(sclbm_release(h));
    free(cp);
    free(hA);
    free(hB);
    free(hA2);
    free(hB2);
    CHECK_HIP(hipFree(dA));
    CHECK_HIP(hipFree(dB));
    CHECK_HIP(hipFree(buf));
    printf("capi_check: ok (96x80 FP32, 250 steps, mass drift %.2e %.2e)\n",
           fabs(d1.mass[0] / d0.mass[0] - 1.0), fabs(d1.mass[1] / d0.mass[1] - 1.0));
    return 0;
}
