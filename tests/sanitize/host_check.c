/*
 * host_check.c -- runs the host side of libsclbm.so under AddressSanitizer
 * and UndefinedBehaviorSanitizer, on every path that does no device work:
 * descriptor validation and state sizes, binding (to an address the library
 * never dereferences without a launch), tilings, the time counter,
 * checkpoint sizes and header checks, batch sizing and its refusals (mixed
 * storage, repeated instance, oversized static tables), the index
 * self-test and the error strings.  Prints "ok" and exits 0 on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sclbm.h"

#define FAIL(...)                              \
    do {                                       \
        fprintf(stderr, "host_check: ");       \
        fprintf(stderr, __VA_ARGS__);          \
        fprintf(stderr, "\n");                 \
        exit(1);                               \
    } while (0)
#define EXPECT(call, want)                                                            \
    do {                                                                              \
        int32_t rc_ = (call);                                                         \
        if (rc_ != (want))                                                            \
            FAIL("%s returned %d (%s), expected %d", #call, rc_, sclbm_last_error(),  \
                 (want));                                                              \
    } while (0)

static sclbm_desc desc(int nx, int ny, int storage, int boundary)
{
    sclbm_desc d;
    memset(&d, 0, sizeof d);
    d.nx = nx;
    d.ny = ny;
    d.storage = storage;
    d.boundary = boundary;
    d.tau[0] = d.tau[1] = 1.0;
    d.G_a[0] = -12.55;
    d.G_a[1] = -11.80;
    d.G_r[0] = 11.70;
    d.G_r[1] = 10.95;
    d.G_x = 0.58;
    d.rho0 = d.psi_amp = 0.7;
    d.rho_ref[0] = d.rho_ref[1] = 0.7;
    return d;
}

int main(void)
{
    if (sclbm_selftest() != 0) FAIL("index self-test");
    for (int32_t s = -8; s <= 1; ++s)
        if (!sclbm_strerror(s) || !*sclbm_strerror(s)) FAIL("strerror %d", s);
    /* invalid descriptors */
    sclbm_desc d = desc(0, 10, SCLBM_F32, SCLBM_PERIODIC);
    if (sclbm_state_bytes(&d) != 0) FAIL("nx = 0 accepted");
    d = desc(10, 10, 7, SCLBM_PERIODIC);
    if (sclbm_state_bytes(&d) != 0) FAIL("storage 7 accepted");
    d = desc(10, 1, SCLBM_F32, SCLBM_WALLS_Y);
    if (sclbm_state_bytes(&d) != 0) FAIL("walls with ny = 1 accepted");
    d = desc(50000, 50000, SCLBM_F64, SCLBM_PERIODIC);
    if (sclbm_state_bytes(&d) != 0) FAIL("oversized lattice accepted");
    if (sclbm_state_bytes(NULL) != 0) FAIL("NULL desc accepted");
    /* bind and host-only calls, every storage and boundary */
    sclbm_inst* h[8];
    int k = 0;
    for (int st = 0; st < 4; ++st)
        for (int b = 0; b < 2; ++b, ++k) {
            d = desc(70 + 13 * k, 33 + 7 * k, st, b);
            size_t need = sclbm_state_bytes(&d);
            if (need == 0) FAIL("state bytes %d", k);
            void* fake = (void*)(uintptr_t)((uint64_t)(k + 1) << 36);
            EXPECT(sclbm_bind(&d, fake, need - 1, &h[k]), SCLBM_ESIZE);
            EXPECT(sclbm_bind(&d, fake, need, &h[k]), SCLBM_OK);
            EXPECT(sclbm_step(h[k], 1, NULL), SCLBM_ESTATE);
            sclbm_tiling t;
            EXPECT(sclbm_get_tiling(h[k], &t), SCLBM_OK);
            sclbm_tiling bad = {61, 8, 8, 1, 0, 0};
            EXPECT(sclbm_set_tiling(h[k], &bad), SCLBM_EINVAL);
            sclbm_tiling good = {40, 8, 2, 0, 1, 0};
            EXPECT(sclbm_set_tiling(h[k], &good), SCLBM_OK);
            int64_t tm = -1;
            EXPECT(sclbm_time(h[k], &tm), SCLBM_OK);
            if (tm != 0) FAIL("time %lld", (long long)tm);
            if (sclbm_checkpoint_bytes(h[k]) == 0) FAIL("checkpoint bytes");
            char junk[64];
            memset(junk, 0, sizeof junk);
            EXPECT(sclbm_restore(h[k], junk, sizeof junk, NULL), SCLBM_EINVAL);
        }
    /* batches: sizing and refusals */
    sclbm_tiling tl[3] = {{60, 4, 4, 1, 0, 0}, {60, 4, 4, 1, 0, 0}, {60, 4, 4, 1, 0, 0}};
    sclbm_inst* two[2] = {h[2], h[3]};       /* both FP32 */
    if (sclbm_batch_bytes(two, 2, tl) == 0) FAIL("batch bytes: %s", sclbm_last_error());
    sclbm_inst* mixed[2] = {h[0], h[2]};
    if (sclbm_batch_bytes(mixed, 2, tl) != 0) FAIL("mixed storage accepted");
    sclbm_inst* rep[2] = {h[2], h[2]};
    if (sclbm_batch_bytes(rep, 2, tl) != 0) FAIL("repeated instance accepted");
    int64_t steps[3] = {1, 1, 1};
    EXPECT(sclbm_batch_step_static(rep, 2, tl, steps, NULL), SCLBM_EINVAL);
    EXPECT(sclbm_batch_step_static(two, 2, tl, NULL, NULL), SCLBM_EINVAL);
    EXPECT(sclbm_batch_step_static(two, 2, tl, steps, NULL), SCLBM_ESTATE);
    d = desc(8192, 4096, SCLBM_F16DEV, SCLBM_PERIODIC);
    sclbm_inst* big[3];
    for (int j = 0; j < 3; ++j) {
        void* fake = (void*)(uintptr_t)((uint64_t)(j + 20) << 36);
        EXPECT(sclbm_bind(&d, fake, sclbm_state_bytes(&d), &big[j]), SCLBM_OK);
    }
    sclbm_tiling small[3] = {{32, 4, 4, 1, 0, 0}, {32, 4, 4, 1, 0, 0}, {32, 4, 4, 1, 0, 0}};
    EXPECT(sclbm_batch_step_static(big, 3, small, steps, NULL), SCLBM_ESIZE);
    for (int j = 0; j < 3; ++j) EXPECT(sclbm_release(big[j]), SCLBM_OK);
    for (int j = 0; j < 8; ++j) EXPECT(sclbm_release(h[j]), SCLBM_OK);
    EXPECT(sclbm_release(NULL), SCLBM_OK);
    printf("ok\n");
    return 0;
}
