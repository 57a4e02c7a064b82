// sclbm_batch.cpp -- batched persistent launch (placeholder until the batch
// kernel lands): every entry point reports SCLBM_EUNSUPPORTED.
#include "sclbm.h"

extern "C" {

size_t sclbm_batch_bytes(sclbm_inst* const*, int32_t, const sclbm_tiling*) { return 0; }

int32_t sclbm_batch_plan(sclbm_inst* const*, int32_t, const sclbm_tiling*, void*, size_t, void*,
                         sclbm_batch** out)
{
    if (out) *out = nullptr;
    return SCLBM_EUNSUPPORTED;
}

int32_t sclbm_batch_step(sclbm_batch*, const int64_t*, void*) { return SCLBM_EUNSUPPORTED; }

int32_t sclbm_batch_release(sclbm_batch*) { return SCLBM_OK; }
}
