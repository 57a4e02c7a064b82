// sclbm_dispatch.cpp -- storage-type dispatch of the kernel launchers of
// libsclbm.so.  The kernels of each storage type live in their own
// compilation unit (sclbm_kernels.hip built with -DSCLBM_STORAGE=k).
#include "sclbm_internal.h"

namespace sclbm {

#define SCLBM_DISPATCH(storage, call)          \
    switch (storage) {                         \
    case 0: return call(0);                    \
    case 1: return call(1);                    \
    case 2: return call(2);                    \
    case 3: return call(3);                    \
    }

hipError_t launch_sweep(int storage, int cw, int wt, int mode, const void* inst, int nb,
                        hipStream_t st)
{
    // the walls flag lives in the Geo at the same offset for every storage type
    const int walls = static_cast<const Inst<float, float>*>(inst)->g.walls;
#define CALL(k) launch_sweep_s##k(cw, wt, walls, mode, inst, nb, st)
    SCLBM_DISPATCH(storage, CALL)
#undef CALL
    return hipErrorInvalidValue;
}

int batch_grid(int storage, int kind)
{
#define CALL(k) batch_grid_s##k(kind)
    SCLBM_DISPATCH(storage, CALL)
#undef CALL
    return 0;
}

hipError_t launch_batch(int storage, int kind, const void* insts, const BatchItem* items,
                        int nitems, int64_t max_steps, BatchCtl* ctl, uint32_t spin_limit,
                        int grid, hipStream_t st)
{
#define CALL(k) launch_batch_s##k(kind, insts, items, nitems, max_steps, ctl, spin_limit, grid, st)
    SCLBM_DISPATCH(storage, CALL)
#undef CALL
    return hipErrorInvalidValue;
}

hipError_t launch_batch_step(int storage, int kind, const void* insts, const BatchItem* items,
                             int nitems, int64_t s, hipStream_t st)
{
#define CALL(k) launch_batch_step_s##k(kind, insts, items, nitems, s, st)
    SCLBM_DISPATCH(storage, CALL)
#undef CALL
    return hipErrorInvalidValue;
}

hipError_t launch_init(int storage, const void* inst, const double* rA, const double* rB,
                       const double* ux, const double* uy, int random, uint64_t seed,
                       double mA, double mB, double amp, hipStream_t st)
{
#define CALL(k) launch_init_s##k(inst, rA, rB, ux, uy, random, seed, mA, mB, amp, st)
    SCLBM_DISPATCH(storage, CALL)
#undef CALL
    return hipErrorInvalidValue;
}

}  // namespace sclbm
