// lbm_adjoint_force_noalloc (include/lbm.h): the adjoint call with its workspace
// in a file-scope device array instead of a caller allocation, for callers that
// cannot allocate device memory.
//
// In host code the array's name is only a host-side stand-in; its device address
// is taken once per device with hipGetSymbolAddress (with that device current)
// and kept in g_scratch, and only that address is ever handed to HIP.  Every call
// on a device shares the device's array: calls that overlap on one device race,
// and each call clears what must start at zero itself (the adjoint driver does).
#include <hip/hip_runtime.h>

#include <mutex>

#include "lbm_ctx.h"

namespace {

constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[LBM_ADJOINT_SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};

// Device address of the scratch array on `dev` (looked up on the first call).
lbm_status scratch_on(lbm_ctx *c, int dev, void **out)
{
    if (dev < 0 || dev >= MAX_DEVICES)
        return c->fail(LBM_E_DEVICE, "lbm_adjoint_force_noalloc: device ordinal %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess)
            return c->fail(LBM_E_DEVICE, "lbm_adjoint_force_noalloc: hipGetDevice failed");
        if (cur != dev && hipSetDevice(dev) != hipSuccess)
            return c->fail(LBM_E_DEVICE, "lbm_adjoint_force_noalloc: hipSetDevice(%d) failed", dev);
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return c->fail(LBM_E_DEVICE, "lbm_adjoint_force_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

}  // namespace

extern "C" lbm_status lbm_adjoint_force_noalloc(lbm_ctx *c, int64_t nsteps, int32_t ckpt_every, int32_t obj,
                                                double dir_x, double dir_y, double *J, double *dJ_duin,
                                                double *dJ_dq, double *dJ_duw, double *dJ_dstate,
                                                double *dJ_dinit)
{
    if (!c) return LBM_E_ARG;
    const size_t need = lbm_adjoint_workspace_bytes(c, nsteps, ckpt_every);
    if (need == 0)
        return c->fail(LBM_E_ARG, "lbm_adjoint_force_noalloc: invalid arguments, storage, layout, collision, "
                                  "force form or scheme, or no geometry");
    if (need > (size_t)LBM_ADJOINT_SCRATCH_BYTES)
        return c->fail(LBM_E_NOMEM,
                       "lbm_adjoint_force_noalloc: needs %zu bytes of scratch, more than the static %zu "
                       "(use lbm_adjoint_force with a caller workspace, or fewer steps per checkpoint)",
                       need, (size_t)LBM_ADJOINT_SCRATCH_BYTES);
    void *ws = nullptr;
    lbm_status s = scratch_on(c, c->p.device, &ws);
    if (s) return s;
    return lbm_host::adjoint_force_impl(c, ws, (size_t)LBM_ADJOINT_SCRATCH_BYTES, nsteps, ckpt_every, obj, dir_x,
                                        dir_y, J, dJ_duin, dJ_dq, dJ_duw, dJ_dstate, dJ_dinit, true,
                                        lbm_host::ADJ_BOTH);
}
