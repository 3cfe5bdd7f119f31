// One storage format's launch helpers of the step kernels (lbm_step_kernels.h).
// This file is compiled once per format with -DLBM_ST=0..5; the per-format
// objects build in parallel and lbm_dispatch.cpp picks the one of a context's
// storage.
#include "lbm_step_kernels.h"

#ifndef LBM_ST
#error "compile with -DLBM_ST=<storage format 0..5>"
#endif

#define LBM_CAT_(a, b) a##b
#define LBM_CAT(a, b) LBM_CAT_(a, b)
#define LBM_FN(f) LBM_CAT(f, LBM_ST)

namespace lbm {

hipError_t LBM_FN(launch_bulk_st)(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                                  const void *uin, const Side &side, double *zb, int32_t nz, const BulkConfig &cf,
                                  hipStream_t s, const ForceReduce &fr)
{
    return bulk_dispatch<LBM_ST>(g, ph, A, B, mask, uin, side, zb, nz, cf, s, fr);
}

hipError_t LBM_FN(launch_bulk_fused_st)(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                                        const void *uin, const Side &side, const FuseArgs &fa, double *zb,
                                        int32_t nz, const BulkConfig &cf, hipStream_t s)
{
    return bulk_fused_dispatch<LBM_ST>(g, ph, A, B, mask, uin, side, fa, zb, nz, cf, s);
}

hipError_t LBM_FN(launch_bulk_batch_st)(const BatchInst *insts, const BatchTile *tiles, int64_t ntiles,
                                        const Phys &ph, const void *A, void *B, const mask_t *mask, const void *uin,
                                        const Side &side, double *zb, int32_t nz, bool open, bool force, bool ss,
                                        int rows, hipStream_t s, const ForceReduce &fr)
{
    return bulk_batch_dispatch<LBM_ST>(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, open, force, ss,
                                       rows, s, fr);
}

#if LBM_ST != 4 && LBM_ST != 5
hipError_t LBM_FN(launch_link_st)(const Grid &g, const Phys &ph, const Links &L, const Side &side,
                                  const Reduce &red, double *bank, double *fsum, int block, hipStream_t s,
                                  ForceReduce *defer)
{
    return link_t<LBM_ST>(g, ph, L, side, red, bank, fsum, block, s, defer);
}

hipError_t LBM_FN(launch_refresh_st)(const Grid &g, const Phys &ph, const void *A, const Side &side, bool moments,
                                     hipStream_t s)
{
    return refresh_t<LBM_ST>(g, ph, A, side, moments, s);
}

hipError_t LBM_FN(launch_init_st)(const Grid &g, const Phys &ph, void *A, const mask_t *mask, const double *stage,
                                  int32_t y0, int32_t rows, hipStream_t s)
{
    return init_t<LBM_ST>(g, ph, A, mask, stage, y0, rows, s);
}

hipError_t LBM_FN(launch_moments_st)(const Grid &g, const Phys &ph, const void *A, const mask_t *mask,
                                     double *stage, int32_t y0, int32_t rows, hipStream_t s)
{
    return moments_t<LBM_ST>(g, ph, A, mask, stage, y0, rows, s);
}

hipError_t LBM_FN(launch_moments_out_st)(const Grid &g, const Phys &ph, const void *A, const mask_t *mask, void *rho,
                                         void *ux, void *uy, bool fp64, hipStream_t s)
{
    return moments_out_t<LBM_ST>(g, ph, A, mask, rho, ux, uy, fp64, s);
}

hipError_t LBM_FN(launch_mass_st)(const Grid &g, const Phys &ph, const void *A, const mask_t *mask,
                                  double *partials, int32_t nb, bool maxdev, hipStream_t s)
{
    return mass_t<LBM_ST>(g, ph, A, mask, partials, nb, maxdev, s);
}
#endif

}  // namespace lbm
