// Storage dispatch of the kernel launches (lbm_internal.h): each launch_*
// function calls the helper of the context's storage format, compiled in its own
// object from lbm_kernels.hip.
#include "lbm_internal.h"

namespace lbm {

// ST 4 and 5 (FP32 storage with an FP64 or a plain FP32 collision) share every
// launch but the bulk ones with ST 1: the stored format is the same.
#define LBM_SWITCH(call, bulk)                  \
    switch (storage) {                          \
    case 0: return call(0);                     \
    case 1: return call(1);                     \
    case 2: return call(2);                     \
    case 3: return call(3);                     \
    case 4: return bulk ? call(4) : call(1);    \
    case 5: return bulk ? call(5) : call(1);    \
    default: return hipErrorInvalidValue;       \
    }

hipError_t launch_link(int storage, const Grid &g, const Phys &ph, const Links &L, const Side &side,
                       const Reduce &red, double *bank, double *fsum, int block, hipStream_t s,
                       ForceReduce *defer)
{
    if (block < 64 || block > 1024 || block % 64) return hipErrorInvalidValue;
#define C(K) launch_link_st##K(g, ph, L, side, red, bank, fsum, block, s, defer)
    LBM_SWITCH(C, false)
#undef C
}

hipError_t launch_bulk_fused(int storage, const Grid &g, const Phys &ph, const void *A, void *B,
                             const mask_t *mask, const void *uin, const Side &side, const FuseArgs &fa,
                             double *zb, int32_t nz, const BulkConfig &cf, hipStream_t s)
{
#define C(K) launch_bulk_fused_st##K(g, ph, A, B, mask, uin, side, fa, zb, nz, cf, s)
    LBM_SWITCH(C, true)
#undef C
}

hipError_t launch_bulk(int storage, const Grid &g, const Phys &ph, const void *A, void *B,
                       const mask_t *mask, const void *uin, const Side &side, double *zb, int32_t nz,
                       const BulkConfig &cf, hipStream_t s, const ForceReduce &fr)
{
#define C(K) launch_bulk_st##K(g, ph, A, B, mask, uin, side, zb, nz, cf, s, fr)
    LBM_SWITCH(C, true)
#undef C
}

hipError_t launch_bulk_batch(int storage, const BatchInst *insts, const BatchTile *tiles, int64_t ntiles,
                             const Phys &ph, const void *A, void *B, const mask_t *mask, const void *uin,
                             const Side &side, double *zb, int32_t nz, bool open, bool force, bool store_solid,
                             int rows, hipStream_t s, const ForceReduce &fr)
{
    if (ntiles <= 0) return fr.nw > 0 ? hipErrorInvalidValue : hipSuccess;
    if (rows != 1 && rows != 2) return hipErrorInvalidValue;
#define C(K) launch_bulk_batch_st##K(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, open, force, \
                                     store_solid, rows, s, fr)
    LBM_SWITCH(C, true)
#undef C
}

hipError_t launch_refresh(int storage, const Grid &g, const Phys &ph, const void *A, const Side &side,
                          bool moments, hipStream_t s)
{
#define C(K) launch_refresh_st##K(g, ph, A, side, moments, s)
    LBM_SWITCH(C, false)
#undef C
}

hipError_t launch_init(int storage, const Grid &g, const Phys &ph, void *A, const mask_t *mask,
                       const double *stage, int32_t y0, int32_t rows, hipStream_t s)
{
#define C(K) launch_init_st##K(g, ph, A, mask, stage, y0, rows, s)
    LBM_SWITCH(C, false)
#undef C
}

hipError_t launch_moments_out(int storage, const Grid &g, const Phys &ph, const void *A, const mask_t *mask,
                              void *rho, void *ux, void *uy, bool fp64, hipStream_t s)
{
#define C(K) launch_moments_out_st##K(g, ph, A, mask, rho, ux, uy, fp64, s)
    LBM_SWITCH(C, false)
#undef C
}

hipError_t launch_moments(int storage, const Grid &g, const Phys &ph, const void *A,
                          const mask_t *mask, double *stage, int32_t y0, int32_t rows, hipStream_t s)
{
#define C(K) launch_moments_st##K(g, ph, A, mask, stage, y0, rows, s)
    LBM_SWITCH(C, false)
#undef C
}

int32_t mass_blocks(const Grid &g)
{
    const int64_t N = (int64_t)g.nx * g.ny;
    int64_t b = (N + MASS_THREADS - 1) / MASS_THREADS;
    return (int32_t)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_mass(int storage, const Grid &g, const Phys &ph, const void *A, const mask_t *mask,
                       double *partials, int32_t nb, bool maxdev, hipStream_t s)
{
#define C(K) launch_mass_st##K(g, ph, A, mask, partials, nb, maxdev, s)
    LBM_SWITCH(C, false)
#undef C
}

#undef LBM_SWITCH

}  // namespace lbm
