// Device-side helpers shared by the forward kernels (lbm_kernels.hip) and the
// adjoint kernels (lbm_adjoint.hip): lattice constants, storage codecs and the
// deviation-form equilibrium.  Everything has internal linkage.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {
namespace {

// ---------------------------------------------------------------------------
// Lattice constants (Section 2).  Velocity order as in the paper's MRT matrix.
// ---------------------------------------------------------------------------
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

template <class R>
__device__ constexpr R wgt(int i)
{
    return i == 0 ? R(4) / R(9) : (i <= 4 ? R(1) / R(9) : R(1) / R(36));
}

// runtime-indexed lookups for the link kernel (direction differs per lane):
// component + 1 packed in two bits per direction
constexpr uint32_t pack2(const int *c)
{
    uint32_t r = 0;
    for (int i = 0; i < 9; ++i) r |= (uint32_t)(c[i] + 1) << (2 * i);
    return r;
}
constexpr uint32_t PCX = pack2(CX), PCY = pack2(CY);
__device__ __forceinline__ int cx_of(int i) { return (int)((PCX >> (2 * i)) & 3u) - 1; }
__device__ __forceinline__ int cy_of(int i) { return (int)((PCY >> (2 * i)) & 3u) - 1; }
__device__ __forceinline__ int opp_of(int i)
{
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
}

// ---------------------------------------------------------------------------
// Storage codecs: value stored = (f - w) [* 2^k for the 16-bit forms].
// ---------------------------------------------------------------------------
template <int ST>
struct Codec;

template <>
struct Codec<0> {  // LBM_F64
    using T = double;
    using R = double;
    static __device__ __forceinline__ R ld(T v, float) { return v; }
    static __device__ __forceinline__ T st(R v, float) { return v; }
};

template <>
struct Codec<1> {  // LBM_F32
    using T = float;
    using R = float;
    static __device__ __forceinline__ R ld(T v, float) { return v; }
    static __device__ __forceinline__ T st(R v, float) { return v; }
};

template <>
struct Codec<2> {  // LBM_F16_DEV
    using T = __half;
    using R = float;
    static __device__ __forceinline__ R ld(T v, float inv) { return __half2float(v) * inv; }
    static __device__ __forceinline__ T st(R v, float scale) { return __float2half_rn(v * scale); }
};

template <>
struct Codec<3> {  // LBM_BF16_DEV, bits of a bfloat16 in a uint16
    using T = uint16_t;
    using R = float;
    static __device__ __forceinline__ R ld(T v, float inv)
    {
        return __uint_as_float((uint32_t)v << 16) * inv;
    }
    static __device__ __forceinline__ T st(R v, float scale)
    {
        uint32_t u = __float_as_uint(v * scale);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
        u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
        return (uint16_t)(u >> 16);
    }
};

// Deviation-form arithmetic.  rho = 1 + dr is never formed: in FP32 its rounding
// (2^-24 relative) is systematic for a slowly varying flow and would drift the
// velocity step after step.  Instead
//   u   = j/rho = j + j*(1/rho - 1),  1/rho - 1 = -dr/(1 + dr)
//   f^eq_i - w_i = w_i (dr + P_i + dr P_i),  P_i = 3 e.u + 9/2 (e.u)^2 - 3/2 u.u
// keep every term at the precision of its own (small) magnitude.
template <class R>
__device__ __forceinline__ R inv_rho_m1(R dr)
{
    return -dr / (R(1) + dr);
}

template <class R>
__device__ __forceinline__ R poly(R eu, R usq)
{
    return R(3) * eu + R(4.5) * eu * eu - R(1.5) * usq;
}

template <class R>
__device__ __forceinline__ R deq(R w, R eu, R dr, R usq)
{
    const R P = poly(eu, usq);
    return w * (dr + P + dr * P);
}

}  // namespace
}  // namespace lbm
