// Device-side helpers shared by the forward kernels (lbm_kernels.hip) and the
// adjoint kernels (lbm_adjoint.hip): lattice constants, storage codecs and the
// deviation-form equilibrium.  Everything has internal linkage.
#pragma once

#include <type_traits>

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

// Reg is how the bulk kernel holds a loaded value until it decodes it (T itself,
// except BF16 below); reg() makes one from a stored value, ldr() decodes it.
template <>
struct Codec<0> {  // LBM_F64
    using T = double;
    using R = double;
    using Reg = T;
    static __device__ __forceinline__ R ld(T v, float) { return v; }
    static __device__ __forceinline__ T st(R v, float) { return v; }
    static __device__ __forceinline__ Reg reg(T v) { return v; }
    static __device__ __forceinline__ R ldr(Reg v, float inv) { return ld(v, inv); }
};

template <>
struct Codec<1> {  // LBM_F32
    using T = float;
    using R = float;
    using Reg = T;
    static __device__ __forceinline__ R ld(T v, float) { return v; }
    static __device__ __forceinline__ T st(R v, float) { return v; }
    static __device__ __forceinline__ Reg reg(T v) { return v; }
    static __device__ __forceinline__ R ldr(Reg v, float inv) { return ld(v, inv); }
};

template <>
struct Codec<4> : Codec<1> {  // LBM_F32_WIDE: stored as LBM_F32
};
template <>
struct Codec<5> : Codec<1> {  // LBM_F32_PLAIN: stored as LBM_F32
};

template <>
struct Codec<2> {  // LBM_F16_DEV
    using T = __half;
    using R = float;
    // held zero-extended in 32 bits, as BF16 below
    using Reg = uint32_t;
    static __device__ __forceinline__ R ld(T v, float inv) { return __half2float(v) * inv; }
    static __device__ __forceinline__ T st(R v, float scale) { return __float2half_rn(v * scale); }
    static __device__ __forceinline__ Reg reg(T v) { return (uint32_t)__builtin_bit_cast(uint16_t, v); }
    static __device__ __forceinline__ R ldr(Reg v, float inv)
    {
        return __half2float(__builtin_bit_cast(__half, (uint16_t)v)) * inv;
    }
};

template <>
struct Codec<3> {  // LBM_BF16_DEV
    using T = __bf16;
    using R = float;
    // Held zero-extended in 32 bits: as 16-bit values the nine pulled populations
    // were packed in pairs right after their loads, which made the kernel wait
    // for the loads there instead of behind the node lookups.
    using Reg = uint32_t;
    static __device__ __forceinline__ R ld(T v, float inv) { return (float)v * inv; }
    // FP32 -> BF16 with round to nearest even: one v_cvt_pk_bf16_f32 on gfx950
    static __device__ __forceinline__ T st(R v, float scale) { return (__bf16)(v * scale); }
    static __device__ __forceinline__ Reg reg(T v) { return (uint32_t)__builtin_bit_cast(uint16_t, v); }
    static __device__ __forceinline__ R ldr(Reg v, float inv) { return __uint_as_float(v << 16) * inv; }
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

// 1/rho - 1 with the hardware reciprocal (about 1 ulp), for the bulk kernel's
// velocity; the error is a relative 1e-7 of u (dr / (1 + dr) times 1 ulp).
__device__ __forceinline__ float inv_rho_m1_fast(float dr) { return -dr * __builtin_amdgcn_rcpf(1.0f + dr); }
__device__ __forceinline__ double inv_rho_m1_fast(double dr) { return -dr / (1.0 + dr); }
// 1/x: the hardware reciprocal in FP32 (about 1 ulp), a true division in FP64.
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_fast(double x) { return 1.0 / x; }
// Arithmetic type of the bulk collision: the storage's own arithmetic type (FP64
// for FP64 storage, FP32 otherwise), FP64 for the wide FP32 form, and FP32
// throughout (moments and odd parts too) for the plain FP32 form.  FP32
// feq and f^eq - f carry absolute rounding errors near 1e-9 (the ulp of the
// O(1e-2) deviations); wherever the flow is steady the same error recurs every
// step and adds up like a body force.  FP64 vector FMAs issue at the rate of
// unpacked FP32 ones on this chip; the cost is the wider registers.
template <int ST>
struct Collide {
    using A = typename Codec<ST>::R;  // the collision's arithmetic
    using D = A;                      // its moments and odd (momentum) parts
};
template <>
struct Collide<1> {
    using A = float;
    using D = double;
};
template <>
struct Collide<4> {
    using A = double;
    using D = double;
};
template <>
struct Collide<5> {
    using A = float;
    using D = float;
};

// Element e of a population plane at base.  A plane is smaller than 4 GiB (the
// runtime checks it), so the byte offset fits 32 bits and the access takes the
// scalar-base + 32-bit vector-offset form.
template <class T>
__device__ __forceinline__ T ld_el(const T *__restrict__ base, int32_t e)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                        (uint64_t)((uint32_t)e * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ void st_el(T *__restrict__ base, int32_t e, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (uint64_t)((uint32_t)e * (uint32_t)sizeof(T))) = v;
}
// The same with the byte offset given (an array smaller than 4 GiB at a
// wavefront-uniform base).
template <class T>
__device__ __forceinline__ T ld_at(const T *__restrict__ base, uint32_t byte_off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (uint64_t)byte_off);
}

// The same through the non-temporal path, for data a kernel streams through once
// (the pulled populations of the compact layout, the per-link records).  Such
// lines are not kept in the caches' retained set, so the bulk kernel's 0.7 GB of
// populations and the link records no longer push out of the 256 MB Infinity
// Cache the deposits (M, P) that the link kernel gathers: it runs 10% faster.
template <class T>
__device__ __forceinline__ T ld_at_nt(const T *__restrict__ base, uint32_t byte_off)
{
    static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "2, 4 or 8 bytes");
    using U = typename std::conditional<sizeof(T) == 2, uint16_t,
                                        typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type>::type;
    const U *p = reinterpret_cast<const U *>(reinterpret_cast<const char *>(base) + (uint64_t)byte_off);
    return __builtin_bit_cast(T, __builtin_nontemporal_load(p));
}

// A population plane as a raw buffer resource (base and size in scalar
// registers; 32-bit data format, the gfx9 encoding of the fourth word).  Stores
// through it take a 32-bit vector byte offset and need no vector address
// arithmetic per plane; offsets at or past `bytes` are dropped by the hardware.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t off, __half v)
{
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t off, uint16_t v)
{
    __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)off, 0, 0);
}
__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t off, __bf16 v)
{
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, 0, 0);
}

// Load of a wavefront-uniform element of a table that no kernel writes while it
// runs (segment bases, fluid masks): read through the constant address space it
// always takes the scalar cache, whatever stores, atomics or barriers come
// before it in the kernel.
template <class T>
__device__ __forceinline__ T ld_const(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)p;
}
// A trivially copyable record through the constant address space, word by word.
template <class T>
__device__ __forceinline__ T ld_const_record(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "record of whole words");
    T v;
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
    uint32_t *d = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = q[i];
    return v;
}
// A 16-byte record per lane through the non-temporal vector path (one 16-byte load).
template <class T>
__device__ __forceinline__ T ld_rec_nt(const T *p)
{
    static_assert(sizeof(T) == 16, "16-byte record");
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p)));
}
// A segment-base record field by field (a record load of only the fields used
// can become 12 bytes wide, which the scalar unit has no form for).
__device__ __forceinline__ SegBase ld_seg(const SegBase *p)
{
    return SegBase{ld_const(&p->flagged), ld_const(&p->links), ld_const(&p->pops), ld_const(&p->fluid)};
}

// Inclusive prefix sum over the 64 lanes of a wavefront with DPP row shifts and
// row broadcasts (all lanes must be active).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Sum over the 64 lanes of a wavefront in FP64 with DPP moves of both halves
// (all lanes must be active): pairs, quads, half-rows, rows, then row 1 += row 0
// and row 3 += row 2, then row 3 += row 1.  Lane 63 holds the total (the order
// of the additions is fixed, so the result is deterministic).
// Permutations within a row (every source lane valid): a plain DPP move.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// Row broadcasts into the rows of ROWS; the other rows read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64_rows(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum_to_last(double v)
{
    v += dpp_f64<0xb1>(v);             // quad_perm [1,0,3,2]
    v += dpp_f64<0x4e>(v);             // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);            // row_half_mirror
    v += dpp_f64<0x140>(v);            // row_mirror
    v += dpp_f64_rows<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64_rows<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Offset of node (x, y) in a population plane (see Grid).
__device__ __forceinline__ int32_t node_offset(const Grid &g, int x, int y)
{
    if (!g.compact) return y * g.pitch + x;
    const int32_t s = y * (g.pitch >> 6) + (x >> 6);
    return g.fseg[s].fluid + (int32_t)__popcll(g.fmask[s] & ((1ull << (x & 63)) - 1ull));
}

}  // namespace
}  // namespace lbm
