// HIP kernels (gfx950) of the D2Q9 BGK step with velocity-interpolation-based
// bounce-back walls (arXiv:1903.01111), with their per-storage launch helpers.
// Included by lbm_kernels.hip, which is compiled once per storage format so that
// the formats build in parallel; everything here has internal linkage.
//
// Per time step two launches read the post-collision state A = f+(t):
//   link kernel  -- one lane per fluid->solid link computes the population that
//                   streams out of the solid (Section 3.1, VIBB, or halfway
//                   bounce-back) and writes it into the link's solid-node slot of
//                   A, where the pull of the bulk kernel picks it up; it also
//                   reduces the momentum-exchange force in FP64;
//   bulk kernel  -- one lane per node: pull streaming from A (Section 2,
//                   evolution equation), moments, BGK collision with Guo forcing,
//                   store into B; lanes next to an open column also write the
//                   inlet / outlet column (Section 4.3).
// Populations are kept as deviations f_i - w_i from the rest state, which keeps
// FP32 and 16-bit storage accurate at low Mach number; all collision arithmetic
// is done in that form.
//
// The work is HBM-bound (about 2.8 flop per byte in FP32), so the kernels are
// written for coalescing: SoA planes with rows padded to 64 elements, each
// 64-lane wavefront covering one aligned run of a row.  No MFMA: nothing here is
// a dense contraction.
#pragma once

#include "lbm_device.h"

namespace lbm {
namespace {

// ---------------------------------------------------------------------------
// Link kernel: one lane per link, reading only compact arrays.
// ---------------------------------------------------------------------------

// What the evaluation of one link reads: its record and the deposits it
// points to.
template <int ST>
struct LinkIn {
    using R = typename Codec<ST>::R;
    using T = typename Codec<ST>::T;
    uint32_t meta;
    int32_t sf, sff, pf, pff, pfi;
    R q, uwx, uwy;
    T pfv, pffv, pfiv;
    R drf, ufx, ufy, drff, uffx, uffy;
};

// First round trip: the per-link record of link k, read once per step through
// the non-temporal path.  The per-link arrays hold at most 2^28 entries of at most
// 8 bytes, so byte offsets fit 32 bits (scalar base + 32-bit vector offset).
template <int ST>
__device__ __forceinline__ void link_load_record(const Links &L, int32_t k, LinkIn<ST> &a)
{
    using R = typename Codec<ST>::R;
    const uint32_t o4 = (uint32_t)k * 4u;
    bool done = false;
    if constexpr (sizeof(R) == 4) {
        if (L.crec) {
            // one 16-byte record and its run's bases (shared by the wavefront's lanes)
            const LinkRunBase b = ld_rec_nt(L.cbase + (k >> 6));
            const LinkRec r = ld_rec_nt(L.crec + k);
            a.meta = r.meta;
            a.q = __builtin_bit_cast(R, r.q);
            if (b.sf0 >= 0) {
                a.sf = b.sf0 + (int32_t)(r.d_f & 0xffffu);
                a.pf = b.pf0 + (int32_t)(r.d_f >> 16);
                a.sff = (r.d_ff & 0xffffu) == 0xffffu ? -1 : b.sff0 + (int32_t)(r.d_ff & 0xffffu);
                a.pff = b.pff0 + (int32_t)(r.d_ff >> 16);
            } else {
                a.pf = ld_at_nt(L.pf, o4);
                a.sf = ld_at_nt(L.sf, o4);
                a.sff = ld_at_nt(L.sff, o4);
                a.pff = ld_at_nt(L.pff, o4);
            }
            done = true;
        }
    }
    if (!done) {
        a.meta = ld_at_nt(L.meta, o4);
        a.pf = ld_at_nt(L.pf, o4);
        a.sf = ld_at_nt(L.sf, o4);
        a.sff = ld_at_nt(L.sff, o4);
        a.pff = ld_at_nt(L.pff, o4);
        a.q = ld_at_nt(static_cast<const R *>(L.q), (uint32_t)k * (uint32_t)sizeof(R));
    }
    // f+_i(x_f) of the outgoing direction: Bouzidi (q > 1/2) and Yu links only;
    // -1 (pf is meant) when no link needs it, so that nothing waits for pf here
    a.pfi = L.pfi ? ld_at_nt(L.pfi, o4) : -1;
    a.uwx = a.uwy = R(0);
    if (L.uw) {
        const R *u = static_cast<const R *>(L.uw);
        a.uwx = u[2 * (int64_t)k];
        a.uwy = u[2 * (int64_t)k + 1];
    }
}

// Second round trip: the deposits of x_f and x_ff the record points to.  Those
// of ff are fetched for halfway bounce-back links too (from f's slots, in
// bounds) and not used, so that no load waits on a branch.
template <int ST>
__device__ __forceinline__ void link_load_deposits(const void *Mv, const void *Pv, LinkIn<ST> &a)
{
    using R = typename Codec<ST>::R;
    using T = typename Codec<ST>::T;
    const T *P = static_cast<const T *>(Pv);
    const R *M = static_cast<const R *>(Mv);
    const int32_t sffc = a.sff < 0 ? a.sf : a.sff, pffc = a.sff < 0 ? a.pf : a.pff;
    a.pfv = P[a.pf];
    a.pffv = P[pffc];
    a.pfiv = P[a.pfi < 0 ? a.pf : a.pfi];
    a.drf = M[3 * (int64_t)a.sf];
    a.ufx = M[3 * (int64_t)a.sf + 1];
    a.ufy = M[3 * (int64_t)a.sf + 2];
    a.drff = M[3 * (int64_t)sffc];
    a.uffx = M[3 * (int64_t)sffc + 1];
    a.uffy = M[3 * (int64_t)sffc + 2];
}

// Value of a link (decoded, before storage rounding) from the moments M and the
// populations P deposited by the previous bulk step, by the link's scheme
// (Section 3.1 VIBB; halfway bounce-back, also where x_ff is unusable; Bouzidi;
// Yu), and its momentum-exchange force: the population f+_{i'}(x_f) into the wall
// and f_i(x_f) back, both along e_{i'}, with Galilean-invariant momentum
// exchange (momenta relative to the wall) the term -u_w (f+_{i'} - f_i) added.
template <int ST>
__device__ __forceinline__ typename Codec<ST>::R link_value(const Phys &ph, const LinkIn<ST> &a, double &fx,
                                                            double &fy, int &obj)
{
    using C = Codec<ST>;
    using R = typename C::R;
    const R q = a.q, uwx = a.uwx, uwy = a.uwy;
    const R drf = a.drf, ufx = a.ufx, ufy = a.ufy, drff = a.drff, uffx = a.uffx, uffy = a.uffy;
    const int ip = (int)(a.meta & 15u);
    obj = (int)(a.meta >> 8);
    const int cxp = cx_of(ip), cyp = cy_of(ip);
    const R w = ip <= 4 ? R(1) / R(9) : R(1) / R(36);
    // moving-wall momentum term 6 w_{i'} rho0 e_i.u_w, with e_i = -e_{i'}
    const R wall = -R(6) * w * R(ph.rho0) * (R(cxp) * uwx + R(cyp) * uwy);
    const R fpf = C::ld(a.pfv, ph.inv_scale);
    R v;
    {
        // VIBB from the moments of f and ff at time t, deposited by the previous
        // bulk step; evaluated for every link (no load may sink into a branch),
        // halfway bounce-back links take fpf + wall below instead
        const R fpff = C::ld(a.pffv, ph.inv_scale);
        const R a2q = R(2) * q, b2q = R(1) - R(2) * q;
        // density at the departure point d (extrapolated when q > 1/2)
        const R drd = a2q * drf + b2q * drff;
        // non-equilibrium parts at f and ff, interpolated per unit density and
        // rescaled by rho_d: rho_d/rho_f = 1 + (dr_d - dr_f)/(1 + dr_f)
        const R neqf = fpf - deq(w, R(cxp) * ufx + R(cyp) * ufy, drf, ufx * ufx + ufy * ufy);
        const R neqff = fpff - deq(w, R(cxp) * uffx + R(cyp) * uffy, drff, uffx * uffx + uffy * uffy);
        const R neqd = a2q * (neqf + neqf * ((drd - drf) * rcp_fast(R(1) + drf))) +
                       b2q * (neqff + neqff * ((drd - drff) * rcp_fast(R(1) + drff)));
        // velocity at d: u*_d from (f, ff) or (f, wall), u**_d from (ff, wall)
        R usx, usy;
        if (q <= R(0.5)) {
            usx = a2q * ufx + b2q * uffx;
            usy = a2q * ufy + b2q * uffy;
        } else {
            const R iq = rcp_fast(q), cf = (R(1) - q) * iq, cw = (R(2) * q - R(1)) * iq;
            usx = cf * ufx + cw * uwx;
            usy = cf * ufy + cw * uwy;
        }
        const R inv1q = rcp_fast(R(1) + q);
        const R cff = (R(1) - q) * inv1q, cww = a2q * inv1q;
        const R ussx = cff * uffx + cww * uwx, ussy = cff * uffy + cww * uwy;
        const R third = R(1) / R(3);
        const R udx = (usx + R(2) * ussx) * third, udy = (usy + R(2) * ussy) * third;
        v = deq(w, R(cxp) * udx + R(cyp) * udy, drd, udx * udx + udy * udy) + neqd + wall;
    }
    // the other schemes from the same deposits (deviation form: their weights sum
    // to one, so the rest-state weights cancel)
    const int sch = (int)((a.meta >> 4) & 15u);
    if (sch == LBM_SCHEME_HBB) {
        v = fpf + wall;
    } else if (sch == LBM_SCHEME_BOUZIDI) {
        const R fpff = C::ld(a.pffv, ph.inv_scale), fpi = C::ld(a.pfiv, ph.inv_scale);
        if (q <= R(0.5))
            v = R(2) * q * fpf + (R(1) - R(2) * q) * fpff + wall;
        else
            v = (fpf + wall + (R(2) * q - R(1)) * fpi) * rcp_fast(R(2) * q);
    } else if (sch == LBM_SCHEME_YU) {
        // wall value by interpolation between x_f and x_ff, then the value at x_f
        // between the wall point and x_ff (which receives f+_i(x_f) at t+1)
        const R fpff = C::ld(a.pffv, ph.inv_scale), fpi = C::ld(a.pfiv, ph.inv_scale);
        v = (q * fpf + (R(1) - q) * fpff + wall + q * fpi) * rcp_fast(R(1) + q);
    }
    const double m = (double)fpf + (double)v + 2.0 * (double)w;
    fx = cxp * m;
    fy = cyp * m;
    if (ph.gi_force) {
        const double dm = (double)fpf - (double)v;
        fx -= (double)uwx * dm;
        fy -= (double)uwy * dm;
    }
    return v;
}

// One link start to finish (two round trips).
template <int ST>
__device__ __forceinline__ typename Codec<ST>::R link_eval(const Phys &ph, const Links &L, const void *Mv,
                                                           const void *Pv, int32_t k, double &fx, double &fy,
                                                           int &obj)
{
    LinkIn<ST> a;
    link_load_record<ST>(L, k, a);
    link_load_deposits<ST>(Mv, Pv, a);
    return link_value<ST>(ph, a, fx, fy, obj);
}

// Link kernel: one lane per link.  The kernel is bound by its four deposit
// gathers per link (a wavefront's lanes hit scattered and repeated entries of M
// and P), not by record bytes, arithmetic or wave count; it runs faster the more
// of the deposits the Infinity Cache still holds when it starts (hence the
// non-temporal streaming loads here and in the bulk kernel).
template <int ST>
__global__ __launch_bounds__(1024) void link_kernel(Grid g, Phys ph, Links L, Side side,
                                                    double2 *__restrict__ wpart, int32_t *__restrict__ wobj,
                                                    double *__restrict__ bank, double *__restrict__ fsum)
{
    using C = Codec<ST>;
    using T = typename C::T;
    // XCD k (which gets hardware blocks k, k+8, ...) takes the k-th contiguous
    // run of link blocks: the links of neighbouring rows gather the same lines of
    // M and P, which then sit in one L2 instead of being fetched by all eight.
    const int32_t nb = (int32_t)gridDim.x, q8 = nb >> 3, r8 = nb & 7, k8 = (int32_t)blockIdx.x & 7;
    const int32_t blk = k8 * q8 + (k8 < r8 ? k8 : r8) + ((int32_t)blockIdx.x >> 3);
    const int lane = threadIdx.x & 63;
    // links number below 2^28
    const int32_t n = (int32_t)L.n;
    const int32_t k = blk * (int32_t)blockDim.x + (int32_t)threadIdx.x;
    double fx = 0.0, fy = 0.0;
    int obj = -1;
    if (k < n) {
        const auto v = link_eval<ST>(ph, L, side.M, side.P, k, fx, fy, obj);
        st_el(static_cast<T *>(side.L), L.li_ident ? k : ld_at(L.li, (uint32_t)k * 4u), C::st(v, ph.scale));
    }
    if (!bank) return;  // link values only: no force wanted (uniform over the grid)
    // FP64 reduction per run of 64 links (entry k/64 of the partials; runs past
    // the last link write none).  Links are sorted by object, so a run usually
    // holds one object: it leaves one partial sum for the reduction (no atomics:
    // thousands of wavefronts adding into the same address would serialise).  A
    // run spanning several objects adds per lane.
    const int32_t r0 = k - lane;
    if (r0 >= n) return;  // wavefront-uniform
    const int32_t run = r0 >> 6;
    const int obj0 = __builtin_amdgcn_readlane(obj, 0);
    if (__all(obj == obj0 || obj < 0)) {
        const double sx = wave_sum_to_last(fx), sy = wave_sum_to_last(fy);
        if (lane == 63) {
            wpart[run] = make_double2(sx, sy);
            wobj[run] = obj0;
        }
    } else {
        if (obj >= 0) {
            unsafeAtomicAdd(&bank[2 * obj], fx);
            unsafeAtomicAdd(&bank[2 * obj + 1], fy);
            unsafeAtomicAdd(&fsum[2 * obj], fx);
            unsafeAtomicAdd(&fsum[2 * obj + 1], fy);
        }
        if (lane == 0) wobj[run] = -1;
    }
}

// Sums the wavefront partials of the link kernel per object (they are in object
// order) into this step's force bank and the running sum.  A block of 256 lanes
// takes 256 * CHUNK consecutive partials: each lane sums its chunk per object,
// a wavefront whose lanes end on one object adds them up across its lanes, and a
// block whose four wavefronts end on one object adds them up in LDS, so that the
// common case costs one atomic per block and address (thousands of atomics on
// the same address would serialise).  Runs of other objects are added where
// they close.  The pointers come from distinct __restrict__ kernel arguments:
// the atomics then provably leave the rest of a kernel's inputs untouched, so
// that its wavefront-uniform loads can still use the scalar cache.
constexpr int REDUCE_CHUNK = 16;

__device__ __forceinline__ void add_force(double *__restrict__ bank, double *__restrict__ fsum, int o,
                                          double ax, double ay)
{
    unsafeAtomicAdd(&bank[2 * o], ax);
    unsafeAtomicAdd(&bank[2 * o + 1], ay);
    unsafeAtomicAdd(&fsum[2 * o], ax);
    unsafeAtomicAdd(&fsum[2 * o + 1], ay);
}

// Every thread of the 256-thread block calls it (it synchronises the block).
template <int CHUNK>
__device__ __forceinline__ void force_reduce_block(const double2 *__restrict__ wpart,
                                                   const int32_t *__restrict__ wobj, int64_t nw,
                                                   double *__restrict__ bank, double *__restrict__ fsum,
                                                   int64_t block, int tid)
{
    __shared__ int s_obj[4];
    __shared__ double s_f[4][2];
    const int64_t k0 = (block * 256 + tid) * CHUNK;
    // all loads of the chunk first (one round trip), then the segmented sum
    int ob[CHUNK];
    double2 pv[CHUNK];
#pragma unroll
    for (int k = 0; k < CHUNK; ++k) {
        const bool in = k0 + k < nw;
        ob[k] = in ? wobj[k0 + k] : -1;
        pv[k] = in ? wpart[k0 + k] : make_double2(0.0, 0.0);
    }
    int cur = -1;
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int k = 0; k < CHUNK; ++k) {
        const int o = ob[k];
        if (o < 0) continue;
        if (o != cur) {
            if (cur >= 0) add_force(bank, fsum, cur, ax, ay);
            cur = o;
            ax = ay = 0.0;
        }
        ax += pv[k].x;
        ay += pv[k].y;
    }
    int top = cur;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) top = max(top, __shfl_xor(top, off));
    const bool uni = __all(cur == top || cur < 0);
    if (uni) {
        // top < 0: the wavefront holds nothing
        if (cur < 0) ax = ay = 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            ax += __shfl_xor(ax, off);
            ay += __shfl_xor(ay, off);
        }
    } else if (cur >= 0) {
        add_force(bank, fsum, cur, ax, ay);
    }
    const int wv = tid >> 6;
    if ((tid & 63) == 0) {
        s_obj[wv] = uni ? top : -1;
        s_f[wv][0] = ax;
        s_f[wv][1] = ay;
    }
    __syncthreads();
    if (tid == 0) {
        int o0 = -1;
        bool same = true;
        for (int w = 0; w < 4; ++w) {
            const int o = s_obj[w];
            if (o < 0) continue;
            if (o0 < 0) o0 = o;
            same = same && o == o0;
        }
        if (same && o0 >= 0) {
            double sx = 0.0, sy = 0.0;
            for (int w = 0; w < 4; ++w)
                if (s_obj[w] >= 0) sx += s_f[w][0], sy += s_f[w][1];
            add_force(bank, fsum, o0, sx, sy);
        } else if (!same) {
            for (int w = 0; w < 4; ++w)
                if (s_obj[w] >= 0) add_force(bank, fsum, s_obj[w], s_f[w][0], s_f[w][1]);
        }
    }
}

__global__ __launch_bounds__(256) void force_reduce_kernel(const double2 *__restrict__ wpart,
                                                           const int32_t *__restrict__ wobj, int64_t nw,
                                                           double *__restrict__ bank,
                                                           double *__restrict__ fsum)
{
    force_reduce_block<REDUCE_CHUNK>(wpart, wobj, nw, bank, fsum, blockIdx.x, threadIdx.x);
}

// The reduction folded into the first blocks of the bulk kernel that follows the
// link kernel (block b, thread tid of 256; uniform per block).  A chunk of four
// partials per lane keeps the bulk kernel's register count (and occupancy) as
// it is; a longer one would raise it for every block.
constexpr int FOLD_CHUNK = 4;

__device__ __forceinline__ void force_reduce_part(const double2 *__restrict__ wpart,
                                                  const int32_t *__restrict__ wobj, int64_t nw,
                                                  double *__restrict__ bank, double *__restrict__ fsum,
                                                  int64_t b, int tid)
{
    if (nw <= 0 || b * 256 * FOLD_CHUNK >= nw) return;
    force_reduce_block<FOLD_CHUNK>(wpart, wobj, nw, bank, fsum, b, tid);
}

// ---------------------------------------------------------------------------
// Bulk kernel: pull, moments, BGK + Guo, store.  A block of BX x (256/BX) lanes
// covers BX consecutive nodes of 256/BX rows; every 64-lane wavefront is one
// aligned 64-node run of a row, so each population plane is read and written
// as contiguous runs.  Boundary nodes pull their cut directions from L and
// deposit what the next link kernel needs into M and P; their indices into
// those compact arrays come from per-segment bases plus wavefront prefix sums.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int popc32(uint32_t v) { return __popc(v); }

// LDS access by a 32-bit byte address (the low half of a flat pointer into LDS),
// for the walks below that advance an address by one element per set bit: a bit
// test, a compare and one address update per direction.  opaque() hides a value
// from the optimiser, which would otherwise re-derive the address from a count.
template <class T>
__device__ __forceinline__ uint32_t lds_addr(const T *p)
{
    return (uint32_t)(uintptr_t)p;
}
template <int N>
using uint_of = std::conditional_t<N == 2, uint16_t, std::conditional_t<N == 4, uint32_t, uint64_t>>;
template <class T>
__device__ __forceinline__ T lds_ld(uint32_t a)
{
    using U = uint_of<sizeof(T)>;
    return __builtin_bit_cast(T, *(const __attribute__((address_space(3))) U *)(uintptr_t)a);
}
template <class T>
__device__ __forceinline__ void lds_st(uint32_t a, T v)
{
    using U = uint_of<sizeof(T)>;
    *(__attribute__((address_space(3))) U *)(uintptr_t)a = __builtin_bit_cast(U, v);
}
__device__ __forceinline__ uint32_t opaque(uint32_t v)
{
    asm("" : "+v"(v));
    return v;
}

// e_i . (x, y) without products by 0 or +-1 (i is a constant once the direction
// loops are unrolled): the same value as CX[i] x + CY[i] y, up to the sign of a
// zero result.
template <class A>
__device__ __forceinline__ A edot(int i, A x, A y)
{
    const A sx = CX[i] > 0 ? x : -x, sy = CY[i] > 0 ? y : -y;
    return CX[i] == 0 ? (CY[i] == 0 ? A(0) : sy) : (CY[i] == 0 ? sx : sx + sy);
}

// MRT collision (Section 2) of one node in deviation form: the six non-conserved
// moments of the paper's M (e, epsilon, q_x, q_y, p_xx, p_xy) relax towards the
// moments of the second-order equilibrium at their own rates (s_e, s_eps, s_q and
// omega = 1/tau for the stresses); rho and j are conserved, and the body force
// enters as Guo's source taken to moment space with the factor (1 - s/2):
// e: 6 u.F, epsilon: -6 u.F, q: -F, p_xx: 2 (u_x F_x - u_y F_y), p_xy: u_x F_y +
// u_y F_x, j: F.  The moment changes return to the populations through
// M^-1 = M^T diag(9, 36, 36, 6, 12, 6, 12, 4, 4)^-1 (M's rows are orthogonal),
// in the same direction pairs as the BGK collision: f_i, f_opp change by ev +- od.
// Mass and momentum are conserved by construction (the axis odd parts take what
// the diagonals leave of F/2, the rest population what the pairs leave of the
// mass), and the momentum-carrying parts (q_x, q_y and the odd parts) are formed
// in D from the exact sums of the inputs, for the reason given in the BGK code.
template <class A, class D, bool FORCE>
__device__ __forceinline__ void collide_mrt(A (&f)[9], const Phys &ph, A drho, D jx_d, D jy_d, A ux, A uy, A usq,
                                            A Fx, A Fy)
{
    const A rho = A(1) + drho;
    const A ru2 = usq + drho * usq;  // rho u.u
    const A sax = (f[1] + f[3]) + (f[2] + f[4]), sdg = (f[5] + f[7]) + (f[6] + f[8]);
    // deviations of the moments from those of the rest state, minus the equilibrium's
    const A ne_e = ((sdg + sdg) - sax - A(4) * f[0]) + (drho + drho) - A(3) * ru2;
    const A ne_eps = ((sdg - (sax + sax)) + A(4) * f[0]) - drho + A(3) * ru2;
    const A ne_pxx = ((f[1] + f[3]) - (f[2] + f[4])) - rho * (ux * ux - uy * uy);
    const A ne_pxy = ((f[5] + f[7]) - (f[6] + f[8])) - rho * (ux * uy);
    const D Px = FORCE ? jx_d + D(0.5) * D(Fx) : jx_d, Py = FORCE ? jy_d + D(0.5) * D(Fy) : jy_d;
    const D ne_qx = (D(-2) * (D(f[1]) - D(f[3])) + ((D(f[5]) - D(f[6])) - (D(f[7]) - D(f[8])))) + Px;
    const D ne_qy = (D(-2) * (D(f[2]) - D(f[4])) + ((D(f[5]) + D(f[6])) - (D(f[7]) + D(f[8])))) + Py;
    const A se = A(ph.s_e), seps = A(ph.s_eps), om = A(ph.omega);
    const D sq = D(ph.s_q);
    A de = -se * ne_e, deps = -seps * ne_eps, dpxx = -om * ne_pxx, dpxy = -om * ne_pxy;
    D dqx = -sq * ne_qx, dqy = -sq * ne_qy;
    if (FORCE) {
        const A uF = ux * Fx + uy * Fy;
        de += (A(1) - A(0.5) * se) * (A(6) * uF);
        deps -= (A(1) - A(0.5) * seps) * (A(6) * uF);
        dpxx += (A(1) - A(0.5) * om) * (A(2) * (ux * Fx - uy * Fy));
        dpxy += (A(1) - A(0.5) * om) * (ux * Fy + uy * Fx);
        dqx -= (D(1) - D(0.5) * sq) * D(Fx);
        dqy -= (D(1) - D(0.5) * sq) * D(Fy);
    }
    const A a = de * A(1.0 / 36.0), b = deps * A(1.0 / 36.0), pp = dpxx * A(0.25), rr = dpxy * A(0.25);
    const A ev13 = (pp - a) - (b + b), ev24 = (-pp - a) - (b + b);
    const A ev57 = (a + a) + b + rr, ev68 = (a + a) + b - rr;
    const D cx = FORCE ? D(Fx) * D(1.0 / 6.0) : D(0), cy = FORCE ? D(Fy) * D(1.0 / 6.0) : D(0);
    const D dx = dqx * D(1.0 / 12.0), dy = dqy * D(1.0 / 12.0);
    const D od57 = (cx + dx) + (cy + dy), od68 = (cy + dy) - (cx + dx);
    const D hFx = FORCE ? D(0.5) * D(Fx) : D(0), hFy = FORCE ? D(0.5) * D(Fy) : D(0);
    const D od13 = hFx - (od57 - od68), od24 = hFy - (od57 + od68);
    const A o13 = A(od13), o24 = A(od24), o57 = A(od57), o68 = A(od68);
    f[0] = f[0] - A(2) * ((ev13 + ev24) + (ev57 + ev68));
    f[1] = f[1] + (ev13 + o13);
    f[3] = f[3] + (ev13 - o13);
    f[2] = f[2] + (ev24 + o24);
    f[4] = f[4] + (ev24 - o24);
    f[5] = f[5] + (ev57 + o57);
    f[7] = f[7] + (ev57 - o57);
    f[6] = f[6] + (ev68 + o68);
    f[8] = f[8] + (ev68 - o68);
}

// One node per lane of the lattice described by (g, A, mask), in two halves:
// bulk_issue loads the node's mask word and issues its nine pulls; bulk_finish
// (with ph, B, uin, side) does the rest once they have arrived.  A wavefront can
// issue the pulls of a second row segment before it finishes the first.
template <int ST>
struct Pulled {
    typename Codec<ST>::Reg a[9];  // the pulled populations (stored form, register holding)
    uint32_t own, own_in, own_out;  // byte offsets in a plane: the node, the open columns
    mask_t m;
    bool live;  // the wavefront's row segment lies in the lattice (uniform)
};

// Compact layout, lane `lane` of row segment sx of row yu (x = 64 sx + lane): the
// byte offsets in a plane of (x, r) (rk), of (x-1, r) (lf) and of (x+1, r) (rt) for
// the rows r = y-1, y, y+1.  The fluid rank of (x, r) is the fluid base of the
// segment in that row plus the fluid lanes below this one (v_mbcnt over the
// segment's bitmask).  In plane order a fluid node at x-1 then has rank rk - 1 and
// one at x+1 rank rk + fluid(x); offsets of solid nodes are only kept in bounds
// (their values are discarded).  yu and sx are wavefront-uniform.
template <uint32_t S, bool OPEN>
__device__ __forceinline__ void cmp_ranks(const Grid &g, int yu, int sx, int lane, uint32_t (&rk)[3],
                                          uint32_t (&lf)[3], uint32_t (&rt)[3])
{
    const int nsr = g.pitch >> 6;
    const int rows3[3] = {yu == 0 ? g.ny - 1 : yu - 1, yu, yu == g.ny - 1 ? 0 : yu + 1};
    const uint32_t last = (uint32_t)(g.plane - 1) * S;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int32_t sg = rows3[r] * nsr + sx;
        const uint64_t fm = ld_const(g.fmask + sg);
        rk[r] = S * __builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)fm, (uint32_t)ld_const(&g.fseg[sg].fluid)));
        lf[r] = (rk[r] > S ? rk[r] : S) - S;
        const uint32_t q = rk[r] + S * (uint32_t)((fm >> lane) & 1ull);
        rt[r] = q < last ? q : last;
    }
    if (!OPEN) {
        // periodic wrap in x: x = 0 pulls its e_x > 0 directions from x = nx-1 and
        // x = nx-1 its e_x < 0 directions from x = 0
        if (sx == 0 && lane == 0) {
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int32_t sg = rows3[r] * nsr + nsr - 1;
                lf[r] = S * (uint32_t)(ld_const(&g.fseg[sg].fluid) +
                                        (int32_t)__popcll(ld_const(g.fmask + sg) & ((1ull << ((g.nx - 1) & 63)) - 1ull)));
            }
        }
        if (sx == nsr - 1 && lane == ((g.nx - 1) & 63)) {
#pragma unroll
            for (int r = 0; r < 3; ++r) rt[r] = S * (uint32_t)ld_const(&g.fseg[rows3[r] * nsr].fluid);
        }
    }
}

// cmp_ranks in two halves for the run kernel, which loads the tables of several
// row segments at once (one wait for all of them) before it computes any offsets.
struct SegRows {
    uint64_t fm[3];  // fluid bitmasks of the segment in rows y-1, y, y+1
    int32_t fb[3];   // fluid counts before it in those rows
};

__device__ __forceinline__ void ld_seg_rows(const Grid &g, int yu, int sx, SegRows &t)
{
    const int nsr = g.pitch >> 6;
    const int rows3[3] = {yu == 0 ? g.ny - 1 : yu - 1, yu, yu == g.ny - 1 ? 0 : yu + 1};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const SegRow q = ld_const_record(g.frow + rows3[r] * nsr + sx);
        t.fm[r] = ((uint64_t)q.fm_hi << 32) | q.fm_lo;
        t.fb[r] = q.fluid;
    }
}

// cmp_ranks' offsets of a periodic lattice from tables loaded by ld_seg_rows.
template <uint32_t S>
__device__ __forceinline__ void cmp_ranks_from(const Grid &g, const SegRows &t, int yu, int sx, int lane,
                                               uint32_t (&rk)[3], uint32_t (&lf)[3], uint32_t (&rt)[3])
{
    const int nsr = g.pitch >> 6;
    const int rows3[3] = {yu == 0 ? g.ny - 1 : yu - 1, yu, yu == g.ny - 1 ? 0 : yu + 1};
    const uint32_t last = (uint32_t)(g.plane - 1) * S;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const uint64_t fm = t.fm[r];
        rk[r] = S * __builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fm, (uint32_t)t.fb[r]));
        lf[r] = (rk[r] > S ? rk[r] : S) - S;
        const uint32_t q = rk[r] + S * (uint32_t)((fm >> lane) & 1ull);
        rt[r] = q < last ? q : last;
    }
    // periodic wrap in x, as in cmp_ranks
    if (sx == 0 && lane == 0) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const SegRow q = ld_const_record(g.frow + rows3[r] * nsr + nsr - 1);
            const uint64_t fm = ((uint64_t)q.fm_hi << 32) | q.fm_lo;
            lf[r] = S * (uint32_t)(q.fluid + (int32_t)__popcll(fm & ((1ull << ((g.nx - 1) & 63)) - 1ull)));
        }
    }
    if (sx == nsr - 1 && lane == ((g.nx - 1) & 63)) {
#pragma unroll
        for (int r = 0; r < 3; ++r) rt[r] = S * (uint32_t)ld_const(&g.frow[rows3[r] * nsr].fluid);
    }
}

// The nine pull sources f_i(x, t+1) = f+_i(x - e_i, t) from cmp_ranks' offsets.
__device__ __forceinline__ void cmp_pull_offsets(const uint32_t (&rk)[3], const uint32_t (&lf)[3],
                                                 const uint32_t (&rt)[3], uint32_t (&o)[9])
{
    o[0] = rk[1];
    o[1] = lf[1];
    o[2] = rk[0];
    o[3] = rt[1];
    o[4] = rk[2];
    o[5] = lf[0];
    o[6] = rt[0];
    o[7] = rt[2];
    o[8] = lf[2];
}

template <int ST, bool OPEN, bool CMP>
__device__ __forceinline__ void bulk_issue(const Grid &g, const typename Codec<ST>::T *__restrict__ A,
                                           const mask_t *__restrict__ mask, int x, int y, Pulled<ST> &pl)
{
    using T = typename Codec<ST>::T;
    // a wavefront is one 64-node row segment: leave together if it lies outside
    pl.live = !(y >= g.ny || (x >> 6) >= (g.pitch >> 6));
    if (!pl.live) return;
    const bool inside = x < g.nx;
    const int32_t row = y * g.pitch;
    const mask_t m = inside ? ld_el(mask, row + x) : MASK_SOLID;
    pl.m = m;
    const int64_t P = g.plane;
    constexpr uint32_t S = sizeof(T);
    // The nine pulls f_i(x, t+1) = f+_i(x - e_i, t) are issued before the node
    // type and the link records are known, so that their latency overlaps the
    // record lookups; values of solid lanes, and those of directions whose
    // source is solid (replaced by link values below), are discarded.
    // Padding lanes (x >= nx) load the last column and are discarded too.
    const int xc = inside ? x : g.nx - 1;
    int xm, xp;
    if (OPEN) {
        xm = xc > 0 ? xc - 1 : 0;
        xp = xc < g.nx - 1 ? xc + 1 : g.nx - 1;
    } else {
        xm = xc == 0 ? g.nx - 1 : xc - 1;
        xp = xc == g.nx - 1 ? 0 : xc + 1;
    }
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int32_t rm = ym * g.pitch;
    const int32_t rp = yp * g.pitch;
    const int lane = threadIdx.x & 63;
    // byte offsets in a plane of the nine pull sources and of the node itself (own)
    uint32_t o[9], own, own_in = (uint32_t)row * S, own_out = (uint32_t)(row + g.nx - 1) * S;
    if (CMP) {
        uint32_t rk[3], lf[3], rt[3];
        cmp_ranks<S, OPEN>(g, __builtin_amdgcn_readfirstlane(y), __builtin_amdgcn_readfirstlane(x >> 6), lane, rk,
                           lf, rt);
        if (OPEN) {
            own_in = lf[1];   // (0, y), written by the lane x = 1 (both fluid)
            own_out = rt[1];  // (nx-1, y), written by the lane x = nx-2 (both fluid)
        }
        own = rk[1];
        cmp_pull_offsets(rk, lf, rt, o);
    } else {
        own = (uint32_t)(row + x) * S;
        o[0] = (uint32_t)(row + xc) * S;
        o[1] = (uint32_t)(row + xm) * S;
        o[2] = (uint32_t)(rm + xc) * S;
        o[3] = (uint32_t)(row + xp) * S;
        o[4] = (uint32_t)(rp + xc) * S;
        o[5] = (uint32_t)(rm + xm) * S;
        o[6] = (uint32_t)(rm + xp) * S;
        o[7] = (uint32_t)(rp + xp) * S;
        o[8] = (uint32_t)(rp + xm) * S;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        // compact layout: streamed through once, non-temporal so that the deposits
        // stay cached for the link kernel; dense layout: neighbouring rows reuse the
        // lines, which the non-temporal path would drop (all-fluid lattice 4% slower)
        if (CMP) pl.a[i] = Codec<ST>::reg(ld_at_nt(A + i * P, o[i]));
        else pl.a[i] = Codec<ST>::reg(ld_at(A + i * P, o[i]));
    }
    pl.own = own;
    pl.own_in = own_in;
    pl.own_out = own_out;
}

// With RUN the wavefront is a run of fluid nodes (bulk_run_kernel): rbase holds
// its bases, and x < nx marks the lanes that hold a node.
template <int ST, bool OPEN, bool FORCE, int BX, bool STORE_SOLID, bool CMP = false, bool FUSE = false,
          int COLL = 0, bool RUN = false>
__device__ __forceinline__ void bulk_finish(const Grid &g, const Phys &ph,
                                            typename Codec<ST>::T *__restrict__ B,
                                            const mask_t *__restrict__ mask,
                                            const typename Codec<ST>::R *__restrict__ uin,
                                            const Side &side, int x, int y, int wv,
                                            typename Codec<ST>::R (*lds_m)[3 * 64],
                                            typename Codec<ST>::T (*lds_p)[8 * 64], const Pulled<ST> &pl,
                                            const FuseArgs *fa = nullptr,
                                            typename Codec<ST>::T (*lds_l)[8 * 64] = nullptr,
                                            const SegBase rbase = SegBase{0, 0, 0, 0})
{
    static_assert(!RUN || (CMP && !OPEN && !FUSE), "runs: compact layout, periodic in x, separate links");
    using C = Codec<ST>;
    using T = typename C::T;
    using R = typename C::R;
    if (!pl.live) return;
    const bool inside = x < g.nx;
    const int32_t row = y * g.pitch;
    const mask_t m = pl.m;
    const int64_t P = g.plane;
    constexpr uint32_t S = sizeof(T);
    // the planes of B are written through buffer resources (plane < 4 GiB)
    const uint32_t pbytes = (uint32_t)(P * S);
    const int lane = threadIdx.x & 63;
    const uint32_t own = pl.own, own_in = pl.own_in, own_out = pl.own_out;
    typename C::Reg a[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) a[i] = pl.a[i];
    int32_t seg = 0;
    SegBase sb = rbase;
    if constexpr (!RUN) {
        seg = __builtin_amdgcn_readfirstlane(y * (g.pitch >> 6) + (x >> 6));
        sb = ld_seg(side.seg + seg);
    }
    if (FUSE) {
        // the wavefront's links are entries [lw, lw + nl) of the (node, dir) order
        // (segment bases; no need to wait for the mask words): one per lane,
        // evaluated from the previous step's deposits while the pulls are in
        // flight, handed to the node lanes through LDS; their force goes to the
        // segment's partial
        const int32_t lw = sb.links;
        const int nl = ld_const(&side.seg[seg + 1].links) - lw;
        const Links &L = fa->L;
        double fx = 0.0, fy = 0.0;
        int obj = -1;
        for (int j = lane; j < nl; j += 64) {
            const int32_t k = L.li_ident ? lw + j : L.kof[lw + j];
            double lfx, lfy;
            int o;
            const R v = link_eval<ST>(ph, L, side.M, side.P, k, lfx, lfy, o);
            lds_l[wv][j] = C::st(v, ph.scale);
            if (obj < 0 || o == obj) {
                obj = o;
                fx += lfx;
                fy += lfy;
            } else {
                unsafeAtomicAdd(&fa->bank[2 * o], lfx);
                unsafeAtomicAdd(&fa->bank[2 * o + 1], lfy);
                unsafeAtomicAdd(&fa->fsum[2 * o], lfx);
                unsafeAtomicAdd(&fa->fsum[2 * o + 1], lfy);
            }
        }
        int top = obj;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) top = max(top, __shfl_xor(top, off));
        if (__all(obj == top || obj < 0)) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                fx += __shfl_xor(fx, off);
                fy += __shfl_xor(fy, off);
            }
            if (lane == 0) {
                fa->wpart[seg] = make_double2(fx, fy);
                fa->wobj[seg] = top;
            }
        } else {
            if (obj >= 0) {
                unsafeAtomicAdd(&fa->bank[2 * obj], fx);
                unsafeAtomicAdd(&fa->bank[2 * obj + 1], fy);
                unsafeAtomicAdd(&fa->fsum[2 * obj], fx);
                unsafeAtomicAdd(&fa->fsum[2 * obj + 1], fy);
            }
            if (lane == 0) fa->wobj[seg] = -1;
        }
    }
    const uint64_t flagged = __ballot((m & MASK_SIDE) != 0);
    const int32_t slot = sb.flagged + (int32_t)__popcll(flagged & ((1ull << lane) - 1ull));
    const uint32_t rec = (m & MASK_SIDE) ? ld_el(side.rec, slot) : 0u;
    // links of this node (mask bits; with RUN, the side record's, as a run holds no
    // mask words): exclusive wavefront prefix -> first L entry
    const uint32_t lk = (RUN ? rec : (uint32_t)m) & MASK_LINKS;
    // deposited populations of this node (side record), counted in the high half
    // (with RUN the side record also gives the links, so that both prefixes come
    // from one scan: a run holds at most 512 links, and the low half does not
    // carry into the high one)
    uint32_t linc, inc = 0u;
    if constexpr (RUN) {
        const uint32_t both = wave_inclusive_scan((uint32_t)popc32(lk) | ((uint32_t)popc32(rec >> 8) << 16));
        linc = both & 0xffffu;
        inc = both & 0xffff0000u;
    } else {
        linc = wave_inclusive_scan((uint32_t)popc32(lk));
    }
    const int32_t lbase = sb.links + (int32_t)(linc - (uint32_t)popc32(lk));
    // where x - e_i is solid, the link (x, i') with i' = opp(i) (bit i'-1 of the
    // mask word) supplies the population: its load is issued now, while the
    // side record is still in flight (with FUSE, or RUN, the wavefront's link
    // values are already in LDS, in (node, dir) order from entry sb.links on)
    if (FUSE || RUN) {
        const int32_t lw = sb.links;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the node's link values are consecutive in direction order: walk its
        // link bits with an LDS address that advances past each value taken
        constexpr int OPPD[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        uint32_t la = lds_addr(&lds_l[wv][0]) + (uint32_t)(lbase - lw) * S;
#pragma unroll
        for (int d = 1; d < 9; ++d) {
            const uint32_t t = opaque((lk >> (d - 1)) & 1u);
            if (t) a[OPPD[d]] = C::reg(lds_ld<T>(la));
            la = opaque(la + t * S);
        }
    } else {
        // a node's links are consecutive L entries in direction order: walk them
        // (byte offsets: the link array is smaller than 4 GiB)
        const T *Lv = static_cast<const T *>(side.L);
        constexpr int OPPD[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        uint32_t lb = (uint32_t)lbase * S;
#pragma unroll
        for (int d = 1; d < 9; ++d)
            if (lk & (1u << (d - 1))) {
                a[OPPD[d]] = C::reg(ld_at(Lv, lb));
                lb += S;
            }
    }
    // deposited populations: exclusive prefix -> first P entry
    const uint32_t cnt = (uint32_t)popc32(rec >> 8) << 16;
    if constexpr (!RUN) inc = wave_inclusive_scan(cnt);
    const uint32_t exc = inc - cnt;
    const int32_t pbase = sb.pops + (int32_t)(exc >> 16);
    const int wave_pops = (int)((uint32_t)__builtin_amdgcn_readlane((int)inc, 63) >> 16);
    const int wave_flagged = (int)__popcll(flagged);
    // the open columns are written by their neighbour lanes: fetch their records,
    // and keep their deposits out of the wavefront's coalesced flush
    uint32_t rec_in = 0, rec_out = 0;
    int32_t pb_in = 0, pb_out = 0, slot_out = 0;
    int m_lo = 0, m_hi = 3 * wave_flagged, p_lo = 0, p_hi = wave_pops;
    if (OPEN) {
        rec_in = (uint32_t)__builtin_amdgcn_readlane((int)rec, 0);
        pb_in = __builtin_amdgcn_readlane(pbase, 0);
        const uint32_t cnt_in = (uint32_t)__builtin_amdgcn_readlane((int)cnt, 0);
        if ((x >> 6) == 0 && (flagged & 1ull)) {
            m_lo = 3;
            p_lo = (int)(cnt_in >> 16);
        }
        const int xe = g.nx - 1;
        const int le = xe & 63;
        const uint32_t r_e = (uint32_t)__builtin_amdgcn_readlane((int)rec, le);
        const int32_t p_e = __builtin_amdgcn_readlane(pbase, le);
        const uint32_t c_e = (uint32_t)__builtin_amdgcn_readlane((int)cnt, le);
        if ((xe >> 6) == (x >> 6)) {
            rec_out = r_e;
            pb_out = p_e;
            slot_out = sb.flagged + (int32_t)__popcll(flagged & ((1ull << le) - 1ull));
            if ((flagged >> le) & 1ull) {
                m_hi -= 3;
                p_hi -= (int)(c_e >> 16);
            }
        } else if (x == g.nx - 2 && (mask[row + xe] & MASK_SIDE)) {
            // x_e starts the next segment of the row
            const SegBase sn = ld_seg(side.seg + seg + 1);
            slot_out = sn.flagged;
            rec_out = side.rec[slot_out];
            pb_out = sn.pops;
        }
    }
    if (!inside) return;
    if (OPEN && (x == 0 || x == g.nx - 1)) return;
    if (m & MASK_SOLID) {
        if (STORE_SOLID && !CMP) {
            // solid slots of B are never read; storing them keeps every cache line
            // of B fully written (no partial-line writes at solid boundaries)
#pragma unroll
            for (int i = 0; i < 9; ++i) st_buf(plane_rsrc(B + i * P, pbytes), own, T(0));
        }
        return;
    }

    const float inv = ph.inv_scale;
    using A = typename Collide<ST>::A;
    // the moments and the momentum-carrying (odd) parts of the collision in D
    using D = typename Collide<ST>::D;
    A f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = A(C::ldr(a[i], inv));

    // In D, these sums of stored values are exact (FP32 inputs in FP64)
    const D drho_d = ((D(f[0]) + D(f[1])) + (D(f[2]) + D(f[3]))) + ((D(f[4]) + D(f[5])) + (D(f[6]) + D(f[7]))) +
                     D(f[8]);
    const D jx_d = (D(f[1]) - D(f[3])) + (D(f[5]) - D(f[6])) + (D(f[8]) - D(f[7]));
    const D jy_d = (D(f[2]) - D(f[4])) + (D(f[5]) + D(f[6])) - (D(f[7]) + D(f[8]));
    const A drho = A(drho_d), jx = A(jx_d), jy = A(jy_d);
    const A ir = inv_rho_m1_fast(drho);
    A ux = jx + jx * ir, uy = jy + jy * ir;
    A Fx = A(0), Fy = A(0);
    if (FORCE) {
        // force density F = rho g; velocity shifted by half the force (Guo)
        Fx = A(ph.gx) + drho * A(ph.gx);
        Fy = A(ph.gy) + drho * A(ph.gy);
        ux += A(0.5) * A(ph.gx);
        uy += A(0.5) * A(ph.gy);
    }
    const A usq = ux * ux + uy * uy;
    if constexpr (COLL == 1) {
        collide_mrt<A, D, FORCE>(f, ph, drho, jx_d, jy_d, ux, uy, usq, Fx, Fy);
    } else {
    const A om = A(ph.omega);
    const A cf = A(1) - A(0.5) * om;
    // BGK + Guo in direction pairs (i, opp(i)), which share e.u up to its sign:
    //   f^eq - w = w (rho P + dr),  P = A +- B,  A = 9/2 (e.u)^2 - 3/2 u.u,  B = 3 e.u,
    // so f^eq_{i,opp} - w = ev +- od with the even part ev = w (rho A + dr) (rho A =
    // A + dr A in deviation form) and the odd part od = w rho B.  Guo's source
    // (1 - omega/2) w [3 (e - u).F + 9 (e.u)(e.F)] splits into gs +- gd with
    // gs = (1 - omega/2) w (9 (e.u)(e.F) - 3 u.F) and gd = 3 (1 - omega/2) w e.F.
    // Mass and momentum are conserved by construction, not through the weights
    // (1/9 and 1/36 are inexact in binary): the odd parts of the two axis pairs are
    // what the diagonal pairs leave of the equilibrium momentum rho u = j + F/2 (and
    // of the source's (1 - omega/2) F), and the rest population takes what the pairs
    // leave of the mass.
    // A population changes by -omega f^neq + source with f^neq = f - f^eq split the
    // same way: (f_i + f_opp)/2 - ev (small terms, exact sum) +- ((f_i - f_opp)/2 - od).
    // The odd part subtracts two O(|u|) numbers; done in FP32, its rounding (the ulp
    // of the O(1e-2) deviations, about 1e-9) recurs every step wherever the flow is
    // steady and adds up like a body force, so the momenta, od and that difference
    // are formed in D (FP64 for FP32 storage); each population then changes by one
    // rounded addition of its small increment.
    const A h15 = A(1.5) * usq;
    const A uF = FORCE ? ux * Fx + uy * Fy : A(0);
    constexpr int PLUS[4] = {1, 2, 5, 6}, MINUS[4] = {3, 4, 7, 8};  // x axis, y axis, two diagonals
    A ev[4], gs[4], gd[4];
    D od[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = PLUS[k];
        const A w = wgt<A>(i);
        const A eu = edot(i, ux, uy);
        const A A2 = A(4.5) * eu * eu - h15;
        ev[k] = w * ((A2 + drho * A2) + drho);
        if (FORCE) {
            const A eF = edot(i, Fx, Fy);
            const A cw = cf * w;
            gs[k] = cw * (A(9) * eu * eF - A(3) * uF);
            if (k >= 2) gd[k] = (A(3) * cw) * eF;
        }
    }
    {
        // diagonal odd parts w rho B = (1/12) rho (e.u), from the exact momenta
        const D Px = FORCE ? jx_d + D(0.5) * D(Fx) : jx_d, Py = FORCE ? jy_d + D(0.5) * D(Fy) : jy_d;
        const D ru2 = Px + Py, ru3 = Py - Px;  // rho e.u of the diagonals (1,1) and (-1,1)
        od[2] = ru2 * D(1.0 / 12.0);
        od[3] = ru3 * D(1.0 / 12.0);
        od[0] = D(0.5) * Px - (od[2] - od[3]);
        od[1] = D(0.5) * Py - (od[2] + od[3]);
    }
    const A ev0 = drho - A(2) * ((ev[0] + ev[1]) + (ev[2] + ev[3]));
    A gs0 = A(0);
    if (FORCE) {
        const A hcf = A(0.5) * cf;
        gd[0] = hcf * Fx - (gd[2] - gd[3]);
        gd[1] = hcf * Fy - (gd[2] + gd[3]);
        gs0 = A(-2) * ((gs[0] + gs[1]) + (gs[2] + gs[3]));
    }
    f[0] = f[0] + (om * (ev0 - f[0]) + gs0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = PLUS[k], j = MINUS[k];
        const A ne = A(0.5) * (f[i] + f[j]) - ev[k];                    // even part of f^neq
        const A no = A(D(0.5) * (D(f[i]) - D(f[j])) - od[k]);           // odd part of f^neq
        const A si = FORCE ? gs[k] + gd[k] : A(0), sj = FORCE ? gs[k] - gd[k] : A(0);
        f[i] = f[i] + (si - om * (ne + no));
        f[j] = f[j] + (sj - om * (ne - no));
    }
    }  // BGK
#pragma unroll
    for (int i = 0; i < 9; ++i) st_buf(plane_rsrc(B + i * P, pbytes), own, C::st(R(f[i]), ph.scale));
    // deposits for the next link kernel, staged in LDS so that the wavefront
    // writes its contiguous ranges of M and P in full lines.  The post-collision
    // moments are the collision's own (rho, u): with Guo's shift the physical
    // velocity of f+ equals the collision velocity.
    R *Mv = static_cast<R *>(side.Mw);
    T *Pv = static_cast<T *>(side.Pw);
    if (m & MASK_SIDE) {
        const int ls = slot - sb.flagged;
        lds_m[wv][3 * ls] = R(drho);
        lds_m[wv][3 * ls + 1] = R(ux);
        lds_m[wv][3 * ls + 2] = R(uy);
        // the deposits in direction order, an LDS address advancing past each
        uint32_t pa = lds_addr(&lds_p[wv][0]) + (exc >> 16) * S;
#pragma unroll
        for (int d = 1; d < 9; ++d) {
            const uint32_t t = opaque((rec >> (d + 7)) & 1u);
            if (t) lds_st<T>(pa, C::st(R(f[d]), ph.scale));
            pa = opaque(pa + t * S);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
        // lanes still running share the flush
        const uint64_t act = __ballot(1);
        const int arank = (int)__popcll(act & ((1ull << lane) - 1ull));
        const int acnt = (int)__popcll(act);
        R *Mw = Mv + 3 * (int64_t)sb.flagged;
        for (int j = m_lo + arank; j < m_hi; j += acnt) Mw[j] = lds_m[wv][j];
        T *Pw = Pv + sb.pops;
        for (int j = p_lo + arank; j < p_hi; j += acnt) Pw[j] = lds_p[wv][j];
    }
    if (OPEN) {
        if (x == 1 && !(mask[row] & MASK_SOLID)) {
            // velocity inlet by non-equilibrium extrapolation:
            // f+(0) = f^eq(rho_1, u_in) + f+(1) - f^eq(rho_1, u_1); its moments are (rho_1, u_in)
            const A vx = A(uin[2 * y]), vy = A(uin[2 * y + 1]);
            const A vsq = vx * vx + vy * vy;
            A f0[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const A w = wgt<A>(i);
                const A ev = A(CX[i]) * vx + A(CY[i]) * vy;
                const A eu = A(CX[i]) * ux + A(CY[i]) * uy;
                const A dp = poly(ev, vsq) - poly(eu, usq);
                f0[i] = f[i] + w * (dp + drho * dp);
                st_buf(plane_rsrc(B + i * P, pbytes), own_in, C::st(R(f0[i]), ph.scale));
            }
            if (flagged & 1ull) {
                const int32_t k = sb.flagged;
                Mv[3 * k] = R(drho);
                Mv[3 * k + 1] = R(vx);
                Mv[3 * k + 2] = R(vy);
#pragma unroll
                for (int d = 1; d < 9; ++d) {
                    const uint32_t bit = 1u << (d + 7);
                    if (rec_in & bit)
                        Pv[pb_in + popc32((rec_in >> 8) & ((1u << (d - 1)) - 1u))] = C::st(R(f0[d]), ph.scale);
                }
            }
        }
        const mask_t me = mask[row + g.nx - 1];
        if (x == g.nx - 2 && !(me & MASK_SOLID)) {
            // zero-gradient outlet: copy every population of the last fluid column
#pragma unroll
            for (int i = 0; i < 9; ++i) st_buf(plane_rsrc(B + i * P, pbytes), own_out, C::st(R(f[i]), ph.scale));
            if (me & MASK_SIDE) {
                Mv[3 * slot_out] = R(drho);
                Mv[3 * slot_out + 1] = R(ux);
                Mv[3 * slot_out + 2] = R(uy);
#pragma unroll
                for (int d = 1; d < 9; ++d) {
                    const uint32_t bit = 1u << (d + 7);
                    if (rec_out & bit)
                        Pv[pb_out + popc32((rec_out >> 8) & ((1u << (d - 1)) - 1u))] = C::st(R(f[d]), ph.scale);
                }
            }
        }
    }
}

// Both halves back to back: one row segment per wavefront.
template <int ST, bool OPEN, bool FORCE, int BX, bool STORE_SOLID, bool CMP = false, bool FUSE = false,
          int COLL = 0>
__device__ __forceinline__ void bulk_body(const Grid &g, const Phys &ph,
                                          const typename Codec<ST>::T *__restrict__ A,
                                          typename Codec<ST>::T *__restrict__ B,
                                          const mask_t *__restrict__ mask,
                                          const typename Codec<ST>::R *__restrict__ uin,
                                          const Side &side, int x, int y, int wv,
                                          typename Codec<ST>::R (*lds_m)[3 * 64],
                                          typename Codec<ST>::T (*lds_p)[8 * 64],
                                          const FuseArgs *fa = nullptr,
                                          typename Codec<ST>::T (*lds_l)[8 * 64] = nullptr)
{
    Pulled<ST> pl;
    bulk_issue<ST, OPEN, CMP>(g, A, mask, x, y, pl);
    // keep the pulls ahead of everything that waits for the mask word (the
    // scheduler would otherwise hoist the ballot of bulk_finish above them and
    // expose the mask's latency)
    __builtin_amdgcn_sched_barrier(0);
    bulk_finish<ST, OPEN, FORCE, BX, STORE_SOLID, CMP, FUSE, COLL>(g, ph, B, mask, uin, side, x, y, wv, lds_m,
                                                                    lds_p, pl, fa, lds_l);
}

// clears the force bank of the next step (all blocks share the work)
__device__ __forceinline__ void zero_bank_part(double *__restrict__ zb, int32_t nz, int64_t block,
                                               int64_t nblocks, int tid)
{
    if (block * 256 >= nz) return;  // most blocks: nothing to clear (uniform)
    for (int64_t k = block * 256 + tid; k < nz; k += nblocks * 256) zb[k] = 0.0;
}

template <int ST, bool OPEN, bool FORCE, int BX, bool STORE_SOLID, bool CMP, int ROWS, int COLL>
__global__ __launch_bounds__(256) void bulk_kernel(Grid g, Phys ph,
                                                   const typename Codec<ST>::T *__restrict__ A,
                                                   typename Codec<ST>::T *__restrict__ B,
                                                   const mask_t *__restrict__ mask,
                                                   const typename Codec<ST>::R *__restrict__ uin,
                                                   Side side, double *__restrict__ zero_bank,
                                                   int32_t n_zero, int32_t xcd, double inv_nbx,
                                                   const double2 *__restrict__ red_part,
                                                   const int32_t *__restrict__ red_obj, int64_t red_n,
                                                   double *__restrict__ red_bank, double *__restrict__ red_sum)
{
    using R = typename Codec<ST>::R;
    using T = typename Codec<ST>::T;
    constexpr int BY = 256 / BX;
    // per wavefront: deposits of up to 64 nodes (3 moments, up to 8 populations each)
    __shared__ R lds_m[4][3 * 64];
    __shared__ T lds_p[4][8 * 64];
    const int tid = threadIdx.y * BX + threadIdx.x;
    const int64_t nb = (int64_t)gridDim.x * gridDim.y;
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    zero_bank_part(zero_bank, n_zero, b, nb, tid);
    force_reduce_part(red_part, red_obj, red_n, red_bank, red_sum, b, tid);
    // Workgroups go to the 8 XCDs round robin (block b to XCD b mod 8).  With xcd,
    // XCD k takes the k-th contiguous run of tiles in row-major order instead, so
    // the rows a tile pulls from, and the cache lines it shares with the tiles
    // beside it, were mostly touched by the same XCD and sit in its L2.
    int tx = blockIdx.x, ty = blockIdx.y;
    if (xcd) {
        const int32_t n = (int32_t)nb, q = n >> 3, r = n & 7, k = (int32_t)b & 7;
        const int32_t tile = k * q + (k < r ? k : r) + ((int32_t)b >> 3);
        // tile / gridDim.x in double: exact for tile < 2^31 (no integer divide)
        ty = (int)((tile + 0.5) * inv_nbx);
        tx = tile - ty * (int)gridDim.x;
        if (tx < 0) tx += gridDim.x, --ty;
        if (tx >= (int)gridDim.x) tx -= gridDim.x, ++ty;
    }
    const int x = tx * BX + threadIdx.x;
    if (ROWS == 1) {
        bulk_body<ST, OPEN, FORCE, BX, STORE_SOLID, CMP, false, COLL>(g, ph, A, B, mask, uin, side, x,
                                                                      ty * BY + threadIdx.y, tid >> 6, lds_m, lds_p);
    } else {
        // two row segments per wavefront (rows y and y + BY of a BX x 2BY tile):
        // the second one's pulls are in flight while the first is finished
        const int y0 = ty * 2 * BY + threadIdx.y, y1 = y0 + BY;
        Pulled<ST> p0, p1;
        bulk_issue<ST, OPEN, CMP>(g, A, mask, x, y0, p0);
        bulk_issue<ST, OPEN, CMP>(g, A, mask, x, y1, p1);
        __builtin_amdgcn_sched_barrier(0);
        bulk_finish<ST, OPEN, FORCE, BX, STORE_SOLID, CMP, false, COLL>(g, ph, B, mask, uin, side, x, y0, tid >> 6,
                                                                        lds_m, lds_p, p0);
        // the first segment's deposit flush has read the wavefront's LDS staging
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        bulk_finish<ST, OPEN, FORCE, BX, STORE_SOLID, CMP, false, COLL>(g, ph, B, mask, uin, side, x, y1, tid >> 6,
                                                                        lds_m, lds_p, p1);
    }
}

// Runs of fluid nodes (compact layout, periodic in x): wavefront w of the launch
// takes the fluid nodes 64w .. 64w+63 in plane order instead of one 64-node row
// segment, so that every lane holds a fluid node (a porous row segment holds 38 of
// 64 on average) and each plane is read at the node itself and written in
// 256-byte-aligned runs of full cache lines.  The run spans a few row segments;
// the wavefront first walks them with one lane per node of the segment (as in the
// segment mapping), computes there the pull offsets of each fluid node, and hands
// them through LDS to the lane that takes the node.  The side records, link values
// and deposits of a run are contiguous ranges like those of a segment, with bases
// from the run table.  The open columns are excluded: they are written by their
// neighbour lanes, which a run may place in another wavefront.
// At most 96 scalar registers: the preloaded tables push the MRT instantiations to
// 98, which leaves room for 7 wavefronts per SIMD instead of 8 (its bulk kernel
// took 178 us against 167 us with the cap, two registers spilled to vector lanes).
constexpr int RUN_PRE = 3;  // row segments whose tables a run loads up front

// The nine pull offsets (bytes) of fluid node k, the lane-th node of run w, from
// its neighbour word (g.nbr): the ranks of (x, y-1) and (x, y+1) relative to k are
// the run's bases (g.nbr_run) plus the word's 7-bit excesses, and with whether those
// nodes are fluid they give the same offsets as the segment walk (cmp_ranks).  A
// node with the word 0xffff (the first and last row and column, whose periodic
// wraps the words do not hold, and the nodes of a run whose differences spread too
// far) reads its nine offsets from the table g.nbr_slow, at the run's base plus the
// run's earlier such nodes.  A lane without a node (live false) gets offset 0
// everywhere.  Called by the whole wavefront (a ballot).
template <uint32_t S>
__device__ __forceinline__ void nbr_offsets(const Grid &g, int32_t w, int32_t k, bool live, uint32_t (&o)[9])
{
    const int lane = threadIdx.x & 63;
    const int32_t dm0 = ld_const(&g.nbr_run[w].dm0), dp0 = ld_const(&g.nbr_run[w].dp0);
    const int32_t sb = ld_const(&g.nbr_run[w].slow);
    const uint32_t wd = live ? (uint32_t)ld_at_nt(g.nbr, (uint32_t)k * 2u) : 0u;
    const bool slow = live && wd == 0xffffu;
    const uint64_t sm = __ballot(slow);
    if (slow) {
        const uint32_t e = (uint32_t)(sb + (int32_t)__popcll(sm & ((1ull << lane) - 1ull))) * 9u;
#pragma unroll
        for (int i = 0; i < 9; ++i) o[i] = ld_el(g.nbr_slow, (int32_t)(e + i)) * S;
    } else {
        const uint32_t last = (uint32_t)(g.plane - 1) * S;
        const int32_t kk = live ? k : 0;
        const int32_t dm = dm0 + (int32_t)(wd & 0x7fu), dp = dp0 + (int32_t)((wd >> 8) & 0x7fu);
        const uint32_t rk[3] = {(uint32_t)(kk + dm) * S, (uint32_t)kk * S, (uint32_t)(kk + dp) * S};
        const uint32_t fl3[3] = {(wd >> 7) & 1u, 1u, wd >> 15};
        uint32_t lf[3], rt[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            lf[r] = (rk[r] > S ? rk[r] : S) - S;
            const uint32_t q = rk[r] + S * fl3[r];
            rt[r] = q < last ? q : last;
        }
        cmp_pull_offsets(rk, lf, rt, o);
    }
    if (!live) {
#pragma unroll
        for (int i = 0; i < 9; ++i) o[i] = 0u;
    }
}

// With FUSE the wavefront also evaluates the links of its nodes (from the previous
// step's deposits; no link kernel) and leaves one force partial per run in fa.
// With NBR each lane reads its node's neighbour word (g.nbr) instead of the
// wavefront walking the row segments: no segment tables, no LDS exchange.
template <int ST, bool FORCE, int COLL, bool FUSE, bool NBR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_num_sgpr(96))) void bulk_run_kernel(
    Grid g, Phys ph, const typename Codec<ST>::T *__restrict__ A, typename Codec<ST>::T *__restrict__ B,
    const mask_t *__restrict__ mask, Side side, FuseArgs fa, double *__restrict__ zero_bank, int32_t n_zero,
    int32_t xcd,
    const double2 *__restrict__ red_part, const int32_t *__restrict__ red_obj, int64_t red_n,
    double *__restrict__ red_bank, double *__restrict__ red_sum)
{
    using C = Codec<ST>;
    using R = typename C::R;
    using T = typename C::T;
    constexpr uint32_t S = sizeof(T);
    // per wavefront, in the same bytes one after the other: the pull offsets of its
    // 64 nodes (9 words each), its link values, the deposit staging of bulk_finish
    constexpr int OFF_BYTES = 9 * 64 * 4;
    constexpr int LNK_BYTES = 8 * 64 * (int)sizeof(T);  // at most 8 links per node
    constexpr int DEP_BYTES = 64 * (3 * (int)sizeof(R) + 8 * (int)sizeof(T));
    constexpr int WB0 = OFF_BYTES > DEP_BYTES ? OFF_BYTES : DEP_BYTES;
    constexpr int WB = WB0 > LNK_BYTES ? WB0 : LNK_BYTES;
    __shared__ __align__(16) unsigned char lds[4 * WB];
    const int tid = threadIdx.x;
    const int64_t nb = gridDim.x;
    const int64_t b = blockIdx.x;
    zero_bank_part(zero_bank, n_zero, b, nb, tid);
    force_reduce_part(red_part, red_obj, red_n, red_bank, red_sum, b, tid);
    // with xcd, XCD k takes the k-th contiguous range of blocks (runs of
    // neighbouring nodes), as in bulk_kernel
    int32_t blk = (int32_t)b;
    if (xcd) {
        const int32_t n = (int32_t)nb, q = n >> 3, r = n & 7, k = (int32_t)b & 7;
        blk = k * q + (k < r ? k : r) + ((int32_t)b >> 3);
    }
    const int wv = tid >> 6, lane = tid & 63;
    const int32_t w = __builtin_amdgcn_readfirstlane(blk * 4 + wv);
    if (w >= g.nruns) return;
    const RunBase rb{ld_const(&g.runs[w].flagged), ld_const(&g.runs[w].links), ld_const(&g.runs[w].pops),
                     ld_const(&g.runs[w].seg), ld_const(&g.runs[w].flag_lo), ld_const(&g.runs[w].flag_hi),
                     ld_const(&g.runs[w].nlinks), 0u};
    const uint64_t rflag = ((uint64_t)rb.flag_hi << 32) | rb.flag_lo;
    const int32_t nl = (int32_t)rb.nlinks;
    // FUSE: the run's links are entries [rb.links, rb.links + nl) of the (node, dir)
    // order; the first 64, one per lane, have their records loaded now and the
    // deposits they point to with the pulls
    LinkIn<ST> la;
    const bool hl = FUSE && lane < nl;
    if (hl) link_load_record<ST>(fa.L, fa.L.li_ident ? rb.links + lane : ld_el(fa.L.kof, rb.links + lane), la);
    unsigned char *wl = lds + wv * WB;
    uint32_t *lo = reinterpret_cast<uint32_t *>(wl);
    const int32_t k0 = w * 64;
    const int32_t kend = k0 + 64 < g.n_fluid ? k0 + 64 : g.n_fluid;
    const int nsr = g.pitch >> 6;
    const bool live = k0 + lane < kend;
    uint32_t o[9];
    if constexpr (NBR) {
        nbr_offsets<S>(g, w, k0 + lane, live, o);
    } else {
    {
        // walk the row segments of the run; lane = bit of the segment.  The tables
        // of the first RUN_PRE segments are loaded together (a run spans two or
        // three); a run that reaches beyond them continues one segment at a time.
        auto emit = [&](const SegRows &t, int yu, int sx) {
            uint32_t rk[3], lf[3], rt[3], o[9];
            cmp_ranks_from<S>(g, t, yu, sx, lane, rk, lf, rt);
            cmp_pull_offsets(rk, lf, rt, o);
            const int32_t dst = (int32_t)(rk[1] / S) - k0;
            if (((t.fm[1] >> lane) & 1ull) && dst >= 0 && dst < 64) {
#pragma unroll
                for (int i = 0; i < 9; ++i) lo[i * 64 + dst] = o[i];
            }
        };
        int yu = rb.seg / nsr;
        int sx = rb.seg - yu * nsr;
        SegRows tb[RUN_PRE];
        int yk[RUN_PRE], sk[RUN_PRE];
        bool in[RUN_PRE];
#pragma unroll
        for (int k = 0; k < RUN_PRE; ++k) {
            yk[k] = yu;
            sk[k] = sx;
            in[k] = yu < g.ny;
            if (in[k]) ld_seg_rows(g, yu, sx, tb[k]);
            if (++sx == nsr) {
                sx = 0;
                ++yu;
            }
        }
        bool more = true;
#pragma unroll
        for (int k = 0; k < RUN_PRE; ++k) {
            if (!more || !in[k] || tb[k].fb[1] >= kend) {
                more = false;
            } else if (tb[k].fm[1]) {
                emit(tb[k], yk[k], sk[k]);
            }
        }
        // (yu, sx) is the segment after the preloaded ones: at most the sentinel
        // when the last preloaded one was inside the lattice
        if (more && in[RUN_PRE - 1]) {
            for (;;) {
                const int32_t sg = yu * nsr + sx;
                if (ld_const(&g.frow[sg].fluid) >= kend) break;  // the sentinel ends the last run
                SegRows t;
                ld_seg_rows(g, yu, sx, t);
                if (t.fm[1]) emit(t, yu, sx);
                if (++sx == nsr) {
                    sx = 0;
                    ++yu;
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < 9; ++i) o[i] = live ? lo[i * 64 + lane] : 0u;
    }  // NBR
    // every lane has read its offsets before the bytes are reused for the link
    // values and the deposits
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    Pulled<ST> pl;
    pl.live = true;
    // the node type: fluid, flagged from the run table; its link directions come
    // from its side record in bulk_finish
    pl.m = live ? (((rflag >> lane) & 1ull) ? (mask_t)MASK_SIDE : (mask_t)0) : (mask_t)MASK_SOLID;
    // The run's link values are L entries [rb.links, rb.links + nl): loaded as a
    // contiguous range before the pulls, so that they do not wait for the side
    // records that say which node takes which; staged in LDS for bulk_finish.
    // With FUSE they are evaluated here instead.
    const T *Lv = static_cast<const T *>(side.L);
    T *ll = reinterpret_cast<T *>(wl);
    T l0{}, l1{};
    if constexpr (FUSE) {
        if (hl) link_load_deposits<ST>(side.M, side.P, la);
    } else {
        if (lane < nl) l0 = Lv[rb.links + lane];
        if (lane + 64 < nl) l1 = Lv[rb.links + 64 + lane];
    }
    const int64_t P = g.plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) pl.a[i] = C::reg(ld_at_nt(A + i * P, o[i]));
    if constexpr (FUSE) {
        double fx = 0.0, fy = 0.0;
        int obj = -1;
        if (hl) ll[lane] = C::st(link_value<ST>(ph, la, fx, fy, obj), ph.scale);
        for (int j = 64 + lane; j < nl; j += 64) {  // more than 64 links
            const int32_t kk = fa.L.li_ident ? rb.links + j : ld_el(fa.L.kof, rb.links + j);
            double lfx, lfy;
            int o2;
            ll[j] = C::st(link_eval<ST>(ph, fa.L, side.M, side.P, kk, lfx, lfy, o2), ph.scale);
            if (obj < 0 || o2 == obj) {
                obj = o2;
                fx += lfx;
                fy += lfy;
            } else {
                add_force(fa.bank, fa.fsum, o2, lfx, lfy);
            }
        }
        // the run's force: one partial (entry w) when its links belong to one
        // object, else added per lane
        int top = obj;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) top = max(top, __shfl_xor(top, off));
        if (__all(obj == top || obj < 0)) {
            const double sx = wave_sum_to_last(fx), sy = wave_sum_to_last(fy);
            if (lane == 63) {
                fa.wpart[w] = make_double2(sx, sy);
                fa.wobj[w] = top;
            }
        } else {
            if (obj >= 0) add_force(fa.bank, fa.fsum, obj, fx, fy);
            if (lane == 0) fa.wobj[w] = -1;
        }
    } else {
        if (lane < nl) ll[lane] = l0;
        if (lane + 64 < nl) ll[64 + lane] = l1;
        for (int j = 128 + lane; j < nl; j += 64) ll[j] = Lv[rb.links + j];  // more than 128 links (rare)
    }
    pl.own = (uint32_t)(k0 + lane) * S;
    pl.own_in = 0;
    pl.own_out = 0;
    __builtin_amdgcn_sched_barrier(0);
    bulk_finish<ST, false, FORCE, 256, false, true, false, COLL, true>(
        g, ph, B, mask, nullptr, side, live ? 0 : g.nx, 0, 0, reinterpret_cast<R(*)[3 * 64]>(wl),
        reinterpret_cast<T(*)[8 * 64]>(wl + 64 * 3 * sizeof(R)), pl, nullptr, reinterpret_cast<T(*)[8 * 64]>(wl),
        SegBase{rb.flagged, rb.links, rb.pops, 0});
}

// The same step with the links of each wavefront's nodes evaluated in the
// wavefront itself (FUSE): 256 lanes along x per block.
template <int ST, bool OPEN, bool FORCE, bool STORE_SOLID, bool CMP, int COLL>
__global__ __launch_bounds__(256) void bulk_fused_kernel(Grid g, Phys ph,
                                                         const typename Codec<ST>::T *__restrict__ A,
                                                         typename Codec<ST>::T *__restrict__ B,
                                                         const mask_t *__restrict__ mask,
                                                         const typename Codec<ST>::R *__restrict__ uin,
                                                         Side side, FuseArgs fa, double *__restrict__ zero_bank,
                                                         int32_t n_zero, int32_t xcd, double inv_nbx)
{
    using R = typename Codec<ST>::R;
    using T = typename Codec<ST>::T;
    __shared__ R lds_m[4][3 * 64];
    __shared__ T lds_p[4][8 * 64];
    __shared__ T lds_l[4][8 * 64];
    const int tid = threadIdx.x;
    const int64_t nb = (int64_t)gridDim.x * gridDim.y;
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    zero_bank_part(zero_bank, n_zero, b, nb, tid);
    int tx = blockIdx.x, ty = blockIdx.y;
    if (xcd) {
        const int32_t n = (int32_t)nb, q = n >> 3, r = n & 7, k = (int32_t)b & 7;
        const int32_t tile = k * q + (k < r ? k : r) + ((int32_t)b >> 3);
        ty = (int)((tile + 0.5) * inv_nbx);
        tx = tile - ty * (int)gridDim.x;
        if (tx < 0) tx += gridDim.x, --ty;
        if (tx >= (int)gridDim.x) tx -= gridDim.x, ++ty;
    }
    bulk_body<ST, OPEN, FORCE, 256, STORE_SOLID, CMP, true, COLL>(g, ph, A, B, mask, uin, side,
                                                                  tx * 256 + threadIdx.x, ty, tid >> 6, lds_m, lds_p,
                                                                  &fa, lds_l);
}

// Batched form: one launch over the tiles of many lattices.  Each block reads its
// tile (instance, first row, first column) and the instance's descriptor; the
// populations, masks, inlet rows and segment tables of all instances live in
// shared arrays at per-instance offsets, while side records, deposits and link
// values use global numbering.
template <int ST, bool OPEN, bool FORCE, int BX, bool STORE_SOLID, int ROWS, int COLL>
__global__ __launch_bounds__(256) void bulk_batch_kernel(const BatchInst *__restrict__ insts,
                                                         const BatchTile *__restrict__ tiles, int64_t ntiles,
                                                         Phys ph0,
                                                         const typename Codec<ST>::T *__restrict__ A,
                                                         typename Codec<ST>::T *__restrict__ B,
                                                         const mask_t *__restrict__ mask,
                                                         const typename Codec<ST>::R *__restrict__ uin,
                                                         Side side, double *__restrict__ zero_bank,
                                                         int32_t n_zero, const double2 *__restrict__ red_part,
                                                         const int32_t *__restrict__ red_obj, int64_t red_n,
                                                         double *__restrict__ red_bank,
                                                         double *__restrict__ red_sum)
{
    using R = typename Codec<ST>::R;
    using T = typename Codec<ST>::T;
    __shared__ R lds_m[4][3 * 64];
    __shared__ T lds_p[4][8 * 64];
    const int tid = threadIdx.y * BX + threadIdx.x;
    zero_bank_part(zero_bank, n_zero, blockIdx.x, gridDim.x, tid);
    force_reduce_part(red_part, red_obj, red_n, red_bank, red_sum, blockIdx.x, tid);
    // the tile table and instance records are read through the scalar cache
    auto finish = [&](const BatchTile &t, const BatchInst &I, const Pulled<ST> &pl) {
        Phys ph = ph0;
        ph.omega = I.omega;
        ph.gx = I.gx;
        ph.gy = I.gy;
        Side sd = side;
        sd.seg = side.seg + I.seg_off;
        bulk_finish<ST, OPEN, FORCE, BX, STORE_SOLID, false, false, COLL>(I.g, ph, B + I.pop_off, mask + I.mask_off,
                                                      uin + 2 * (int64_t)I.uin_off, sd, t.x0 + threadIdx.x,
                                                      t.y0 + threadIdx.y, tid >> 6, lds_m, lds_p, pl);
    };
    if (ROWS == 1) {
        const BatchTile t = ld_const_record(tiles + blockIdx.x);
        const BatchInst I = ld_const_record(insts + t.inst);
        Pulled<ST> pl;
        bulk_issue<ST, OPEN, false>(I.g, A + I.pop_off, mask + I.mask_off, t.x0 + threadIdx.x, t.y0 + threadIdx.y,
                                    pl);
        __builtin_amdgcn_sched_barrier(0);
        finish(t, I, pl);
    } else {
        // two tile-table entries per block: the second one's pulls are in flight
        // while the first is finished
        const int64_t k0 = 2 * (int64_t)blockIdx.x;
        const bool has1 = k0 + 1 < ntiles;
        const BatchTile t0 = ld_const_record(tiles + k0), t1 = ld_const_record(tiles + (has1 ? k0 + 1 : k0));
        const BatchInst I0 = ld_const_record(insts + t0.inst), I1 = ld_const_record(insts + t1.inst);
        Pulled<ST> p0, p1;
        bulk_issue<ST, OPEN, false>(I0.g, A + I0.pop_off, mask + I0.mask_off, t0.x0 + threadIdx.x,
                                    t0.y0 + threadIdx.y, p0);
        if (has1)
            bulk_issue<ST, OPEN, false>(I1.g, A + I1.pop_off, mask + I1.mask_off, t1.x0 + threadIdx.x,
                                        t1.y0 + threadIdx.y, p1);
        __builtin_amdgcn_sched_barrier(0);
        finish(t0, I0, p0);
        if (has1) {
            // the first tile's deposit flush has read the wavefront's LDS staging
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            finish(t1, I1, p1);
        }
    }
}

// ---------------------------------------------------------------------------
// Initialisation, deposit refresh, moments and mass.
// ---------------------------------------------------------------------------
template <int ST>
__global__ void refresh_kernel(Grid g, Phys ph, const typename Codec<ST>::T *__restrict__ A, Side side,
                               int moments)
{
    using C = Codec<ST>;
    using T = typename C::T;
    using R = typename C::R;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= side.K) return;
    const int32_t nd = side.mnode[k];
    const int32_t n = node_offset(g, nd % g.pitch, nd / g.pitch);
    const uint32_t rec = side.rec[k];
    T *Pv = static_cast<T *>(side.P);
    int32_t pb = side.pbase[k];
#pragma unroll
    for (int d = 1; d < 9; ++d)
        if (rec & (1u << (d + 7))) Pv[pb++] = A[(int64_t)d * g.plane + n];
    if (!moments) return;
    R dr = R(0), jx = R(0), jy = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R v = C::ld(A[(int64_t)i * g.plane + n], ph.inv_scale);
        dr += v;
        jx += R(CX[i]) * v;
        jy += R(CY[i]) * v;
    }
    const R ir = inv_rho_m1(dr);
    R *Mv = static_cast<R *>(side.M);
    Mv[3 * k] = dr;
    Mv[3 * k + 1] = jx + jx * ir - R(0.5) * R(ph.gx);
    Mv[3 * k + 2] = jy + jy * ir - R(0.5) * R(ph.gy);
}

template <int ST>
__global__ void init_kernel(Grid g, Phys ph, typename Codec<ST>::T *__restrict__ A,
                            const mask_t *__restrict__ mask, const double *__restrict__ stage,
                            int32_t y0, int32_t rows)
{
    using C = Codec<ST>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)rows * g.nx) return;
    const int y = y0 + (int)(k / g.nx), x = (int)(k % g.nx);
    const bool solid = (mask[y * g.pitch + x] & MASK_SOLID) != 0;
    if (solid && g.compact) return;  // no slot
    const int32_t n = node_offset(g, x, y);
    const double rho = stage[3 * k], ux = stage[3 * k + 1], uy = stage[3 * k + 2];
    const double usq = ux * ux + uy * uy;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double eu = CX[i] * ux + CY[i] * uy;
        const double d = solid ? 0.0 : deq<double>(wgt<double>(i), eu, rho - 1.0, usq);
        A[(int64_t)i * g.plane + n] = C::st((typename Codec<ST>::R)d, ph.scale);
    }
}

// Density and physical velocity (Guo's half-force shift) of fluid node (x, y) in
// FP64; 0 for solid nodes.
template <int ST>
__device__ __forceinline__ void node_moments(const Grid &g, const Phys &ph, const typename Codec<ST>::T *__restrict__ A,
                                             const mask_t *__restrict__ mask, int x, int y, double &rho, double &ux,
                                             double &uy)
{
    using C = Codec<ST>;
    if (mask[y * g.pitch + x] & MASK_SOLID) {
        rho = ux = uy = 0.0;
        return;
    }
    const int32_t n = node_offset(g, x, y);
    double dr = 0, jx = 0, jy = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double v = (double)C::ld(A[(int64_t)i * g.plane + n], ph.inv_scale);
        dr += v;
        jx += CX[i] * v;
        jy += CY[i] * v;
    }
    rho = 1.0 + dr;
    ux = jx / rho - 0.5 * ph.gx;
    uy = jy / rho - 0.5 * ph.gy;
}

template <int ST>
__global__ void moments_kernel(Grid g, Phys ph, const typename Codec<ST>::T *__restrict__ A,
                               const mask_t *__restrict__ mask, double *__restrict__ stage,
                               int32_t y0, int32_t rows)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)rows * g.nx) return;
    const int y = y0 + (int)(k / g.nx), x = (int)(k % g.nx);
    node_moments<ST>(g, ph, A, mask, x, y, stage[3 * k], stage[3 * k + 1], stage[3 * k + 2]);
}

// The moments of every node into three caller arrays of ny*nx values (y*nx + x),
// rounded to OT; a null array is skipped.
template <int ST, class OT>
__global__ void moments_out_kernel(Grid g, Phys ph, const typename Codec<ST>::T *__restrict__ A,
                                   const mask_t *__restrict__ mask, OT *__restrict__ rho, OT *__restrict__ ux,
                                   OT *__restrict__ uy)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)g.ny * g.nx) return;
    const int y = (int)(k / g.nx), x = (int)(k % g.nx);
    double r, vx, vy;
    node_moments<ST>(g, ph, A, mask, x, y, r, vx, vy);
    if (rho) rho[k] = (OT)r;
    if (ux) ux[k] = (OT)vx;
    if (uy) uy[k] = (OT)vy;
}


// Per-block FP64 partials over the fluid nodes: MAXDEV = false sums the mass
// sum_i f_i; MAXDEV = true takes max_i |f_i - w_i| (sizes the 16-bit scale).
template <int ST, bool MAXDEV>
__global__ __launch_bounds__(MASS_THREADS) void mass_kernel(Grid g, Phys ph,
                                                           const typename Codec<ST>::T *__restrict__ A,
                                                           const mask_t *__restrict__ mask,
                                                           double *__restrict__ partials)
{
    using C = Codec<ST>;
    __shared__ double red[MASS_THREADS / 64];
    const int64_t N = (int64_t)g.nx * g.ny;
    double s = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * MASS_THREADS + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * MASS_THREADS) {
        const int y = (int)(k / g.nx), x = (int)(k % g.nx);
        if (mask[y * g.pitch + x] & MASK_SOLID) continue;
        const int32_t n = node_offset(g, x, y);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double d = (double)C::ld(A[(int64_t)i * g.plane + n], ph.inv_scale);
            if (MAXDEV) s = fmax(s, fabs(d));
            else s += d + wgt<double>(i);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(s, off);
        s = MAXDEV ? fmax(s, o) : s + o;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < MASS_THREADS / 64; ++k) t = MAXDEV ? fmax(t, red[k]) : t + red[k];
        partials[blockIdx.x] = t;
    }
}

template <int ST>
hipError_t link_t(const Grid &g, const Phys &ph, const Links &L, const Side &side, const Reduce &red,
                  double *bank, double *fsum, int block, hipStream_t s, ForceReduce *defer)
{
    if (defer) *defer = ForceReduce{red.wpart, red.wobj, 0, bank, fsum};
    if (L.n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((L.n + block - 1) / block);
    hipLaunchKernelGGL(link_kernel<ST>, dim3(blocks), dim3(block), 0, s, g, ph, L, side, red.wpart,
                       red.wobj, bank, fsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !bank) return e;
    // one partial per run of 64 links
    const ForceReduce fr{red.wpart, red.wobj, (L.n + 63) / 64, bank, fsum};
    if (defer) {
        *defer = fr;
        return hipSuccess;
    }
    const int64_t lanes = (fr.nw + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
    hipLaunchKernelGGL(force_reduce_kernel, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, fr.wpart,
                       fr.wobj, fr.nw, fr.bank, fr.fsum);
    return hipGetLastError();
}

template <int ST, bool OPEN, bool FORCE, bool SS, bool CMP>
hipError_t bulk_fused_t(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                        const void *uin, const Side &side, const FuseArgs &fa, double *zb, int32_t nz,
                        int32_t xcd, hipStream_t s)
{
    using C = Codec<ST>;
    dim3 grid((g.nx + 255) / 256, g.ny);
    hipLaunchKernelGGL((bulk_fused_kernel<ST, OPEN, FORCE, SS, CMP, 0>), grid, dim3(256), 0, s, g, ph,
                       static_cast<const typename C::T *>(A), static_cast<typename C::T *>(B), mask,
                       static_cast<const typename C::R *>(uin), side, fa, zb, nz, xcd, 1.0 / grid.x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one force partial per 64-node row segment
    const int64_t nw = (int64_t)(g.pitch / 64) * g.ny;
    const int64_t lanes = (nw + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
    hipLaunchKernelGGL(force_reduce_kernel, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, fa.wpart,
                       fa.wobj, nw, fa.bank, fa.fsum);
    return hipGetLastError();
}

template <int ST, bool OPEN, bool FORCE>
hipError_t bulk_fused_shape(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                            const void *uin, const Side &side, const FuseArgs &fa, double *zb, int32_t nz,
                            const BulkConfig &cf, hipStream_t s)
{
    if (cf.block_x != 256) return hipErrorInvalidValue;
    if (g.compact) return bulk_fused_t<ST, OPEN, FORCE, false, true>(g, ph, A, B, mask, uin, side, fa, zb, nz, cf.xcd, s);
    if (cf.store_solid) return bulk_fused_t<ST, OPEN, FORCE, true, false>(g, ph, A, B, mask, uin, side, fa, zb, nz, cf.xcd, s);
    return bulk_fused_t<ST, OPEN, FORCE, false, false>(g, ph, A, B, mask, uin, side, fa, zb, nz, cf.xcd, s);
}

template <int ST, bool FORCE, int COLL, bool FUSE>
hipError_t bulk_run_t(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask, const Side &side,
                      const FuseArgs &fa, double *zb, int32_t nz, int32_t xcd, bool nbr, hipStream_t s,
                      const ForceReduce &fr);

// The fused form (links inside the bulk kernel): BGK in the row-segment mapping,
// BGK or MRT in runs of fluid nodes.
template <int ST>
hipError_t bulk_fused_dispatch(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                               const void *uin, const Side &side, const FuseArgs &fa, double *zb, int32_t nz,
                               const BulkConfig &cf, hipStream_t s)
{
    const bool force = ph.gx != 0.0 || ph.gy != 0.0;
    if (cf.runs) {
        // runs of fluid nodes (BGK or MRT)
        const ForceReduce none{};
#define LBM_RUNF(FV, CV) bulk_run_t<ST, FV, CV, true>(g, ph, A, B, mask, side, fa, zb, nz, cf.xcd, cf.runs == 2, s, none)
        if (ph.coll == LBM_COLLISION_MRT) return force ? LBM_RUNF(true, 1) : LBM_RUNF(false, 1);
        if (ph.coll == LBM_COLLISION_BGK) return force ? LBM_RUNF(true, 0) : LBM_RUNF(false, 0);
#undef LBM_RUNF
        return hipErrorInvalidValue;
    }
    if (ph.coll != LBM_COLLISION_BGK) return hipErrorInvalidValue;
    if (g.x_open)
        return force ? bulk_fused_shape<ST, true, true>(g, ph, A, B, mask, uin, side, fa, zb, nz, cf, s)
                     : bulk_fused_shape<ST, true, false>(g, ph, A, B, mask, uin, side, fa, zb, nz, cf, s);
    return force ? bulk_fused_shape<ST, false, true>(g, ph, A, B, mask, uin, side, fa, zb, nz, cf, s)
                 : bulk_fused_shape<ST, false, false>(g, ph, A, B, mask, uin, side, fa, zb, nz, cf, s);
}

template <int ST, bool OPEN, bool FORCE, int BX, bool SS, bool CMP, int ROWS, int COLL>
hipError_t bulk_t(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                  const void *uin, const Side &side, double *zb, int32_t nz, int32_t xcd, hipStream_t s,
                  const ForceReduce &fr)
{
    using C = Codec<ST>;
    constexpr int BY = 256 / BX;
    dim3 grid((g.nx + BX - 1) / BX, (g.ny + ROWS * BY - 1) / (ROWS * BY));
    const int64_t nb = (int64_t)grid.x * grid.y;
    if (fr.nw > nb * 256 * FOLD_CHUNK) return hipErrorInvalidValue;  // more partials than lanes
    hipLaunchKernelGGL((bulk_kernel<ST, OPEN, FORCE, BX, SS, CMP, ROWS, COLL>), grid, dim3(BX, BY), 0, s, g, ph,
                       static_cast<const typename C::T *>(A), static_cast<typename C::T *>(B), mask,
                       static_cast<const typename C::R *>(uin), side, zb, nz, xcd, 1.0 / grid.x, fr.wpart,
                       fr.wobj, fr.nw, fr.bank, fr.fsum);
    return hipGetLastError();
}

// Launch shapes: BGK in every shape; MRT with 256-lane rows (one or two row
// segments per wavefront, both layouts, with or without solid stores).
template <int ST, bool OPEN, bool FORCE, int COLL>
hipError_t bulk_shape(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                      const void *uin, const Side &side, double *zb, int32_t nz, const BulkConfig &cf,
                      hipStream_t s, const ForceReduce &fr)
{
#define LBM_BULK(BXV, SSV, CMPV, ROWSV) \
    bulk_t<ST, OPEN, FORCE, BXV, SSV, CMPV, ROWSV, COLL>(g, ph, A, B, mask, uin, side, zb, nz, cf.xcd, s, fr)
    if (cf.rows == 2 || COLL != LBM_COLLISION_BGK) {
        if (cf.block_x != 256) return hipErrorInvalidValue;
        // no solid slots to store in the compact layout
        if (g.compact) return cf.rows == 2 ? LBM_BULK(256, false, true, 2) : LBM_BULK(256, false, true, 1);
        if (cf.rows == 2) return cf.store_solid ? LBM_BULK(256, true, false, 2) : LBM_BULK(256, false, false, 2);
        return cf.store_solid ? LBM_BULK(256, true, false, 1) : LBM_BULK(256, false, false, 1);
    }
    if constexpr (COLL == LBM_COLLISION_BGK) {
        if (g.compact) {
            if (cf.block_x == 64) return LBM_BULK(64, false, true, 1);
            if (cf.block_x == 128) return LBM_BULK(128, false, true, 1);
            if (cf.block_x == 256) return LBM_BULK(256, false, true, 1);
            return hipErrorInvalidValue;
        }
        if (cf.block_x == 64) return cf.store_solid ? LBM_BULK(64, true, false, 1) : LBM_BULK(64, false, false, 1);
        if (cf.block_x == 128) return cf.store_solid ? LBM_BULK(128, true, false, 1) : LBM_BULK(128, false, false, 1);
        if (cf.block_x == 256) return cf.store_solid ? LBM_BULK(256, true, false, 1) : LBM_BULK(256, false, false, 1);
    }
#undef LBM_BULK
    return hipErrorInvalidValue;
}

template <int ST, bool FORCE, int COLL, bool FUSE>
hipError_t bulk_run_t(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask, const Side &side,
                      const FuseArgs &fa, double *zb, int32_t nz, int32_t xcd, bool nbr, hipStream_t s,
                      const ForceReduce &fr)
{
    using C = Codec<ST>;
    if (!g.compact || g.x_open || !g.runs || g.nruns < 0) return hipErrorInvalidValue;
    if (nbr && !g.nbr) return hipErrorInvalidValue;  // no neighbour words for this geometry
    // four runs per block; at least enough blocks for the force partials and one
    // to clear the force bank
    constexpr int64_t per_block = 256 * FOLD_CHUNK;
    int64_t nb = ((int64_t)g.nruns + 3) / 4;
    if (nb * per_block < fr.nw) nb = (fr.nw + per_block - 1) / per_block;
    if (nb < 1) nb = 1;
    if (nbr)
        hipLaunchKernelGGL((bulk_run_kernel<ST, FORCE, COLL, FUSE, true>), dim3((unsigned)nb), dim3(256), 0, s, g,
                           ph, static_cast<const typename C::T *>(A), static_cast<typename C::T *>(B), mask, side, fa,
                           zb, nz, xcd, fr.wpart, fr.wobj, fr.nw, fr.bank, fr.fsum);
    else
        hipLaunchKernelGGL((bulk_run_kernel<ST, FORCE, COLL, FUSE, false>), dim3((unsigned)nb), dim3(256), 0, s, g,
                           ph, static_cast<const typename C::T *>(A), static_cast<typename C::T *>(B), mask, side, fa,
                           zb, nz, xcd, fr.wpart, fr.wobj, fr.nw, fr.bank, fr.fsum);
    hipError_t e = hipGetLastError();
    if (!FUSE || e != hipSuccess || g.nruns == 0) return e;
    // the fused form's force partials, one per run
    const int64_t nw = g.nruns;
    const int64_t lanes = (nw + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
    hipLaunchKernelGGL(force_reduce_kernel, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, fa.wpart,
                       fa.wobj, nw, fa.bank, fa.fsum);
    return hipGetLastError();
}

template <int ST, int COLL>
hipError_t bulk_coll(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                     const void *uin, const Side &side, double *zb, int32_t nz, const BulkConfig &cf,
                     hipStream_t s, const ForceReduce &fr)
{
    const bool force = ph.gx != 0.0 || ph.gy != 0.0;
    if (cf.runs)
        return force ? bulk_run_t<ST, true, COLL, false>(g, ph, A, B, mask, side, FuseArgs{}, zb, nz, cf.xcd,
                                                         cf.runs == 2, s, fr)
                     : bulk_run_t<ST, false, COLL, false>(g, ph, A, B, mask, side, FuseArgs{}, zb, nz, cf.xcd,
                                                          cf.runs == 2, s, fr);
    if (g.x_open)
        return force ? bulk_shape<ST, true, true, COLL>(g, ph, A, B, mask, uin, side, zb, nz, cf, s, fr)
                     : bulk_shape<ST, true, false, COLL>(g, ph, A, B, mask, uin, side, zb, nz, cf, s, fr);
    return force ? bulk_shape<ST, false, true, COLL>(g, ph, A, B, mask, uin, side, zb, nz, cf, s, fr)
                 : bulk_shape<ST, false, false, COLL>(g, ph, A, B, mask, uin, side, zb, nz, cf, s, fr);
}

template <int ST>
hipError_t bulk_dispatch(const Grid &g, const Phys &ph, const void *A, void *B, const mask_t *mask,
                         const void *uin, const Side &side, double *zb, int32_t nz, const BulkConfig &cf,
                         hipStream_t s, const ForceReduce &fr)
{
    if (ph.coll == LBM_COLLISION_MRT)
        return bulk_coll<ST, LBM_COLLISION_MRT>(g, ph, A, B, mask, uin, side, zb, nz, cf, s, fr);
    if (ph.coll == LBM_COLLISION_BGK)
        return bulk_coll<ST, LBM_COLLISION_BGK>(g, ph, A, B, mask, uin, side, zb, nz, cf, s, fr);
    return hipErrorInvalidValue;
}

template <int ST, bool OPEN, bool FORCE, bool SS, int ROWS, int COLL>
hipError_t bulk_batch_t(const BatchInst *insts, const BatchTile *tiles, int64_t ntiles, const Phys &ph,
                        const void *A, void *B, const mask_t *mask, const void *uin, const Side &side,
                        double *zb, int32_t nz, hipStream_t s, const ForceReduce &fr)
{
    using C = Codec<ST>;
    constexpr int BX = BATCH_BX, BY = 256 / BATCH_BX;
    const int64_t nb = (ntiles + ROWS - 1) / ROWS;
    if (fr.nw > nb * 256 * FOLD_CHUNK) return hipErrorInvalidValue;  // more partials than lanes
    hipLaunchKernelGGL((bulk_batch_kernel<ST, OPEN, FORCE, BX, SS, ROWS, COLL>), dim3((unsigned)nb), dim3(BX, BY),
                       0, s, insts, tiles, ntiles, ph, static_cast<const typename C::T *>(A),
                       static_cast<typename C::T *>(B), mask, static_cast<const typename C::R *>(uin), side,
                       zb, nz, fr.wpart, fr.wobj, fr.nw, fr.bank, fr.fsum);
    return hipGetLastError();
}

template <int ST, bool OPEN, bool FORCE, int COLL>
hipError_t bulk_batch_shape(const BatchInst *insts, const BatchTile *tiles, int64_t ntiles, const Phys &ph,
                            const void *A, void *B, const mask_t *mask, const void *uin, const Side &side,
                            double *zb, int32_t nz, bool ss, int rows, hipStream_t s, const ForceReduce &fr)
{
#define LBM_BATCH(SSV, ROWSV) \
    bulk_batch_t<ST, OPEN, FORCE, SSV, ROWSV, COLL>(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, s, fr)
    if (rows == 2) return ss ? LBM_BATCH(true, 2) : LBM_BATCH(false, 2);
    return ss ? LBM_BATCH(true, 1) : LBM_BATCH(false, 1);
#undef LBM_BATCH
}

template <int ST, int COLL>
hipError_t bulk_batch_coll(const BatchInst *insts, const BatchTile *tiles, int64_t ntiles, const Phys &ph,
                           const void *A, void *B, const mask_t *mask, const void *uin, const Side &side,
                           double *zb, int32_t nz, bool open, bool force, bool ss, int rows, hipStream_t s,
                           const ForceReduce &fr)
{
    if (open)
        return force ? bulk_batch_shape<ST, true, true, COLL>(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, ss, rows, s, fr)
                     : bulk_batch_shape<ST, true, false, COLL>(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, ss, rows, s, fr);
    return force ? bulk_batch_shape<ST, false, true, COLL>(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, ss, rows, s, fr)
                 : bulk_batch_shape<ST, false, false, COLL>(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, ss, rows, s, fr);
}

template <int ST>
hipError_t bulk_batch_dispatch(const BatchInst *insts, const BatchTile *tiles, int64_t ntiles,
                               const Phys &ph, const void *A, void *B, const mask_t *mask, const void *uin,
                               const Side &side, double *zb, int32_t nz, bool open, bool force, bool ss,
                               int rows, hipStream_t s, const ForceReduce &fr)
{
    if (ph.coll == LBM_COLLISION_MRT)
        return bulk_batch_coll<ST, LBM_COLLISION_MRT>(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, open,
                                                      force, ss, rows, s, fr);
    if (ph.coll == LBM_COLLISION_BGK)
        return bulk_batch_coll<ST, LBM_COLLISION_BGK>(insts, tiles, ntiles, ph, A, B, mask, uin, side, zb, nz, open,
                                                      force, ss, rows, s, fr);
    return hipErrorInvalidValue;
}

template <int ST>
hipError_t refresh_t(const Grid &g, const Phys &ph, const void *A, const Side &side, bool moments,
                     hipStream_t s)
{
    if (side.K == 0) return hipSuccess;
    hipLaunchKernelGGL(refresh_kernel<ST>, dim3((unsigned)((side.K + 255) / 256)), dim3(256), 0, s, g,
                       ph, static_cast<const typename Codec<ST>::T *>(A), side, moments ? 1 : 0);
    return hipGetLastError();
}


template <int ST>
hipError_t init_t(const Grid &g, const Phys &ph, void *A, const mask_t *mask, const double *stage,
                  int32_t y0, int32_t rows, hipStream_t s)
{
    const int64_t n = (int64_t)rows * g.nx;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel<ST>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, ph,
                       static_cast<typename Codec<ST>::T *>(A), mask, stage, y0, rows);
    return hipGetLastError();
}
template <int ST>
hipError_t moments_t(const Grid &g, const Phys &ph, const void *A, const mask_t *mask,
                     double *stage, int32_t y0, int32_t rows, hipStream_t s)
{
    const int64_t n = (int64_t)rows * g.nx;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(moments_kernel<ST>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, ph,
                       static_cast<const typename Codec<ST>::T *>(A), mask, stage, y0, rows);
    return hipGetLastError();
}
template <int ST>
hipError_t moments_out_t(const Grid &g, const Phys &ph, const void *A, const mask_t *mask, void *rho, void *ux,
                         void *uy, bool fp64, hipStream_t s)
{
    const int64_t n = (int64_t)g.ny * g.nx;
    if (n == 0 || (!rho && !ux && !uy)) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    const auto *a = static_cast<const typename Codec<ST>::T *>(A);
    if (fp64)
        hipLaunchKernelGGL((moments_out_kernel<ST, double>), grid, block, 0, s, g, ph, a, mask,
                           static_cast<double *>(rho), static_cast<double *>(ux), static_cast<double *>(uy));
    else
        hipLaunchKernelGGL((moments_out_kernel<ST, float>), grid, block, 0, s, g, ph, a, mask,
                           static_cast<float *>(rho), static_cast<float *>(ux), static_cast<float *>(uy));
    return hipGetLastError();
}
template <int ST>
hipError_t mass_t(const Grid &g, const Phys &ph, const void *A, const mask_t *mask,
                  double *partials, int32_t nb, bool maxdev, hipStream_t s)
{
    if (maxdev)
        hipLaunchKernelGGL((mass_kernel<ST, true>), dim3(nb), dim3(MASS_THREADS), 0, s, g, ph,
                           static_cast<const typename Codec<ST>::T *>(A), mask, partials);
    else
        hipLaunchKernelGGL((mass_kernel<ST, false>), dim3(nb), dim3(MASS_THREADS), 0, s, g, ph,
                           static_cast<const typename Codec<ST>::T *>(A), mask, partials);
    return hipGetLastError();
}

}  // namespace
}  // namespace lbm
