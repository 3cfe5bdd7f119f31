// Adjoint (reverse-mode) kernels of the D2Q9 BGK step with VIBB walls
// (arXiv:1903.01111): the transpose of the linearised step, run backwards over
// a recomputed trajectory.
//
// Forward step t -> t+1 on the post-collision state S_t (Sections 2, 3.1, 4.3):
//   v_l      = VIBB(S_t at x_f and x_ff, q_l, u_w,l)         every link l
//   f_i(x)   = S_t(x - e_i, i), or v_l where x - e_i is solid  interior nodes
//   S''(x)   = BGK + Guo collision of f(x)
//   S_t+1    = S'' on interior nodes; inlet column from S''(1, y) and u_in(y);
//              outlet column = S''(nx-2, y)
//   F_t      = sum_l e_i'(S_t(x_f, i') + v_l)                   force of step t
// Adjoint, with lambda_t = dJ/dS_t and C_t(x) = dJ/df(x) (pre-collision):
//   adj_bulk  (one lane per node, step t): lambda_t+1(x) is gathered from C_t+1
//             of the nodes that pulled from x plus the node's side record (the
//             link adjoints of step t+1); open columns fold into their
//             neighbour lanes; the collision Jacobian^T gives C_t(x), whose
//             cut directions go to the links (Lbar);
//   adj_link  (one lane per link): Lbar plus the force weight is the adjoint of
//             v_l; the VIBB Jacobian^T spreads it over the moments and the
//             populations of x_f and x_ff (side records, FP64 atomics) and adds
//             v-bar dv/dq and v-bar dv/du_w to FP64 accumulators; the same lane
//             recomputes the link values of the preceding step for adj_bulk.
// No MFMA: the reverse step is as memory-bound as the forward one.
#include "lbm_device.h"

namespace lbm {
namespace {

constexpr int SIG = 12;  // doubles per flagged node: alpha, beta_x, beta_y, gamma_1..8, pad

// f^eq_i per unit density and its velocity gradient (Section 2, Eq. feq):
//   phi_i(u) = w_i (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u)
//   grad phi_i(u) = w_i (3 e + 9 (e.u) e - 3 u)
template <class R>
__device__ __forceinline__ R phi(R w, R ex, R ey, R ux, R uy)
{
    const R eu = ex * ux + ey * uy;
    return w * (R(1) + poly(eu, ux * ux + uy * uy));
}
template <class R>
__device__ __forceinline__ void gphi(R w, R ex, R ey, R ux, R uy, R &gx, R &gy)
{
    const R eu = ex * ux + ey * uy;
    gx = w * (R(3) * ex + R(9) * eu * ex - R(3) * ux);
    gy = w * (R(3) * ey + R(9) * eu * ey - R(3) * uy);
}

// Moments of a post-collision node from its nine stored deviations:
// dr = rho - 1, (tx, ty) = j/rho, (ux, uy) = j/rho - g/2 (physical velocity).
template <int ST>
struct NodeState {
    using R = typename Codec<ST>::R;
    R d[9];
    R dr, tx, ty, ux, uy;
    __device__ __forceinline__ void load(const typename Codec<ST>::T *__restrict__ S, int64_t plane,
                                         int32_t off, const Phys &ph)
    {
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = Codec<ST>::ld(S[i * plane + off], ph.inv_scale);
        dr = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
        const R jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
        const R jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
        const R ir = inv_rho_m1(dr);
        tx = jx + jx * ir;
        ty = jy + jy * ir;
        ux = tx - R(0.5) * R(ph.gx);
        uy = ty - R(0.5) * R(ph.gy);
    }
    // runtime-indexed population (the link direction differs per lane)
    __device__ __forceinline__ R pop(int i) const
    {
        R v = d[0];
#pragma unroll
        for (int k = 1; k < 9; ++k)
            if (k == i) v = d[k];
        return v;
    }
};

// Adds the adjoint (rho-bar, u-bar, f+_i'-bar) of one node's moments and one of
// its populations to the node's side record, in the form the reverse bulk
// kernel consumes: lambda_j += alpha + beta.e_j (+ gamma_j), since
// d rho / d f_j = 1 and d u / d f_j = (e_j - j/rho)/rho.
template <class R>
__device__ __forceinline__ void add_record(double *__restrict__ rec, R rbar, R ubx, R uby, R pbar, int ip,
                                           R rho, R tx, R ty)
{
    const R irho = R(1) / rho;
    unsafeAtomicAdd(&rec[0], (double)(rbar - (ubx * tx + uby * ty) * irho));
    unsafeAtomicAdd(&rec[1], (double)(ubx * irho));
    unsafeAtomicAdd(&rec[2], (double)(uby * irho));
    unsafeAtomicAdd(&rec[2 + ip], (double)pbar);
}

// ---------------------------------------------------------------------------
// Link adjoint: one lane per link.  With Sn (= S_t+1) it back-propagates the
// link's adjoint of step t+1; with Sc (= S_t) it recomputes the link value of
// step t into Lf for the reverse bulk kernel of step t.
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(256) void adj_link_kernel(Grid g, Phys ph, Links L, const int32_t *__restrict__ mnode,
                                                       const typename Codec<ST>::T *__restrict__ Sn,
                                                       const typename Codec<ST>::T *__restrict__ Sc,
                                                       typename Codec<ST>::R *__restrict__ Lf,
                                                       const typename Codec<ST>::R *__restrict__ Lbar,
                                                       double *__restrict__ sig, double *__restrict__ dq,
                                                       double *__restrict__ duw, int32_t obj, double djx,
                                                       double djy)
{
    using R = typename Codec<ST>::R;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L.n) return;
    const uint32_t meta = L.meta[l];
    const int ip = (int)(meta & 15u);
    const int ob = (int)(meta >> 8);
    const R ex = R(cx_of(ip)), ey = R(cy_of(ip));
    const R w = ip <= 4 ? R(1) / R(9) : R(1) / R(36);
    const R q = static_cast<const R *>(L.q)[l];
    R uwx = R(0), uwy = R(0);
    if (L.uw) {
        uwx = static_cast<const R *>(L.uw)[2 * l];
        uwy = static_cast<const R *>(L.uw)[2 * l + 1];
    }
    const R rho0 = R(ph.rho0);
    const int32_t sf = L.sf[l], sff = L.sff[l];
    const int32_t of = mnode[sf];
    const int32_t off = sff >= 0 ? mnode[sff] : -1;
    const int32_t li = L.li[l];
    const R a2q = R(2) * q, b2q = R(1) - R(2) * q;
    const bool first = q <= R(0.5);
    // coefficients of u_d = u*_d/3 + 2 u**_d/3 on u_f, u_ff and u_w
    const R inv1q = R(1) / (R(1) + q);
    const R cuf = first ? a2q / R(3) : (R(1) - q) / (R(3) * q);
    const R cuff = (first ? b2q / R(3) : R(0)) + R(2) / R(3) * (R(1) - q) * inv1q;
    const R cuw = (first ? R(0) : (R(2) * q - R(1)) / (R(3) * q)) + R(2) / R(3) * a2q * inv1q;
    // moving-wall term 6 w rho0 e_i.u_w with e_i = -e_i'
    const R wgx = -R(6) * w * rho0 * ex, wgy = -R(6) * w * rho0 * ey;

    if (Sn) {
        NodeState<ST> nf;
        nf.load(Sn, g.plane, of, ph);
        const R fterm = ob == obj ? R(djx) * ex + R(djy) * ey : R(0);
        const R vbar = Lbar[li] + fterm;
        const R rf = R(1) + nf.dr;
        double *recf = sig + (int64_t)SIG * sf;
        if (off < 0) {
            // halfway bounce-back: v = f+_i'(x_f) + wall
            add_record(recf, R(0), R(0), R(0), vbar + fterm, ip, rf, nf.tx, nf.ty);
            duw[2 * l] += (double)(vbar * wgx);
            duw[2 * l + 1] += (double)(vbar * wgy);
        } else {
            NodeState<ST> nff;
            nff.load(Sn, g.plane, off, ph);
            const R rff = R(1) + nff.dr;
            const R rd = a2q * rf + b2q * rff;
            const R neqf = nf.pop(ip) - deq(w, ex * nf.ux + ey * nf.uy, nf.dr, nf.ux * nf.ux + nf.uy * nf.uy);
            const R neqff =
                nff.pop(ip) - deq(w, ex * nff.ux + ey * nff.uy, nff.dr, nff.ux * nff.ux + nff.uy * nff.uy);
            const R sf_ = neqf / rf, sff_ = neqff / rff;  // non-equilibrium per unit density
            const R r = a2q * sf_ + b2q * sff_;
            // u*_d, u**_d, u_d
            R usx, usy;
            if (first) {
                usx = a2q * nf.ux + b2q * nff.ux;
                usy = a2q * nf.uy + b2q * nff.uy;
            } else {
                usx = ((R(1) - q) * nf.ux + (R(2) * q - R(1)) * uwx) / q;
                usy = ((R(1) - q) * nf.uy + (R(2) * q - R(1)) * uwy) / q;
            }
            const R ussx = ((R(1) - q) * nff.ux + a2q * uwx) * inv1q;
            const R ussy = ((R(1) - q) * nff.uy + a2q * uwy) * inv1q;
            const R udx = (usx + R(2) * ussx) / R(3), udy = (usy + R(2) * ussy) / R(3);
            // v = rho_d phi(u_d) + rho_d r + wall
            R gdx, gdy;
            gphi(w, ex, ey, udx, udy, gdx, gdy);
            const R rbd = vbar * (phi(w, ex, ey, udx, udy) + r);
            const R ubx = vbar * rd * gdx, uby = vbar * rd * gdy;
            const R nbf = vbar * rd * a2q / rf, nbff = vbar * rd * b2q / rff;
            R gfx, gfy, gffx, gffy;
            gphi(w, ex, ey, nf.ux, nf.uy, gfx, gfy);
            gphi(w, ex, ey, nff.ux, nff.uy, gffx, gffy);
            // x_f: rho_d, the non-equilibrium part (through f+_i', rho_f and u_f) and u_d
            const R rbf = a2q * rbd - nbf * (sf_ + phi(w, ex, ey, nf.ux, nf.uy));
            const R ubfx = -nbf * rf * gfx + ubx * cuf, ubfy = -nbf * rf * gfy + uby * cuf;
            add_record(recf, rbf, ubfx, ubfy, nbf + fterm, ip, rf, nf.tx, nf.ty);
            const R rbff = b2q * rbd - nbff * (sff_ + phi(w, ex, ey, nff.ux, nff.uy));
            const R ubffx = -nbff * rff * gffx + ubx * cuff, ubffy = -nbff * rff * gffy + uby * cuff;
            add_record(sig + (int64_t)SIG * sff, rbff, ubffx, ubffy, nbff, ip, rff, nff.tx, nff.ty);
            // parameters: q (both velocity branches, rho_d and the non-equilibrium weights), u_w
            R dusx, dusy;
            if (first) {
                dusx = R(2) * (nf.ux - nff.ux);
                dusy = R(2) * (nf.uy - nff.uy);
            } else {
                dusx = (uwx - nf.ux) / (q * q);
                dusy = (uwy - nf.uy) / (q * q);
            }
            const R c2 = R(2) * inv1q * inv1q;
            const R dudqx = dusx / R(3) + R(2) / R(3) * c2 * (uwx - nff.ux);
            const R dudqy = dusy / R(3) + R(2) / R(3) * c2 * (uwy - nff.uy);
            const R gq = R(2) * rbd * (nf.dr - nff.dr) + ubx * dudqx + uby * dudqy +
                         R(2) * vbar * rd * (sf_ - sff_);
            dq[l] += (double)gq;
            duw[2 * l] += (double)(ubx * cuw + vbar * wgx);
            duw[2 * l + 1] += (double)(uby * cuw + vbar * wgy);
        }
    }

    if (Sc) {
        // link value of step t, as the forward link kernel computes it
        NodeState<ST> nf;
        nf.load(Sc, g.plane, of, ph);
        const R wall = wgx * uwx + wgy * uwy;
        R v;
        if (off < 0) {
            v = nf.pop(ip) + wall;
        } else {
            NodeState<ST> nff;
            nff.load(Sc, g.plane, off, ph);
            const R drd = a2q * nf.dr + b2q * nff.dr;
            const R neqf = nf.pop(ip) - deq(w, ex * nf.ux + ey * nf.uy, nf.dr, nf.ux * nf.ux + nf.uy * nf.uy);
            const R neqff =
                nff.pop(ip) - deq(w, ex * nff.ux + ey * nff.uy, nff.dr, nff.ux * nff.ux + nff.uy * nff.uy);
            const R neqd = a2q * (neqf + neqf * ((drd - nf.dr) / (R(1) + nf.dr))) +
                           b2q * (neqff + neqff * ((drd - nff.dr) / (R(1) + nff.dr)));
            R usx, usy;
            if (first) {
                usx = a2q * nf.ux + b2q * nff.ux;
                usy = a2q * nf.uy + b2q * nff.uy;
            } else {
                const R cf = (R(1) - q) / q, cw = (R(2) * q - R(1)) / q;
                usx = cf * nf.ux + cw * uwx;
                usy = cf * nf.uy + cw * uwy;
            }
            const R cff = (R(1) - q) * inv1q, cww = a2q * inv1q;
            const R ussx = cff * nff.ux + cww * uwx, ussy = cff * nff.uy + cww * uwy;
            const R udx = (usx + R(2) * ussx) / R(3), udy = (usy + R(2) * ussy) / R(3);
            v = deq(w, ex * udx + ey * udy, drd, udx * udx + udy * udy) + neqd + wall;
        }
        Lf[li] = v;
    }
}

// ---------------------------------------------------------------------------
// Reverse bulk kernel.  Blocks of 64 x 4 lanes: each wavefront is one aligned
// 64-node run of a row (the segment of the flagged-node numbering).
// ---------------------------------------------------------------------------

// Wavefront bookkeeping shared by the reverse kernels: the lane's node, its mask
// word, its side-record slot and its first link entry.
struct AdjLane {
    int x, y, lane;
    int32_t row;
    mask_t m;
    int32_t slot, lbase;
    bool inside;
};

__device__ __forceinline__ bool adj_lane(const Grid &g, const mask_t *__restrict__ mask,
                                         const SegBase *__restrict__ segb, AdjLane &a)
{
    a.lane = threadIdx.x & 63;
    a.x = blockIdx.x * 64 + a.lane;
    a.y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (a.y >= g.ny) return false;  // whole wavefront
    a.inside = a.x < g.nx;
    a.row = a.y * g.pitch;
    a.m = a.inside ? mask[a.row + a.x] : MASK_SOLID;
    const int32_t seg = __builtin_amdgcn_readfirstlane(a.y * (g.pitch >> 6) + (a.x >> 6));
    const SegBase sb = segb[seg];
    const uint64_t flagged = __ballot((a.m & MASK_SIDE) != 0);
    a.slot = sb.flagged + (int32_t)__popcll(flagged & ((1ull << a.lane) - 1ull));
    const uint32_t lk = a.m & MASK_LINKS;
    uint32_t linc = (uint32_t)__popc(lk);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(linc, off);
        if (a.lane >= off) linc += t;
    }
    a.lbase = sb.links + (int32_t)(linc - (uint32_t)__popc(lk));
    return true;
}

// Side record of a flagged node added to lambda (and cleared for the next step
// when `clear`).
template <class R>
__device__ __forceinline__ void take_record(double *__restrict__ rec, R *lam, bool clear)
{
    const double al = rec[0], bx = rec[1], by = rec[2];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        double v = al + bx * CX[i] + by * CY[i];
        if (i > 0) v += rec[2 + i];
        lam[i] += R(v);
    }
    if (clear)
#pragma unroll
        for (int k = 0; k < SIG; ++k) rec[k] = 0.0;
}

// lambda of an open-column node (x0 = 0 or nx-1) gathered from C of the nodes of
// the neighbour column that pulled from it (direction sign sx = +1 / -1).
template <class R>
__device__ __forceinline__ void column_lambda(const Grid &g, const mask_t *__restrict__ mask,
                                              const R *__restrict__ Cin, int x0, int y, int sx, R *lam)
{
    const int xn = x0 + sx;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        lam[i] = R(0);
        if (CX[i] != sx) continue;
        const int yn = y + CY[i] < 0 ? g.ny - 1 : (y + CY[i] >= g.ny ? 0 : y + CY[i]);
        const int32_t o = yn * g.pitch + xn;
        if (!(mask[o] & MASK_SOLID)) lam[i] = Cin[(int64_t)i * g.plane + o];
    }
}

template <int ST, bool OPEN, bool FORCE>
__global__ __launch_bounds__(256) void adj_bulk_kernel(Grid g, Phys ph, const typename Codec<ST>::T *__restrict__ S,
                                                       const typename Codec<ST>::R *__restrict__ Lf,
                                                       const typename Codec<ST>::R *__restrict__ Cin,
                                                       typename Codec<ST>::R *__restrict__ Cout,
                                                       typename Codec<ST>::R *__restrict__ Lbar,
                                                       double *__restrict__ sig, const mask_t *__restrict__ mask,
                                                       const SegBase *__restrict__ segb,
                                                       const int32_t *__restrict__ colslot,
                                                       const typename Codec<ST>::R *__restrict__ uin,
                                                       double *__restrict__ duin)
{
    using C = Codec<ST>;
    using R = typename C::R;
    AdjLane a;
    if (!adj_lane(g, mask, segb, a)) return;
    if (!a.inside || (a.m & MASK_SOLID)) return;
    const int x = a.x, y = a.y;
    if (OPEN && (x == 0 || x == g.nx - 1)) return;
    const int64_t P = g.plane;
    const int32_t row = a.row;
    int xm, xp;
    if (OPEN) {
        xm = x - 1;
        xp = x + 1;
    } else {
        xm = x == 0 ? g.nx - 1 : x - 1;
        xp = x == g.nx - 1 ? 0 : x + 1;
    }
    const int32_t rm = (y == 0 ? g.ny - 1 : y - 1) * g.pitch;
    const int32_t rp = (y == g.ny - 1 ? 0 : y + 1) * g.pitch;
    const uint32_t lk = a.m & MASK_LINKS;
    constexpr int OPPI[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    // offsets of x - e_i (pull sources) and x + e_i (nodes that pulled from x)
    const int32_t src[9] = {row + x, row + xm, rm + x, row + xp, rp + x, rm + xm, rm + xp, rp + xp, rp + xm};
    const int32_t dst[9] = {row + x, row + xp, rp + x, row + xm, rm + x, rp + xp, rp + xm, rm + xm, rm + xp};

    // pre-collision populations of step t
    R f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint32_t bit = i ? 1u << (OPPI[i] - 1) : 0u;
        if (lk & bit) f[i] = Lf[a.lbase + __popc(lk & (bit - 1u))];
        else f[i] = C::ld(S[i * P + src[i]], ph.inv_scale);
    }
    // adjoint of S_t+1 at this node: C_t+1 of the node that pulled each population
    // (none where x + e_i is solid -- a link reads it -- or an open column)
    R lam[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const bool cut = i && (lk & (1u << (i - 1)));
        const bool col = OPEN && CX[i] != 0 && ((CX[i] > 0 ? xp : xm) == 0 || (CX[i] > 0 ? xp : xm) == g.nx - 1);
        lam[i] = (cut || col) ? R(0) : Cin[i * P + dst[i]];
    }
    if (a.m & MASK_SIDE) take_record(sig + (int64_t)SIG * a.slot, lam, true);

    // moments and collision velocity of the pre-collision state
    const R dr = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const R ir = inv_rho_m1(dr);
    const R tx = jx + jx * ir, ty = jy + jy * ir;  // j/rho
    const R gx = FORCE ? R(ph.gx) : R(0), gy = FORCE ? R(ph.gy) : R(0);
    const R ux = tx + R(0.5) * gx, uy = ty + R(0.5) * gy;
    const R rho = R(1) + dr;

    if (OPEN) {
        if (x == 1 && !(mask[row] & MASK_SOLID)) {
            // inlet f+(0) = rho1 phi(u_in) + S''(1) - rho1 phi(u1), with (rho1, u1) the
            // moments of S''(1): rho and the collision velocity u (j/rho of S'' is u + g/2)
            R l0[9];
            column_lambda(g, mask, Cin, 0, y, 1, l0);
            const int32_t cs = colslot[y];
            if (cs >= 0) take_record(sig + (int64_t)SIG * cs, l0, true);
            const R vx = uin[2 * y], vy = uin[2 * y + 1];
            const R t1x = ux + R(0.5) * gx, t1y = uy + R(0.5) * gy;
            R s0 = R(0), gux = R(0), guy = R(0), gvx = R(0), gvy = R(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const R w = wgt<R>(i), ex = R(CX[i]), ey = R(CY[i]);
                s0 += l0[i] * w * (poly(ex * vx + ey * vy, vx * vx + vy * vy) - poly(ex * ux + ey * uy, ux * ux + uy * uy));
                R ax, ay;
                gphi(w, ex, ey, ux, uy, ax, ay);
                gux += l0[i] * ax;
                guy += l0[i] * ay;
                gphi(w, ex, ey, vx, vy, ax, ay);
                gvx += l0[i] * ax;
                gvy += l0[i] * ay;
            }
#pragma unroll
            for (int j = 0; j < 9; ++j)
                lam[j] += l0[j] + s0 - (gux * (R(CX[j]) - t1x) + guy * (R(CY[j]) - t1y));
            duin[2 * y] += (double)(rho * gvx);
            duin[2 * y + 1] += (double)(rho * gvy);
        }
        if (x == g.nx - 2 && !(mask[row + g.nx - 1] & MASK_SOLID)) {
            // outlet f+(nx-1) = S''(nx-2)
            R le[9];
            column_lambda(g, mask, Cin, g.nx - 1, y, -1, le);
            const int32_t cs = colslot[g.ny + y];
            if (cs >= 0) take_record(sig + (int64_t)SIG * cs, le, true);
#pragma unroll
            for (int j = 0; j < 9; ++j) lam[j] += le[j];
        }
    }

    // BGK + Guo collision transposed:
    //   f+_i = f_i - omega (f_i - rho phi_i(u)) + (1 - omega/2) rho s_i(u),
    //   s_i(u) = w_i [3 (e_i - u) + 9 (e_i.u) e_i].g,  u = j/rho + g/2
    // so C_j = (1 - omega) lam_j + G_rho + G_u.(e_j - j/rho)/rho with
    //   G_rho = sum_i lam_i (omega phi_i + (1 - omega/2) s_i),
    //   G_u   = rho sum_i lam_i (omega grad phi_i + (1 - omega/2) grad s_i).
    const R om = R(ph.omega);
    const R cf = R(1) - R(0.5) * om;
    R Gr = R(0), Gx = R(0), Gy = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R w = wgt<R>(i), ex = R(CX[i]), ey = R(CY[i]);
        const R eu = ex * ux + ey * uy;
        Gr += lam[i] * om * w * (R(1) + poly(eu, ux * ux + uy * uy));
        Gx += lam[i] * om * w * (R(3) * ex + R(9) * eu * ex - R(3) * ux);
        Gy += lam[i] * om * w * (R(3) * ey + R(9) * eu * ey - R(3) * uy);
        if (FORCE) {
            const R eg = ex * gx + ey * gy;
            Gr += lam[i] * cf * w * ((R(3) * (ex - ux) + R(9) * eu * ex) * gx + (R(3) * (ey - uy) + R(9) * eu * ey) * gy);
            Gx += lam[i] * cf * w * (-R(3) * gx + R(9) * ex * eg);
            Gy += lam[i] * cf * w * (-R(3) * gy + R(9) * ey * eg);
        }
    }
    // (Gx, Gy) = G_u / rho
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const R c = (R(1) - om) * lam[j] + Gr + Gx * (R(CX[j]) - tx) + Gy * (R(CY[j]) - ty);
        Cout[j * P + row + x] = c;
        const uint32_t bit = j ? 1u << (OPPI[j] - 1) : 0u;
        if (lk & bit) Lbar[a.lbase + __popc(lk & (bit - 1u))] = c;
    }
}

// ---------------------------------------------------------------------------
// lambda_0 = dJ/dS_0 at every fluid node (open columns included) and its chain
// to the fields of an equilibrium initial state f+ = rho phi(u).
// ---------------------------------------------------------------------------
template <int ST, bool OPEN>
__global__ __launch_bounds__(256) void adj_final_kernel(Grid g, Phys ph, const typename Codec<ST>::T *__restrict__ S,
                                                        const typename Codec<ST>::R *__restrict__ Cin,
                                                        const double *__restrict__ sig,
                                                        const mask_t *__restrict__ mask,
                                                        const SegBase *__restrict__ segb, double *__restrict__ dstate,
                                                        double *__restrict__ dinit, int64_t dplane)
{
    using C = Codec<ST>;
    using R = typename C::R;
    AdjLane a;
    if (!adj_lane(g, mask, segb, a)) return;
    if (!a.inside) return;
    const int x = a.x, y = a.y;
    const int32_t o = a.row + x;
    if (a.m & MASK_SOLID) {
        for (int i = 0; i < 9; ++i) dstate[i * dplane + o] = 0.0;
        for (int k = 0; k < 3; ++k) dinit[k * dplane + o] = 0.0;
        return;
    }
    R lam[9];
    if (OPEN && x == 0) {
        column_lambda(g, mask, Cin, 0, y, 1, lam);
    } else if (OPEN && x == g.nx - 1) {
        column_lambda(g, mask, Cin, g.nx - 1, y, -1, lam);
    } else {
        const uint32_t lk = a.m & MASK_LINKS;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xn = x + CX[i], yn = y + CY[i];
            if (!OPEN) xn = xn < 0 ? g.nx - 1 : (xn >= g.nx ? 0 : xn);
            yn = yn < 0 ? g.ny - 1 : (yn >= g.ny ? 0 : yn);
            const bool cut = i && (lk & (1u << (i - 1)));
            const bool col = OPEN && (xn == 0 || xn == g.nx - 1);
            lam[i] = (cut || col) ? R(0) : Cin[i * g.plane + yn * g.pitch + xn];
        }
    }
    if (a.m & MASK_SIDE) take_record(const_cast<double *>(sig) + (int64_t)SIG * a.slot, lam, false);
    R d[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        d[i] = C::ld(S[i * g.plane + o], ph.inv_scale);
        dstate[i * dplane + o] = (double)lam[i];
    }
    const R dr = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    const R jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    const R jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
    const R ir = inv_rho_m1(dr);
    const R tx = jx + jx * ir, ty = jy + jy * ir;
    R rb = R(0), bx = R(0), by = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R w = wgt<R>(i), ex = R(CX[i]), ey = R(CY[i]);
        rb += lam[i] * phi(w, ex, ey, tx, ty);
        R ax, ay;
        gphi(w, ex, ey, tx, ty, ax, ay);
        bx += lam[i] * ax;
        by += lam[i] * ay;
    }
    const R rho = R(1) + dr;
    dinit[o] = (double)rb;
    dinit[dplane + o] = (double)(rho * bx);
    dinit[2 * dplane + o] = (double)(rho * by);
}

template <int ST>
void adj_link_t(const Grid &g, const Phys &ph, const Links &L, const int32_t *mnode, const void *Sn, const void *Sc,
                void *Lf, const void *Lbar, double *sig, double *dq, double *duw, int32_t obj, double djx,
                double djy, hipStream_t s)
{
    using T = typename Codec<ST>::T;
    using R = typename Codec<ST>::R;
    const unsigned blocks = (unsigned)((L.n + 255) / 256);
    hipLaunchKernelGGL(adj_link_kernel<ST>, dim3(blocks), dim3(256), 0, s, g, ph, L, mnode,
                       static_cast<const T *>(Sn), static_cast<const T *>(Sc), static_cast<R *>(Lf),
                       static_cast<const R *>(Lbar), sig, dq, duw, obj, djx, djy);
}

template <int ST, bool OPEN, bool FORCE>
void adj_bulk_t(const Grid &g, const Phys &ph, const void *S, const void *Lf, const void *Cin, void *Cout,
                void *Lbar, double *sig, const mask_t *mask, const SegBase *seg, const int32_t *colslot,
                const void *uin, double *duin, hipStream_t s)
{
    using T = typename Codec<ST>::T;
    using R = typename Codec<ST>::R;
    const dim3 grid((unsigned)(g.pitch / 64), (unsigned)((g.ny + 3) / 4));
    hipLaunchKernelGGL((adj_bulk_kernel<ST, OPEN, FORCE>), grid, dim3(256), 0, s, g, ph,
                       static_cast<const T *>(S), static_cast<const R *>(Lf), static_cast<const R *>(Cin),
                       static_cast<R *>(Cout), static_cast<R *>(Lbar), sig, mask, seg, colslot,
                       static_cast<const R *>(uin), duin);
}

template <int ST, bool OPEN>
void adj_final_t(const Grid &g, const Phys &ph, const void *S, const void *Cin, const double *sig,
                 const mask_t *mask, const SegBase *seg, double *dstate, double *dinit, int64_t dplane,
                 hipStream_t s)
{
    using T = typename Codec<ST>::T;
    using R = typename Codec<ST>::R;
    const dim3 grid((unsigned)(g.pitch / 64), (unsigned)((g.ny + 3) / 4));
    hipLaunchKernelGGL((adj_final_kernel<ST, OPEN>), grid, dim3(256), 0, s, g, ph, static_cast<const T *>(S),
                       static_cast<const R *>(Cin), sig, mask, seg, dstate, dinit, dplane);
}

}  // namespace

hipError_t launch_adj_link(int storage, const Grid &g, const Phys &ph, const Links &L, const int32_t *mnode,
                           const void *Sn, const void *Sc, void *Lf, const void *Lbar, double *sig, double *dq,
                           double *duw, int32_t obj, double djx, double djy, hipStream_t s)
{
    if (L.n == 0) return hipSuccess;
    if (storage == 0) adj_link_t<0>(g, ph, L, mnode, Sn, Sc, Lf, Lbar, sig, dq, duw, obj, djx, djy, s);
    else adj_link_t<1>(g, ph, L, mnode, Sn, Sc, Lf, Lbar, sig, dq, duw, obj, djx, djy, s);
    return hipGetLastError();
}

hipError_t launch_adj_bulk(int storage, const Grid &g, const Phys &ph, const void *S, const void *Lf,
                           const void *Cin, void *Cout, void *Lbar, double *sig, const mask_t *mask,
                           const SegBase *seg, const int32_t *colslot, const void *uin, double *duin,
                           hipStream_t s)
{
    const bool open = g.x_open != 0, force = ph.gx != 0.0 || ph.gy != 0.0;
#define ADJ_BULK(ST, O, F) adj_bulk_t<ST, O, F>(g, ph, S, Lf, Cin, Cout, Lbar, sig, mask, seg, colslot, uin, duin, s)
    if (storage == 0) {
        if (open) force ? ADJ_BULK(0, true, true) : ADJ_BULK(0, true, false);
        else force ? ADJ_BULK(0, false, true) : ADJ_BULK(0, false, false);
    } else {
        if (open) force ? ADJ_BULK(1, true, true) : ADJ_BULK(1, true, false);
        else force ? ADJ_BULK(1, false, true) : ADJ_BULK(1, false, false);
    }
#undef ADJ_BULK
    return hipGetLastError();
}

hipError_t launch_adj_final(int storage, const Grid &g, const Phys &ph, const void *S, const void *Cin,
                            const double *sig, const mask_t *mask, const SegBase *seg, double *dstate,
                            double *dinit, int64_t dplane, hipStream_t s)
{
    const bool open = g.x_open != 0;
    if (storage == 0) {
        if (open) adj_final_t<0, true>(g, ph, S, Cin, sig, mask, seg, dstate, dinit, dplane, s);
        else adj_final_t<0, false>(g, ph, S, Cin, sig, mask, seg, dstate, dinit, dplane, s);
    } else {
        if (open) adj_final_t<1, true>(g, ph, S, Cin, sig, mask, seg, dstate, dinit, dplane, s);
        else adj_final_t<1, false>(g, ph, S, Cin, sig, mask, seg, dstate, dinit, dplane, s);
    }
    return hipGetLastError();
}

}  // namespace lbm
