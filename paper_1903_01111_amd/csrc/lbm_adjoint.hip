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
// Adjoint, with lambda_t = dJ/dS_t and C_t(x) = dJ/df(x) (pre-collision), one
// launch per reverse step t (one lane per node):
//   lambda_t+1(x) is gathered from C_t+1 of the nodes that pulled from x, plus
//   the node's side record of step t+1 (what the links of step t+1 sent back);
//   the open columns fold into their neighbour lanes (inlet adds dJ/du_in);
//   the pre-collision state is rebuilt from S_t (pulls, and the values of the
//   node's own links); the collision Jacobian^T gives C_t(x);
//   a boundary node then takes the adjoint of each of its links, C_t in the
//   link's direction plus the force weight, through the VIBB Jacobian^T into the
//   side records of step t of x_f and x_ff (FP64 atomics) and into the FP64
//   accumulators of dJ/dq and dJ/du_w.
// Side records are double-buffered by step parity: a launch consumes (and
// clears) those of step t+1 and fills those of step t.
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

// Moments of a post-collision node from its nine stored deviations, and its
// population in one link direction ip: dr = rho - 1, (tx, ty) = j/rho,
// (ux, uy) = j/rho - g/2 (physical velocity).  The direction's population is a
// load of its own (a runtime index into the nine registers would go through
// scratch memory).
template <int ST>
struct NodeState {
    using R = typename Codec<ST>::R;
    R dr, tx, ty, ux, uy, pip;
    __device__ __forceinline__ void load(const typename Codec<ST>::T *__restrict__ S, int64_t plane,
                                         int32_t off, int ip, const Phys &ph)
    {
        R d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = Codec<ST>::ld(S[i * plane + off], ph.inv_scale);
        pip = Codec<ST>::ld(S[ip * plane + off], ph.inv_scale);
        dr = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
        const R jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
        const R jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
        const R ir = inv_rho_m1(dr);
        tx = jx + jx * ir;
        ty = jy + jy * ir;
        ux = tx - R(0.5) * R(ph.gx);
        uy = ty - R(0.5) * R(ph.gy);
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
// Links.  The links of a wavefront's 64 nodes are a contiguous run of the
// per-link records in (node, dir) order (the order of the link bits of the
// mask words); the wavefront spreads them over its lanes, one link per lane,
// and hands values to the owning node lanes (and adjoints back) through LDS.
// ---------------------------------------------------------------------------
template <class R>
struct AdjLinkRec {
    int32_t k;       // position in the (obj, node, dir) order: the dq / duw entry
    int32_t off_f;   // plane offset of x_f
    int32_t off_ff;  // plane offset of x_ff, or -1 (halfway bounce-back)
    int32_t sf;      // side slot of x_f
    int32_t sff;     // side slot of x_ff
    uint32_t meta;   // dir | obj << 8
    R q, uwx, uwy;
};

template <class R>
__global__ __launch_bounds__(256) void adj_setup_kernel(Links L, const int32_t *__restrict__ mnode,
                                                        AdjLinkRec<R> *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L.n) return;
    AdjLinkRec<R> r;
    r.k = (int32_t)k;
    r.sf = L.sf[k];
    r.off_f = mnode[r.sf];
    r.sff = L.sff[k];
    r.off_ff = r.sff >= 0 ? mnode[r.sff] : -1;
    r.meta = L.meta[k];
    r.q = static_cast<const R *>(L.q)[k];
    r.uwx = L.uw ? static_cast<const R *>(L.uw)[2 * k] : R(0);
    r.uwy = L.uw ? static_cast<const R *>(L.uw)[2 * k + 1] : R(0);
    out[L.li[k]] = r;
}

// Value of a VIBB link (Section 3.1) from the states of x_f and x_ff, in the
// deviation form of the forward link kernel (without the moving-wall term).
template <int ST>
__device__ __forceinline__ typename Codec<ST>::R vibb_value(const NodeState<ST> &nf, const NodeState<ST> &nff,
                                                            int ip, typename Codec<ST>::R q,
                                                            typename Codec<ST>::R uwx, typename Codec<ST>::R uwy)
{
    using R = typename Codec<ST>::R;
    const R ex = R(cx_of(ip)), ey = R(cy_of(ip));
    const R w = ip <= 4 ? R(1) / R(9) : R(1) / R(36);
    const R a2q = R(2) * q, b2q = R(1) - R(2) * q;
    const R drd = a2q * nf.dr + b2q * nff.dr;
    const R neqf = nf.pip - deq(w, ex * nf.ux + ey * nf.uy, nf.dr, nf.ux * nf.ux + nf.uy * nf.uy);
    const R neqff = nff.pip - deq(w, ex * nff.ux + ey * nff.uy, nff.dr, nff.ux * nff.ux + nff.uy * nff.uy);
    const R neqd = a2q * (neqf + neqf * ((drd - nf.dr) / (R(1) + nf.dr))) +
                   b2q * (neqff + neqff * ((drd - nff.dr) / (R(1) + nff.dr)));
    R usx, usy;
    if (q <= R(0.5)) {
        usx = a2q * nf.ux + b2q * nff.ux;
        usy = a2q * nf.uy + b2q * nff.uy;
    } else {
        const R cf = (R(1) - q) / q, cw = (R(2) * q - R(1)) / q;
        usx = cf * nf.ux + cw * uwx;
        usy = cf * nf.uy + cw * uwy;
    }
    const R inv1q = R(1) / (R(1) + q);
    const R cff = (R(1) - q) * inv1q, cww = a2q * inv1q;
    const R ussx = cff * nff.ux + cww * uwx, ussy = cff * nff.uy + cww * uwy;
    const R udx = (usx + R(2) * ussx) / R(3), udy = (usy + R(2) * ussy) / R(3);
    return deq(w, ex * udx + ey * udy, drd, udx * udx + udy * udy) + neqd;
}

// Adjoint of a VIBB link value: v-bar (which includes the force weight fterm of
// v) spread over the moments and the populations f+_i' of x_f and x_ff (side
// records recf, recff; fterm also weighs f+_i'(x_f) in the force) and over q and
// u_w (FP64 accumulators of the link).
//   v = rho_d phi_i'(u_d) + rho_d r + wall,   rho_d = 2q rho_f + (1-2q) rho_ff,
//   r = 2q n_f/rho_f + (1-2q) n_ff/rho_ff,   n = f+_i' - rho phi_i'(u),
//   u_d = u*_d/3 + 2 u**_d/3 (two branches of u*_d).
template <int ST>
__device__ __forceinline__ void vibb_adjoint(const NodeState<ST> &nf, const NodeState<ST> &nff, int ip,
                                             typename Codec<ST>::R q, typename Codec<ST>::R uwx,
                                             typename Codec<ST>::R uwy, typename Codec<ST>::R vbar,
                                             typename Codec<ST>::R fterm, typename Codec<ST>::R wgx,
                                             typename Codec<ST>::R wgy, double *__restrict__ recf,
                                             double *__restrict__ recff, double *__restrict__ dq,
                                             double *__restrict__ duw)
{
    using R = typename Codec<ST>::R;
    const R ex = R(cx_of(ip)), ey = R(cy_of(ip));
    const R w = ip <= 4 ? R(1) / R(9) : R(1) / R(36);
    const R a2q = R(2) * q, b2q = R(1) - R(2) * q;
    const bool first = q <= R(0.5);
    const R inv1q = R(1) / (R(1) + q);
    // coefficients of u_d on u_f, u_ff and u_w
    const R cuf = first ? a2q / R(3) : (R(1) - q) / (R(3) * q);
    const R cuff = (first ? b2q / R(3) : R(0)) + R(2) / R(3) * (R(1) - q) * inv1q;
    const R cuw = (first ? R(0) : (R(2) * q - R(1)) / (R(3) * q)) + R(2) / R(3) * a2q * inv1q;
    const R rf = R(1) + nf.dr, rff = R(1) + nff.dr;
    const R rd = a2q * rf + b2q * rff;
    const R neqf = nf.pip - deq(w, ex * nf.ux + ey * nf.uy, nf.dr, nf.ux * nf.ux + nf.uy * nf.uy);
    const R neqff = nff.pip - deq(w, ex * nff.ux + ey * nff.uy, nff.dr, nff.ux * nff.ux + nff.uy * nff.uy);
    const R sf = neqf / rf, sff = neqff / rff;  // non-equilibrium per unit density
    const R r = a2q * sf + b2q * sff;
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
    R gdx, gdy;
    gphi(w, ex, ey, udx, udy, gdx, gdy);
    const R rbd = vbar * (phi(w, ex, ey, udx, udy) + r);  // rho_d-bar
    const R ubx = vbar * rd * gdx, uby = vbar * rd * gdy;  // u_d-bar
    const R nbf = vbar * rd * a2q / rf, nbff = vbar * rd * b2q / rff;
    R gfx, gfy, gffx, gffy;
    gphi(w, ex, ey, nf.ux, nf.uy, gfx, gfy);
    gphi(w, ex, ey, nff.ux, nff.uy, gffx, gffy);
    const R rbf = a2q * rbd - nbf * (sf + phi(w, ex, ey, nf.ux, nf.uy));
    add_record(recf, rbf, -nbf * rf * gfx + ubx * cuf, -nbf * rf * gfy + uby * cuf, nbf + fterm, ip, rf, nf.tx,
               nf.ty);
    const R rbff = b2q * rbd - nbff * (sff + phi(w, ex, ey, nff.ux, nff.uy));
    add_record(recff, rbff, -nbff * rff * gffx + ubx * cuff, -nbff * rff * gffy + uby * cuff, nbff, ip, rff,
               nff.tx, nff.ty);
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
    *dq += (double)(R(2) * rbd * (nf.dr - nff.dr) + ubx * dudqx + uby * dudqy + R(2) * vbar * rd * (sf - sff));
    duw[0] += (double)(ubx * cuw + vbar * wgx);
    duw[1] += (double)(uby * cuw + vbar * wgy);
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
    const uint32_t linc = wave_inclusive_scan((uint32_t)__popc(lk));
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
__global__ __launch_bounds__(256) void adj_step_kernel(Grid g, Phys ph, const typename Codec<ST>::T *__restrict__ S,
                                                       const typename Codec<ST>::R *__restrict__ Cin,
                                                       typename Codec<ST>::R *__restrict__ Cout,
                                                       double *__restrict__ sig_in, double *__restrict__ sig_out,
                                                       const AdjLinkRec<typename Codec<ST>::R> *__restrict__ lrec,
                                                       const mask_t *__restrict__ mask,
                                                       const SegBase *__restrict__ segb,
                                                       const int32_t *__restrict__ colslot,
                                                       const typename Codec<ST>::R *__restrict__ uin,
                                                       double *__restrict__ duin, double *__restrict__ dq,
                                                       double *__restrict__ duw, int32_t obj, double djx, double djy)
{
    using C = Codec<ST>;
    using R = typename C::R;
    AdjLane a;
    if (!adj_lane(g, mask, segb, a)) return;  // whole wavefront
    const int x = a.x, y = a.y;
    const bool active = a.inside && !(a.m & MASK_SOLID) && !(OPEN && (x == 0 || x == g.nx - 1));
    const int64_t P = g.plane;
    const int32_t row = a.row;
    int xm, xp;
    if (OPEN) {
        xm = x > 0 ? x - 1 : 0;
        xp = x < g.nx - 1 ? x + 1 : g.nx - 1;
    } else {
        xm = x == 0 ? g.nx - 1 : x - 1;
        xp = x == g.nx - 1 ? 0 : x + 1;
    }
    const int32_t rm = (y == 0 ? g.ny - 1 : y - 1) * g.pitch;
    const int32_t rp = (y == g.ny - 1 ? 0 : y + 1) * g.pitch;
    constexpr int OPPI[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    // offsets of x - e_i (pull sources) and x + e_i (nodes that pulled from x)
    const int32_t src[9] = {row + x, row + xm, rm + x, row + xp, rp + x, rm + xm, rm + xp, rp + xp, rp + xm};
    const int32_t dst[9] = {row + x, row + xp, rp + x, row + xm, rm + x, rp + xp, rp + xm, rm + xm, rm + xp};
    const R rho0 = R(ph.rho0);

    // the wavefront's links: records [lw, lw + nw) of the (node, dir) order
    __shared__ R lds[4][8 * 64];
    const int wv = threadIdx.x >> 6;
    const uint32_t lk = active ? a.m & MASK_LINKS : 0u;
    const int32_t lw = __builtin_amdgcn_readfirstlane(__shfl(a.lbase, 0));
    const int nw = __shfl(a.lbase + __popc(a.m & MASK_LINKS), 63) - lw;
    // link values of step t, one link per lane
    for (int j = a.lane; j < nw; j += 64) {
        const AdjLinkRec<R> r = lrec[lw + j];
        const int d = (int)(r.meta & 15u);
        const R w = d <= 4 ? R(1) / R(9) : R(1) / R(36);
        const R wall = -R(6) * w * rho0 * (R(cx_of(d)) * r.uwx + R(cy_of(d)) * r.uwy);
        NodeState<ST> nf;
        nf.load(S, P, r.off_f, d, ph);
        R v;
        if (r.off_ff < 0) {
            v = nf.pip + wall;
        } else {
            NodeState<ST> nff;
            nff.load(S, P, r.off_ff, d, ph);
            v = vibb_value(nf, nff, d, r.q, r.uwx, r.uwy) + wall;
        }
        lds[wv][j] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int lo = a.lbase - lw;  // this node's first link in the wavefront's run

    // pre-collision populations of step t: pulls, and the values of this node's
    // links where x - e_i is solid
    R c[9];
    if (active) {
        R f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const uint32_t bit = i ? 1u << (OPPI[i] - 1) : 0u;
            f[i] = (lk & bit) ? lds[wv][lo + __popc(lk & (bit - 1u))] : C::ld(S[i * P + src[i]], ph.inv_scale);
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
        if (a.m & MASK_SIDE) take_record(sig_in + (int64_t)SIG * a.slot, lam, true);

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
                if (cs >= 0) take_record(sig_in + (int64_t)SIG * cs, l0, true);
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
                if (cs >= 0) take_record(sig_in + (int64_t)SIG * cs, le, true);
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
        R Gr = R(0), Gx = R(0), Gy = R(0);  // G_rho and G_u / rho
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
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            c[j] = (R(1) - om) * lam[j] + Gr + Gx * (R(CX[j]) - tx) + Gy * (R(CY[j]) - ty);
            Cout[j * P + row + x] = c[j];
        }
    }
    // the adjoints of the link values go back to the link lanes
    if (active) {
#pragma unroll
        for (int j = 1; j < 9; ++j) {
            const uint32_t bit = 1u << (OPPI[j] - 1);
            if (lk & bit) lds[wv][lo + __popc(lk & (bit - 1u))] = c[j];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // adjoint of the link values of step t (with the force weight of the step),
    // one link per lane, into the side records of step t and the accumulators
    for (int j = a.lane; j < nw; j += 64) {
        const AdjLinkRec<R> r = lrec[lw + j];
        const int d = (int)(r.meta & 15u);
        const R ex = R(cx_of(d)), ey = R(cy_of(d));
        const R w = d <= 4 ? R(1) / R(9) : R(1) / R(36);
        const R wgx = -R(6) * w * rho0 * ex, wgy = -R(6) * w * rho0 * ey;
        const R fterm = (int)(r.meta >> 8) == obj ? R(djx) * ex + R(djy) * ey : R(0);
        const R vbar = lds[wv][j] + fterm;
        NodeState<ST> nf;
        nf.load(S, P, r.off_f, d, ph);
        double *recf = sig_out + (int64_t)SIG * r.sf;
        if (r.off_ff < 0) {
            // halfway bounce-back: v = f+_i'(x_f) + wall
            add_record(recf, R(0), R(0), R(0), vbar + fterm, d, R(1) + nf.dr, nf.tx, nf.ty);
            duw[2 * r.k] += (double)(vbar * wgx);
            duw[2 * r.k + 1] += (double)(vbar * wgy);
        } else {
            NodeState<ST> nff;
            nff.load(S, P, r.off_ff, d, ph);
            vibb_adjoint(nf, nff, d, r.q, r.uwx, r.uwy, vbar, fterm, wgx, wgy, recf,
                         sig_out + (int64_t)SIG * r.sff, dq + r.k, duw + 2 * r.k);
        }
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
void adj_setup_t(const Links &L, const int32_t *mnode, void *lrec, hipStream_t s)
{
    using R = typename Codec<ST>::R;
    hipLaunchKernelGGL(adj_setup_kernel<R>, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, s, L, mnode,
                       static_cast<AdjLinkRec<R> *>(lrec));
}

template <int ST, bool OPEN, bool FORCE>
void adj_step_t(const Grid &g, const Phys &ph, const void *S, const void *Cin, void *Cout, double *sig_in,
                double *sig_out, const void *lrec, const mask_t *mask, const SegBase *seg, const int32_t *colslot,
                const void *uin, double *duin, double *dq, double *duw, int32_t obj, double djx, double djy,
                hipStream_t s)
{
    using T = typename Codec<ST>::T;
    using R = typename Codec<ST>::R;
    const dim3 grid((unsigned)(g.pitch / 64), (unsigned)((g.ny + 3) / 4));
    hipLaunchKernelGGL((adj_step_kernel<ST, OPEN, FORCE>), grid, dim3(256), 0, s, g, ph,
                       static_cast<const T *>(S), static_cast<const R *>(Cin), static_cast<R *>(Cout), sig_in,
                       sig_out, static_cast<const AdjLinkRec<R> *>(lrec), mask, seg, colslot,
                       static_cast<const R *>(uin), duin, dq, duw, obj, djx, djy);
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

size_t adj_link_record_bytes(int storage)
{
    return storage == 0 ? sizeof(AdjLinkRec<double>) : sizeof(AdjLinkRec<float>);
}

hipError_t launch_adj_setup(int storage, const Links &L, const int32_t *mnode, void *lrec, hipStream_t s)
{
    if (L.n == 0) return hipSuccess;
    if (storage == 0) adj_setup_t<0>(L, mnode, lrec, s);
    else adj_setup_t<1>(L, mnode, lrec, s);
    return hipGetLastError();
}

hipError_t launch_adj_step(int storage, const Grid &g, const Phys &ph, const void *S, const void *Cin, void *Cout,
                           double *sig_in, double *sig_out, const void *lrec, const mask_t *mask,
                           const SegBase *seg, const int32_t *colslot, const void *uin, double *duin, double *dq,
                           double *duw, int32_t obj, double djx, double djy, hipStream_t s)
{
    const bool open = g.x_open != 0, force = ph.gx != 0.0 || ph.gy != 0.0;
#define ADJ_STEP(ST, O, F) \
    adj_step_t<ST, O, F>(g, ph, S, Cin, Cout, sig_in, sig_out, lrec, mask, seg, colslot, uin, duin, dq, duw, obj, djx, djy, s)
    if (storage == 0) {
        if (open) force ? ADJ_STEP(0, true, true) : ADJ_STEP(0, true, false);
        else force ? ADJ_STEP(0, false, true) : ADJ_STEP(0, false, false);
    } else {
        if (open) force ? ADJ_STEP(1, true, true) : ADJ_STEP(1, true, false);
        else force ? ADJ_STEP(1, false, true) : ADJ_STEP(1, false, false);
    }
#undef ADJ_STEP
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
