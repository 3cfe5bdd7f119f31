// Host runtime of the C ABI declared in include/lbm.h: argument and geometry
// validation, workspace layout, link preprocessing, the step loop (HIP graph
// replay of a fixed number of steps), read-back, checkpoints and kernel timing.
// All arithmetic of a time step runs in the HIP kernels (lbm_kernels.hip).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "lbm_ctx.h"

namespace lbm_host {

thread_local std::string g_thread_error = "no error";

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t elem_bytes(int storage)
{
    switch (storage) {
    case LBM_F64: return 8;
    case LBM_F32:
    case LBM_F32_WIDE:
    case LBM_F32_PLAIN: return 4;
    default: return 2;
    }
}
size_t real_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }
bool storage_is_16bit(int storage) { return storage == LBM_F16_DEV || storage == LBM_BF16_DEV; }


// device bytes per link of capacity (link arrays, and up to two flagged nodes
// with their side moments)
size_t bytes_per_link(int storage)
{
    return 53 + 15 * real_bytes(storage) + 7 * elem_bytes(storage);
}

// Room of the neighbour words' offset table: the first and last row and column
// (the periodic wraps), plus 16 runs of 64 nodes whose rank differences spread too
// far for the 16-bit words.
int64_t nbr_table_room(int64_t pitch, int64_t ny)
{
    return 2 * pitch + 2 * ny + 16 * 64;
}

// Plane stride: rows padded to 64 elements; the plane size in 256-byte units is
// kept odd so that the nine planes do not start on the same memory channel.
Layout make_layout(const lbm_params &p, int64_t max_links)
{
    Layout L{};
    const size_t eb = elem_bytes(p.storage), rb = real_bytes(p.storage);
    L.pitch = (p.nx + 63) / 64 * 64;
    size_t pb = align256((size_t)L.pitch * p.ny * eb);
    if ((pb / 256) % 2 == 0) pb += 256;
    L.plane = (int64_t)(pb / eb);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.off_A = take(9 * pb);
    L.off_B = take(9 * pb);
    L.off_mask = take((size_t)L.pitch * p.ny * sizeof(lbm::mask_t));
    L.off_seg = take(((size_t)(L.pitch / 64) * p.ny + 1) * sizeof(lbm::SegBase));
    L.off_fmask = take((size_t)(L.pitch / 64) * p.ny * sizeof(uint64_t));
    // runs of 64 fluid nodes: at most one per segment, plus the sentinel
    L.off_runs = take(((size_t)(L.pitch / 64) * p.ny + 1) * sizeof(lbm::RunBase));
    L.off_frow = take(((size_t)(L.pitch / 64) * p.ny + 1) * sizeof(lbm::SegRow));
    // neighbour words: one per fluid node, and nine offsets per node of the first and
    // last row and column
    L.off_nbr = take((size_t)L.pitch * p.ny * sizeof(uint16_t));
    L.off_nbrr = take(((size_t)(L.pitch / 64) * p.ny + 1) * sizeof(lbm::NbrRun));
    L.off_nbrs = take((size_t)nbr_table_room(L.pitch, p.ny) * 9 * sizeof(uint32_t));
    const size_t nl = (size_t)std::max<int64_t>(max_links, 0);
    L.off_meta = take(nl * 4);
    L.off_q = take(nl * rb);
    L.off_uw = take(nl * 2 * rb);
    L.off_sf = take(nl * 4);
    L.off_sff = take(nl * 4);
    L.off_pf = take(nl * 4);
    L.off_pff = take(nl * 4);
    L.off_pfi = take(nl * 4);
    L.off_crec = take(rb == 4 ? nl * sizeof(lbm::LinkRec) : 0);
    L.off_cbase = take(rb == 4 ? (nl / 64 + 1) * sizeof(lbm::LinkRunBase) : 0);
    L.off_li = take(nl * 4);
    L.off_kof = take(nl * 4);
    L.off_L = take(nl * eb);
    // at most two flagged nodes and three deposited populations per link
    L.off_rec = take(2 * nl * 2);
    L.off_mnode = take(2 * nl * 4);
    L.off_pbase = take(2 * nl * 4);
    L.off_M = take(2 * nl * 3 * rb);
    L.off_P = take(3 * nl * eb);
    L.off_M2 = take(2 * nl * 3 * rb);
    L.off_P2 = take(3 * nl * eb);
    // force partials: one per 64 links (link kernel) or per row segment (fused bulk)
    L.wave_cap = std::max<int64_t>((int64_t)(nl + 63) / 64, (int64_t)(L.pitch / 64) * p.ny) + 16;
    L.off_wpart = take((size_t)L.wave_cap * 16);
    L.off_wobj = take((size_t)L.wave_cap * 4);
    L.off_uin = take((size_t)p.ny * 2 * rb);
    L.off_force = take((size_t)p.n_obj * 6 * sizeof(double));
    L.off_partials = take(1024 * sizeof(double));
    L.off_stage = take((size_t)std::min<int64_t>((int64_t)p.nx * p.ny, STAGE_NODES) * 3 *
                       sizeof(double) + (size_t)p.nx * 3 * sizeof(double));
    L.total = o;
    return L;
}

bool params_ok(const lbm_params *p, std::string *why)
{
    char m[256];
    if (!p) {
        *why = "null params";
        return false;
    }
    if (p->nx < 1 || p->ny < 1) {
        *why = "nx and ny must be >= 1";
        return false;
    }
    const int64_t pitch = (p->nx + 63) / 64 * 64;
    if (pitch * p->ny >= ((int64_t)1 << 31) / 2) {
        *why = "lattice too large for 32-bit plane offsets";
        return false;
    }
    if (p->x_bc != LBM_X_PERIODIC && p->x_bc != LBM_X_OPEN) {
        *why = "x_bc must be LBM_X_PERIODIC or LBM_X_OPEN";
        return false;
    }
    if (p->x_bc == LBM_X_OPEN && p->nx < 3) {
        *why = "an open lattice needs nx >= 3";
        return false;
    }
    if (p->storage < LBM_F64 || p->storage > LBM_F32_PLAIN) {
        *why = "unknown storage";
        return false;
    }
    if ((pitch * p->ny * (int64_t)elem_bytes(p->storage) + 512) >= ((int64_t)1 << 32)) {
        *why = "a population plane must be smaller than 4 GiB (the kernels use 32-bit byte offsets)";
        return false;
    }
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) {
        std::snprintf(m, sizeof m, "tau must be finite and > 1/2 (got %g)", p->tau);
        *why = m;
        return false;
    }
    if (!std::isfinite(p->gx) || !std::isfinite(p->gy) || !std::isfinite(p->rho0)) {
        *why = "gx, gy and rho0 must be finite";
        return false;
    }
    if (p->n_obj < 1 || p->n_obj > (1 << 23)) {
        *why = "n_obj must be in [1, 2^23]";
        return false;
    }
    if (p->dev_scale_log2 < -30 || p->dev_scale_log2 > 30) {
        *why = "dev_scale_log2 must be in [-30, 30]";
        return false;
    }
    if (p->layout != LBM_LAYOUT_DENSE && p->layout != LBM_LAYOUT_COMPACT) {
        *why = "layout must be LBM_LAYOUT_DENSE or LBM_LAYOUT_COMPACT";
        return false;
    }
    if (p->collision != LBM_COLLISION_BGK && p->collision != LBM_COLLISION_MRT) {
        *why = "collision must be LBM_COLLISION_BGK or LBM_COLLISION_MRT";
        return false;
    }
    if (p->collision == LBM_COLLISION_MRT) {
        for (double s : {p->s_e, p->s_eps, p->s_q})
            if (!(s > 0.0 && s < 2.0)) {
                std::snprintf(m, sizeof m, "MRT rates s_e, s_eps, s_q must lie in (0, 2) (got %g, %g, %g)",
                              p->s_e, p->s_eps, p->s_q);
                *why = m;
                return false;
            }
    }
    if (p->force_form != LBM_FORCE_PLAIN && p->force_form != LBM_FORCE_GALILEAN) {
        *why = "force_form must be LBM_FORCE_PLAIN or LBM_FORCE_GALILEAN";
        return false;
    }
    return true;
}



// Validates mask and links; on success fills the device-ready link arrays
// (sorted by object, then node, then direction).
lbm_status prepare_geometry(const lbm_params &p, const uint8_t *mask, int64_t n, const int32_t *node,
                            const int8_t *dir, const double *q, const double *uw,
                            const int32_t *obj, const int8_t *scheme, int32_t pitch, Prepared *out,
                            std::string *why)
{
    char m[256];
    const int nx = p.nx, ny = p.ny;
    const bool open = p.x_bc == LBM_X_OPEN;
    const int64_t N = (int64_t)nx * ny;
    if (!mask || n < 0 || (n > 0 && (!node || !dir || !q))) {
        *why = "null mask or link array";
        return LBM_E_ARG;
    }
    for (int64_t k = 0; k < N; ++k)
        if (mask[k] > 1) {
            std::snprintf(m, sizeof m, "mask[%lld] = %d is not 0 or 1", (long long)k, mask[k]);
            *why = m;
            return LBM_E_GEOM;
        }
    if (open)
        for (int y = 0; y < ny; ++y) {
            const int64_t r = (int64_t)y * nx;
            if ((!mask[r] && mask[r + 1]) || (!mask[r + nx - 1] && mask[r + nx - 2])) {
                std::snprintf(m, sizeof m, "open column node of row %d has a solid neighbour column", y);
                *why = m;
                return LBM_E_GEOM;
            }
        }
    std::vector<uint16_t> have((size_t)N, 0);
    for (int64_t l = 0; l < n; ++l) {
        const int32_t nd = node[l];
        const int d = dir[l];
        if (nd < 0 || nd >= N || d < 1 || d > 8) {
            std::snprintf(m, sizeof m, "link %lld: node or dir out of range", (long long)l);
            *why = m;
            return LBM_E_GEOM;
        }
        const int x = nd % nx, y = nd / nx;
        if (mask[nd] || (open && (x == 0 || x == nx - 1))) {
            std::snprintf(m, sizeof m, "link %lld: node %d is solid or an open column", (long long)l, nd);
            *why = m;
            return LBM_E_GEOM;
        }
        int xs = x + EXR[d];
        if (open && (xs < 0 || xs >= nx)) {
            std::snprintf(m, sizeof m, "link %lld: leaves the open lattice", (long long)l);
            *why = m;
            return LBM_E_GEOM;
        }
        xs = (xs + nx) % nx;
        const int ys = (y + EYR[d] + ny) % ny;
        if (!mask[(int64_t)ys * nx + xs]) {
            std::snprintf(m, sizeof m, "link %lld: node %d + e_%d is not solid", (long long)l, nd, d);
            *why = m;
            return LBM_E_GEOM;
        }
        if (!(q[l] > 0.0 && q[l] <= 1.0)) {
            std::snprintf(m, sizeof m, "link %lld: q = %g outside (0, 1]", (long long)l, q[l]);
            *why = m;
            return LBM_E_GEOM;
        }
        if (uw && (!std::isfinite(uw[2 * l]) || !std::isfinite(uw[2 * l + 1]))) {
            std::snprintf(m, sizeof m, "link %lld: non-finite wall velocity", (long long)l);
            *why = m;
            return LBM_E_GEOM;
        }
        if (obj && (obj[l] < 0 || obj[l] >= p.n_obj)) {
            std::snprintf(m, sizeof m, "link %lld: obj %d outside [0, %d)", (long long)l, obj[l], p.n_obj);
            *why = m;
            return LBM_E_GEOM;
        }
        if (scheme && (scheme[l] < LBM_SCHEME_VIBB || scheme[l] > LBM_SCHEME_YU)) {
            std::snprintf(m, sizeof m, "link %lld: unknown scheme %d", (long long)l, scheme[l]);
            *why = m;
            return LBM_E_GEOM;
        }
        if (have[nd] & (1u << d)) {
            std::snprintf(m, sizeof m, "link %lld: duplicate (node %d, dir %d)", (long long)l, nd, d);
            *why = m;
            return LBM_E_GEOM;
        }
        have[nd] |= (uint16_t)(1u << d);
    }
    // every pull from a solid node must be covered by a link
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int64_t nd = (int64_t)y * nx + x;
            if (mask[nd] || (open && (x == 0 || x == nx - 1))) continue;
            for (int i = 1; i < 9; ++i) {
                const int xs = (x - EXR[i] + nx) % nx, ys = (y - EYR[i] + ny) % ny;
                if (mask[(int64_t)ys * nx + xs] && !(have[nd] & (1u << OPPR[i]))) {
                    std::snprintf(m, sizeof m, "node %lld pulls direction %d from a solid node with no link",
                                  (long long)nd, i);
                    *why = m;
                    return LBM_E_GEOM;
                }
            }
        }
    if (!out) return LBM_OK;
    // scheme evaluated per link and its second node (-1: not read).  A scheme that
    // needs x_ff (VIBB, Yu, Bouzidi for q <= 1/2) falls back to halfway bounce-back
    // where x_ff is solid or off an open edge; Bouzidi for q > 1/2 and Yu also read
    // f+_i(x_f) of the outgoing direction i = opp(dir).
    std::vector<int32_t> ffo(n);  // plane offset of x_ff
    std::vector<uint8_t> eff(n);  // scheme evaluated
    out->n_fallback = 0;
    out->has_pfi = out->has_ext_scheme = false;
    for (int64_t l = 0; l < n; ++l) {
        const int nd = node[l], d = dir[l], x = nd % nx, y = nd / nx;
        int xf2 = x - EXR[d];
        const int yf2 = (y - EYR[d] + ny) % ny;
        bool ff_ok = !(open && (xf2 < 0 || xf2 >= nx));
        xf2 = (xf2 + nx) % nx;
        if (ff_ok && mask[(int64_t)yf2 * nx + xf2]) ff_ok = false;
        int sch = scheme ? scheme[l] : LBM_SCHEME_VIBB;
        out->has_ext_scheme |= sch == LBM_SCHEME_BOUZIDI || sch == LBM_SCHEME_YU;
        const bool needs_ff = sch == LBM_SCHEME_VIBB || sch == LBM_SCHEME_YU ||
                              (sch == LBM_SCHEME_BOUZIDI && q[l] <= 0.5);
        if (needs_ff && !ff_ok) {
            ++out->n_fallback;
            sch = LBM_SCHEME_HBB;
        }
        eff[l] = (uint8_t)sch;
        ffo[l] = (needs_ff && ff_ok) ? yf2 * pitch + xf2 : -1;
    }
    auto needs_pfi = [&](int64_t l) {
        return eff[l] == LBM_SCHEME_YU || (eff[l] == LBM_SCHEME_BOUZIDI && q[l] > 0.5);
    };
    // padded mask; padding columns count as solid and are never streamed
    const size_t plane_n = (size_t)pitch * ny;
    out->mask.assign(plane_n, lbm::MASK_SOLID);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            out->mask[(size_t)y * pitch + x] = mask[(int64_t)y * nx + x] ? lbm::MASK_SOLID : lbm::mask_t(0);
    // per-node record bits: link directions at x_f, deposited populations at x_f and x_ff
    std::vector<uint16_t> bits(plane_n, 0);
    for (int64_t l = 0; l < n; ++l) {
        const int nd = node[l], d = dir[l];
        const int32_t of = (nd / nx) * pitch + nd % nx;
        bits[of] |= (uint16_t)((1u << (d - 1)) | (1u << (d + 7)));
        if (ffo[l] >= 0) bits[ffo[l]] |= (uint16_t)(1u << (d + 7));
        if (needs_pfi(l)) bits[of] |= (uint16_t)(1u << (OPPR[d] + 7));
    }
    // slots, segment bases, deposit bases
    const int64_t nseg = (int64_t)(pitch / 64) * ny;
    out->seg.assign((size_t)nseg, lbm::SegBase{0, 0, 0, 0});
    out->rec.clear();
    out->mnode.clear();
    out->pbase.clear();
    std::vector<int32_t> slot(plane_n, -1);
    int32_t nlinks = 0, npops = 0;
    out->fmask.assign((size_t)nseg, 0);
    int32_t nfluid = 0;
    for (int64_t sg = 0; sg < nseg; ++sg) {
        out->seg[sg] = lbm::SegBase{(int32_t)out->rec.size(), nlinks, npops, nfluid};
        for (int b = 0; b < 64; ++b)
            if (!(out->mask[sg * 64 + b] & lbm::MASK_SOLID)) out->fmask[sg] |= 1ull << b;
        nfluid += __builtin_popcountll(out->fmask[sg]);
        for (int64_t o = sg * 64; o < sg * 64 + 64; ++o) {
            if (!bits[o]) continue;
            out->mask[o] |= (lbm::mask_t)(lbm::MASK_SIDE | (bits[o] & lbm::MASK_LINKS));
            slot[o] = (int32_t)out->rec.size();
            out->rec.push_back(bits[o]);
            out->mnode.push_back((int32_t)o);
            out->pbase.push_back(npops);
            nlinks += __builtin_popcount(bits[o] & 0xffu);
            npops += __builtin_popcount(bits[o] >> 8);
        }
    }
    // sentinel after the last segment: the totals
    out->seg.push_back(lbm::SegBase{(int32_t)out->rec.size(), nlinks, npops, nfluid});
    out->frow.resize((size_t)nseg + 1);
    for (int64_t sg = 0; sg <= nseg; ++sg) {
        const uint64_t fm = sg < nseg ? out->fmask[sg] : 0;
        out->frow[sg] = lbm::SegRow{(uint32_t)fm, (uint32_t)(fm >> 32), out->seg[sg].fluid, 0};
    }
    // runs of 64 fluid nodes in plane order: the counts before each run's first node
    out->n_fluid = nfluid;
    out->runs.clear();
    {
        int32_t fl = 0, nl = 0, np = 0, nf = 0;
        for (int64_t o = 0; o < (int64_t)plane_n; ++o) {
            if (out->mask[o] & lbm::MASK_SOLID) continue;
            const int j = nf & 63;
            if (j == 0) out->runs.push_back(lbm::RunBase{fl, nl, np, (int32_t)(o / 64), 0u, 0u, 0u, 0u});
            ++nf;
            if (bits[o]) {
                (j < 32 ? out->runs.back().flag_lo : out->runs.back().flag_hi) |= 1u << (j & 31);
                ++fl;
                nl += __builtin_popcount(bits[o] & 0xffu);
                np += __builtin_popcount(bits[o] >> 8);
            }
        }
        out->runs.push_back(lbm::RunBase{fl, nl, np, (int32_t)nseg, 0u, 0u, 0u, 0u});
        for (size_t r = 0; r + 1 < out->runs.size(); ++r)
            out->runs[r].nlinks = (uint32_t)(out->runs[r + 1].links - out->runs[r].links);
    }
    // Neighbour words for runs that read their pull offsets instead of computing
    // them from the segment tables (periodic x only; the x-open layout has no runs).
    // For fluid node k at (x, y) let dm and dp be the fluid ranks of (x, y-1) and
    // (x, y+1) relative to k.  Within a run of 64 nodes they vary little, so each
    // run stores the smallest dm and dp of its nodes (NbrRun) and each node a 16-bit
    // word: dm and dp above those bases in 7 bits each, and whether (x, y-1) and
    // (x, y+1) are fluid.  The nodes of the first and last row and column (periodic
    // wraps), and every node of a run whose differences spread over more than 126,
    // have the word 0xffff instead and their nine pull offsets in a table, in plane
    // order (the run stores how many entries precede it).
    out->nbr.clear();
    out->nbr_run.clear();
    out->nbr_slow.clear();
    if (p.x_bc != LBM_X_OPEN && p.layout == LBM_LAYOUT_COMPACT) {
        const int64_t nsr = pitch / 64;
        auto fluid_at = [&](int xx, int yy) { return !(out->mask[(size_t)yy * pitch + xx] & lbm::MASK_SOLID); };
        // rank of (x, r): fluid nodes before it in plane order
        auto rank = [&](int xx, int yy) -> int64_t {
            const int64_t sg = yy * nsr + xx / 64;
            return out->seg[sg].fluid + __builtin_popcountll(out->fmask[sg] & ((1ull << (xx & 63)) - 1ull));
        };
        const int64_t last = make_layout(p, 0).plane;  // the plane's element count bounds every offset
        struct Node {
            int x, y;
            int64_t dm, dp;
            bool fm, fp, edge;
        };
        std::vector<Node> run;
        run.reserve(64);
        auto flush = [&]() {
            if (run.empty()) return;
            int64_t m0 = INT64_MAX, m1 = INT64_MIN, p0 = INT64_MAX, p1 = INT64_MIN;
            for (const Node &n : run)
                if (!n.edge) {
                    m0 = std::min(m0, n.dm), m1 = std::max(m1, n.dm);
                    p0 = std::min(p0, n.dp), p1 = std::max(p1, n.dp);
                }
            const bool wide = m0 != INT64_MAX && (m1 - m0 > 126 || p1 - p0 > 126 || m0 < INT32_MIN ||
                                                   m0 > INT32_MAX || p0 < INT32_MIN || p0 > INT32_MAX);
            if (m0 == INT64_MAX || wide) m0 = p0 = 0;
            out->nbr_run.push_back(lbm::NbrRun{(int32_t)m0, (int32_t)p0, (int32_t)(out->nbr_slow.size() / 9), 0});
            for (const Node &n : run) {
                if (!n.edge && !wide) {
                    out->nbr.push_back((uint16_t)((uint32_t)(n.dm - m0) | ((uint32_t)n.fm << 7) |
                                                  ((uint32_t)(n.dp - p0) << 8) | ((uint32_t)n.fp << 15)));
                    continue;
                }
                // the nine offsets as the segment walk computes them (elements)
                const int x = n.x, y = n.y;
                const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
                const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
                const int rows[3] = {ym, y, yp};
                int64_t rk[3], lf[3], rt[3];
                for (int r = 0; r < 3; ++r) {
                    rk[r] = rank(x, rows[r]);
                    lf[r] = x == 0 ? rank(xm, rows[r]) : std::max<int64_t>(rk[r] - 1, 0);
                    rt[r] = x == nx - 1 ? rank(xp, rows[r])
                                        : std::min<int64_t>(rk[r] + (fluid_at(x, rows[r]) ? 1 : 0), last - 1);
                }
                const int64_t o9[9] = {rk[1], lf[1], rk[0], rt[1], rk[2], lf[0], rt[0], rt[2], lf[2]};
                for (int i = 0; i < 9; ++i) out->nbr_slow.push_back((uint32_t)o9[i]);
                out->nbr.push_back((uint16_t)0xffffu);
            }
            run.clear();
        };
        out->nbr.reserve((size_t)nfluid);
        int64_t k = 0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!fluid_at(x, y)) continue;
                const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
                run.push_back(Node{x, y, rank(x, ym) - k, rank(x, yp) - k, fluid_at(x, ym), fluid_at(x, yp),
                                   y == 0 || y == ny - 1 || x == 0 || x == nx - 1});
                if (run.size() == 64) flush();
                ++k;
            }
        flush();
        out->nbr_run.push_back(lbm::NbrRun{0, 0, (int32_t)(out->nbr_slow.size() / 9), 0});  // sentinel
        // table entries beyond the workspace's room: no neighbour words
        if ((int64_t)out->nbr_slow.size() / 9 > nbr_table_room(pitch, ny)) {
            out->nbr.clear();
            out->nbr_run.clear();
            out->nbr_slow.clear();
        }
    }
    out->n_pops = npops;
    auto rank_below = [](uint32_t set, int d) { return __builtin_popcount(set & ((1u << (d - 1)) - 1u)); };
    // links in (obj, node, dir) order; L entry = rank in (node, dir) order
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        const int oa = obj ? obj[a] : 0, ob = obj ? obj[b] : 0;
        if (oa != ob) return oa < ob;
        if (node[a] != node[b]) return node[a] < node[b];
        return dir[a] < dir[b];
    });
    out->order = order;
    out->meta.resize(n);
    out->q.resize(n);
    out->sf.assign(n, -1);
    out->sff.assign(n, -1);
    out->pf.resize(n);
    out->pff.assign(n, -1);
    out->pfi.resize(n);
    out->li.resize(n);
    out->has_uw = false;
    if (uw)
        for (int64_t l = 0; l < n && !out->has_uw; ++l)
            out->has_uw = uw[2 * l] != 0.0 || uw[2 * l + 1] != 0.0;
    out->uw.assign(out->has_uw ? 2 * n : 0, 0.0);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t l = order[k];
        const int nd = node[l], d = dir[l];
        const int32_t of = (nd / nx) * pitch + nd % nx;
        const int32_t sfo = slot[of];
        out->meta[k] = (uint32_t)d | ((uint32_t)eff[l] << 4) | ((uint32_t)(obj ? obj[l] : 0) << 8);
        out->q[k] = q[l];
        if (out->has_uw) {
            out->uw[2 * k] = uw[2 * l];
            out->uw[2 * k + 1] = uw[2 * l + 1];
        }
        out->sf[k] = sfo;
        out->pf[k] = out->pbase[sfo] + rank_below(out->rec[sfo] >> 8, d);
        out->pfi[k] = out->pf[k];
        if (needs_pfi(l)) {
            out->pfi[k] = out->pbase[sfo] + rank_below(out->rec[sfo] >> 8, OPPR[d]);
            out->has_pfi = true;
        }
        if (ffo[l] >= 0) {
            const int32_t sff = slot[ffo[l]];
            out->sff[k] = sff;
            out->pff[k] = out->pbase[sff] + rank_below(out->rec[sff] >> 8, d);
        }
    }
    // L entry of a link: links of earlier nodes plus the link's rank at its node
    std::vector<int32_t> links_before(out->rec.size());
    {
        int32_t acc = 0;
        for (size_t k = 0; k < out->rec.size(); ++k) {
            links_before[k] = acc;
            acc += __builtin_popcount(out->rec[k] & 0xffu);
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        const int d = (int)(out->meta[k] & 15u);
        const int32_t sfo = out->sf[k];
        out->li[k] = links_before[sfo] + rank_below(out->rec[sfo] & 0xffu, d);
    }
    return LBM_OK;
}

void build_link_records(size_t n, const uint32_t *meta, const float *q, const int32_t *sf, const int32_t *sff,
                        const int32_t *pf, const int32_t *pff, std::vector<lbm::LinkRec> *crec,
                        std::vector<lbm::LinkRunBase> *cbase)
{
    crec->assign(n, lbm::LinkRec{0u, 0u, 0u, 0u});
    cbase->assign(n / 64 + 1, lbm::LinkRunBase{-1, 0, 0, 0});
    for (size_t r = 0; r * 64 < n; ++r) {
        const size_t a = r * 64, e = std::min(n, a + 64);
        int64_t sf0 = INT64_MAX, pf0 = INT64_MAX, sff0 = INT64_MAX, pff0 = INT64_MAX;
        int64_t sf1 = INT64_MIN, pf1 = INT64_MIN, sff1 = INT64_MIN, pff1 = INT64_MIN;
        for (size_t k = a; k < e; ++k) {
            sf0 = std::min<int64_t>(sf0, sf[k]), sf1 = std::max<int64_t>(sf1, sf[k]);
            pf0 = std::min<int64_t>(pf0, pf[k]), pf1 = std::max<int64_t>(pf1, pf[k]);
            if (sff[k] >= 0) {
                sff0 = std::min<int64_t>(sff0, sff[k]), sff1 = std::max<int64_t>(sff1, sff[k]);
                pff0 = std::min<int64_t>(pff0, pff[k]), pff1 = std::max<int64_t>(pff1, pff[k]);
            }
        }
        if (sff0 == INT64_MAX) sff0 = sff1 = pff0 = pff1 = 0;
        // 0xffff is kept free in the x_ff slot excess: it marks a link without x_ff
        const bool fit = sf1 - sf0 <= 0xffff && pf1 - pf0 <= 0xffff && sff1 - sff0 < 0xffff && pff1 - pff0 <= 0xffff;
        if (fit) (*cbase)[r] = lbm::LinkRunBase{(int32_t)sf0, (int32_t)pf0, (int32_t)sff0, (int32_t)pff0};
        for (size_t k = a; k < e; ++k) {
            uint32_t qb;
            std::memcpy(&qb, &q[k], 4);
            uint32_t df = 0u, dff = 0u;
            if (fit) {
                df = (uint32_t)(sf[k] - sf0) | ((uint32_t)(pf[k] - pf0) << 16);
                dff = sff[k] >= 0 ? (uint32_t)(sff[k] - sff0) | ((uint32_t)(pff[k] - pff0) << 16) : 0xffffu;
            }
            (*crec)[k] = lbm::LinkRec{meta[k], qb, df, dff};
        }
    }
}

}  // namespace lbm_host

using namespace lbm_host;


extern "C" void lbm_set_thread_error(const char *msg) { g_thread_error = msg; }

lbm_status lbm_host::enqueue_step(lbm_ctx *c, bool timed)
{
    lbm_status s = enqueue_step_to(c, c->cur, c->nxt, timed);
    if (s) return s;
    std::swap(c->cur, c->nxt);
    return LBM_OK;
}

lbm_status lbm_host::enqueue_step_to(lbm_ctx *c, const void *A, void *B, bool timed)
{
    const lbm::Grid g = c->grid();
    const lbm::Phys ph = c->phys();
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (timed) {
        while (c->events.size() < c->ev_used + 3) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return c->fail(LBM_E_DEVICE, "hipEventCreate failed");
            c->events.push_back(e);
        }
        e0 = c->events[c->ev_used];
        e1 = c->events[c->ev_used + 1];
        e2 = c->events[c->ev_used + 2];
        c->ev_used += 3;
        hipEventRecord(e0, c->stream);
    }
    const lbm::Side sd = c->side_par(c->dpar);
    lbm_status s;
    if (c->kcfg.bulk_fused) {
        // links inside the bulk kernel: the link interval of the timing is empty
        if (timed) hipEventRecord(e1, c->stream);
        const lbm::Reduce red = c->reduce();
        const lbm::FuseArgs fa{c->links(), red.wpart, red.wobj, c->bank(c->step), c->fsum()};
        s = c->hip(lbm::launch_bulk_fused(c->p.storage, g, ph, A, B, c->mask(), c->ws + c->lay.off_uin, sd, fa,
                                          c->bank(c->step + 1), 2 * c->p.n_obj, c->bulk_config(), c->stream),
                   "fused bulk kernel launch");
        if (s) return s;
    } else {
        // the force reduction over the link kernel's partials runs in the bulk launch
        lbm::ForceReduce fr{};
        s = c->hip(lbm::launch_link(c->p.storage, g, ph, c->links(), sd, c->reduce(), c->bank(c->step), c->fsum(),
                                    c->kcfg.link_block, c->stream, &fr),
                   "link kernel launch");
        if (s) return s;
        if (timed) hipEventRecord(e1, c->stream);
        s = c->hip(lbm::launch_bulk(c->p.storage, g, ph, A, B, c->mask(), c->ws + c->lay.off_uin, sd,
                                    c->bank(c->step + 1), 2 * c->p.n_obj, c->bulk_config(), c->stream, fr),
                   "bulk kernel launch");
        if (s) return s;
    }
    if (timed) hipEventRecord(e2, c->stream);
    c->dpar ^= 1;
    ++c->step;
    ++c->nsum;
    return LBM_OK;
}

namespace {

lbm_status collect_times(lbm_ctx *c)
{
    if (c->ev_used == 0) return LBM_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return c->fail(LBM_E_DEVICE, "sync failed");
    for (size_t k = 0; k + 2 < c->ev_used; k += 3) {
        float a = 0, b = 0;
        hipEventElapsedTime(&a, c->events[k], c->events[k + 1]);
        hipEventElapsedTime(&b, c->events[k + 1], c->events[k + 2]);
        c->link_ms += a;
        c->bulk_ms += b;
        ++c->prof_steps;
    }
    c->ev_used = 0;
    return LBM_OK;
}

// Captures kcfg.graph_steps steps on a private stream (the caller's stream may be the
// null stream, which cannot be captured); the graph is launched on the caller's
// stream.
lbm_status build_graph(lbm_ctx *c)
{
    c->drop_graph();
    if (!c->cap_stream &&
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        return c->fail(LBM_E_DEVICE, "hipStreamCreateWithFlags failed");
    }
    void *start = c->cur;
    const int64_t step0 = c->step, nsum0 = c->nsum;
    const int dpar0 = c->dpar;
    hipGraph_t graph = nullptr;
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    lbm_status s = c->hip(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed),
                          "hipStreamBeginCapture");
    if (s) {
        c->stream = user;
        return s;
    }
    for (int k = 0; k < c->kcfg.graph_steps && !s; ++k) s = enqueue_step(c, false);
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    c->stream = user;
    // capture only records; restore the host-side counters
    c->step = step0;
    c->nsum = nsum0;
    c->dpar = dpar0;
    if (c->cur != start) std::swap(c->cur, c->nxt);
    if (s) {
        if (graph) hipGraphDestroy(graph);
        return s;
    }
    if ((s = c->hip(e, "hipStreamEndCapture"))) return s;
    e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if ((s = c->hip(e, "hipGraphInstantiate"))) {
        c->gexec = nullptr;
        return s;
    }
    c->graph_cur = start;
    c->graph_dpar = dpar0;
    return LBM_OK;
}

lbm_status check_finite(lbm_ctx *c, const double *v, size_t n, const char *what)
{
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return c->fail(LBM_E_UNSTABLE, "non-finite %s read back", what);
    return LBM_OK;
}

}  // namespace

extern "C" {

const char *lbm_last_error(const lbm_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_thread_error.c_str();
}

lbm_status lbm_check_geometry(const lbm_params *p, const uint8_t *mask, int64_t n_links,
                              const int32_t *node, const int8_t *dir, const double *q,
                              const double *uw, const int32_t *obj, const int8_t *scheme,
                              int64_t *n_fallback)
{
    std::string why;
    if (!params_ok(p, &why)) {
        g_thread_error = "lbm_check_geometry: " + why;
        return LBM_E_ARG;
    }
    Prepared prep;
    const int32_t pitch = (p->nx + 63) / 64 * 64;
    lbm_status s = prepare_geometry(*p, mask, n_links, node, dir, q, uw, obj, scheme, pitch,
                                    n_fallback ? &prep : nullptr, &why);
    if (s) {
        g_thread_error = "lbm_check_geometry: " + why;
        return s;
    }
    if (n_fallback) *n_fallback = prep.n_fallback;
    return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_params *p, int64_t max_links)
{
    std::string why;
    if (!params_ok(p, &why) || max_links < 0 || max_links > LBM_MAX_LINKS) return 0;
    return make_layout(*p, max_links).total;
}

lbm_status lbm_create(const lbm_params *p, void *workspace, size_t bytes, lbm_ctx **out)
{
    std::string why;
    if (!out) {
        g_thread_error = "lbm_create: null output pointer";
        return LBM_E_ARG;
    }
    *out = nullptr;
    if (!params_ok(p, &why)) {
        g_thread_error = "lbm_create: " + why;
        return LBM_E_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        g_thread_error = "lbm_create: no HIP device available";
        return LBM_E_DEVICE;
    }
    if (p->device < 0 || p->device >= ndev) {
        g_thread_error = "lbm_create: device ordinal out of range";
        return LBM_E_ARG;
    }
    if (!workspace || ((uintptr_t)workspace & 255)) {
        g_thread_error = "lbm_create: workspace must be non-null and 256-byte aligned";
        return LBM_E_ARG;
    }
    // largest link capacity the workspace holds (layout size is monotone in it)
    if (bytes < make_layout(*p, 0).total) {
        g_thread_error = "lbm_create: workspace too small";
        return LBM_E_NOMEM;
    }
    int64_t lo = 0, hi = (int64_t)(bytes / bytes_per_link(p->storage)) + 1;
    while (make_layout(*p, hi).total <= bytes) hi *= 2;
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(*p, mid).total <= bytes) lo = mid;
        else hi = mid;
    }
    const int64_t cap = std::min<int64_t>(lo, LBM_MAX_LINKS);
    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) {
        g_thread_error = "lbm_create: out of host memory";
        return LBM_E_NOMEM;
    }
    c->p = *p;
    c->lay = make_layout(*p, cap);
    c->max_links = cap;
    c->ws = static_cast<char *>(workspace);
    c->ws_bytes = bytes;
    c->stream = static_cast<hipStream_t>(p->stream);
    c->cur = c->ws + c->lay.off_A;
    c->nxt = c->ws + c->lay.off_B;
    if (hipSetDevice(p->device) != hipSuccess) {
        delete c;
        g_thread_error = "lbm_create: hipSetDevice failed";
        return LBM_E_DEVICE;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_get_params(const lbm_ctx *c, lbm_params *out)
{
    if (!c || !out) return LBM_E_ARG;
    *out = c->p;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx *c)
{
    if (!c) return;
    c->drop_graph();
    for (hipEvent_t e : c->events) hipEventDestroy(e);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
}

lbm_status lbm_set_geometry(lbm_ctx *c, const uint8_t *mask, int64_t n_links, const int32_t *node,
                            const int8_t *dir, const double *q, const double *uw, const int32_t *obj,
                            const int8_t *scheme)
{
    if (!c) return LBM_E_ARG;
    c->adj.valid = false;
    std::string why;
    Prepared prep;
    lbm_status s = prepare_geometry(c->p, mask, n_links, node, dir, q, uw, obj, scheme, c->lay.pitch,
                                    &prep, &why);
    if (s) return c->fail(s, "lbm_set_geometry: %s", why.c_str());
    if (n_links > c->max_links)
        return c->fail(LBM_E_NOMEM, "lbm_set_geometry: %lld links exceed the workspace capacity %lld",
                       (long long)n_links, (long long)c->max_links);
    c->drop_graph();
    const hipStream_t st = c->stream;
    if ((s = c->hip(hipMemcpyAsync(c->mask(), prep.mask.data(), prep.mask.size() * sizeof(lbm::mask_t),
                                   hipMemcpyHostToDevice, st), "mask upload")))
        return s;
    const size_t n = (size_t)n_links;
    const size_t rb = real_bytes(c->p.storage);
    std::vector<float> qf, uwf;
    const void *qsrc = prep.q.data(), *uwsrc = prep.uw.data();
    if (rb == 4) {
        qf.assign(prep.q.begin(), prep.q.end());
        uwf.assign(prep.uw.begin(), prep.uw.end());
        qsrc = qf.data();
        uwsrc = uwf.data();
    }
    const size_t K = prep.rec.size();
    // link index of each (node, dir) rank, for the fused bulk kernel
    std::vector<int32_t> kof(n);
    for (size_t k = 0; k < n; ++k) kof[prep.li[k]] = (int32_t)k;
    // compact link records (4-byte reals)
    std::vector<lbm::LinkRec> crec;
    std::vector<lbm::LinkRunBase> cbase;
    if (rb == 4)
        build_link_records(n, prep.meta.data(), qf.data(), prep.sf.data(), prep.sff.data(), prep.pf.data(),
                           prep.pff.data(), &crec, &cbase);
    struct Up {
        size_t off;
        const void *src;
        size_t bytes;
    } ups[] = {{c->lay.off_meta, prep.meta.data(), n * 4},
               {c->lay.off_q, qsrc, n * rb},
               {c->lay.off_uw, uwsrc, prep.has_uw ? 2 * n * rb : 0},
               {c->lay.off_sf, prep.sf.data(), n * 4},
               {c->lay.off_sff, prep.sff.data(), n * 4},
               {c->lay.off_pf, prep.pf.data(), n * 4},
               {c->lay.off_pff, prep.pff.data(), n * 4},
               {c->lay.off_pfi, prep.pfi.data(), prep.has_pfi ? n * 4 : 0},
               {c->lay.off_crec, crec.data(), crec.size() * sizeof(lbm::LinkRec)},
               {c->lay.off_cbase, cbase.data(), cbase.size() * sizeof(lbm::LinkRunBase)},
               {c->lay.off_li, prep.li.data(), n * 4},
               {c->lay.off_kof, kof.data(), kof.size() * 4},
               {c->lay.off_rec, prep.rec.data(), K * 2},
               {c->lay.off_mnode, prep.mnode.data(), K * 4},
               {c->lay.off_pbase, prep.pbase.data(), K * 4},
               {c->lay.off_seg, prep.seg.data(), prep.seg.size() * sizeof(lbm::SegBase)},
               {c->lay.off_fmask, prep.fmask.data(), prep.fmask.size() * sizeof(uint64_t)},
               {c->lay.off_runs, prep.runs.data(), prep.runs.size() * sizeof(lbm::RunBase)},
               {c->lay.off_frow, prep.frow.data(), prep.frow.size() * sizeof(lbm::SegRow)},
               {c->lay.off_nbr, prep.nbr.data(), prep.nbr.size() * sizeof(uint16_t)},
               {c->lay.off_nbrr, prep.nbr_run.data(), prep.nbr_run.size() * sizeof(lbm::NbrRun)},
               {c->lay.off_nbrs, prep.nbr_slow.data(), prep.nbr_slow.size() * sizeof(uint32_t)}};
    for (const Up &u : ups)
        if (u.bytes && (s = c->hip(hipMemcpyAsync(c->ws + u.off, u.src, u.bytes,
                                                  hipMemcpyHostToDevice, st), "link upload")))
            return s;
    // both population buffers start at zero (solid slots included)
    if ((s = c->hip(hipMemsetAsync(c->ws + c->lay.off_A, 0, c->lay.off_mask - c->lay.off_A, st),
                    "population clear")))
        return s;
    if ((s = c->hip(hipMemsetAsync(c->force(), 0, (size_t)c->p.n_obj * 6 * sizeof(double), st),
                    "force clear")))
        return s;
    if ((s = c->hip(hipStreamSynchronize(st), "geometry upload")))  // host vectors die here
        return s;
    c->n_links = n_links;
    c->link_order = prep.order;
    c->li_ident = true;
    for (int64_t k = 0; k < n_links && c->li_ident; ++k) c->li_ident = prep.li[k] == k;
    c->colslot.assign(c->p.x_bc == LBM_X_OPEN ? 2 * (size_t)c->p.ny : 0, -1);
    if (c->p.x_bc == LBM_X_OPEN)
        for (int y = 0; y < c->p.ny; ++y)
            for (int side = 0; side < 2; ++side) {
                const int32_t o = y * c->lay.pitch + (side ? c->p.nx - 1 : 0);
                auto it = std::lower_bound(prep.mnode.begin(), prep.mnode.end(), o);
                if (it != prep.mnode.end() && *it == o)
                    c->colslot[(size_t)side * c->p.ny + y] = (int32_t)(it - prep.mnode.begin());
            }
    c->n_moment_nodes = (int64_t)prep.rec.size();
    c->n_fluid = prep.n_fluid;
    c->nruns = (int32_t)prep.runs.size() - 1;
    c->has_nbr = !prep.nbr.empty() || prep.n_fluid == 0;
    if (c->kcfg.bulk_runs == 2 && !c->has_nbr) c->kcfg.bulk_runs = 1;  // offsets from the segment tables
    c->has_uw = prep.has_uw;
    c->has_pfi = prep.has_pfi;
    c->has_crec = rb == 4 && n > 0;
    c->has_ext_scheme = prep.has_ext_scheme;
    c->have_geom = true;
    c->have_init = false;
    c->cur = c->ws + c->lay.off_A;
    c->nxt = c->ws + c->lay.off_B;
    c->dpar = 0;
    c->step = 0;
    c->nsum = 0;
    return LBM_OK;
}

lbm_status lbm_set_inlet(lbm_ctx *c, const double *ux, const double *uy)
{
    if (!c) return LBM_E_ARG;
    const int ny = c->p.ny;
    std::vector<double> v((size_t)2 * ny, 0.0);
    for (int y = 0; y < ny; ++y) {
        v[2 * y] = ux ? ux[y] : 0.0;
        v[2 * y + 1] = uy ? uy[y] : 0.0;
        if (!std::isfinite(v[2 * y]) || !std::isfinite(v[2 * y + 1]))
            return c->fail(LBM_E_ARG, "lbm_set_inlet: non-finite velocity in row %d", y);
    }
    lbm_status s;
    if (real_bytes(c->p.storage) == 4) {
        std::vector<float> f(v.begin(), v.end());
        s = c->hip(hipMemcpyAsync(c->ws + c->lay.off_uin, f.data(), f.size() * 4,
                                  hipMemcpyHostToDevice, c->stream), "inlet upload");
        if (!s) s = c->hip(hipStreamSynchronize(c->stream), "inlet upload");
    } else {
        s = c->hip(hipMemcpyAsync(c->ws + c->lay.off_uin, v.data(), v.size() * 8,
                                  hipMemcpyHostToDevice, c->stream), "inlet upload");
        if (!s) s = c->hip(hipStreamSynchronize(c->stream), "inlet upload");
    }
    return s;
}

lbm_status lbm_init_equilibrium(lbm_ctx *c, const double *rho, const double *ux, const double *uy)
{
    if (!c) return LBM_E_ARG;
    c->adj.valid = false;
    if (!c->have_geom) return c->fail(LBM_E_STATE, "lbm_init_equilibrium before lbm_set_geometry");
    c->drop_graph();
    const int nx = c->p.nx, ny = c->p.ny;
    const int rows_per = (int)std::max<int64_t>(1, STAGE_NODES / nx);
    std::vector<double> h;
    lbm_status s;
    for (int y0 = 0; y0 < ny; y0 += rows_per) {
        const int rows = std::min(rows_per, ny - y0);
        h.assign((size_t)3 * rows * nx, 0.0);
        for (int64_t k = 0; k < (int64_t)rows * nx; ++k) {
            const int64_t n = (int64_t)y0 * nx + k;
            h[3 * k] = rho ? rho[n] : c->p.rho0;
            h[3 * k + 1] = ux ? ux[n] : 0.0;
            h[3 * k + 2] = uy ? uy[n] : 0.0;
            if (!std::isfinite(h[3 * k]) || !std::isfinite(h[3 * k + 1]) || !std::isfinite(h[3 * k + 2]))
                return c->fail(LBM_E_ARG, "lbm_init_equilibrium: non-finite value at node %lld",
                               (long long)n);
        }
        if ((s = c->hip(hipMemcpyAsync(c->stage(), h.data(), h.size() * 8, hipMemcpyHostToDevice,
                                       c->stream), "init upload")))
            return s;
        if ((s = c->hip(lbm::launch_init(c->p.storage, c->grid(), c->phys(), c->cur, c->mask(),
                                         c->stage(), y0, rows, c->stream), "init kernel")))
            return s;
        if ((s = c->hip(hipStreamSynchronize(c->stream), "init")))  // h is reused
            return s;
    }
    if ((s = c->hip(lbm::launch_refresh(c->p.storage, c->grid(), c->phys(), c->cur, c->side(), true,
                                        c->stream), "deposit refresh")))
        return s;
    c->have_init = true;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t n)
{
    if (!c) return LBM_E_ARG;
    if (n < 0) return c->fail(LBM_E_ARG, "lbm_step: negative step count");
    if (!c->have_geom || !c->have_init)
        return c->fail(LBM_E_STATE, "lbm_step before lbm_set_geometry and initialisation");
    lbm_status s;
    if (c->prof) {
        for (int64_t k = 0; k < n; ++k)
            if ((s = enqueue_step(c, true))) return s;
        if (c->ev_used > 3 * 256) return collect_times(c);
        return LBM_OK;
    }
    while (n > 0) {
        const int gs = c->kcfg.graph_steps;
        if (n >= gs) {
            if (!c->gexec || c->graph_cur != c->cur || c->graph_dpar != c->dpar) {
                if ((s = build_graph(c))) return s;
            }
            if ((s = c->hip(hipGraphLaunch(c->gexec, c->stream), "hipGraphLaunch"))) return s;
            c->step += gs;
            c->nsum += gs;  // graph_steps is even: buffers return to their roles
            n -= gs;
        } else {
            if ((s = enqueue_step(c, false))) return s;
            --n;
        }
    }
    return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx *c)
{
    if (!c) return LBM_E_ARG;
    return c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

int64_t lbm_step_count(const lbm_ctx *c) { return c ? c->step : -1; }

lbm_status lbm_moments(lbm_ctx *c, double *rho, double *ux, double *uy)
{
    if (!c) return LBM_E_ARG;
    if (!c->have_geom || !c->have_init) return c->fail(LBM_E_STATE, "lbm_moments before initialisation");
    const int nx = c->p.nx, ny = c->p.ny;
    const int rows_per = (int)std::max<int64_t>(1, STAGE_NODES / nx);
    std::vector<double> h;
    lbm_status s;
    for (int y0 = 0; y0 < ny; y0 += rows_per) {
        const int rows = std::min(rows_per, ny - y0);
        h.resize((size_t)3 * rows * nx);
        if ((s = c->hip(lbm::launch_moments(c->p.storage, c->grid(), c->phys(), c->cur, c->mask(),
                                            c->stage(), y0, rows, c->stream), "moments kernel")))
            return s;
        if ((s = c->hip(hipMemcpyAsync(h.data(), c->stage(), h.size() * 8, hipMemcpyDeviceToHost,
                                       c->stream), "moments read-back")))
            return s;
        if ((s = c->hip(hipStreamSynchronize(c->stream), "moments"))) return s;
        if ((s = check_finite(c, h.data(), h.size(), "moment"))) return s;
        for (int64_t k = 0; k < (int64_t)rows * nx; ++k) {
            const int64_t n = (int64_t)y0 * nx + k;
            if (rho) rho[n] = h[3 * k];
            if (ux) ux[n] = h[3 * k + 1];
            if (uy) uy[n] = h[3 * k + 2];
        }
    }
    return LBM_OK;
}

lbm_status lbm_moments_device(lbm_ctx *c, void *rho, void *ux, void *uy, int32_t fp64)
{
    if (!c) return LBM_E_ARG;
    if (!c->have_geom || !c->have_init)
        return c->fail(LBM_E_STATE, "lbm_moments_device before initialisation");
    return c->hip(lbm::launch_moments_out(c->p.storage, c->grid(), c->phys(), c->cur, c->mask(), rho, ux, uy,
                                          fp64 != 0, c->stream),
                  "moments kernel");
}

namespace {
double half_to_double(uint16_t h)
{
    const int sgn = h >> 15, ex = (h >> 10) & 31, man = h & 1023;
    double v;
    if (ex == 0) v = std::ldexp((double)man, -24);
    else if (ex == 31) v = man ? NAN : INFINITY;
    else v = std::ldexp((double)(man | 1024), ex - 25);
    return sgn ? -v : v;
}
double bf16_to_double(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
}  // namespace

lbm_status lbm_populations(lbm_ctx *c, double *f)
{
    if (!c || !f) return LBM_E_ARG;
    if (!c->have_geom || !c->have_init) return c->fail(LBM_E_STATE, "lbm_populations before initialisation");
    const int nx = c->p.nx, ny = c->p.ny, pitch = c->lay.pitch;
    const size_t eb = elem_bytes(c->p.storage);
    const double inv = std::ldexp(1.0, storage_is_16bit(c->p.storage) ? -c->p.dev_scale_log2 : 0);
    std::vector<lbm::mask_t> mask((size_t)pitch * ny);
    std::vector<char> plane((size_t)pitch * ny * eb);
    lbm_status s;
    if ((s = c->hip(hipMemcpy(mask.data(), c->mask(), mask.size() * sizeof(lbm::mask_t), hipMemcpyDeviceToHost),
                    "mask read")))
        return s;
    if ((s = c->hip(hipStreamSynchronize(c->stream), "populations"))) return s;
    // plane offset of every node: y*pitch + x, or its fluid rank in the compact layout
    std::vector<int64_t> off((size_t)pitch * ny);
    {
        int64_t r = 0;
        for (size_t k = 0; k < off.size(); ++k) {
            off[k] = c->p.layout == LBM_LAYOUT_COMPACT ? r : (int64_t)k;
            if (!(mask[k] & lbm::MASK_SOLID)) ++r;
        }
    }
    for (int i = 0; i < 9; ++i) {
        const char *src = static_cast<const char *>(c->cur) + (size_t)i * c->lay.plane * eb;
        if ((s = c->hip(hipMemcpy(plane.data(), src, plane.size(), hipMemcpyDeviceToHost), "plane read")))
            return s;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t k = (size_t)off[(size_t)y * pitch + x];
                double d;
                switch (c->p.storage) {
                case LBM_F64: std::memcpy(&d, &plane[k * 8], 8); break;
                case LBM_F32:
                case LBM_F32_WIDE:
                case LBM_F32_PLAIN: {
                    float v;
                    std::memcpy(&v, &plane[k * 4], 4);
                    d = v;
                    break;
                }
                case LBM_F16_DEV: {
                    uint16_t v;
                    std::memcpy(&v, &plane[k * 2], 2);
                    d = half_to_double(v) * inv;
                    break;
                }
                default: {
                    uint16_t v;
                    std::memcpy(&v, &plane[k * 2], 2);
                    d = bf16_to_double(v) * inv;
                }
                }
                f[((size_t)y * nx + x) * 9 + i] =
                    (mask[(size_t)y * pitch + x] & lbm::MASK_SOLID) ? 0.0 : d + WR[i];
            }
    }
    return LBM_OK;
}

lbm_status lbm_force(lbm_ctx *c, int32_t obj, double last[2], double sum[2], int64_t *nsum)
{
    if (!c) return LBM_E_ARG;
    if (obj < 0 || obj >= c->p.n_obj) return c->fail(LBM_E_ARG, "lbm_force: obj %d out of range", obj);
    double h[4] = {0, 0, 0, 0};
    lbm_status s;
    if (c->step > 0 &&
        (s = c->hip(hipMemcpyAsync(h, c->bank(c->step - 1) + 2 * obj, 16, hipMemcpyDeviceToHost,
                                   c->stream), "force read")))
        return s;
    if ((s = c->hip(hipMemcpyAsync(h + 2, c->fsum() + 2 * obj, 16, hipMemcpyDeviceToHost, c->stream),
                    "force read")))
        return s;
    if ((s = c->hip(hipStreamSynchronize(c->stream), "force read"))) return s;
    if ((s = check_finite(c, h, 4, "force"))) return s;
    if (last) last[0] = h[0], last[1] = h[1];
    if (sum) sum[0] = h[2], sum[1] = h[3];
    if (nsum) *nsum = c->nsum;
    return LBM_OK;
}

lbm_status lbm_force_reset(lbm_ctx *c)
{
    if (!c) return LBM_E_ARG;
    lbm_status s = c->hip(hipMemsetAsync(c->fsum(), 0, (size_t)c->p.n_obj * 2 * sizeof(double), c->stream),
                          "force reset");
    if (s) return s;
    c->nsum = 0;
    return LBM_OK;
}

namespace {
lbm_status reduce_state(lbm_ctx *c, bool maxdev, double *out)
{
    if (!c || !out) return LBM_E_ARG;
    if (!c->have_geom || !c->have_init) return c->fail(LBM_E_STATE, "reduction before initialisation");
    const int nb = lbm::mass_blocks(c->grid());
    std::vector<double> h(nb);
    lbm_status s;
    if ((s = c->hip(lbm::launch_mass(c->p.storage, c->grid(), c->phys(), c->cur, c->mask(), c->partials(),
                                     nb, maxdev, c->stream), "reduction kernel")))
        return s;
    if ((s = c->hip(hipMemcpyAsync(h.data(), c->partials(), nb * 8, hipMemcpyDeviceToHost, c->stream),
                    "reduction read")))
        return s;
    if ((s = c->hip(hipStreamSynchronize(c->stream), "reduction"))) return s;
    double t = 0;
    for (double v : h) t = maxdev ? std::fmax(t, v) : t + v;
    if (!std::isfinite(t)) return c->fail(LBM_E_UNSTABLE, "non-finite populations");
    *out = t;
    return LBM_OK;
}
}  // namespace

lbm_status lbm_mass(lbm_ctx *c, double *m) { return reduce_state(c, false, m); }

lbm_status lbm_max_deviation(lbm_ctx *c, double *d) { return reduce_state(c, true, d); }

// Checkpoint layout: {step, nsum} | populations (nine planes, storage precision) |
// force accumulators | side moments of the flagged nodes (they are part of the
// state: recomputing them from rounded populations would not resume bitwise).
size_t lbm_state_bytes(const lbm_ctx *c)
{
    if (!c) return 0;
    return 9 * (size_t)c->lay.plane * elem_bytes(c->p.storage) + 6 * (size_t)c->p.n_obj * sizeof(double) +
           2 * sizeof(int64_t) + (size_t)c->n_moment_nodes * 3 * real_bytes(c->p.storage);
}

lbm_status lbm_state_layout(const lbm_ctx *c, int32_t *pitch, int64_t *plane_elems, int32_t *elem)
{
    if (!c) return LBM_E_ARG;
    if (pitch) *pitch = c->lay.pitch;
    if (plane_elems) *plane_elems = c->lay.plane;
    if (elem) *elem = (int32_t)elem_bytes(c->p.storage);
    return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx *c, void *host, size_t bytes)
{
    if (!c || !host) return LBM_E_ARG;
    if (bytes < lbm_state_bytes(c)) return c->fail(LBM_E_ARG, "lbm_get_state: buffer too small");
    if (!c->have_geom || !c->have_init) return c->fail(LBM_E_STATE, "lbm_get_state before initialisation");
    char *h = static_cast<char *>(host);
    const size_t pb = 9 * (size_t)c->lay.plane * elem_bytes(c->p.storage);
    int64_t hdr[2] = {c->step, c->nsum};
    std::memcpy(h, hdr, sizeof hdr);
    lbm_status s;
    if ((s = c->hip(hipStreamSynchronize(c->stream), "state"))) return s;
    if ((s = c->hip(hipMemcpy(h + sizeof hdr, c->cur, pb, hipMemcpyDeviceToHost), "state read"))) return s;
    const size_t fb = 6 * (size_t)c->p.n_obj * 8;
    if ((s = c->hip(hipMemcpy(h + sizeof hdr + pb, c->force(), fb, hipMemcpyDeviceToHost), "state read")))
        return s;
    return c->hip(hipMemcpy(h + sizeof hdr + pb + fb, c->side().M,
                            (size_t)c->n_moment_nodes * 3 * real_bytes(c->p.storage),
                            hipMemcpyDeviceToHost), "state read");
}

lbm_status lbm_set_state(lbm_ctx *c, const void *host, size_t bytes)
{
    if (c) c->adj.valid = false;
    if (!c || !host) return LBM_E_ARG;
    if (!c->have_geom) return c->fail(LBM_E_STATE, "lbm_set_state before lbm_set_geometry");
    if (bytes < lbm_state_bytes(c)) return c->fail(LBM_E_ARG, "lbm_set_state: buffer too small");
    c->drop_graph();
    const char *h = static_cast<const char *>(host);
    const size_t pb = 9 * (size_t)c->lay.plane * elem_bytes(c->p.storage);
    int64_t hdr[2];
    std::memcpy(hdr, h, sizeof hdr);
    lbm_status s;
    if ((s = c->hip(hipStreamSynchronize(c->stream), "state"))) return s;
    // the step parity selects the buffer roles and the force bank
    c->cur = c->ws + ((hdr[0] & 1) ? c->lay.off_B : c->lay.off_A);
    c->nxt = c->ws + ((hdr[0] & 1) ? c->lay.off_A : c->lay.off_B);
    if ((s = c->hip(hipMemcpy(c->cur, h + sizeof hdr, pb, hipMemcpyHostToDevice), "state write"))) return s;
    const size_t fb = 6 * (size_t)c->p.n_obj * 8;
    if ((s = c->hip(hipMemcpy(c->force(), h + sizeof hdr + pb, fb, hipMemcpyHostToDevice), "state write")))
        return s;
    if ((s = c->hip(hipMemcpy(c->side().M, h + sizeof hdr + pb + fb,
                              (size_t)c->n_moment_nodes * 3 * real_bytes(c->p.storage),
                              hipMemcpyHostToDevice), "state write")))
        return s;
    // the deposited populations are copies of stored values: rebuilt exactly
    if ((s = c->hip(lbm::launch_refresh(c->p.storage, c->grid(), c->phys(), c->cur, c->side(), false,
                                        c->stream), "deposit refresh")))
        return s;
    c->step = hdr[0];
    c->nsum = hdr[1];
    c->have_init = true;
    return LBM_OK;
}

lbm_status lbm_set_profiling(lbm_ctx *c, int32_t on)
{
    if (!c) return LBM_E_ARG;
    lbm_status s = collect_times(c);
    if (s) return s;
    c->prof = on != 0;
    c->link_ms = c->bulk_ms = 0;
    c->prof_steps = 0;
    return LBM_OK;
}

lbm_status lbm_get_kernel_config(const lbm_ctx *c, lbm_kernel_config *cfg)
{
    if (!c || !cfg) return LBM_E_ARG;
    *cfg = c->kcfg;
    return LBM_OK;
}

lbm_status lbm_set_kernel_config(lbm_ctx *c, const lbm_kernel_config *cfg)
{
    if (!c || !cfg) return LBM_E_ARG;
    const int bx = cfg->bulk_block_x;
    if ((bx != 64 && bx != 128 && bx != 256) || (cfg->bulk_store_solid != 0 && cfg->bulk_store_solid != 1) ||
        (cfg->bulk_xcd != 0 && cfg->bulk_xcd != 1) || (cfg->bulk_fused != 0 && cfg->bulk_fused != 1) ||
        (cfg->bulk_fused && bx != 256) || cfg->bulk_rows < 0 || cfg->bulk_rows > 2 ||
        (cfg->bulk_rows == 2 && (bx != 256 || cfg->bulk_fused)) ||
        cfg->link_block < 64 || cfg->link_block > 1024 || cfg->link_block % 64 ||
        cfg->graph_steps < 2 || cfg->graph_steps > 1024 || cfg->graph_steps % 2)
        return c->fail(LBM_E_ARG, "lbm_set_kernel_config: unsupported configuration");
    if (c->p.collision == LBM_COLLISION_MRT && (bx != 256 || (cfg->bulk_fused && !cfg->bulk_runs)))
        return c->fail(LBM_E_ARG, "lbm_set_kernel_config: MRT runs with bulk_block_x 256, and fused only with "
                                  "bulk_runs");
    if (cfg->bulk_runs < 0 || cfg->bulk_runs > 2)
        return c->fail(LBM_E_ARG, "lbm_set_kernel_config: bulk_runs must be 0, 1 or 2");
    if (cfg->bulk_runs && (c->p.layout != LBM_LAYOUT_COMPACT || c->p.x_bc == LBM_X_OPEN))
        return c->fail(LBM_E_ARG, "lbm_set_kernel_config: bulk_runs needs the compact layout and a periodic x "
                                  "direction");
    if (cfg->bulk_runs == 2 && !c->has_nbr)
        return c->fail(LBM_E_ARG, "lbm_set_kernel_config: bulk_runs 2 needs the neighbour words of a geometry "
                                  "(set one first; not built when the first and last row and column hold too "
                                  "many fluid nodes)");
    c->drop_graph();
    c->kcfg = *cfg;
    return LBM_OK;
}

// Autotune cache: with the environment variable VIBB_TUNE_CACHE naming a file,
// lbm_autotune first looks for the lattice's key there and applies the stored
// configuration without timing trials; after a tuning run it appends the choice as
// one JSON line {"key": "...", "config": [8 ints], "ms": t}.  The key holds what
// the choice depends on: device architecture, lattice size and boundary, storage,
// layout, collision, body force, link and fluid counts, moving walls and closures.
// Every configuration computes the same result, so a stale or foreign entry can
// only cost speed.  Lines that do not parse are ignored.
namespace {

std::string tune_key(const lbm_ctx *c)
{
    hipDeviceProp_t prop{};
    const char *arch = hipGetDeviceProperties(&prop, c->p.device) == hipSuccess ? prop.gcnArchName : "unknown";
    char k[512];
    std::snprintf(k, sizeof k, "v1:%s:%dx%d:x%d:s%d:l%d:c%d:f%d:n%lld:k%d:o%d:u%d:e%d", arch, c->p.nx, c->p.ny,
                  c->p.x_bc, c->p.storage, c->p.layout, c->p.collision,
                  (c->p.gx != 0.0 || c->p.gy != 0.0) ? 1 : 0, (long long)c->n_links, c->n_fluid, c->p.n_obj,
                  c->has_uw ? 1 : 0, c->has_ext_scheme ? 1 : 0);
    for (char *q = k; *q; ++q)
        if (*q == '"' || *q == '\\' || *q == '\n') *q = '_';
    return k;
}

bool tune_lookup(const char *path, const std::string &key, lbm_kernel_config *cfg, double *ms)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    const std::string tag = "{\"key\": \"" + key + "\", \"config\": [";
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, tag.c_str(), tag.size()) != 0) continue;
        lbm_kernel_config k{};
        double t = 0;
        if (std::sscanf(line + tag.size(), "%d, %d, %d, %d, %d, %d, %d, %d], \"ms\": %lf", &k.bulk_block_x,
                        &k.bulk_store_solid, &k.link_block, &k.graph_steps, &k.bulk_xcd, &k.bulk_fused, &k.bulk_rows,
                        &k.bulk_runs, &t) == 9) {
            *cfg = k;  // the last matching line wins
            *ms = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const char *path, const std::string &key, const lbm_kernel_config &k, double ms)
{
    char line[1024];
    const int n = std::snprintf(line, sizeof line,
                                "{\"key\": \"%s\", \"config\": [%d, %d, %d, %d, %d, %d, %d, %d], \"ms\": %.6g}\n",
                                key.c_str(), k.bulk_block_x, k.bulk_store_solid, k.link_block, k.graph_steps,
                                k.bulk_xcd, k.bulk_fused, k.bulk_rows, k.bulk_runs, ms);
    if (n <= 0 || n >= (int)sizeof line) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;  // an unwritable cache only costs the next run its trials
    std::fputs(line, f);  // one write per line (append mode)
    std::fclose(f);
}

}  // namespace

// Times every bulk shape and link block size on the current state (steps_per_trial
// steps each, HIP events on the context's stream), keeps the fastest and restores
// the state, so the run continues as if no trial had been made.
lbm_status lbm_autotune(lbm_ctx *c, int32_t steps_per_trial, lbm_kernel_config *chosen,
                        double *best_ms_per_step)
{
    if (!c || steps_per_trial < 1) return LBM_E_ARG;
    if (!c->have_geom || !c->have_init) return c->fail(LBM_E_STATE, "lbm_autotune before initialisation");
    const char *cache = std::getenv("VIBB_TUNE_CACHE");
    std::string key;
    if (cache && *cache) {
        key = tune_key(c);
        lbm_kernel_config k{};
        double ms = 0;
        if (tune_lookup(cache, key, &k, &ms) && lbm_set_kernel_config(c, &k) == LBM_OK) {
            if (chosen) *chosen = k;
            if (best_ms_per_step) *best_ms_per_step = ms;
            return LBM_OK;
        }
    }
    std::vector<char> saved(lbm_state_bytes(c));
    lbm_status s = lbm_get_state(c, saved.data(), saved.size());
    if (s) return s;
    const bool prof = c->prof;
    if ((s = lbm_set_profiling(c, 0))) return s;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return c->fail(LBM_E_DEVICE, "hipEventCreate failed");
    const lbm_kernel_config base = c->kcfg;
    lbm_kernel_config best = base;
    double best_ms = 1e300;
    auto trial = [&](const lbm_kernel_config &k, double *ms) -> lbm_status {
        lbm_status r = lbm_set_kernel_config(c, &k);
        if (r) return r;
        for (int w = 0; w < 2; ++w)
            if ((r = enqueue_step(c, false))) return r;
        hipEventRecord(e0, c->stream);
        for (int t = 0; t < steps_per_trial; ++t)
            if ((r = enqueue_step(c, false))) return r;
        hipEventRecord(e1, c->stream);
        if ((r = c->hip(hipEventSynchronize(e1), "autotune"))) return r;
        float f = 0;
        hipEventElapsedTime(&f, e0, e1);
        *ms = f / steps_per_trial;
        return LBM_OK;
    };
    for (int bx : {64, 128, 256})
        for (int ss : {0, 1})
            for (int xo : {0, 1})
                for (int rows : {1, 2}) {
                    if (s || (ss && c->p.layout == LBM_LAYOUT_COMPACT)) continue;  // no solid slots there
                    if (rows == 2 && bx != 256) continue;
                    if (c->p.collision == LBM_COLLISION_MRT && bx != 256) continue;
                    lbm_kernel_config k = best;
                    k.bulk_block_x = bx;
                    k.bulk_store_solid = ss;
                    k.bulk_xcd = xo;
                    k.bulk_fused = 0;
                    k.bulk_rows = rows;
                    k.bulk_runs = 0;
                    double ms;
                    if ((s = trial(k, &ms))) break;
                    if (ms < best_ms) best_ms = ms, best = k;
                }
    // runs of 64 fluid nodes per wavefront (compact layout, periodic in x), with
    // offsets from the segment tables or from the neighbour words
    for (int ru : {1, 2})
        for (int xo : {0, 1}) {
            if (s || c->p.layout != LBM_LAYOUT_COMPACT || c->p.x_bc == LBM_X_OPEN) break;
            if (ru == 2 && !c->has_nbr) break;
            lbm_kernel_config k = best;
            k.bulk_block_x = 256;
            k.bulk_store_solid = 0;
            k.bulk_xcd = xo;
            k.bulk_fused = 0;
            k.bulk_rows = 1;
            k.bulk_runs = ru;
            double ms;
            if ((s = trial(k, &ms))) break;
            if (ms < best_ms) best_ms = ms, best = k;
        }
    for (int lb : {128, 256, 512, 1024}) {
        if (s) break;
        lbm_kernel_config k = best;
        k.link_block = lb;
        double ms;
        if ((s = trial(k, &ms))) break;
        if (ms < best_ms) best_ms = ms, best = k;
    }
    // links evaluated inside the bulk kernel (256-lane blocks)
    const lbm_kernel_config unfused = best;
    for (int ss : {0, 1})
        for (int xo : {0, 1}) {
            if (s || (ss && c->p.layout == LBM_LAYOUT_COMPACT) || c->p.collision != LBM_COLLISION_BGK) continue;
            lbm_kernel_config k = unfused;
            k.bulk_fused = 1;
            k.bulk_rows = 1;
            k.bulk_runs = 0;
            k.bulk_block_x = 256;
            k.bulk_store_solid = ss;
            k.bulk_xcd = xo;
            double ms;
            if ((s = trial(k, &ms))) break;
            if (ms < best_ms) best_ms = ms, best = k;
        }
    // links inside the run kernel (compact layout, periodic in x), with the run
    // form the unfused trials chose
    for (int xo : {0, 1}) {
        if (s || c->p.layout != LBM_LAYOUT_COMPACT || c->p.x_bc == LBM_X_OPEN) break;
        lbm_kernel_config k = unfused;
        k.bulk_fused = 1;
        k.bulk_runs = unfused.bulk_runs ? unfused.bulk_runs : 1;
        k.bulk_rows = 1;
        k.bulk_block_x = 256;
        k.bulk_store_solid = 0;
        k.bulk_xcd = xo;
        double ms;
        if ((s = trial(k, &ms))) break;
        if (ms < best_ms) best_ms = ms, best = k;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    lbm_status r = lbm_set_kernel_config(c, s ? &base : &best);
    if (!r) r = lbm_set_state(c, saved.data(), saved.size());
    if (!r) r = lbm_set_profiling(c, prof ? 1 : 0);
    if (s) return s;
    if (r) return r;
    if (cache && *cache) tune_store(cache, key, best, best_ms);
    if (chosen) *chosen = best;
    if (best_ms_per_step) *best_ms_per_step = best_ms;
    return LBM_OK;
}

lbm_status lbm_kernel_times(lbm_ctx *c, double *link_ms, double *bulk_ms, int64_t *n_steps)
{
    if (!c) return LBM_E_ARG;
    lbm_status s = collect_times(c);
    if (s) return s;
    if (link_ms) *link_ms = c->link_ms;
    if (bulk_ms) *bulk_ms = c->bulk_ms;
    if (n_steps) *n_steps = c->prof_steps;
    return LBM_OK;
}

}  // extern "C"
