// Batched form of the C ABI (include/lbm.h, lbm_batch_*): many lattices of uneven
// size advanced together, one link launch and one bulk launch per step for all
// of them (HIP graph replay of a fixed number of steps).
//
// Every instance keeps its own population planes, mask words, segment table and
// inlet rows at per-instance offsets of shared buffers; the boundary data that the
// kernels exchange (side records, deposits, link values, force accumulators) is
// numbered globally across instances, so the link kernel and the force reduction
// run unchanged over the concatenated link list.  The bulk kernel reads a tile
// table (instance, row, column of every 256-node block) and the instance
// descriptors.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_host.h"
#include "lbm_internal.h"

using namespace lbm_host;

namespace {

struct InstLayout {
    int32_t pitch;
    int64_t plane;     // elements per plane
    int64_t pop_off;   // element offset of plane 0 in A and B
    int64_t mask_off;  // mask words
    int32_t seg_off, nseg;
    int32_t uin_off;   // inlet rows
    int32_t obj_off;   // first global object
    int64_t max_links;
};

}  // namespace

struct lbm_batch {
    int32_t n = 0;
    std::vector<lbm_params> p;
    std::vector<InstLayout> il;
    int32_t storage = 1, x_bc = 0;
    bool forced = false;  // some instance has a body force
    int64_t n_obj = 0, max_links = 0, pop_elems = 0, mask_words = 0, nseg = 0, uin_rows = 0, ntiles = 0,
            stage_nodes = 0;
    hipStream_t stream = nullptr, cap_stream = nullptr;
    std::string err = "no error";
    char *ws = nullptr;
    size_t bytes = 0;
    // workspace offsets
    size_t off_A = 0, off_B = 0, off_mask = 0, off_seg = 0, off_meta = 0, off_q = 0, off_uw = 0, off_sf = 0,
           off_sff = 0, off_pf = 0, off_pff = 0, off_pfi = 0, off_crec = 0, off_cbase = 0, off_li = 0, off_L = 0, off_rec = 0, off_mnode = 0,
           off_pbase = 0, off_M = 0, off_P = 0, off_wpart = 0, off_wobj = 0, off_uin = 0, off_force = 0,
           off_insts = 0, off_tiles = 0, off_partials = 0, off_stage = 0, total = 0;
    // geometry, per instance until the batch is assembled
    std::vector<Prepared> prep;
    std::vector<char> has_geom, has_init;
    bool assembled = false;
    // global numbering after assembly
    std::vector<int64_t> slot_off, pop_base, link_off;
    int64_t n_links = 0, n_flagged = 0, n_pops = 0;
    bool has_uw = false, has_pfi = false;
    void *cur = nullptr, *nxt = nullptr;
    int64_t step = 0, nsum = 0;
    lbm_batch_kernel_config kcfg{1, 1, 256, 16};
    hipGraphExec_t gexec = nullptr;
    void *graph_cur = nullptr;

    lbm_status fail(lbm_status s, const char *fmt, ...)
    {
        char m[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(m, sizeof m, fmt, ap);
        va_end(ap);
        err = m;
        return s;
    }
    lbm_status hip(hipError_t e, const char *what)
    {
        if (e == hipSuccess) return LBM_OK;
        return fail(LBM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    }
    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        graph_cur = nullptr;
    }
    lbm::Phys phys(int i) const
    {
        const float sc = std::ldexp(1.0f, lbm_host::storage_is_16bit(storage) ? p[0].dev_scale_log2 : 0);
        return lbm::Phys{1.0 / p[i].tau, p[i].gx, p[i].gy, p[0].rho0, sc, 1.0f / sc, p[0].s_e, p[0].s_eps,
                         p[0].s_q, p[0].force_form == LBM_FORCE_GALILEAN ? 1 : 0, p[0].collision};
    }
    lbm::Grid grid(int i) const
    {
        return lbm::Grid{p[i].nx, p[i].ny, il[i].pitch, x_bc == LBM_X_OPEN ? 1 : 0, il[i].plane, 0, 0, nullptr,
                         nullptr};
    }
    size_t eb() const { return elem_bytes(storage); }
    size_t rb() const { return real_bytes(storage); }
    lbm::mask_t *mask(int i) const { return reinterpret_cast<lbm::mask_t *>(ws + off_mask) + il[i].mask_off; }
    char *pops(void *base, int i) const { return static_cast<char *>(base) + il[i].pop_off * eb(); }
    double *force() const { return reinterpret_cast<double *>(ws + off_force); }
    double *bank(int64_t t) const { return force() + (size_t)(t & 1) * 2 * n_obj; }
    double *fsum() const { return force() + 4 * (size_t)n_obj; }
    double *stage() const { return reinterpret_cast<double *>(ws + off_stage); }
    lbm::Side side_global() const
    {
        return lbm::Side{ws + off_M, ws + off_P, ws + off_L, reinterpret_cast<const uint16_t *>(ws + off_rec),
                         reinterpret_cast<const lbm::SegBase *>(ws + off_seg),
                         reinterpret_cast<const int32_t *>(ws + off_mnode),
                         reinterpret_cast<const int32_t *>(ws + off_pbase), n_flagged, ws + off_M, ws + off_P};
    }
    // the flagged nodes of instance i alone (its records, deposits and local node offsets)
    lbm::Side side_of(int i) const
    {
        const int64_t so = slot_off[i];
        return lbm::Side{ws + off_M + (size_t)so * 3 * rb(), ws + off_P + (size_t)pop_base[i] * eb(),
                         ws + off_L, reinterpret_cast<const uint16_t *>(ws + off_rec) + so,
                         reinterpret_cast<const lbm::SegBase *>(ws + off_seg) + il[i].seg_off,
                         reinterpret_cast<const int32_t *>(ws + off_mnode) + so,
                         reinterpret_cast<const int32_t *>(ws + off_pbase) + so,
                         (int64_t)prep[i].rec.size(), ws + off_M + (size_t)so * 3 * rb(),
                         ws + off_P + (size_t)pop_base[i] * eb()};
    }
    lbm::Links links() const
    {
        auto i32 = [&](size_t off) { return reinterpret_cast<const int32_t *>(ws + off); };
        return lbm::Links{reinterpret_cast<const uint32_t *>(ws + off_meta), ws + off_q,
                          has_uw ? ws + off_uw : nullptr, i32(off_sf), i32(off_sff), i32(off_pf), i32(off_pff),
                          i32(off_li), n_links, 0, 0, nullptr, has_pfi ? i32(off_pfi) : nullptr,
                          rb() == 4 && n_links > 0 ? reinterpret_cast<const lbm::LinkRec *>(ws + off_crec) : nullptr,
                          reinterpret_cast<const lbm::LinkRunBase *>(ws + off_cbase)};
    }
};

namespace {

// Lays the batch out in a workspace starting at 0; returns the total size.
size_t layout(lbm_batch *b)
{
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t eb = b->eb(), rb = b->rb();
    b->pop_elems = b->mask_words = b->nseg = b->uin_rows = b->n_obj = b->max_links = b->ntiles = 0;
    b->stage_nodes = 0;
    for (int i = 0; i < b->n; ++i) {
        InstLayout &L = b->il[i];
        const lbm_params &p = b->p[i];
        L.pitch = (p.nx + 63) / 64 * 64;
        size_t pb = align256((size_t)L.pitch * p.ny * eb);
        if ((pb / 256) % 2 == 0) pb += 256;
        L.plane = (int64_t)(pb / eb);
        L.pop_off = b->pop_elems;
        b->pop_elems += 9 * L.plane;
        L.mask_off = b->mask_words;
        b->mask_words += (int64_t)L.pitch * p.ny;
        L.nseg = (L.pitch / 64) * p.ny;
        L.seg_off = (int32_t)b->nseg;
        b->nseg += L.nseg;
        L.uin_off = (int32_t)b->uin_rows;
        b->uin_rows += p.ny;
        L.obj_off = (int32_t)b->n_obj;
        b->n_obj += p.n_obj;
        b->max_links += L.max_links;
        b->ntiles += (int64_t)((p.nx + lbm::BATCH_BX - 1) / lbm::BATCH_BX) * p.ny;
        b->stage_nodes = std::max<int64_t>(b->stage_nodes, std::min<int64_t>((int64_t)p.nx * p.ny, 1 << 20) +
                                                               p.nx);
    }
    const size_t nl = (size_t)b->max_links;
    b->off_A = take((size_t)b->pop_elems * eb);
    b->off_B = take((size_t)b->pop_elems * eb);
    b->off_mask = take((size_t)b->mask_words * sizeof(lbm::mask_t));
    b->off_seg = take((size_t)b->nseg * sizeof(lbm::SegBase));
    b->off_meta = take(nl * 4);
    b->off_q = take(nl * rb);
    b->off_uw = take(nl * 2 * rb);
    b->off_sf = take(nl * 4);
    b->off_sff = take(nl * 4);
    b->off_pf = take(nl * 4);
    b->off_pff = take(nl * 4);
    b->off_pfi = take(nl * 4);
    b->off_crec = take(rb == 4 ? nl * sizeof(lbm::LinkRec) : 0);
    b->off_cbase = take(rb == 4 ? (nl / 64 + 1) * sizeof(lbm::LinkRunBase) : 0);
    b->off_li = take(nl * 4);
    b->off_L = take(nl * eb);
    b->off_rec = take(2 * nl * 2);
    b->off_mnode = take(2 * nl * 4);
    b->off_pbase = take(2 * nl * 4);
    b->off_M = take(2 * nl * 3 * rb);
    b->off_P = take(3 * nl * eb);
    const size_t waves = (nl + 63) / 64 + 16;
    b->off_wpart = take(waves * 16);
    b->off_wobj = take(waves * 4);
    b->off_uin = take((size_t)b->uin_rows * 2 * rb);
    b->off_force = take((size_t)b->n_obj * 6 * sizeof(double));
    b->off_insts = take((size_t)b->n * sizeof(lbm::BatchInst));
    b->off_tiles = take((size_t)b->ntiles * sizeof(lbm::BatchTile));
    b->off_partials = take(1024 * sizeof(double));
    b->off_stage = take((size_t)b->stage_nodes * 3 * sizeof(double));
    b->total = o;
    return o;
}

bool batch_params_ok(int32_t n, const lbm_params *p, const int64_t *max_links, std::string *why)
{
    if (n < 1 || !p || !max_links) {
        *why = "need n >= 1 instances, params and link capacities";
        return false;
    }
    int64_t total_links = 0;
    for (int i = 0; i < n; ++i) {
        if (max_links[i] >= 0) total_links += max_links[i];
        if (total_links > LBM_MAX_LINKS) {
            *why = "the link capacities sum to more than LBM_MAX_LINKS";
            return false;
        }
    }
    for (int i = 0; i < n; ++i) {
        std::string w;
        if (!params_ok(&p[i], &w)) {
            *why = "instance " + std::to_string(i) + ": " + w;
            return false;
        }
        if (max_links[i] < 0) {
            *why = "instance " + std::to_string(i) + ": negative link capacity";
            return false;
        }
        if (p[i].layout != LBM_LAYOUT_DENSE) {
            *why = "instance " + std::to_string(i) + ": the batched form uses the dense layout";
            return false;
        }
        if (p[i].storage != p[0].storage || p[i].x_bc != p[0].x_bc || p[i].rho0 != p[0].rho0 ||
            p[i].dev_scale_log2 != p[0].dev_scale_log2 || p[i].device != p[0].device ||
            p[i].stream != p[0].stream || p[i].collision != p[0].collision ||
            p[i].force_form != p[0].force_form ||
            (p[0].collision == LBM_COLLISION_MRT &&
             (p[i].s_e != p[0].s_e || p[i].s_eps != p[0].s_eps || p[i].s_q != p[0].s_q))) {
            *why = "instance " + std::to_string(i) +
                   ": storage, x_bc, rho0, dev_scale_log2, device, stream, collision, force_form and the MRT "
                   "rates must match instance 0";
            return false;
        }
    }
    return true;
}

// Concatenates the per-instance geometries into the global arrays and uploads
// them with the instance descriptors and the tile table.
lbm_status assemble(lbm_batch *b)
{
    for (int i = 0; i < b->n; ++i)
        if (!b->has_geom[i]) return b->fail(LBM_E_STATE, "instance %d has no geometry", i);
    b->drop_graph();
    b->slot_off.assign(b->n, 0);
    b->pop_base.assign(b->n, 0);
    b->link_off.assign(b->n, 0);
    int64_t slots = 0, pops = 0, links = 0;
    b->has_uw = b->has_pfi = false;
    for (int i = 0; i < b->n; ++i) {
        b->slot_off[i] = slots;
        b->pop_base[i] = pops;
        b->link_off[i] = links;
        slots += (int64_t)b->prep[i].rec.size();
        pops += b->prep[i].n_pops;
        links += (int64_t)b->prep[i].meta.size();
        b->has_uw |= b->prep[i].has_uw;
        b->has_pfi |= b->prep[i].has_pfi;
    }
    if (slots >= INT32_MAX || pops >= INT32_MAX || links >= INT32_MAX)
        return b->fail(LBM_E_NOMEM, "batch too large for 32-bit link numbering");
    b->n_links = links;
    b->n_flagged = slots;
    b->n_pops = pops;
    std::vector<uint32_t> meta;
    std::vector<double> q, uw;
    std::vector<int32_t> sf, sff, pf, pff, pfi, li, mnode, pbase;
    std::vector<uint16_t> rec;
    std::vector<lbm::SegBase> seg;
    meta.reserve(links);
    for (int i = 0; i < b->n; ++i) {
        const Prepared &P = b->prep[i];
        const int32_t so = (int32_t)b->slot_off[i], po = (int32_t)b->pop_base[i], lo = (int32_t)b->link_off[i];
        const uint32_t oo = (uint32_t)b->il[i].obj_off;
        for (size_t k = 0; k < P.meta.size(); ++k) {
            meta.push_back((P.meta[k] & 255u) | (((P.meta[k] >> 8) + oo) << 8));
            q.push_back(P.q[k]);
            if (b->has_uw) {
                uw.push_back(P.has_uw ? P.uw[2 * k] : 0.0);
                uw.push_back(P.has_uw ? P.uw[2 * k + 1] : 0.0);
            }
            sf.push_back(P.sf[k] + so);
            sff.push_back(P.sff[k] >= 0 ? P.sff[k] + so : -1);
            pf.push_back(P.pf[k] + po);
            pff.push_back(P.pff[k] >= 0 ? P.pff[k] + po : -1);
            if (b->has_pfi) pfi.push_back((P.has_pfi ? P.pfi[k] : P.pf[k]) + po);
            li.push_back(P.li[k] + lo);
        }
        rec.insert(rec.end(), P.rec.begin(), P.rec.end());
        mnode.insert(mnode.end(), P.mnode.begin(), P.mnode.end());
        pbase.insert(pbase.end(), P.pbase.begin(), P.pbase.end());
        for (size_t k = 0; k + 1 < P.seg.size(); ++k) {  // the instance's sentinel is not copied
            const lbm::SegBase &sb = P.seg[k];
            seg.push_back(lbm::SegBase{sb.flagged + so, sb.links + lo, sb.pops + po, 0});
        }
    }
    std::vector<lbm::BatchInst> insts(b->n);
    std::vector<lbm::BatchTile> tiles;
    tiles.reserve(b->ntiles);
    for (int i = 0; i < b->n; ++i) {
        insts[i] = lbm::BatchInst{b->grid(i), b->il[i].pop_off, b->il[i].mask_off, b->il[i].seg_off,
                                  b->il[i].uin_off, 1.0 / b->p[i].tau, b->p[i].gx, b->p[i].gy};
        for (int y = 0; y < b->p[i].ny; ++y)
            for (int x0 = 0; x0 < b->p[i].nx; x0 += lbm::BATCH_BX) tiles.push_back(lbm::BatchTile{i, y, x0, 0});
    }
    const size_t rb = b->rb();
    std::vector<float> qf, uwf;
    const void *qsrc = q.data(), *uwsrc = uw.data();
    if (rb == 4) {
        qf.assign(q.begin(), q.end());
        uwf.assign(uw.begin(), uw.end());
        qsrc = qf.data();
        uwsrc = uwf.data();
    }
    const size_t n = (size_t)links;
    // compact link records (4-byte reals) over the batch's global numbering
    std::vector<lbm::LinkRec> crec;
    std::vector<lbm::LinkRunBase> cbase;
    if (rb == 4)
        build_link_records(n, meta.data(), qf.data(), sf.data(), sff.data(), pf.data(), pff.data(), &crec, &cbase);
    struct Up {
        size_t off;
        const void *src;
        size_t bytes;
    } ups[] = {{b->off_meta, meta.data(), n * 4},
               {b->off_q, qsrc, n * rb},
               {b->off_uw, uwsrc, b->has_uw ? 2 * n * rb : 0},
               {b->off_sf, sf.data(), n * 4},
               {b->off_sff, sff.data(), n * 4},
               {b->off_pf, pf.data(), n * 4},
               {b->off_pff, pff.data(), n * 4},
               {b->off_pfi, pfi.data(), b->has_pfi ? n * 4 : 0},
               {b->off_li, li.data(), n * 4},
               {b->off_crec, crec.data(), crec.size() * sizeof(lbm::LinkRec)},
               {b->off_cbase, cbase.data(), cbase.size() * sizeof(lbm::LinkRunBase)},
               {b->off_rec, rec.data(), rec.size() * 2},
               {b->off_mnode, mnode.data(), mnode.size() * 4},
               {b->off_pbase, pbase.data(), pbase.size() * 4},
               {b->off_seg, seg.data(), seg.size() * sizeof(lbm::SegBase)},
               {b->off_insts, insts.data(), insts.size() * sizeof(lbm::BatchInst)},
               {b->off_tiles, tiles.data(), tiles.size() * sizeof(lbm::BatchTile)}};
    lbm_status s;
    for (const Up &u : ups)
        if (u.bytes && (s = b->hip(hipMemcpyAsync(b->ws + u.off, u.src, u.bytes, hipMemcpyHostToDevice, b->stream),
                                   "batch upload")))
            return s;
    if ((s = b->hip(hipStreamSynchronize(b->stream), "batch upload"))) return s;
    b->assembled = true;
    // deposits of every initialised instance from its populations
    for (int i = 0; i < b->n; ++i)
        if (b->has_init[i] &&
            (s = b->hip(lbm::launch_refresh(b->storage, b->grid(i), b->phys(i), b->pops(b->cur, i), b->side_of(i),
                                            true, b->stream), "batch deposit refresh")))
            return s;
    return LBM_OK;
}

lbm_status enqueue_batch_step(lbm_batch *b)
{
    const lbm::Side side = b->side_global();
    lbm::Reduce red{reinterpret_cast<double2 *>(b->ws + b->off_wpart), reinterpret_cast<int32_t *>(b->ws + b->off_wobj)};
    // the force reduction over the link kernel's partials runs in the bulk launch
    lbm::ForceReduce fr{};
    lbm_status s = b->hip(lbm::launch_link(b->storage, b->grid(0), b->phys(0), b->links(), side, red,
                                           b->bank(b->step), b->fsum(), b->kcfg.link_block, b->stream, &fr),
                          "batch link launch");
    if (s) return s;
    s = b->hip(lbm::launch_bulk_batch(b->storage, reinterpret_cast<const lbm::BatchInst *>(b->ws + b->off_insts),
                                      reinterpret_cast<const lbm::BatchTile *>(b->ws + b->off_tiles), b->ntiles,
                                      b->phys(0), b->cur, b->nxt, reinterpret_cast<const lbm::mask_t *>(b->ws + b->off_mask),
                                      b->ws + b->off_uin, side, b->bank(b->step + 1), (int32_t)(2 * b->n_obj),
                                      b->x_bc == LBM_X_OPEN, b->forced, b->kcfg.bulk_store_solid != 0,
                                      b->kcfg.bulk_rows == 2 ? 2 : 1, b->stream, fr),
               "batch bulk launch");
    if (s) return s;
    std::swap(b->cur, b->nxt);
    ++b->step;
    ++b->nsum;
    return LBM_OK;
}

lbm_status build_batch_graph(lbm_batch *b)
{
    b->drop_graph();
    if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        b->cap_stream = nullptr;
        return b->fail(LBM_E_DEVICE, "hipStreamCreateWithFlags failed");
    }
    void *start = b->cur;
    const int64_t step0 = b->step, nsum0 = b->nsum;
    hipStream_t user = b->stream;
    b->stream = b->cap_stream;
    hipGraph_t graph = nullptr;
    lbm_status s = b->hip(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    if (s) {
        b->stream = user;
        return s;
    }
    for (int k = 0; k < b->kcfg.graph_steps && !s; ++k) s = enqueue_batch_step(b);
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    b->stream = user;
    b->step = step0;
    b->nsum = nsum0;
    if (b->cur != start) std::swap(b->cur, b->nxt);
    if (s) {
        if (graph) hipGraphDestroy(graph);
        return s;
    }
    if ((s = b->hip(e, "hipStreamEndCapture"))) return s;
    e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if ((s = b->hip(e, "hipGraphInstantiate"))) {
        b->gexec = nullptr;
        return s;
    }
    b->graph_cur = start;
    return LBM_OK;
}

bool inst_ok(lbm_batch *b, int32_t i)
{
    if (!b || i < 0 || i >= b->n) {
        if (b) b->fail(LBM_E_ARG, "instance %d out of range", i);
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_thread_error.c_str(); }

size_t lbm_batch_workspace_bytes(int32_t n, const lbm_params *p, const int64_t *max_links)
{
    std::string why;
    if (!batch_params_ok(n, p, max_links, &why)) return 0;
    lbm_batch b;
    b.n = n;
    b.p.assign(p, p + n);
    b.il.resize(n);
    b.storage = p[0].storage;
    for (int i = 0; i < n; ++i) b.il[i].max_links = max_links[i];
    return layout(&b);
}

lbm_status lbm_batch_create(int32_t n, const lbm_params *p, const int64_t *max_links, void *workspace,
                            size_t bytes, lbm_batch **out)
{
    std::string why;
    if (!out) {
        g_thread_error = "lbm_batch_create: null output pointer";
        return LBM_E_ARG;
    }
    *out = nullptr;
    if (!batch_params_ok(n, p, max_links, &why)) {
        g_thread_error = "lbm_batch_create: " + why;
        return LBM_E_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        g_thread_error = "lbm_batch_create: no HIP device available";
        return LBM_E_DEVICE;
    }
    if (!workspace || ((uintptr_t)workspace & 255)) {
        g_thread_error = "lbm_batch_create: workspace must be non-null and 256-byte aligned";
        return LBM_E_ARG;
    }
    lbm_batch *b = new (std::nothrow) lbm_batch;
    if (!b) {
        g_thread_error = "lbm_batch_create: out of host memory";
        return LBM_E_NOMEM;
    }
    b->n = n;
    b->p.assign(p, p + n);
    b->il.resize(n);
    b->storage = p[0].storage;
    b->x_bc = p[0].x_bc;
    for (int i = 0; i < n; ++i) {
        b->il[i].max_links = max_links[i];
        b->forced |= p[i].gx != 0.0 || p[i].gy != 0.0;
    }
    if (layout(b) > bytes) {
        delete b;
        g_thread_error = "lbm_batch_create: workspace too small";
        return LBM_E_NOMEM;
    }
    b->ws = static_cast<char *>(workspace);
    b->bytes = bytes;
    b->stream = static_cast<hipStream_t>(p[0].stream);
    b->prep.resize(n);
    b->has_geom.assign(n, 0);
    b->has_init.assign(n, 0);
    b->cur = b->ws + b->off_A;
    b->nxt = b->ws + b->off_B;
    if (hipSetDevice(p[0].device) != hipSuccess) {
        delete b;
        g_thread_error = "lbm_batch_create: hipSetDevice failed";
        return LBM_E_DEVICE;
    }
    lbm_status s = b->hip(hipMemsetAsync(b->ws, 0, b->off_mask, b->stream), "batch clear");
    if (!s) s = b->hip(hipMemsetAsync(b->force(), 0, (size_t)b->n_obj * 6 * 8, b->stream), "batch clear");
    if (!s) s = b->hip(hipStreamSynchronize(b->stream), "batch clear");
    if (s) {
        g_thread_error = "lbm_batch_create: " + b->err;
        delete b;
        return s;
    }
    *out = b;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return;
    b->drop_graph();
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

lbm_status lbm_batch_set_geometry(lbm_batch *b, int32_t i, const uint8_t *mask, int64_t n_links,
                                  const int32_t *node, const int8_t *dir, const double *q, const double *uw,
                                  const int32_t *obj, const int8_t *scheme)
{
    if (!inst_ok(b, i)) return LBM_E_ARG;
    std::string why;
    Prepared prep;
    lbm_status s = prepare_geometry(b->p[i], mask, n_links, node, dir, q, uw, obj, scheme, b->il[i].pitch, &prep,
                                    &why);
    if (s) return b->fail(s, "lbm_batch_set_geometry(%d): %s", i, why.c_str());
    if (n_links > b->il[i].max_links)
        return b->fail(LBM_E_NOMEM, "lbm_batch_set_geometry(%d): %lld links exceed the capacity %lld", i,
                       (long long)n_links, (long long)b->il[i].max_links);
    b->drop_graph();
    if ((s = b->hip(hipMemcpyAsync(b->mask(i), prep.mask.data(), prep.mask.size() * sizeof(lbm::mask_t),
                                   hipMemcpyHostToDevice, b->stream), "batch mask upload")))
        return s;
    if ((s = b->hip(hipStreamSynchronize(b->stream), "batch mask upload"))) return s;
    b->prep[i] = std::move(prep);
    b->has_geom[i] = 1;
    b->has_init[i] = 0;
    b->assembled = false;
    return LBM_OK;
}

lbm_status lbm_batch_set_inlet(lbm_batch *b, int32_t i, const double *ux, const double *uy)
{
    if (!inst_ok(b, i)) return LBM_E_ARG;
    const int ny = b->p[i].ny;
    std::vector<double> v((size_t)2 * ny, 0.0);
    for (int y = 0; y < ny; ++y) {
        v[2 * y] = ux ? ux[y] : 0.0;
        v[2 * y + 1] = uy ? uy[y] : 0.0;
        if (!std::isfinite(v[2 * y]) || !std::isfinite(v[2 * y + 1]))
            return b->fail(LBM_E_ARG, "lbm_batch_set_inlet(%d): non-finite velocity in row %d", i, y);
    }
    char *dst = b->ws + b->off_uin + (size_t)b->il[i].uin_off * 2 * b->rb();
    lbm_status s;
    if (b->rb() == 4) {
        std::vector<float> f(v.begin(), v.end());
        s = b->hip(hipMemcpyAsync(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice, b->stream), "inlet upload");
        if (!s) s = b->hip(hipStreamSynchronize(b->stream), "inlet upload");
    } else {
        s = b->hip(hipMemcpyAsync(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice, b->stream), "inlet upload");
        if (!s) s = b->hip(hipStreamSynchronize(b->stream), "inlet upload");
    }
    return s;
}

lbm_status lbm_batch_init_equilibrium(lbm_batch *b, int32_t i, const double *rho, const double *ux,
                                      const double *uy)
{
    if (!inst_ok(b, i)) return LBM_E_ARG;
    if (!b->has_geom[i]) return b->fail(LBM_E_STATE, "lbm_batch_init_equilibrium(%d) before its geometry", i);
    b->drop_graph();
    const int nx = b->p[i].nx, ny = b->p[i].ny;
    const int rows_per = (int)std::max<int64_t>(1, (1 << 20) / nx);
    std::vector<double> h;
    lbm_status s;
    for (int y0 = 0; y0 < ny; y0 += rows_per) {
        const int rows = std::min(rows_per, ny - y0);
        h.assign((size_t)3 * rows * nx, 0.0);
        for (int64_t k = 0; k < (int64_t)rows * nx; ++k) {
            const int64_t nd = (int64_t)y0 * nx + k;
            h[3 * k] = rho ? rho[nd] : b->p[i].rho0;
            h[3 * k + 1] = ux ? ux[nd] : 0.0;
            h[3 * k + 2] = uy ? uy[nd] : 0.0;
            if (!std::isfinite(h[3 * k]) || !std::isfinite(h[3 * k + 1]) || !std::isfinite(h[3 * k + 2]))
                return b->fail(LBM_E_ARG, "lbm_batch_init_equilibrium(%d): non-finite value", i);
        }
        if ((s = b->hip(hipMemcpyAsync(b->stage(), h.data(), h.size() * 8, hipMemcpyHostToDevice, b->stream),
                        "init upload")))
            return s;
        if ((s = b->hip(lbm::launch_init(b->storage, b->grid(i), b->phys(i), b->pops(b->cur, i), b->mask(i),
                                         b->stage(), y0, rows, b->stream), "init kernel")))
            return s;
        if ((s = b->hip(hipStreamSynchronize(b->stream), "init"))) return s;
    }
    b->has_init[i] = 1;
    if (b->assembled &&
        (s = b->hip(lbm::launch_refresh(b->storage, b->grid(i), b->phys(i), b->pops(b->cur, i), b->side_of(i), true,
                                        b->stream), "deposit refresh")))
        return s;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t n)
{
    if (!b) return LBM_E_ARG;
    if (n < 0) return b->fail(LBM_E_ARG, "lbm_batch_step: negative step count");
    lbm_status s;
    for (int i = 0; i < b->n; ++i)
        if (!b->has_geom[i] || !b->has_init[i])
            return b->fail(LBM_E_STATE, "lbm_batch_step: instance %d lacks geometry or initialisation", i);
    if (!b->assembled && (s = assemble(b))) return s;
    while (n > 0) {
        if (n >= b->kcfg.graph_steps) {
            if (!b->gexec || b->graph_cur != b->cur)
                if ((s = build_batch_graph(b))) return s;
            if ((s = b->hip(hipGraphLaunch(b->gexec, b->stream), "hipGraphLaunch"))) return s;
            b->step += b->kcfg.graph_steps;
            b->nsum += b->kcfg.graph_steps;
            n -= b->kcfg.graph_steps;
        } else {
            if ((s = enqueue_batch_step(b))) return s;
            --n;
        }
    }
    return LBM_OK;
}

lbm_status lbm_batch_sync(lbm_batch *b)
{
    if (!b) return LBM_E_ARG;
    return b->hip(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
}

lbm_status lbm_batch_moments(lbm_batch *b, int32_t i, double *rho, double *ux, double *uy)
{
    if (!inst_ok(b, i)) return LBM_E_ARG;
    if (!b->has_geom[i] || !b->has_init[i]) return b->fail(LBM_E_STATE, "lbm_batch_moments(%d) before init", i);
    const int nx = b->p[i].nx, ny = b->p[i].ny;
    const int rows_per = (int)std::max<int64_t>(1, (1 << 20) / nx);
    std::vector<double> h;
    lbm_status s;
    for (int y0 = 0; y0 < ny; y0 += rows_per) {
        const int rows = std::min(rows_per, ny - y0);
        h.resize((size_t)3 * rows * nx);
        if ((s = b->hip(lbm::launch_moments(b->storage, b->grid(i), b->phys(i), b->pops(b->cur, i), b->mask(i),
                                            b->stage(), y0, rows, b->stream), "moments kernel")))
            return s;
        if ((s = b->hip(hipMemcpyAsync(h.data(), b->stage(), h.size() * 8, hipMemcpyDeviceToHost, b->stream),
                        "moments read")))
            return s;
        if ((s = b->hip(hipStreamSynchronize(b->stream), "moments"))) return s;
        for (int64_t k = 0; k < (int64_t)rows * nx; ++k) {
            if (!std::isfinite(h[3 * k]) || !std::isfinite(h[3 * k + 1]) || !std::isfinite(h[3 * k + 2]))
                return b->fail(LBM_E_UNSTABLE, "instance %d: non-finite moment read back", i);
            const int64_t nd = (int64_t)y0 * nx + k;
            if (rho) rho[nd] = h[3 * k];
            if (ux) ux[nd] = h[3 * k + 1];
            if (uy) uy[nd] = h[3 * k + 2];
        }
    }
    return LBM_OK;
}

lbm_status lbm_batch_force(lbm_batch *b, int32_t i, int32_t obj, double last[2], double sum[2], int64_t *nsum)
{
    if (!inst_ok(b, i)) return LBM_E_ARG;
    if (obj < 0 || obj >= b->p[i].n_obj) return b->fail(LBM_E_ARG, "lbm_batch_force: obj %d out of range", obj);
    const int64_t go = b->il[i].obj_off + obj;
    double h[4] = {0, 0, 0, 0};
    lbm_status s;
    if (b->step > 0 &&
        (s = b->hip(hipMemcpyAsync(h, b->bank(b->step - 1) + 2 * go, 16, hipMemcpyDeviceToHost, b->stream),
                    "force read")))
        return s;
    if ((s = b->hip(hipMemcpyAsync(h + 2, b->fsum() + 2 * go, 16, hipMemcpyDeviceToHost, b->stream), "force read")))
        return s;
    if ((s = b->hip(hipStreamSynchronize(b->stream), "force read"))) return s;
    for (double v : h)
        if (!std::isfinite(v)) return b->fail(LBM_E_UNSTABLE, "instance %d: non-finite force", i);
    if (last) last[0] = h[0], last[1] = h[1];
    if (sum) sum[0] = h[2], sum[1] = h[3];
    if (nsum) *nsum = b->nsum;
    return LBM_OK;
}

lbm_status lbm_batch_force_reset(lbm_batch *b)
{
    if (!b) return LBM_E_ARG;
    lbm_status s = b->hip(hipMemsetAsync(b->fsum(), 0, (size_t)b->n_obj * 2 * 8, b->stream), "force reset");
    if (s) return s;
    b->nsum = 0;
    return LBM_OK;
}

int64_t lbm_batch_step_count(const lbm_batch *b) { return b ? b->step : -1; }

lbm_status lbm_batch_get_kernel_config(const lbm_batch *b, lbm_batch_kernel_config *cfg)
{
    if (!b || !cfg) return LBM_E_ARG;
    *cfg = b->kcfg;
    return LBM_OK;
}

lbm_status lbm_batch_set_kernel_config(lbm_batch *b, const lbm_batch_kernel_config *cfg)
{
    if (!b || !cfg) return LBM_E_ARG;
    if ((cfg->bulk_store_solid != 0 && cfg->bulk_store_solid != 1) || cfg->bulk_rows < 0 || cfg->bulk_rows > 2 ||
        cfg->link_block < 64 || cfg->link_block > 1024 || cfg->link_block % 64 || cfg->graph_steps < 2 ||
        cfg->graph_steps > 1024 || cfg->graph_steps % 2)
        return b->fail(LBM_E_ARG, "lbm_batch_set_kernel_config: unsupported configuration");
    b->drop_graph();
    b->kcfg = *cfg;
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *b, int32_t steps_per_trial, lbm_batch_kernel_config *chosen,
                              double *best_ms_per_step)
{
    if (!b || steps_per_trial < 1) return LBM_E_ARG;
    for (int i = 0; i < b->n; ++i)
        if (!b->has_geom[i] || !b->has_init[i])
            return b->fail(LBM_E_STATE, "lbm_batch_autotune: instance %d lacks geometry or initialisation", i);
    lbm_status s;
    if (!b->assembled && (s = assemble(b))) return s;
    // the state the trials start from: populations, deposits, forces and counters
    const size_t pop_bytes = (size_t)b->pop_elems * b->eb();
    const size_t m_bytes = (size_t)b->n_flagged * 3 * b->rb(), p_bytes = (size_t)b->n_pops * b->eb();
    const size_t f_bytes = (size_t)b->n_obj * 6 * sizeof(double);
    std::vector<char> saved;
    try {
        saved.resize(pop_bytes + m_bytes + p_bytes + f_bytes);
    } catch (const std::bad_alloc &) {
        return b->fail(LBM_E_NOMEM, "lbm_batch_autotune: no host memory for the saved state");
    }
    char *h = saved.data();
    const struct {
        size_t host_off;
        char *dev;
        size_t bytes;
    } parts[4] = {{0, static_cast<char *>(b->cur), pop_bytes},
                  {pop_bytes, b->ws + b->off_M, m_bytes},
                  {pop_bytes + m_bytes, b->ws + b->off_P, p_bytes},
                  {pop_bytes + m_bytes + p_bytes, b->ws + b->off_force, f_bytes}};
    for (const auto &pt : parts)
        if (pt.bytes && (s = b->hip(hipMemcpyAsync(h + pt.host_off, pt.dev, pt.bytes, hipMemcpyDeviceToHost,
                                                   b->stream), "autotune save")))
            return s;
    if ((s = b->hip(hipStreamSynchronize(b->stream), "autotune save"))) return s;
    const int64_t step0 = b->step, nsum0 = b->nsum;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return b->fail(LBM_E_DEVICE, "hipEventCreate failed");
    const lbm_batch_kernel_config base = b->kcfg;
    lbm_batch_kernel_config best = base;
    double best_ms = 1e300;
    auto trial = [&](const lbm_batch_kernel_config &k, double *ms) -> lbm_status {
        lbm_status r = lbm_batch_set_kernel_config(b, &k);
        if (r) return r;
        for (int w = 0; w < 2; ++w)
            if ((r = enqueue_batch_step(b))) return r;
        hipEventRecord(e0, b->stream);
        for (int t = 0; t < steps_per_trial; ++t)
            if ((r = enqueue_batch_step(b))) return r;
        hipEventRecord(e1, b->stream);
        if ((r = b->hip(hipEventSynchronize(e1), "autotune"))) return r;
        float f = 0;
        hipEventElapsedTime(&f, e0, e1);
        *ms = f / steps_per_trial;
        return LBM_OK;
    };
    s = LBM_OK;
    for (int ss : {0, 1})
        for (int rows : {1, 2}) {
            if (s) break;
            lbm_batch_kernel_config k = best;
            k.bulk_store_solid = ss;
            k.bulk_rows = rows;
            double ms;
            if ((s = trial(k, &ms))) break;
            if (ms < best_ms) best_ms = ms, best = k;
        }
    for (int lb : {128, 256, 512, 1024}) {
        if (s) break;
        lbm_batch_kernel_config k = best;
        k.link_block = lb;
        double ms;
        if ((s = trial(k, &ms))) break;
        if (ms < best_ms) best_ms = ms, best = k;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    // back to the saved state (whichever buffer is current now)
    lbm_status r = lbm_batch_set_kernel_config(b, s ? &base : &best);
    const char *devs[4] = {static_cast<char *>(b->cur), b->ws + b->off_M, b->ws + b->off_P, b->ws + b->off_force};
    for (int k = 0; k < 4 && !r; ++k)
        if (parts[k].bytes)
            r = b->hip(hipMemcpyAsync(const_cast<char *>(devs[k]), h + parts[k].host_off, parts[k].bytes,
                                      hipMemcpyHostToDevice, b->stream), "autotune restore");
    if (!r) r = b->hip(hipStreamSynchronize(b->stream), "autotune restore");
    b->step = step0;
    b->nsum = nsum0;
    b->drop_graph();
    if (s) return s;
    if (r) return r;
    if (chosen) *chosen = best;
    if (best_ms_per_step) *best_ms_per_step = best_ms;
    return LBM_OK;
}

}  // extern "C"
