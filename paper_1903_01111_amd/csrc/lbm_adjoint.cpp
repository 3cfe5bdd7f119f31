// Host driver of the adjoint form (lbm_adjoint_force in include/lbm.h): forward
// sweep with checkpoints, then segment by segment a recomputation of the states
// from the segment's checkpoint and the reverse sweep through them.  All
// arithmetic runs in the HIP kernels (lbm_kernels.hip, lbm_adjoint.hip).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lbm_ctx.h"

using namespace lbm_host;

namespace {

constexpr int SIG = 12;  // doubles per side record (lbm_adjoint.hip)

// Caller workspace of one adjoint call.
struct AdjLayout {
    size_t state;     // bytes of one state (nine planes)
    int64_t n_ck;     // checkpoints: states 0, k, 2k, ...
    int64_t n_tape;   // recomputed states of a segment besides its checkpoint
    int64_t dplane;   // doubles per plane of the gradient fields
    size_t mbytes;    // bytes of one copy of the side moments
    size_t off_ck, off_ckM, off_tape, off_C0, off_C1, off_lrec, off_sig, off_dq, off_duw, off_duin,
        off_colslot, off_dstate, off_dinit, total;
};

bool adj_layout(const lbm_ctx *c, int64_t nsteps, int32_t k, AdjLayout *L)
{
    if (!c || nsteps < 1 || k < 1) return false;
    const size_t eb = elem_bytes(c->p.storage);
    const size_t nl = (size_t)std::max<int64_t>(c->n_links, 1);
    const size_t K = (size_t)std::max<int64_t>(c->n_moment_nodes, 1);
    L->state = align256(9 * (size_t)c->lay.plane * eb);
    L->n_ck = (nsteps + k - 1) / k;
    L->n_tape = std::min<int64_t>(k, nsteps) - 1;
    L->dplane = (int64_t)c->lay.pitch * c->p.ny;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L->mbytes = align256(K * 3 * real_bytes(c->p.storage));
    L->off_ck = take((size_t)L->n_ck * L->state);
    // side moments of every checkpoint, and of the final state at [n_ck]
    L->off_ckM = take((size_t)(L->n_ck + 1) * L->mbytes);
    L->off_tape = take((size_t)L->n_tape * L->state);
    L->off_C0 = take(L->state);
    L->off_C1 = take(L->state);
    L->off_lrec = take(nl * lbm::adj_link_record_bytes(c->p.storage));
    L->off_sig = take(2 * K * SIG * sizeof(double));  // steps of even / odd parity
    L->off_dq = take(nl * sizeof(double));
    L->off_duw = take(2 * nl * sizeof(double));
    L->off_duin = take(2 * (size_t)c->p.ny * sizeof(double));
    L->off_colslot = take(2 * (size_t)c->p.ny * sizeof(int32_t));
    L->off_dstate = take(9 * (size_t)L->dplane * sizeof(double));
    L->off_dinit = take(3 * (size_t)L->dplane * sizeof(double));
    L->total = o;
    return true;
}

}  // namespace

extern "C" {

size_t lbm_adjoint_workspace_bytes(const lbm_ctx *c, int64_t nsteps, int32_t ckpt_every)
{
    AdjLayout L;
    if (!c || !c->have_geom || (c->p.storage != LBM_F64 && c->p.storage != LBM_F32) ||
        c->p.layout != LBM_LAYOUT_DENSE || c->p.collision != LBM_COLLISION_BGK ||
        c->p.force_form != LBM_FORCE_PLAIN || c->has_ext_scheme)
        return 0;
    if (!adj_layout(c, nsteps, ckpt_every, &L)) return 0;
    return L.total;
}

lbm_status lbm_adjoint_force(lbm_ctx *c, void *wsv, size_t ws_bytes, int64_t nsteps, int32_t k, int32_t obj,
                             double dir_x, double dir_y, double *J, double *dJ_duin, double *dJ_dq,
                             double *dJ_duw, double *dJ_dstate, double *dJ_dinit)
{
    return adjoint_force_impl(c, wsv, ws_bytes, nsteps, k, obj, dir_x, dir_y, J, dJ_duin, dJ_dq, dJ_duw, dJ_dstate,
                              dJ_dinit, false, ADJ_BOTH);
}

lbm_status lbm_adjoint_forward(lbm_ctx *c, void *ws, size_t ws_bytes, int64_t nsteps, int32_t ckpt_every,
                               int32_t obj, double dir_x, double dir_y, double *J)
{
    return adjoint_force_impl(c, ws, ws_bytes, nsteps, ckpt_every, obj, dir_x, dir_y, J, nullptr, nullptr, nullptr,
                              nullptr, nullptr, false, ADJ_FORWARD);
}

lbm_status lbm_adjoint_backward(lbm_ctx *c, void *ws, size_t ws_bytes, double *dJ_duin, double *dJ_dq,
                                double *dJ_duw, double *dJ_dstate, double *dJ_dinit)
{
    if (!c) return LBM_E_ARG;
    if (!c->adj.valid || c->adj.ws != ws || c->adj.bytes != ws_bytes || c->step != c->adj.step_end)
        return c->fail(LBM_E_STATE, "lbm_adjoint_backward without a matching lbm_adjoint_forward on this workspace "
                                    "(or the context changed in between)");
    return adjoint_force_impl(c, ws, ws_bytes, c->adj.nsteps, c->adj.k, c->adj.obj, c->adj.dir_x, c->adj.dir_y,
                              nullptr, dJ_duin, dJ_dq, dJ_duw, dJ_dstate, dJ_dinit, false, ADJ_BACKWARD);
}

}  // extern "C"

// The adjoint call over a device workspace ws.  With no_alloc, nothing is
// allocated on the host or the device: the forward sweep launches the step
// kernels directly instead of through the context's HIP graph (whose
// instantiation allocates), and the results are read back through a fixed stack
// buffer.  Both forms compute bitwise the same results.
lbm_status lbm_host::adjoint_force_impl(lbm_ctx *c, void *wsv, size_t ws_bytes, int64_t nsteps, int32_t k,
                                        int32_t obj, double dir_x, double dir_y, double *J, double *dJ_duin,
                                        double *dJ_dq, double *dJ_duw, double *dJ_dstate, double *dJ_dinit,
                                        bool no_alloc, int phase)
{
    if (!c) return LBM_E_ARG;
    if (phase != ADJ_BACKWARD) c->adj.valid = false;
    if (!c->have_geom || !c->have_init)
        return c->fail(LBM_E_STATE, "lbm_adjoint_force before lbm_set_geometry and initialisation");
    if (c->p.storage != LBM_F64 && c->p.storage != LBM_F32)
        return c->fail(LBM_E_ARG, "lbm_adjoint_force: FP64 or FP32 storage only");
    if (c->p.layout != LBM_LAYOUT_DENSE) return c->fail(LBM_E_ARG, "lbm_adjoint_force: dense layout only");
    if (c->p.collision != LBM_COLLISION_BGK) return c->fail(LBM_E_ARG, "lbm_adjoint_force: BGK collision only");
    if (c->p.force_form != LBM_FORCE_PLAIN)
        return c->fail(LBM_E_ARG, "lbm_adjoint_force: the plain momentum exchange only");
    if (c->has_ext_scheme)
        return c->fail(LBM_E_ARG, "lbm_adjoint_force: VIBB and halfway bounce-back links only");
    if (nsteps < 1 || k < 1) return c->fail(LBM_E_ARG, "lbm_adjoint_force: nsteps and ckpt_every must be >= 1");
    if (obj < 0 || obj >= c->p.n_obj) return c->fail(LBM_E_ARG, "lbm_adjoint_force: obj out of range");
    if (!std::isfinite(dir_x) || !std::isfinite(dir_y))
        return c->fail(LBM_E_ARG, "lbm_adjoint_force: non-finite direction");
    AdjLayout L;
    adj_layout(c, nsteps, k, &L);
    if (!wsv || ((uintptr_t)wsv & 255)) return c->fail(LBM_E_ARG, "lbm_adjoint_force: workspace null or misaligned");
    if (ws_bytes < L.total)
        return c->fail(LBM_E_ARG, "lbm_adjoint_force: workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    char *ws = static_cast<char *>(wsv);
    const hipStream_t st = c->stream;
    const lbm::Grid g = c->grid();
    const lbm::Phys ph = c->phys();
    const int storage = c->p.storage;
    const size_t nl = (size_t)c->n_links;
    lbm_status s;
    auto ck = [&](int64_t j) -> void * { return ws + L.off_ck + (size_t)j * L.state; };
    auto ckM = [&](int64_t j) -> void * { return ws + L.off_ckM + (size_t)j * L.mbytes; };
    const size_t mb = (size_t)c->n_moment_nodes * 3 * real_bytes(storage);
    auto tape = [&](int64_t j) -> void * { return ws + L.off_tape + (size_t)j * L.state; };
    auto state = [&](int64_t t) -> void * { return t % k == 0 ? ck(t / k) : tape(t % k - 1); };
    const int64_t K = std::max<int64_t>(c->n_moment_nodes, 1);
    double *sig = reinterpret_cast<double *>(ws + L.off_sig);
    double *sigp[2] = {sig, sig + K * SIG};  // side records of steps of even / odd parity
    double *dq = reinterpret_cast<double *>(ws + L.off_dq);
    double *duw = reinterpret_cast<double *>(ws + L.off_duw);
    double *duin = reinterpret_cast<double *>(ws + L.off_duin);
    int32_t *colslot = reinterpret_cast<int32_t *>(ws + L.off_colslot);
    void *Cb[2] = {ws + L.off_C0, ws + L.off_C1};

    // forward sweep: checkpoints every k steps (the state and the side moments the
    // next link kernel reads); J from the running force sum
    double Jv = c->adj.J;
    if (phase != ADJ_BACKWARD) {
        double last[2], sum0[2], sum1[2];
        int64_t ns;
        if ((s = lbm_force(c, obj, last, sum0, &ns))) return s;
        for (int64_t j = 0; j < L.n_ck; ++j) {
            if ((s = c->hip(hipMemcpyAsync(ck(j), c->cur, 9 * (size_t)c->lay.plane * elem_bytes(storage),
                                           hipMemcpyDeviceToDevice, st), "checkpoint copy")))
                return s;
            if (mb && (s = c->hip(hipMemcpyAsync(ckM(j), c->side().M, mb, hipMemcpyDeviceToDevice, st),
                                  "checkpoint copy")))
                return s;
            if (j + 1 < L.n_ck) {
                if (no_alloc) {
                    for (int32_t t = 0; t < k; ++t)
                        if ((s = enqueue_step(c, false))) return s;
                } else if ((s = lbm_step(c, k))) {
                    return s;
                }
                continue;
            }
            // the last segment is written straight into the tape: the reverse sweep
            // starts on it without recomputing it
            for (int64_t t = j * k; t < nsteps; ++t) {
                const void *A = t == j * k ? c->cur : state(t);
                void *Bn = t + 1 < nsteps ? state(t + 1) : c->nxt;
                if ((s = enqueue_step_to(c, A, Bn, false))) return s;
            }
            std::swap(c->cur, c->nxt);
        }
        if (mb && (s = c->hip(hipMemcpyAsync(ckM(L.n_ck), c->side().M, mb, hipMemcpyDeviceToDevice, st),
                              "checkpoint copy")))
            return s;
        if ((s = lbm_force(c, obj, last, sum1, &ns))) return s;
        Jv = (dir_x * (sum1[0] - sum0[0]) + dir_y * (sum1[1] - sum0[1])) / (double)nsteps;
    }
    if (phase == ADJ_FORWARD) {
        if (!std::isfinite(Jv)) return c->fail(LBM_E_UNSTABLE, "lbm_adjoint_forward: non-finite objective");
        if (J) *J = Jv;
        c->adj.valid = true;
        c->adj.ws = wsv;
        c->adj.bytes = ws_bytes;
        c->adj.nsteps = nsteps;
        c->adj.step_end = c->step;
        c->adj.k = k;
        c->adj.obj = obj;
        c->adj.dir_x = dir_x;
        c->adj.dir_y = dir_y;
        c->adj.J = Jv;
        return LBM_OK;
    }
    c->adj.valid = false;

    // reverse sweep
    struct Z {
        void *p;
        size_t n;
    } zs[] = {{Cb[0], L.state}, {Cb[1], L.state}, {sig, 2 * (size_t)K * SIG * sizeof(double)},
              {dq, nl * sizeof(double)},
              {duw, 2 * nl * sizeof(double)}, {duin, 2 * (size_t)c->p.ny * sizeof(double)}};
    for (const Z &z : zs)
        if (z.n && (s = c->hip(hipMemsetAsync(z.p, 0, z.n, st), "adjoint clear"))) return s;
    if (!c->colslot.empty() &&
        (s = c->hip(hipMemcpyAsync(colslot, c->colslot.data(), c->colslot.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st), "column slots")))
        return s;
    const lbm::Links links = c->links();
    // the recomputation reads and deposits in the current state's pair (the link
    // kernel of a step reads before the bulk kernel overwrites)
    lbm::Side side = c->side();
    side.Mw = side.M;
    side.Pw = side.P;
    const int32_t *mnode = side.mnode;
    const lbm::SegBase *seg = side.seg;
    if ((s = c->hip(lbm::launch_adj_setup(storage, links, mnode, ws + L.off_lrec, st), "adjoint setup")))
        return s;
    const double djx = dir_x / (double)nsteps, djy = dir_y / (double)nsteps;
    for (int64_t sgm = L.n_ck - 1; sgm >= 0; --sgm) {
        const int64_t t0 = sgm * k, t1 = std::min<int64_t>(t0 + k, nsteps);
        if (t1 - t0 > 1 && sgm + 1 < L.n_ck) {
            // recompute the segment's states from its checkpoint: same kernels, launch
            // shapes and side data as the forward sweep, so bitwise the same states
            if (mb && (s = c->hip(hipMemcpyAsync(side.M, ckM(sgm), mb, hipMemcpyDeviceToDevice, st),
                                  "checkpoint restore")))
                return s;
            if ((s = c->hip(lbm::launch_refresh(storage, g, ph, ck(sgm), side, false, st), "refresh")))
                return s;
            for (int64_t t = t0; t + 1 < t1; ++t) {
                // no force: only the states are wanted
                if ((s = c->hip(lbm::launch_link(storage, g, ph, links, side, c->reduce(), nullptr, nullptr,
                                                 c->kcfg.link_block, st), "link kernel")))
                    return s;
                if ((s = c->hip(lbm::launch_bulk(storage, g, ph, state(t), state(t + 1), c->mask(),
                                                 c->ws + c->lay.off_uin, side, nullptr, 0, c->bulk_config(),
                                                 st), "bulk kernel")))
                    return s;
            }
        }
        for (int64_t t = t1 - 1; t >= t0; --t)
            if ((s = c->hip(lbm::launch_adj_step(storage, g, ph, state(t), Cb[(t + 1) & 1], Cb[t & 1],
                                                 sigp[(t + 1) & 1], sigp[t & 1], ws + L.off_lrec, c->mask(), seg,
                                                 c->colslot.empty() ? nullptr : colslot, c->ws + c->lay.off_uin,
                                                 duin, dq, duw, obj, djx, djy, st), "adjoint step kernel")))
                return s;
    }
    double *dstate = reinterpret_cast<double *>(ws + L.off_dstate);
    double *dinit = reinterpret_cast<double *>(ws + L.off_dinit);
    if ((s = c->hip(lbm::launch_adj_final(storage, g, ph, state(0), Cb[0], sigp[0], c->mask(), seg, dstate, dinit,
                                          L.dplane, st), "adjoint final kernel")))
        return s;
    // the recomputation overwrote the context's deposits: restore them for its
    // current state, so that its next steps are those of an uninterrupted run
    if (mb && (s = c->hip(hipMemcpyAsync(side.M, ckM(L.n_ck), mb, hipMemcpyDeviceToDevice, st),
                          "checkpoint restore")))
        return s;
    if ((s = c->hip(lbm::launch_refresh(storage, g, ph, c->cur, side, false, st), "refresh")))
        return s;

    if ((s = c->hip(hipStreamSynchronize(st), "adjoint"))) return s;
    if (!std::isfinite(Jv)) return c->fail(LBM_E_UNSTABLE, "lbm_adjoint_force: non-finite objective");
    if (J) *J = Jv;
    const int nx = c->p.nx, ny = c->p.ny, pitch = c->lay.pitch;
    if (no_alloc) {
        // every output through a stack buffer, chunk by chunk: dst(j, v) stores
        // element j of the device array
        double buf[2048];
        auto stream_out = [&](const double *src, size_t n, auto &&dst) -> lbm_status {
            for (size_t j0 = 0; j0 < n; j0 += 2048) {
                const size_t m = std::min<size_t>(2048, n - j0);
                lbm_status r = c->hip(hipMemcpyAsync(buf, src + j0, m * sizeof(double), hipMemcpyDeviceToHost, st),
                                      "gradient read-back");
                if (!r) r = c->hip(hipStreamSynchronize(st), "gradient read-back");
                if (r) return r;
                for (size_t j = 0; j < m; ++j) {
                    if (!std::isfinite(buf[j])) return c->fail(LBM_E_UNSTABLE, "lbm_adjoint_force: non-finite gradient");
                    dst(j0 + j, buf[j]);
                }
            }
            return LBM_OK;
        };
        if (dJ_duin && (s = stream_out(duin, 2 * (size_t)ny, [&](size_t j, double v) { dJ_duin[j] = v; })))
            return s;
        if (dJ_dq && (s = stream_out(dq, nl, [&](size_t j, double v) { dJ_dq[c->link_order[j]] = v; }))) return s;
        if (dJ_duw && (s = stream_out(duw, 2 * nl, [&](size_t j, double v) {
                           dJ_duw[2 * c->link_order[j / 2] + (j & 1)] = v;
                       })))
            return s;
        for (int i = 0; i < 9 && dJ_dstate; ++i)
            for (int y = 0; y < ny; ++y)
                if ((s = stream_out(dstate + (size_t)i * L.dplane + (size_t)y * pitch, (size_t)nx,
                                    [&](size_t x, double v) { dJ_dstate[((size_t)y * nx + x) * 9 + i] = v; })))
                    return s;
        for (int i = 0; i < 3 && dJ_dinit; ++i)
            for (int y = 0; y < ny; ++y)
                if ((s = stream_out(dinit + (size_t)i * L.dplane + (size_t)y * pitch, (size_t)nx,
                                    [&](size_t x, double v) { dJ_dinit[((size_t)y * nx + x) * 3 + i] = v; })))
                    return s;
        return LBM_OK;
    }
    // read-back
    std::vector<double> h;
    auto fetch = [&](const void *src, size_t n) -> lbm_status {
        h.resize(n);
        if (n == 0) return LBM_OK;
        lbm_status r = c->hip(hipMemcpyAsync(h.data(), src, n * sizeof(double), hipMemcpyDeviceToHost, st),
                              "gradient read-back");
        if (!r) r = c->hip(hipStreamSynchronize(st), "gradient read-back");
        if (!r)
            for (double v : h)
                if (!std::isfinite(v)) return c->fail(LBM_E_UNSTABLE, "lbm_adjoint_force: non-finite gradient");
        return r;
    };
    if (dJ_duin) {
        if ((s = fetch(duin, 2 * (size_t)c->p.ny))) return s;
        std::copy(h.begin(), h.end(), dJ_duin);
    }
    if (dJ_dq) {
        if ((s = fetch(dq, nl))) return s;
        for (size_t j = 0; j < nl; ++j) dJ_dq[c->link_order[j]] = h[j];
    }
    if (dJ_duw) {
        if ((s = fetch(duw, 2 * nl))) return s;
        for (size_t j = 0; j < nl; ++j) {
            dJ_duw[2 * c->link_order[j]] = h[2 * j];
            dJ_duw[2 * c->link_order[j] + 1] = h[2 * j + 1];
        }
    }
    if (dJ_dstate) {
        for (int i = 0; i < 9; ++i) {
            if ((s = fetch(dstate + (size_t)i * L.dplane, (size_t)L.dplane))) return s;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    dJ_dstate[((size_t)y * nx + x) * 9 + i] = h[(size_t)y * pitch + x];
        }
    }
    if (dJ_dinit) {
        for (int i = 0; i < 3; ++i) {
            if ((s = fetch(dinit + (size_t)i * L.dplane, (size_t)L.dplane))) return s;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    dJ_dinit[((size_t)y * nx + x) * 3 + i] = h[(size_t)y * pitch + x];
        }
    }
    return LBM_OK;
}
