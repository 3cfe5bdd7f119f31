// Internal state of a lattice context (struct lbm_ctx of the C ABI) and its
// device workspace layout, shared by the runtime (lbm_runtime.cpp) and the
// adjoint driver (lbm_adjoint.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_host.h"
#include "lbm_internal.h"

namespace lbm_host {

struct Layout {
    int32_t pitch;
    int64_t plane;  // elements per population plane
    size_t off_A, off_B, off_mask, off_seg, off_fmask, off_runs, off_frow, off_nbr, off_nbrr, off_nbrs, off_meta, off_q, off_uw, off_sf, off_sff, off_pf, off_pff,
        off_pfi, off_crec, off_cbase, off_li, off_kof, off_L, off_rec, off_mnode, off_pbase, off_M, off_P, off_M2, off_P2, off_wpart,
        off_wobj, off_uin,
        off_force, off_partials, off_stage, total;
    int64_t wave_cap;  // wavefront partials of the link kernel
};

size_t bytes_per_link(int storage);
Layout make_layout(const lbm_params &p, int64_t max_links);

}  // namespace lbm_host

struct lbm_ctx {
    lbm_params p{};
    lbm_host::Layout lay{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream the step graph is captured on
    std::string err = "no error";
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t max_links = 0, n_links = 0, n_moment_nodes = 0;
    bool has_uw = false, have_geom = false, have_init = false;
    bool has_pfi = false;       // some link needs f+_i(x_f) (Bouzidi, Yu)
    bool has_crec = false;      // compact link records uploaded (4-byte reals)
    bool has_ext_scheme = false;  // some link uses Bouzidi or Yu
    bool li_ident = false;  // links in (node, dir) order: L entry = link index
    // caller's index of each device link (links are kept in (obj, node, dir) order)
    std::vector<int64_t> link_order;
    // flagged slot of the inlet node (0, y) at [y] and of the outlet node
    // (nx-1, y) at [ny + y], or -1 (open lattices only)
    std::vector<int32_t> colslot;
    void *cur = nullptr, *nxt = nullptr;
    int64_t step = 0, nsum = 0;
    lbm_kernel_config kcfg{256, 0, 256, 16, 0, 0, 1, 0};
    int32_t nruns = 0, n_fluid = 0;  // runs of 64 fluid nodes (compact layout)
    bool has_nbr = false;             // neighbour words built (periodic x)
    // deposits (M, P) are double-buffered: dpar selects the pair the links of the
    // next step read; the bulk kernel deposits into the other one
    int dpar = 0;
    // graph of kcfg.graph_steps steps starting from buffer `graph_cur` and deposit
    // parity `graph_dpar`
    hipGraphExec_t gexec = nullptr;
    void *graph_cur = nullptr;
    int graph_dpar = 0;
    // an adjoint call split in two (lbm_adjoint_forward, then lbm_adjoint_backward):
    // what the forward half left in its workspace; any change of the state between
    // the halves (steps, geometry, initialisation, a restored checkpoint) voids it
    struct {
        bool valid = false;
        void *ws = nullptr;
        size_t bytes = 0;
        int64_t nsteps = 0, step_end = 0;
        int32_t k = 0, obj = 0;
        double dir_x = 0, dir_y = 0, J = 0;
    } adj;
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> events;
    size_t ev_used = 0;
    double link_ms = 0, bulk_ms = 0;
    int64_t prof_steps = 0;

    lbm::Grid grid() const
    {
        return lbm::Grid{p.nx, p.ny, lay.pitch, p.x_bc == LBM_X_OPEN ? 1 : 0, lay.plane,
                         p.layout == LBM_LAYOUT_COMPACT ? 1 : 0, 0,
                         reinterpret_cast<const lbm::SegBase *>(ws + lay.off_seg),
                         reinterpret_cast<const uint64_t *>(ws + lay.off_fmask),
                         reinterpret_cast<const lbm::RunBase *>(ws + lay.off_runs),
                         reinterpret_cast<const lbm::SegRow *>(ws + lay.off_frow), nruns, n_fluid,
                         has_nbr ? reinterpret_cast<const uint16_t *>(ws + lay.off_nbr) : nullptr,
                         reinterpret_cast<const lbm::NbrRun *>(ws + lay.off_nbrr),
                         reinterpret_cast<const uint32_t *>(ws + lay.off_nbrs)};
    }
    lbm::Phys phys() const
    {
        const float sc = std::ldexp(1.0f, lbm_host::storage_is_16bit(p.storage) ? p.dev_scale_log2 : 0);
        return lbm::Phys{1.0 / p.tau, p.gx, p.gy, p.rho0, sc, 1.0f / sc, p.s_e, p.s_eps, p.s_q,
                         p.force_form == LBM_FORCE_GALILEAN ? 1 : 0, p.collision};
    }
    lbm::Links links() const
    {
        auto i32 = [&](size_t off) { return reinterpret_cast<const int32_t *>(ws + off); };
        return lbm::Links{reinterpret_cast<const uint32_t *>(ws + lay.off_meta), ws + lay.off_q,
                          has_uw ? ws + lay.off_uw : nullptr, i32(lay.off_sf), i32(lay.off_sff),
                          i32(lay.off_pf), i32(lay.off_pff), i32(lay.off_li), n_links, li_ident ? 1 : 0, 0,
                          li_ident ? nullptr : i32(lay.off_kof), has_pfi ? i32(lay.off_pfi) : nullptr,
                          has_crec ? reinterpret_cast<const lbm::LinkRec *>(ws + lay.off_crec) : nullptr,
                          reinterpret_cast<const lbm::LinkRunBase *>(ws + lay.off_cbase)};
    }
    lbm::Reduce reduce() const
    {
        return lbm::Reduce{reinterpret_cast<double2 *>(ws + lay.off_wpart),
                           reinterpret_cast<int32_t *>(ws + lay.off_wobj)};
    }
    lbm::BulkConfig bulk_config() const
    {
        return lbm::BulkConfig{kcfg.bulk_block_x, kcfg.bulk_store_solid, kcfg.bulk_xcd, kcfg.bulk_fused,
                               kcfg.bulk_rows == 2 ? 2 : 1, kcfg.bulk_runs};
    }
    // deposits read with parity p (and written into the other pair)
    lbm::Side side_par(int p) const
    {
        char *Mr = ws + (p ? lay.off_M2 : lay.off_M), *Pr = ws + (p ? lay.off_P2 : lay.off_P);
        char *Mw = ws + (p ? lay.off_M : lay.off_M2), *Pw = ws + (p ? lay.off_P : lay.off_P2);
        return lbm::Side{Mr, Pr, ws + lay.off_L,
                         reinterpret_cast<const uint16_t *>(ws + lay.off_rec),
                         reinterpret_cast<const lbm::SegBase *>(ws + lay.off_seg),
                         reinterpret_cast<const int32_t *>(ws + lay.off_mnode),
                         reinterpret_cast<const int32_t *>(ws + lay.off_pbase), n_moment_nodes, Mw, Pw};
    }
    // the deposits of the current state
    lbm::Side side() const { return side_par(dpar); }
    lbm::mask_t *mask() const { return reinterpret_cast<lbm::mask_t *>(ws + lay.off_mask); }
    double *force() const { return reinterpret_cast<double *>(ws + lay.off_force); }
    double *bank(int64_t t) const { return force() + (size_t)(t & 1) * 2 * p.n_obj; }
    double *fsum() const { return force() + 4 * (size_t)p.n_obj; }
    double *stage() const { return reinterpret_cast<double *>(ws + lay.off_stage); }
    double *partials() const { return reinterpret_cast<double *>(ws + lay.off_partials); }

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
        if (gexec) hipGraphExecDestroy(gexec);
        gexec = nullptr;
        graph_cur = nullptr;
    }
};

namespace lbm_host {
// One forward step on the context's own buffers (link + bulk launches); with
// timed, HIP events bracket both launches for lbm_kernel_times.
lbm_status enqueue_step(lbm_ctx *c, bool timed);
// The same step from state A into B (any buffers of the context's layout); the
// context's own buffers are left as they are.
lbm_status enqueue_step_to(lbm_ctx *c, const void *A, void *B, bool timed);

// The adjoint call (lbm_adjoint.cpp) over a device workspace: phase selects the
// whole call, its forward half only (checkpoints and J, kept pending in the
// context) or its backward half only (from the pending forward half); with
// no_alloc nothing is allocated on the device or the host.
enum { ADJ_BOTH = 0, ADJ_FORWARD = 1, ADJ_BACKWARD = 2 };
lbm_status adjoint_force_impl(lbm_ctx *c, void *wsv, size_t ws_bytes, int64_t nsteps, int32_t k, int32_t obj,
                              double dir_x, double dir_y, double *J, double *dJ_duin, double *dJ_dq,
                              double *dJ_duw, double *dJ_dstate, double *dJ_dinit, bool no_alloc, int phase);
}  // namespace lbm_host
