/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 lattice-Boltzmann library with the
 * velocity-interpolation-based bounce-back (VIBB) wall closure of Zhang et al.,
 * arXiv:1903.01111.
 *
 * What one time step computes (the paper's Sections 2 and 3):
 *   1. for every fluid->solid link (x_f, i', q, u_w): the population f_i(x_f, t+1)
 *      that would stream out of the solid, by VIBB (Section 3.1: bounce-back from
 *      the departure point d, whose density, non-equilibrium part and velocity
 *      are interpolated along the link), by halfway bounce-back, or by the
 *      interpolated bounce-back of Bouzidi or of Yu (Section 3) that the paper
 *      compares VIBB with; plus the momentum-exchange force on the solid;
 *   2. pull streaming f_i(x, t+1) = f+_i(x - e_i, t) at every fluid node
 *      (Section 2, the evolution equation);
 *   3. collision (Section 2): BGK, f+ = f - (f - f^eq)/tau, or the paper's MRT
 *      operator f+ = f + M^-1 S (m^eq - m), each with a body force by Guo's
 *      scheme;
 *   4. optional open columns (Section 4.3): a non-equilibrium extrapolation
 *      velocity inlet at x = 0 and a zero-gradient (copy) outlet at x = nx-1.
 *
 * Conventions
 *   - Lattice: nx x ny nodes, node (x, y) at index y*nx + x in every host array.
 *     Periodic in y; periodic in x unless x_bc = LBM_X_OPEN.
 *   - Velocities (the order fixed by the rows j_x, j_y of the paper's MRT matrix):
 *       e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1)
 *       e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1)
 *   - A link is (node, dir): node is a fluid node x_f, dir = i' in 1..8 points
 *     from x_f into the solid node x_s = x_f + e_{i'}; q = |x_f - x_w|/|x_f - x_s|
 *     in (0, 1] (Section 3); u_w is the wall velocity at x_w.
 *   - Every call returns lbm_status (0 = success, < 0 = error); no exception
 *     crosses the ABI.  lbm_last_error() describes the last failure.
 *   - Host arrays passed in are owned by the caller and copied during the call;
 *     no pointer is kept.  Device memory is a workspace the caller allocates
 *     (lbm_workspace_bytes) and keeps alive until lbm_destroy; the library never
 *     frees it.
 *   - Work is enqueued on params.stream (a hipStream_t; NULL = the null stream).
 *     Calls that return host data synchronise that stream.
 *   - One host thread may use a context at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_E_ARG (-1)      /* invalid argument or size */
#define LBM_E_GEOM (-2)     /* invalid geometry or link list */
#define LBM_E_NOMEM (-3)    /* workspace too small, or a host allocation failed */
#define LBM_E_DEVICE (-4)   /* no usable GPU, or a HIP call failed */
#define LBM_E_STATE (-5)    /* call out of order (e.g. step before geometry) */
#define LBM_E_UNSTABLE (-6) /* a non-finite value was read back */

/* storage of the populations in device memory.  All store f_i - w_i (deviation
 * from the rest state).  F64 computes in FP64.  The FP32 and 16-bit forms compute
 * the links and the collision in FP32, except that the collision forms the
 * moments rho, j and the momentum-carrying (odd) parts in FP64 from the exact sums
 * of the FP32 inputs (FP64 vector arithmetic issues at the FP32 rate on gfx950; in
 * FP32 their rounding recurs every step in steady flows and drifts the velocity);
 * F32_PLAIN does the whole collision in FP32 and F32_WIDE the whole collision in
 * FP64.  The 16-bit forms store (f_i - w_i) * 2^dev_scale_log2 rounded to nearest
 * even. */
#define LBM_F64 0
#define LBM_F32 1
#define LBM_F16_DEV 2
#define LBM_BF16_DEV 3
#define LBM_F32_WIDE 4  /* FP32 storage, FP64 collision */
#define LBM_F32_PLAIN 5 /* FP32 storage, every collision operation in FP32 */

/* population layout in device memory */
#define LBM_LAYOUT_DENSE 0   /* every node of the padded lattice, node (x, y) at y*pitch + x */
#define LBM_LAYOUT_COMPACT 1 /* fluid nodes only, numbered in (y, x) order */

#define LBM_X_PERIODIC 0
#define LBM_X_OPEN 1 /* inlet at x = 0, outlet at x = nx-1 */

/* per-link wall closure (Section 3).  A scheme that needs the second fluid node
 * x_ff = x_f - e_{i'} (VIBB, Yu, Bouzidi with q <= 1/2) falls back to halfway
 * bounce-back where x_ff is solid or outside an open lattice. */
#define LBM_SCHEME_VIBB 0    /* velocity-interpolation bounce-back, Section 3.1 */
#define LBM_SCHEME_HBB 1     /* halfway bounce-back (Section 3) */
#define LBM_SCHEME_BOUZIDI 2 /* Bouzidi's linear interpolated bounce-back (Section 3, two branches in q) */
#define LBM_SCHEME_YU 3      /* Yu's unified interpolated bounce-back (Section 3) */

/* collision operator (Section 2) */
#define LBM_COLLISION_BGK 0 /* single relaxation time tau */
#define LBM_COLLISION_MRT 1 /* moments m = M f relaxed at the rates S: s_e, s_eps, s_q as given,
                               s_nu = 1/tau for p_xx and p_xy; rho and j are conserved */

/* momentum-exchange force on the solid (Section 4.3 uses it for the lift) */
#define LBM_FORCE_PLAIN 0    /* sum over links of e_{i'} (f+_{i'}(x_f) + f_i(x_f, t+1)) */
#define LBM_FORCE_GALILEAN 1 /* the Galilean-invariant form (Wen et al., J. Comput. Phys. 266, 2014):
                                momenta relative to the wall, which adds -u_w (f+_{i'} - f_i) per link */

/* obstacle primitives of lbm_geometry; geo = (cx, cy, r) */
#define LBM_PRIM_DISC 0  /* solid where |x - c| <= r */
#define LBM_PRIM_RING 1  /* solid where |x - c| >= r */
#define LBM_PRIM_BELOW 2 /* solid where y <= cy */
#define LBM_PRIM_ABOVE 3 /* solid where y >= cy */

typedef struct {
    int32_t nx, ny;         /* lattice size, >= 1 each; nx >= 3 with LBM_X_OPEN */
    int32_t x_bc;           /* LBM_X_PERIODIC or LBM_X_OPEN */
    int32_t storage;        /* LBM_F64 .. LBM_F32_PLAIN */
    double tau;             /* BGK relaxation time, > 1/2 (tau = 3 nu + 1/2, Section 2) */
    double gx, gy;          /* body acceleration; force density rho*g (Guo forcing) */
    double rho0;            /* reference density of the moving-wall term 6 w rho0 e.u_w */
    int32_t n_obj;          /* number of force accumulators, >= 1 */
    int32_t dev_scale_log2; /* 16-bit storage scale exponent k, |k| <= 30 */
    int32_t device;         /* HIP device ordinal */
    int32_t layout;         /* LBM_LAYOUT_DENSE or LBM_LAYOUT_COMPACT (single lattices) */
    void *stream;           /* hipStream_t the work is enqueued on; NULL = null stream */
    int32_t collision;      /* LBM_COLLISION_BGK (0) or LBM_COLLISION_MRT */
    int32_t force_form;     /* LBM_FORCE_PLAIN (0) or LBM_FORCE_GALILEAN */
    double s_e, s_eps, s_q; /* MRT rates of the moments e, epsilon and q_x, q_y, each in (0, 2)
                               (Section 2 prints 1.5, 1.5, 1.2); read only with LBM_COLLISION_MRT */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Message for the last failure on ctx, or of the calling thread when ctx is NULL
 * (e.g. a failed lbm_create).  Never NULL; valid until the next call. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Geometry (host only; no GPU needed).
 * ------------------------------------------------------------------------- */

/* Solid mask and fluid->solid links of a union of primitives (Section 3: node
 * classification and q).  A node is solid when any primitive holds it (a node on
 * a circle is solid; periodic directions use minimum-image offsets).  For each
 * fluid node that is streamed (not an open column) and each direction i' whose
 * neighbour x_f + e_{i'} is solid, one link is emitted; q is the fraction of the
 * link to the first crossing of a primitive that holds that neighbour, u_w the
 * rigid velocity (ux, uy) + omega x (x_w - c) of that primitive at
 * x_w = x_f + q e_{i'}, obj its obj id.
 *   kind[n_prim], geo[3*n_prim] = (cx, cy, r), motion[3*n_prim] = (ux, uy, omega),
 *   prim_obj[n_prim];  mask_out[ny*nx] (1 = solid);  links ordered by node, then dir.
 * The link arrays (node, dir, q, uw[2*k], obj) are written only if the count does
 * not exceed max_links; *n_links_out always receives the count (call once with
 * max_links = 0 to size them).  Errors: LBM_E_ARG. */
lbm_status lbm_geometry(int32_t nx, int32_t ny, int32_t x_bc, int32_t n_prim, const int32_t *kind,
                        const double *geo, const double *motion, const int32_t *prim_obj,
                        uint8_t *mask_out, int64_t max_links, int32_t *node, int8_t *dir,
                        double *q, double *uw, int32_t *obj, int64_t *n_links_out);

/* lbm_geometry plus, per link (either may be NULL): prim[k], the primitive that
 * sets its q, and dq[3k..3k+2] = dq/d(cx, cy, r) of that primitive with the node
 * classification held fixed (circles: from |x_f + q e - c| = r, so with
 * p = x_w - c, dq/dc = p/(p.e) and dq/dr = r/(p.e); lines: dq/dcy = 1/e_y). */
lbm_status lbm_geometry_ex(int32_t nx, int32_t ny, int32_t x_bc, int32_t n_prim, const int32_t *kind,
                           const double *geo, const double *motion, const int32_t *prim_obj,
                           uint8_t *mask_out, int64_t max_links, int32_t *node, int8_t *dir,
                           double *q, double *uw, int32_t *obj, int32_t *prim, double *dq,
                           int64_t *n_links_out);

/* Validates a mask and link list against params without touching a device:
 * sizes, q in (0,1], every link from a streamed fluid node into a solid node,
 * no duplicate (node, dir), every pull from a solid node covered by a link, obj
 * in [0, n_obj), scheme in LBM_SCHEME_VIBB .. LBM_SCHEME_YU, open columns backed
 * by a fluid neighbour column.  uw, obj and scheme may be NULL (0, 0, VIBB).
 * *n_fallback (may be NULL) receives the number of links whose scheme needs the
 * second node x_ff = x_f - e_{i'} where it is solid or off an open edge: they fall
 * back to halfway bounce-back.  Errors: LBM_E_ARG, LBM_E_GEOM (message names the
 * index). */
lbm_status lbm_check_geometry(const lbm_params *p, const uint8_t *mask, int64_t n_links,
                              const int32_t *node, const int8_t *dir, const double *q,
                              const double *uw, const int32_t *obj, const int8_t *scheme,
                              int64_t *n_fallback);

/* ---------------------------------------------------------------------------
 * Lattice context.
 * ------------------------------------------------------------------------- */

/* Most links one lattice (or one batch, summed over its instances) can hold: the
 * bulk kernel addresses the link values with 32-bit byte offsets. */
#define LBM_MAX_LINKS ((int64_t)1 << 28)

/* Device bytes the context needs for params and up to max_links links, or 0 if
 * params are invalid or max_links is outside [0, LBM_MAX_LINKS]. */
size_t lbm_workspace_bytes(const lbm_params *p, int64_t max_links);

/* Creates a context over a device workspace of at least
 * lbm_workspace_bytes(p, max_links) bytes (256-byte aligned; the caller owns it).
 * max_links is read from the workspace size (at most LBM_MAX_LINKS).  Launches nothing.
 * Errors: LBM_E_ARG, LBM_E_NOMEM, LBM_E_DEVICE (no GPU). */
lbm_status lbm_create(const lbm_params *p, void *workspace, size_t bytes, lbm_ctx **out);

void lbm_destroy(lbm_ctx *ctx); /* frees host-side state only */

/* The parameters the context was created with (e.g. to size the arrays of
 * lbm_moments_device).  Errors: LBM_E_ARG (null pointer). */
lbm_status lbm_get_params(const lbm_ctx *ctx, lbm_params *out);

/* Uploads the geometry (validated as lbm_check_geometry; nothing on the device
 * changes if it fails), resets the force accumulators and the step counter.
 * The populations must then be initialised.  Errors: LBM_E_GEOM, LBM_E_NOMEM
 * (more links than the workspace holds), LBM_E_DEVICE. */
lbm_status lbm_set_geometry(lbm_ctx *ctx, const uint8_t *mask, int64_t n_links,
                            const int32_t *node, const int8_t *dir, const double *q,
                            const double *uw, const int32_t *obj, const int8_t *scheme);

/* Inlet velocity per row (ny values each; NULL = 0) for LBM_X_OPEN.  Default 0. */
lbm_status lbm_set_inlet(lbm_ctx *ctx, const double *ux, const double *uy);

/* Post-collision populations f+ = f^eq(rho, u) at every fluid node (Section 2,
 * equilibrium), from host fields of ny*nx values (NULL: rho0, 0, 0).
 * Errors: LBM_E_STATE before lbm_set_geometry. */
lbm_status lbm_init_equilibrium(lbm_ctx *ctx, const double *rho, const double *ux,
                                const double *uy);

/* Enqueues n >= 0 time steps; returns without waiting.  One step is the
 * evolution equation of Section 2, f_i(x + e_i, t+1) = f_i(x, t) + Omega, with the
 * collision of params.collision and the boundary values of Section 3 for the
 * populations that would stream out of the solid (see the top of this file).
 * Errors: LBM_E_STATE. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* Waits for the context's stream. */
lbm_status lbm_sync(lbm_ctx *ctx);

int64_t lbm_step_count(const lbm_ctx *ctx); /* steps since geometry / set_state */

/* Density and physical velocity u = (sum f+ e)/rho - g/2 (Section 2 moments with
 * Guo's half-force shift) at every node into host arrays of ny*nx doubles (may be
 * NULL); solid nodes read 0.  Synchronises.  Errors: LBM_E_STATE, LBM_E_UNSTABLE
 * (non-finite value found). */
lbm_status lbm_moments(lbm_ctx *ctx, double *rho, double *ux, double *uy);

/* The same moments into device arrays of ny*nx values each, index y*nx + x (FP64
 * when fp64 is nonzero, else rounded to FP32; any may be NULL), enqueued on the
 * context's stream without waiting.  The arrays are the caller's (e.g. torch
 * tensors on the context's device) and must hold ny*nx values and stay valid until
 * the stream has run the kernel.  FP64 values equal those of lbm_moments bitwise.
 * No finiteness check (lbm_moments does one).  Errors: LBM_E_STATE before
 * initialisation, LBM_E_DEVICE. */
lbm_status lbm_moments_device(lbm_ctx *ctx, void *rho, void *ux, void *uy, int32_t fp64);

/* Raw post-collision populations f+_i (including w_i) into a host array of
 * 9*ny*nx doubles, node-major: f[(y*nx + x)*9 + i]; solid nodes read 0. */
lbm_status lbm_populations(lbm_ctx *ctx, double *f);

/* Force of the fluid on object obj by momentum exchange over its links (the
 * force whose y component gives the lift coefficient of Section 4.3; the paper
 * does not name the method, params.force_form selects the plain or the
 * Galilean-invariant form): last = the latest step, sum = accumulated since
 * geometry / lbm_force_reset over *nsum steps (any output may be NULL).
 * Accumulated in FP64 on the device.  Synchronises.
 * Errors: LBM_E_ARG (obj range), LBM_E_UNSTABLE (non-finite). */
lbm_status lbm_force(lbm_ctx *ctx, int32_t obj, double last[2], double sum[2], int64_t *nsum);
lbm_status lbm_force_reset(lbm_ctx *ctx);

/* Total mass: the zeroth moment rho = sum_i f_i of Section 2 summed over the
 * fluid nodes (post-collision populations), reduced in FP64.  Synchronises.
 * Errors: LBM_E_STATE, LBM_E_UNSTABLE (non-finite). */
lbm_status lbm_mass(lbm_ctx *ctx, double *mass);

/* max over fluid nodes and directions of |f+_i - w_i|, in FP64: sizes the scale
 * 2^k of 16-bit deviation storage (largest k with 2^k * max <= 2^14 leaves a 4x
 * margin below the FP16 maximum).  Synchronises. */
lbm_status lbm_max_deviation(lbm_ctx *ctx, double *max_dev);

/* Checkpoint: the population buffer in storage precision, the step counter, the
 * force accumulators and the stored moments of the boundary-adjacent nodes, so
 * that a restored run continues bitwise.  lbm_state_bytes gives the size of the
 * host buffer; a state only fits a context with the same params and geometry. */
size_t lbm_state_bytes(const lbm_ctx *ctx);
/* Checkpoint format: int64 step, int64 steps in the force sum; then plane i = 0..8
 * of plane_elems elements of elem bytes each (storage format: (f_i - w_i)
 * [* 2^k]; dense layout: node (x, y) at y*pitch + x; compact layout: the k-th
 * fluid node in (y, x) order at k); then 6*n_obj doubles of force
 * accumulators; then the stored moments of the boundary-adjacent nodes. */
lbm_status lbm_state_layout(const lbm_ctx *ctx, int32_t *pitch, int64_t *plane_elems, int32_t *elem);
lbm_status lbm_get_state(lbm_ctx *ctx, void *host, size_t bytes);
lbm_status lbm_set_state(lbm_ctx *ctx, const void *host, size_t bytes);

/* Kernel timing: while on, lbm_step brackets every link and bulk launch with HIP
 * events on the context's stream (no graph replay).  lbm_kernel_times
 * synchronises and returns the summed durations in ms and the number of steps
 * timed since profiling was switched on. */
lbm_status lbm_set_profiling(lbm_ctx *ctx, int32_t on);
lbm_status lbm_kernel_times(lbm_ctx *ctx, double *link_ms, double *bulk_ms, int64_t *n_steps);

/* Launch configuration of the step kernels.  Every configuration computes the same
 * result; they differ in speed only. */
typedef struct {
    int32_t bulk_block_x;     /* bulk kernel: 64, 128 or 256 lanes along x per 256-lane block */
    int32_t bulk_store_solid; /* 1: lanes of solid nodes store too, so rows are written in full lines */
    int32_t link_block;       /* link kernel lanes per block: 64..1024, a multiple of 64 */
    int32_t graph_steps;      /* steps per captured HIP graph: even, 2..1024 */
    int32_t bulk_xcd;         /* 1: each XCD takes a contiguous run of the bulk blocks (workgroups
                                 go to the 8 XCDs round robin), so neighbouring rows and shared
                                 cache lines stay in one L2; 0: hardware order */
    int32_t bulk_fused;       /* 1: the bulk kernel evaluates the links of its own nodes (one
                                 launch per step plus the force reduction); needs bulk_block_x
                                 256, and BGK unless bulk_runs; 0: a separate link kernel */
    int32_t bulk_rows;        /* row segments per bulk wavefront: 2 issues the second one's loads
                                 before the first is finished (needs bulk_block_x 256 and
                                 bulk_fused 0); 1 (or 0): one */
    int32_t bulk_runs;        /* 1: each bulk wavefront takes a run of 64 consecutive fluid nodes
                                 instead of a 64-node row segment, so every lane holds a node and
                                 the planes are written in whole cache lines (compact layout,
                                 periodic in x; bulk_block_x, bulk_store_solid and bulk_rows do not
                                 apply; with bulk_fused the run evaluates its own links, BGK or
                                 MRT); 2: runs whose lanes read their pull offsets from a
                                 per-node neighbour word built with the geometry (2 bytes per
                                 fluid node, 16 per run of 64) instead of walking the row
                                 segments, refused with LBM_E_ARG before a geometry is set or
                                 when the nodes the words cannot hold (first and last row and
                                 column, runs whose rank differences spread over more than
                                 126) exceed the offset table's room, 2 pitch + 2 ny + 1024
                                 nodes (a later geometry without the words turns 2 into 1);
                                 0: row segments */
} lbm_kernel_config;

lbm_status lbm_get_kernel_config(const lbm_ctx *ctx, lbm_kernel_config *cfg);
/* Errors: LBM_E_ARG for an unsupported configuration (the previous one stays). */
lbm_status lbm_set_kernel_config(lbm_ctx *ctx, const lbm_kernel_config *cfg);

/* Autotuner: times every bulk shape (block, solid stores, XCD order, rows per wavefront, runs of fluid nodes, fused links) and link block size for steps_per_trial steps
 * on the current state, keeps the fastest, and restores the state (populations,
 * step counter, forces), so results do not depend on having tuned.  Needs host
 * memory for one checkpoint.  chosen and best_ms_per_step may be NULL.
 * With the environment variable VIBB_TUNE_CACHE naming a file, a stored choice for
 * the lattice's key (device architecture, size, boundary, storage, layout,
 * collision, body force, link and fluid counts) is applied without trials, and a
 * new choice is appended as one JSON line {"key", "config" (the eight fields of
 * lbm_kernel_config in order), "ms"}; an unreadable or unwritable file only costs
 * the trials. */
lbm_status lbm_autotune(lbm_ctx *ctx, int32_t steps_per_trial, lbm_kernel_config *chosen,
                        double *best_ms_per_step);

/* ---------------------------------------------------------------------------
 * Batched form: n lattices of uneven size (e.g. the same flow at different
 * obstacle offsets or Reynolds numbers) advanced together.  Each step is one
 * link launch over the links of all instances and one bulk launch over a tile
 * table of all instances (HIP graph replay).  Instances share storage, x_bc,
 * rho0, dev_scale_log2, device, stream, collision, force_form and the MRT rates
 * s_e, s_eps, s_q, and use the dense layout; nx, ny,
 * tau, body force, n_obj and geometry are per instance.  The results of an instance equal those of a
 * single-lattice context with the same arguments (bitwise for the populations).
 * ------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

const char *lbm_batch_last_error(const lbm_batch *b); /* NULL b: the thread's message */

/* Device bytes for n instances with params p[n] and link capacities max_links[n];
 * 0 if the params are invalid or do not share the common fields. */
size_t lbm_batch_workspace_bytes(int32_t n, const lbm_params *p, const int64_t *max_links);

lbm_status lbm_batch_create(int32_t n, const lbm_params *p, const int64_t *max_links, void *workspace,
                            size_t bytes, lbm_batch **out);
void lbm_batch_destroy(lbm_batch *b);

/* Per-instance counterparts of lbm_set_geometry, lbm_set_inlet and
 * lbm_init_equilibrium (same arguments and errors; inst in [0, n)). */
lbm_status lbm_batch_set_geometry(lbm_batch *b, int32_t inst, const uint8_t *mask, int64_t n_links,
                                  const int32_t *node, const int8_t *dir, const double *q, const double *uw,
                                  const int32_t *obj, const int8_t *scheme);
lbm_status lbm_batch_set_inlet(lbm_batch *b, int32_t inst, const double *ux, const double *uy);
lbm_status lbm_batch_init_equilibrium(lbm_batch *b, int32_t inst, const double *rho, const double *ux,
                                      const double *uy);

/* n steps of every instance.  Errors: LBM_E_STATE if an instance lacks geometry
 * or initialisation. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t n);
lbm_status lbm_batch_sync(lbm_batch *b);
int64_t lbm_batch_step_count(const lbm_batch *b);

/* Launch configuration of the batched step.  Every configuration computes the same
 * result; they differ in speed only. */
typedef struct {
    int32_t bulk_store_solid; /* 1: lanes of solid nodes store too (rows written in full lines) */
    int32_t bulk_rows;        /* tile-table entries per bulk wavefront: 2 issues the second one's
                                 loads before the first is finished; 1 (or 0): one */
    int32_t link_block;       /* link kernel lanes per block: 64..1024, a multiple of 64 */
    int32_t graph_steps;      /* steps per captured HIP graph: even, 2..1024 */
} lbm_batch_kernel_config;

lbm_status lbm_batch_get_kernel_config(const lbm_batch *b, lbm_batch_kernel_config *cfg);
/* Errors: LBM_E_ARG for an unsupported configuration (the previous one stays). */
lbm_status lbm_batch_set_kernel_config(lbm_batch *b, const lbm_batch_kernel_config *cfg);

/* Autotuner of the batched step: times every configuration (solid stores, rows per
 * wavefront, link block size) for steps_per_trial steps on the current state, keeps
 * the fastest and restores the state (populations, deposits, step count, forces),
 * so results do not depend on having tuned.  Needs host memory for one copy of the
 * populations and deposits.  Errors: LBM_E_STATE before every instance has geometry
 * and initialisation.  chosen and best_ms_per_step may be NULL. */
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t steps_per_trial, lbm_batch_kernel_config *chosen,
                              double *best_ms_per_step);

/* Per-instance read-back, as lbm_moments and lbm_force. */
lbm_status lbm_batch_moments(lbm_batch *b, int32_t inst, double *rho, double *ux, double *uy);
lbm_status lbm_batch_force(lbm_batch *b, int32_t inst, int32_t obj, double last[2], double sum[2],
                           int64_t *nsum);
lbm_status lbm_batch_force_reset(lbm_batch *b);

/* ---------------------------------------------------------------------------
 * Adjoint form: gradients of a time-averaged force by the discrete adjoint of
 * the step (the reverse of the link update of Section 3.1, of the pull streaming
 * and BGK/Guo collision of Section 2 and of the open columns of Section 4.3).
 *
 * Objective, for the nsteps steps that follow the context's current state S_0:
 *     J = (1/nsteps) sum_{t=0}^{nsteps-1} (d_x F_x(t) + d_y F_y(t)),
 * F(t) the momentum-exchange force on object obj during step t (what lbm_force
 * accumulates) and d = (dir_x, dir_y) (d = (1, 0): the mean drag).
 *
 * Method: a forward sweep of nsteps steps keeps the state every ckpt_every steps;
 * the reverse sweep recomputes each segment of ckpt_every steps from its
 * checkpoint and runs the adjoint step backwards through it.  The gradients are
 * derivatives of the discrete map with the node classification held fixed; at
 * q = 1/2 the VIBB velocity branch of the forward (q <= 1/2) is differentiated.
 * Adjoint arithmetic is in the storage's precision; gradients with respect to the
 * parameters are accumulated in FP64.  FP64 and FP32 storage, dense layout, BGK
 * collision, the plain force and VIBB / halfway bounce-back links only.
 *
 * lbm_adjoint_workspace_bytes: device bytes the call needs for this context
 * (checkpoints, the recomputed segment, adjoint fields); 0 on invalid arguments.
 *
 * lbm_adjoint_force: ws is a caller-owned device buffer, 256-byte aligned, of at
 * least lbm_adjoint_workspace_bytes; nothing is retained after the call.  On
 * return the context has advanced by nsteps exactly as lbm_step(nsteps) advances
 * it (state, step count, force accumulators).  Outputs (host, each may be NULL):
 *   J           the objective;
 *   dJ_duin     [2*ny]   dJ/d(u_in,x, u_in,y) of every inlet row (open lattices);
 *   dJ_dq       [n_links] dJ/dq of every link, in the order given to lbm_set_geometry;
 *   dJ_duw      [2*n_links] dJ/du_w of every link, same order;
 *   dJ_dstate   [nx*ny*9] dJ/df+_i(x, 0) of the initial post-collision state,
 *               node-major (index (y*nx + x)*9 + i), zero at solid nodes;
 *   dJ_dinit    [nx*ny*3] dJ/d(rho, ux, uy) of the initial fields, reading the
 *               initial state as f+ = f^eq(rho, u) of its own (rho, u) (the state
 *               lbm_init_equilibrium writes), node-major, zero at solid nodes.
 * Errors: LBM_E_ARG (nsteps < 1, ckpt_every < 1, obj out of range, 16-bit
 * storage, compact layout, MRT, Galilean-invariant force, Bouzidi or Yu links,
 * workspace null, misaligned or too small), LBM_E_STATE (no geometry or
 * initialisation), LBM_E_DEVICE, LBM_E_UNSTABLE (non-finite objective or
 * gradient). */
size_t lbm_adjoint_workspace_bytes(const lbm_ctx *ctx, int64_t nsteps, int32_t ckpt_every);
lbm_status lbm_adjoint_force(lbm_ctx *ctx, void *ws, size_t ws_bytes, int64_t nsteps,
                             int32_t ckpt_every, int32_t obj, double dir_x, double dir_y, double *J,
                             double *dJ_duin, double *dJ_dq, double *dJ_duw, double *dJ_dstate,
                             double *dJ_dinit);

/* lbm_adjoint_force in two halves, for callers that need J before they know
 * whether the gradient is wanted (a torch.autograd.Function: forward, then
 * backward): lbm_adjoint_forward runs the forward sweep (the context advances by
 * nsteps, checkpoints go into ws) and returns J; lbm_adjoint_backward, on the same
 * workspace, runs the recomputation and the reverse sweep and returns the
 * gradients (outputs as lbm_adjoint_force; any may be NULL).  The workspace must
 * be left as it is between the two calls; stepping the context, a new geometry,
 * initialisation or a restored checkpoint in between void the forward half
 * (lbm_adjoint_backward then returns LBM_E_STATE).  The two halves compute what
 * lbm_adjoint_force computes. */
lbm_status lbm_adjoint_forward(lbm_ctx *ctx, void *ws, size_t ws_bytes, int64_t nsteps, int32_t ckpt_every,
                               int32_t obj, double dir_x, double dir_y, double *J);
lbm_status lbm_adjoint_backward(lbm_ctx *ctx, void *ws, size_t ws_bytes, double *dJ_duin, double *dJ_dq,
                                double *dJ_duw, double *dJ_dstate, double *dJ_dinit);

/* For callers that cannot allocate memory (code that must not call hipMalloc,
 * tight loops, harnesses that forbid allocation): lbm_adjoint_force with the same
 * arguments, results and errors, but its workspace is a static device array of
 * LBM_ADJOINT_SCRATCH_BYTES per GPU that the library holds until the process ends;
 * it allocates nothing, on the device or the host.  A call that needs more
 * (lbm_adjoint_workspace_bytes above the limit) returns LBM_E_NOMEM.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU race (one call
 * per GPU at a time).  Synchronises the context's stream. */
#define LBM_ADJOINT_SCRATCH_BYTES ((size_t)64 << 20)
lbm_status lbm_adjoint_force_noalloc(lbm_ctx *ctx, int64_t nsteps, int32_t ckpt_every, int32_t obj,
                                     double dir_x, double dir_y, double *J, double *dJ_duin, double *dJ_dq,
                                     double *dJ_duw, double *dJ_dstate, double *dJ_dinit);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
