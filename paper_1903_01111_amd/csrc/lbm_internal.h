// Internal interface between the host runtime (lbm_runtime.cpp) and the HIP
// kernels (lbm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

// Device population layout: nine planes of `plane` elements, plane i holding
// f_i - w_i of node (x, y) at offset y*pitch + x.  pitch >= nx is a multiple of
// 64 elements, so a 64-lane wavefront reads one aligned run of a row.
struct SegBase;
struct RunBase;
struct SegRow;
struct NbrRun;

// With compact set, plane i holds only the fluid nodes, the k-th fluid node in
// (y, x) order at offset k: a node's offset is the fluid count before its
// 64-node row segment (fseg[s].fluid) plus the fluid nodes below it in the
// segment (popcount of the segment's fluid bitmask fmask[s]).
struct Grid {
    int32_t nx, ny, pitch, x_open;
    int64_t plane;
    int32_t compact, pad;
    const SegBase *fseg;    // [ny * pitch / 64] (compact layout)
    const uint64_t *fmask;  // [ny * pitch / 64] (compact layout)
    const RunBase *runs;    // [nruns + 1] (compact layout): see RunBase
    const SegRow *frow;     // [ny * pitch / 64 + 1] (compact layout): fmask and fseg.fluid in one record
    int32_t nruns;          // runs of 64 fluid nodes: ceil(n_fluid / 64)
    int32_t n_fluid;
    // per fluid node (compact layout, periodic x): the fluid ranks of (x, y-1) and
    // (x, y+1) relative to the node's own, minus its run's bases (nbr_run), in bits
    // 0-6 and 8-14, whether those nodes are fluid in bits 7 and 15; 0xffff: the
    // node's nine pull offsets (elements) are the next entry of nbr_slow after the
    // run's base and the run's earlier such nodes
    const uint16_t *nbr;
    const NbrRun *nbr_run;  // [nruns + 1]
    const uint32_t *nbr_slow;
};

struct Phys {
    double omega;     // 1/tau (BGK rate; MRT rate of p_xx and p_xy)
    double gx, gy;    // body acceleration
    double rho0;      // reference density of the moving-wall term
    float scale;      // 2^k for 16-bit storage (1 otherwise)
    float inv_scale;  // 2^-k
    double s_e, s_eps, s_q;  // MRT rates of e, epsilon and q_x, q_y
    int32_t gi_force;        // Galilean-invariant momentum exchange
    int32_t coll;            // LBM_COLLISION_BGK or LBM_COLLISION_MRT
};

// Per-node mask word: bits 0..7 the directions d (bit d-1) of the node's links
// (the pulls of directions opp(d) come from link values), bit 8 solid, bit 9
// "side record" -- the node is x_f of a link or x_ff of a VIBB link.  Flagged
// nodes are numbered (slot) in plane order: the slot of a node is
// seg[y*pitch/64 + x/64].flagged (flagged nodes before its 64-node row segment)
// plus the flagged lanes below it in its wavefront.
using mask_t = uint16_t;
constexpr mask_t MASK_LINKS = 0xff, MASK_SOLID = 0x100, MASK_SIDE = 0x200;

// Per 64-node row segment: flagged nodes, links and deposited populations that
// come before it in plane order.
struct SegBase {
    int32_t flagged, links, pops, fluid;
};

// Run w of the compact layout is the fluid nodes 64w .. 64w+63 in plane order.
// Counts before its first node: flagged nodes (side records), links in (node, dir)
// order and deposited populations; seg is the row segment of its first node; bit j
// of (flag_hi, flag_lo) is set when node 64w + j is flagged (has a side record);
// nlinks is the number of links of the run's nodes.  Entry nruns holds the totals.
// A row segment's fluid bitmask and the fluid count before it, in one 16-byte
// record (one scalar load); entry ny * pitch / 64 holds the total fluid count.
struct SegRow {
    uint32_t fm_lo, fm_hi;
    int32_t fluid, pad;
};

// Per run of 64 fluid nodes: the bases of its nodes' neighbour words and the
// offset-table entries that precede it.
struct NbrRun {
    int32_t dm0, dp0, slow, pad;
};

struct RunBase {
    int32_t flagged, links, pops, seg;
    uint32_t flag_lo, flag_hi, nlinks, pad;
};

// Data exchanged between the bulk kernel and the link kernel through compact
// arrays, so that neither touches the population planes at random:
//  - after collision the bulk kernel deposits, for every flagged node, its
//    moments (rho - 1, ux, uy) into M and the post-collision populations the
//    links will need (rec bits 8..15) into P;
//  - the link kernel reads M and P and writes the value of every link into L,
//    in (node, dir) order;
//  - the next bulk kernel pulls direction i of a node from L instead of from the
//    solid neighbour x - e_i (rec bits 0..7 mark the node's link directions).
//  M and P are what the links read this step; the bulk kernel deposits into Mw
//  and Pw (the same arrays, or the other of a double-buffered pair when the bulk
//  kernel evaluates the links of its own nodes).
struct Side {
    void *M;                 // real[3K]
    void *P;                 // storage[NP]
    void *L;                 // storage[n_links]
    const uint16_t *rec;     // [K] bit d-1: link in direction d; bit d+7: population d deposited
    const SegBase *seg;      // [ny * pitch / 64]
    const int32_t *mnode;    // [K] plane offset of each flagged node
    const int32_t *pbase;    // [K] first P entry of each flagged node
    int64_t K;
    void *Mw;                // deposits of this step: real[3K]
    void *Pw;                // storage[NP]
};

// Links in (obj, node, dir) order, so a wavefront usually serves one object.
// The scheme in bits 4..7 of meta is the one evaluated: LBM_SCHEME_HBB also for a
// link whose scheme needs x_ff where x_ff is unusable (then sff = -1).
// Compact link record (storages with 4-byte reals): the direction word, q's bits,
// and the M slots and P entries of x_f and x_ff as 16-bit excesses over the bases
// of the link's run of 64 links (d_f: slot | entry << 16; d_ff likewise, slot
// 0xffff: no x_ff).  A run whose excesses do not fit 16 bits has sf0 = -1 and its
// links are read from the separate arrays.
struct LinkRec {
    uint32_t meta, q, d_f, d_ff;
};
struct LinkRunBase {
    int32_t sf0, pf0, sff0, pff0;
};

struct Links {
    const uint32_t *meta;  // dir | (scheme << 4) | (obj << 8)
    const void *q;         // real[n]
    const void *uw;        // real[2n] or nullptr (still walls)
    const int32_t *sf;     // moment slot of x_f
    const int32_t *sff;    // moment slot of x_ff, or -1: halfway bounce-back
    const int32_t *pf;     // P entry of f+_{i'}(x_f)
    const int32_t *pff;    // P entry of f+_{i'}(x_ff) (VIBB links)
    const int32_t *li;     // rank of the link in (node, dir) order: its L entry
    int64_t n;
    int32_t li_ident;      // 1: li[l] == l for every link (one object), li is not read
    int32_t pad;
    const int32_t *kof;    // inverse of li (null when li_ident)
    const int32_t *pfi;    // P entry of f+_i(x_f), i = opp(dir) (Bouzidi and Yu links; others
                           // repeat pf), or null when no link needs it
    const LinkRec *crec;   // [n] compact records, or null (read meta, q, sf, sff, pf, pff)
    const LinkRunBase *cbase;  // [n / 64 + 1] their bases
};

// Partial forces of the link kernel, one per run of 64 links, reduced per object
// by the first blocks of the next bulk launch (or by force_reduce_kernel): one
// entry per 64 links of capacity.
struct Reduce {
    double2 *wpart;
    int32_t *wobj;
};

// A pending force reduction: nw wavefront partials (wpart, wobj) summed per object
// into bank and fsum.  nw = 0: nothing to do.
struct ForceReduce {
    const double2 *wpart;
    const int32_t *wobj;
    int64_t nw;
    double *bank;
    double *fsum;
};

// Launch shape of the bulk kernel (chosen by the autotuner).
struct BulkConfig {
    int32_t block_x;      // 64, 128 or 256 lanes along x; 256/block_x rows
    int32_t store_solid;  // lanes of solid nodes store zeros too (full-line writes)
    int32_t xcd;          // contiguous runs of blocks per XCD (see bulk_kernel)
    int32_t fused;        // the bulk kernel evaluates the links of its nodes (no link kernel)
    int32_t rows;         // row segments per wavefront: 1, or 2 (block_x 256, not fused)
    int32_t runs;         // one run of 64 fluid nodes per wavefront (compact layout, periodic x)
};

// What the fused bulk kernel needs for the links: link arrays, the per-segment
// force partials (one per 64-node row segment, reduced by force_reduce_kernel
// into force_bank and force_sum) and the banks for wavefronts that mix objects.
struct FuseArgs {
    Links L;
    double2 *wpart;
    int32_t *wobj;
    double *bank;
    double *fsum;
};

// Link values of one step into side.L and, unless force_bank is null, the force
// of every object added to force_bank and force_sum.  With defer non-null the
// reduction of the per-64-link partials is not launched but described in
// *defer, for the bulk launch that follows (nw = 0 when there is none).
hipError_t launch_link(int storage, const Grid &g, const Phys &ph, const Links &L, const Side &side,
                       const Reduce &red, double *force_bank, double *force_sum, int block,
                       hipStream_t s, ForceReduce *defer = nullptr);

// One bulk step; fr is a reduction deferred by launch_link, done by the first
// blocks of the launch.
hipError_t launch_bulk(int storage, const Grid &g, const Phys &ph, const void *A, void *B,
                       const mask_t *mask, const void *uin, const Side &side, double *zero_bank,
                       int32_t n_zero, const BulkConfig &cf, hipStream_t s,
                       const ForceReduce &fr = ForceReduce{nullptr, nullptr, 0, nullptr, nullptr});

// One whole step with the links evaluated inside the bulk kernel (cf.fused): the
// bulk launch, then the force reduction over its segment partials.  side.M/P
// must hold this step's deposits and side.Mw/Pw other arrays.
hipError_t launch_bulk_fused(int storage, const Grid &g, const Phys &ph, const void *A, void *B,
                             const mask_t *mask, const void *uin, const Side &side, const FuseArgs &fa,
                             double *zero_bank, int32_t n_zero, const BulkConfig &cf, hipStream_t s);

// Batched form: per-instance descriptor and per-block tile.
struct BatchInst {
    Grid g;            // the instance's lattice (plane = its own plane stride)
    int64_t pop_off;   // element offset of its plane 0 in the shared population buffers
    int64_t mask_off;  // element offset of its mask words
    int32_t seg_off;   // first entry of its segment table
    int32_t uin_off;   // first inlet row
    double omega, gx, gy;
};
struct BatchTile {
    int32_t inst, y0, x0, pad;
};
constexpr int BATCH_BX = 256;  // lanes along x per batched block (one row)

hipError_t launch_bulk_batch(int storage, const BatchInst *insts, const BatchTile *tiles, int64_t ntiles,
                             const Phys &ph, const void *A, void *B, const mask_t *mask, const void *uin,
                             const Side &side, double *zero_bank, int32_t n_zero, bool open, bool force,
                             bool store_solid, int rows, hipStream_t s, const ForceReduce &fr);

// Rebuilds the deposited populations P (and, with moments, M) of every flagged
// node from the populations in A: after initialisation or a restored checkpoint.
hipError_t launch_refresh(int storage, const Grid &g, const Phys &ph, const void *A,
                          const Side &side, bool moments, hipStream_t s);

// Equilibrium initialisation of rows [y0, y0+rows) of A from staged doubles
// (rho, ux, uy interleaved per node, rows*nx nodes).
hipError_t launch_init(int storage, const Grid &g, const Phys &ph, void *A, const mask_t *mask,
                       const double *stage, int32_t y0, int32_t rows, hipStream_t s);

// Moments of rows [y0, y0+rows) into staged doubles (rho, ux, uy per node).
hipError_t launch_moments(int storage, const Grid &g, const Phys &ph, const void *A,
                          const mask_t *mask, double *stage, int32_t y0, int32_t rows,
                          hipStream_t s);

// Moments of every node into three device arrays of ny*nx values (y*nx + x), FP64
// or FP32; null arrays are skipped.
hipError_t launch_moments_out(int storage, const Grid &g, const Phys &ph, const void *A, const mask_t *mask,
                              void *rho, void *ux, void *uy, bool fp64, hipStream_t s);

// Per-block FP64 partials over the fluid nodes: the mass (sum) or, with maxdev,
// max |f_i - w_i|; n_partials = number of blocks used.
hipError_t launch_mass(int storage, const Grid &g, const Phys &ph, const void *A,
                       const mask_t *mask, double *partials, int32_t n_partials, bool maxdev,
                       hipStream_t s);

int32_t mass_blocks(const Grid &g);
constexpr int MASS_THREADS = 256;  // lanes per block of the mass / deviation reduction

// The launch helpers of one storage format, defined by lbm_kernels.hip compiled
// with LBM_ST = 0..5 (one object per format, so that the formats build in
// parallel); the launch_* functions above dispatch on the storage.  Formats 4 and
// 5 (FP32 storage with an FP64 or a plain FP32 collision) define only the bulk
// launches and share the others with format 1.
#define LBM_ST_DECLS(K)                                                                                       \
    hipError_t launch_link_st##K(const Grid &, const Phys &, const Links &, const Side &, const Reduce &,      \
                                 double *, double *, int, hipStream_t, ForceReduce *);                         \
    hipError_t launch_bulk_st##K(const Grid &, const Phys &, const void *, void *, const mask_t *, const void *, \
                                 const Side &, double *, int32_t, const BulkConfig &, hipStream_t,             \
                                 const ForceReduce &);                                                         \
    hipError_t launch_bulk_fused_st##K(const Grid &, const Phys &, const void *, void *, const mask_t *,         \
                                       const void *, const Side &, const FuseArgs &, double *, int32_t,          \
                                       const BulkConfig &, hipStream_t);                                       \
    hipError_t launch_bulk_batch_st##K(const BatchInst *, const BatchTile *, int64_t, const Phys &, const void *, \
                                       void *, const mask_t *, const void *, const Side &, double *, int32_t,   \
                                       bool, bool, bool, int, hipStream_t, const ForceReduce &);               \
    hipError_t launch_refresh_st##K(const Grid &, const Phys &, const void *, const Side &, bool, hipStream_t); \
    hipError_t launch_init_st##K(const Grid &, const Phys &, void *, const mask_t *, const double *, int32_t,  \
                                 int32_t, hipStream_t);                                                        \
    hipError_t launch_moments_st##K(const Grid &, const Phys &, const void *, const mask_t *, double *, int32_t, \
                                    int32_t, hipStream_t);                                                     \
    hipError_t launch_moments_out_st##K(const Grid &, const Phys &, const void *, const mask_t *, void *, void *, \
                                        void *, bool, hipStream_t);                                            \
    hipError_t launch_mass_st##K(const Grid &, const Phys &, const void *, const mask_t *, double *, int32_t,   \
                                 bool, hipStream_t);
LBM_ST_DECLS(0)
LBM_ST_DECLS(1)
LBM_ST_DECLS(2)
LBM_ST_DECLS(3)
LBM_ST_DECLS(4)
LBM_ST_DECLS(5)

// ---------------------------------------------------------------------------
// Adjoint kernels (lbm_adjoint.hip); FP64 and FP32 storage only.  Side records
// hold 12 doubles per flagged node.
// ---------------------------------------------------------------------------

// Bytes of one per-link record of the adjoint.
size_t adj_link_record_bytes(int storage);

// Per-link records of the adjoint, in (node, dir) order, from the link arrays.
hipError_t launch_adj_setup(int storage, const Links &L, const int32_t *mnode, void *lrec, hipStream_t s);

// One reverse step t, one lane per node: from the adjoint Cin of the
// pre-collision populations of step t+1 and the side records sig_in of step t+1
// (consumed and cleared), the adjoint Cout of the pre-collision populations of
// step t (state S of step t), the side records sig_out of step t (added to) and
// the FP64 accumulators dq, duw (per link) and duin (per inlet row).  The force
// weight (djx, djy) applies to the links of object obj.  colslot: side slots of
// the inlet and outlet column nodes (open lattices).
hipError_t launch_adj_step(int storage, const Grid &g, const Phys &ph, const void *S, const void *Cin, void *Cout,
                           double *sig_in, double *sig_out, const void *lrec, const mask_t *mask,
                           const SegBase *seg, const int32_t *colslot, const void *uin, double *duin, double *dq,
                           double *duw, int32_t obj, double djx, double djy, hipStream_t s);

// dJ/dS_0 (nine planes of dplane doubles) and dJ/d(rho, ux, uy) of an
// equilibrium initial state (three planes) from Cin and the side records of
// step 0.
hipError_t launch_adj_final(int storage, const Grid &g, const Phys &ph, const void *S, const void *Cin,
                            const double *sig, const mask_t *mask, const SegBase *seg, double *dstate,
                            double *dinit, int64_t dplane, hipStream_t s);

}  // namespace lbm
