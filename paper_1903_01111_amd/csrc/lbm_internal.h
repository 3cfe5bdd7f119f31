// Internal interface between the host runtime (lbm_runtime.cpp) and the HIP
// kernels (lbm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace lbm {

// Device population layout: nine planes of `plane` elements, plane i holding
// f_i - w_i of node (x, y) at offset y*pitch + x.  pitch >= nx is a multiple of
// 64 elements, so a 64-lane wavefront reads one aligned run of a row.
struct Grid {
    int32_t nx, ny, pitch, x_open;
    int64_t plane;
};

struct Phys {
    double omega;     // 1/tau
    double gx, gy;    // body acceleration
    double rho0;      // reference density of the moving-wall term
    float scale;      // 2^k for 16-bit storage (1 otherwise)
    float inv_scale;  // 2^-k
};

// Mask byte of a node: bit 0 solid, bit 1 "moments wanted" (the node is x_f or
// x_ff of some VIBB link).  The bulk kernel stores (rho - 1, ux, uy) of every
// flagged node after collision; the link kernel of the next step reads them
// instead of gathering the nine populations of both nodes.  The slot of a
// flagged node is its rank in plane order: seg_base[y*pitch/64 + x/64] (flagged
// nodes before that 64-node row segment) plus the flagged lanes below it in its
// wavefront.
constexpr uint8_t MASK_SOLID = 1, MASK_MOMENTS = 2;

struct Side {
    void *M;                  // real[3K]: rho - 1, ux, uy (physical velocity)
    const int32_t *seg_base;  // [ny * pitch / 64]
    const int32_t *mnode;     // [K] plane offset of each flagged node
    int64_t K;
};

// Compacted boundary links, sorted by (obj, node).  Indices are offsets inside
// a plane.  meta = dir | (obj << 8).
struct Links {
    const int32_t *nf;   // x_f
    const int32_t *nff;  // x_ff = x_f - e_{i'}, or -1: halfway bounce-back
    const int32_t *ns;   // x_s = x_f + e_{i'}: its slot of plane i = opp(i')
                         // receives f_i(x_f, t+1) for the next pull
    const int32_t *sf;   // moment slot of x_f (VIBB links)
    const int32_t *sff;  // moment slot of x_ff (VIBB links)
    const uint32_t *meta;
    const void *q;       // real[n]
    const void *uw;      // real[2n] or nullptr (still walls)
    int64_t n;
};

// Wavefront partial forces of the link kernel, reduced per object by a second
// launch: capacity one entry per 64 links of capacity, rounded up to a block.
struct Reduce {
    double2 *wpart;
    int32_t *wobj;
};

// Launch shape of the bulk kernel (chosen by the autotuner).
struct BulkConfig {
    int32_t block_x;      // 64, 128 or 256 lanes along x; 256/block_x rows
    int32_t store_solid;  // lanes of solid nodes store zeros too (full-line writes)
};

hipError_t launch_link(int storage, const Grid &g, const Phys &ph, void *A, const Links &L,
                       const void *M, const Reduce &red, double *force_bank, double *force_sum,
                       int block, hipStream_t s);

hipError_t launch_bulk(int storage, const Grid &g, const Phys &ph, const void *A, void *B,
                       const uint8_t *mask, const void *uin, const Side &side, double *zero_bank,
                       int32_t n_zero, const BulkConfig &cf, hipStream_t s);

// Recomputes the side moments of every flagged node from the populations in A
// (after initialisation or a restored checkpoint).
hipError_t launch_refresh(int storage, const Grid &g, const Phys &ph, const void *A,
                          const Side &side, hipStream_t s);

// Equilibrium initialisation of rows [y0, y0+rows) of A from staged doubles
// (rho, ux, uy interleaved per node, rows*nx nodes).
hipError_t launch_init(int storage, const Grid &g, const Phys &ph, void *A, const uint8_t *mask,
                       const double *stage, int32_t y0, int32_t rows, hipStream_t s);

// Moments of rows [y0, y0+rows) into staged doubles (rho, ux, uy per node).
hipError_t launch_moments(int storage, const Grid &g, const Phys &ph, const void *A,
                          const uint8_t *mask, double *stage, int32_t y0, int32_t rows,
                          hipStream_t s);

// Per-block FP64 partial sums of the mass; n_partials = number of blocks used.
hipError_t launch_mass(int storage, const Grid &g, const Phys &ph, const void *A,
                       const uint8_t *mask, double *partials, int32_t n_partials, hipStream_t s);

int32_t mass_blocks(const Grid &g);

}  // namespace lbm
