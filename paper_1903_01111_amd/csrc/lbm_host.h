// Host-side helpers shared by the lattice runtime (lbm_runtime.cpp) and the
// batched runtime (lbm_batch.cpp): validation and preprocessing of geometries.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

namespace lbm_host {

extern thread_local std::string g_thread_error;

inline constexpr int EXR[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
inline constexpr int EYR[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
inline constexpr int OPPR[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
inline constexpr double WR[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

inline constexpr int64_t STAGE_NODES = 1 << 20;  // nodes per read-back / init chunk


size_t align256(size_t v);
size_t elem_bytes(int storage);
size_t real_bytes(int storage);
bool storage_is_16bit(int storage);  // FP16 or BF16 deviations scaled by 2^dev_scale_log2

// Rejects invalid lattice parameters with a reason.
bool params_ok(const lbm_params *p, std::string *why);

// Device-ready form of a validated geometry (see prepare_geometry).
struct Prepared {
    // per link, in (obj, node, dir) order
    std::vector<uint32_t> meta;
    std::vector<double> q, uw;
    std::vector<int32_t> sf, sff, pf, pff, pfi, li;
    std::vector<int64_t> order;  // caller's index of each link
    // per flagged node, in plane order
    std::vector<uint16_t> rec;
    std::vector<int32_t> mnode, pbase;
    std::vector<lbm::mask_t> mask;         // padded to the pitch: link bits, solid bit, side bit
    std::vector<lbm::SegBase> seg;         // per 64-node row segment, plus a sentinel with the totals
    std::vector<uint64_t> fmask;           // per segment: its fluid nodes (bit = lane)
    std::vector<lbm::RunBase> runs;        // per run of 64 fluid nodes, plus a sentinel with the totals
    std::vector<lbm::SegRow> frow;         // per segment: fmask and fluid base in one record, plus a sentinel
    std::vector<uint16_t> nbr;             // per fluid node: neighbour word (empty: not available)
    std::vector<lbm::NbrRun> nbr_run;      // per run of 64 fluid nodes: word bases, plus a sentinel
    std::vector<uint32_t> nbr_slow;        // nine pull offsets per table entry of the neighbour words
    int32_t n_fluid = 0;
    int64_t n_pops = 0;
    bool has_uw = false;
    bool has_pfi = false;       // some link reads f+_i(x_f) (Bouzidi, Yu): pfi is filled
    bool has_ext_scheme = false;  // some link uses Bouzidi or Yu
    int64_t n_fallback = 0;
};

// Validates mask and links against p (see lbm_check_geometry); with out, also
// builds the link arrays (object, node, direction order), the side records and
// segment bases of the flagged nodes for a row pitch of `pitch`.
lbm_status prepare_geometry(const lbm_params &p, const uint8_t *mask, int64_t n, const int32_t *node,
                            const int8_t *dir, const double *q, const double *uw, const int32_t *obj,
                            const int8_t *scheme, int32_t pitch, Prepared *out, std::string *why);

// Compact link records of n links (4-byte reals): per run of 64 links the bases
// (the smallest M slot and P entry of x_f and of x_ff), per link the direction
// word, q's bits and the 16-bit excesses over the bases; runs that do not fit are
// marked (sf0 = -1) and keep only the direction word and q.  crec gets n entries,
// cbase n / 64 + 1.
void build_link_records(size_t n, const uint32_t *meta, const float *q, const int32_t *sf, const int32_t *sff,
                        const int32_t *pf, const int32_t *pff, std::vector<lbm::LinkRec> *crec,
                        std::vector<lbm::LinkRunBase> *cbase);

}  // namespace lbm_host
