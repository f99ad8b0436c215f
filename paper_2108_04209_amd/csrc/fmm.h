// fmm.h -- triangular far-field compression of the secular sums (internal).
#pragma once

#include <vector>

#include "common.h"

namespace sdc {

constexpr int FMM_P = 16;          // Chebyshev nodes per box (equivalent sources)
constexpr int FMM_NEAR_MAX = 24;   // near leaves per target leaf
constexpr int FMM_FAR_MAX = 64;    // far boxes per side per target leaf

// Per batch: the problems that use the FMM, their trees, and per-leaf interaction lists.
// Problem q (in FMM numbering) owns boxes [box_off[q], box_off[q+1]) in heap order over its
// leaves (level h has 2^h boxes; box (h, i) covers leaves [i 2^(H-h), (i+1) 2^(H-h))), and
// leaves [leaf_off[q], leaf_off[q+1]).
struct FmmArgs {
    const int64_t *off;
    int leaf;                 // poles per leaf
    double sep;               // separation ratio for the far field
    const int32_t *fmm_prob;  // [nfmm] batch problem index
    const int32_t *fmm_of;    // [nprob] FMM index of a problem, -1 for direct
    const int32_t *box_off;   // [nfmm + 1]
    const int32_t *leaf_off;  // [nfmm + 1]
    const int32_t *height;    // [nfmm] tree height H (levels 0..H)
    const double2 *dw;        // (d_j, w_j) of the batch (from validation)
    const double *z2;         // sum of w per problem
    const int32_t *status;
    double2 *eq;              // [boxes][FMM_P] equivalent sources (node, weight)
    double2 *box_ab;          // [boxes] (first pole, last pole) of the box
    int32_t *near_lo, *near_hi;   // [leaves][FMM_NEAR_MAX] pole ranges of near leaves
    int32_t *far_l, *far_r;       // [leaves][FMM_FAR_MAX] far box ids (global)
    int32_t *cnt;             // [leaves][3] counts (near, far left, far right); -1 = direct
    int nboxes, nleaves;
    const int32_t *box_fmm;   // [nboxes] owning FMM problem of each box
    const int32_t *leaf_fmm;  // [nleaves] owning FMM problem of each leaf
};

// Host side: the FMM layout of one batch for one leaf size (device buffers owned here).
struct FmmPlan {
    int leaf = 0;
    int crossover = 0;               // problems with n >= crossover use the FMM
    int nfmm = 0, nboxes = 0, nleaves = 0;
    std::vector<int32_t> fmm_prob_h, fmm_of_h, box_off_h, leaf_off_h;
    int32_t *fmm_prob = nullptr, *fmm_of = nullptr, *box_off = nullptr, *leaf_off = nullptr;
    int32_t *height = nullptr, *box_fmm = nullptr, *leaf_fmm = nullptr;
    double2 *eq = nullptr, *box_ab = nullptr;
    int32_t *near_lo = nullptr, *near_hi = nullptr, *far_l = nullptr, *far_r = nullptr;
    int32_t *cnt = nullptr;
    // work items: 64-root pieces of the target leaves (a piece never crosses a leaf)
    int sub = TILE;                    // roots per work item
    int nitems = 0;
    int split = 1;                     // wavefronts per work item (they share its lists)
    std::vector<int32_t> item_off_h;   // FMM problem q owns items [item_off[q], item_off[q+1])
    Tile *leaf_lpt = nullptr;          // work items, longest problems first
    Tile *leaf_nat = nullptr;          // ... in problem order
    std::vector<Tile *> dir_lpt;       // direct chunks of the other problems, per cut length
    std::vector<int32_t> dir_count;
    std::vector<void *> allocs;
};

hipError_t launch_fmm_build(const FmmArgs &f, hipStream_t s);
hipError_t launch_secular_fmm(const SolveArgs &a, const FmmArgs &f, int split, Queue *q,
                              int grid, hipStream_t s);

}  // namespace sdc
