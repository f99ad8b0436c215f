// fmm.h -- triangular far-field compression of the secular sums (internal).
#pragma once

#include <vector>

#include "common.h"

namespace sdc {

constexpr int FMM_P = 16;          // Chebyshev nodes per box (equivalent sources)
constexpr int FMM_NEAR_MAX = 24;   // near leaves (and so near ranges) per target leaf
constexpr int FMM_FAR_MAX = 64;    // far boxes per side per target leaf
constexpr int FMM_PL = 20;         // Chebyshev terms of a target leaf's local expansion
constexpr int FMM_LOC = 4 * FMM_PL; // local expansion of a target leaf: psi, psi', phi, phi'
                                    // far fields, FMM_PL Chebyshev coefficients each

// Chebyshev nodes (first kind) of a P-point grid on [-1, 1], cos((2q + 1) pi / 2P), and the
// barycentric weights of the first FMM_P of them, (-1)^q sin((2q + 1) pi / 2P)
__device__ __forceinline__ double cheb_node(int q, int P = FMM_P) {
    return cos((2.0 * q + 1.0) * 3.14159265358979323846 / (2.0 * P));
}
__device__ __forceinline__ double cheb_bary(int q) {
    return ((q & 1) ? -1.0 : 1.0) * sin((2.0 * q + 1.0) * 3.14159265358979323846 / (2.0 * FMM_P));
}
// Per batch: the problems that use the FMM, their trees, and per-leaf interaction lists.
// Problem q (in FMM numbering) owns boxes [box_off[q], box_off[q+1]) in heap order over its
// leaves (level h has 2^h boxes; box (h, i) covers leaves [i 2^(H-h), (i+1) 2^(H-h))), and
// leaves [leaf_off[q], leaf_off[q+1]).
struct FmmArgs {
    const int64_t *off;
    int leaf;                 // poles per leaf
    double sep;               // separation ratio for the far field (times the box's width)
    double sep_loc;           // separation from the target interval, times its width, of the
                              // sources that enter a target leaf's local expansion
    const int32_t *fmm_prob;  // [nfmm] batch problem index
    const int32_t *fmm_of;    // [nprob] FMM index of a problem, -1 for direct
    const int32_t *box_off;   // [nfmm + 1]
    const int32_t *leaf_off;  // [nfmm + 1]
    const int32_t *height;    // [nfmm] tree height H (levels 0..H)
    const double2 *dw;        // (d_j, w_j) of the batch (from validation); .x alone for geometry
    const double *tail;       // [nprob] bound of the last root above d_{n-1}
    const int32_t *status;
    int32_t *used;            // [nboxes] == gen if some target leaf of the current lists lists
                              // the box as far field
    int gen;                  // the current lists' number: the lists kernel tags the boxes it
                              // uses with it, so no pass clears the flags between builds
    double2 *eq;              // [boxes][FMM_P] equivalent sources (node, weight)
    int32_t *near_lo, *near_hi;   // [leaves][FMM_NEAR_MAX] pole ranges: runs of adjacent near leaves
    int32_t *near_lf;             // [leaves][FMM_NEAR_MAX] 1: the range lies sep_loc target widths
                                  // (and a tile of indices) from the target interval, so its
                                  // poles enter the local expansion instead of the solver's
                                  // direct sums (the other consumers sum every near range)
    int32_t *far_l, *far_r;       // [leaves][FMM_FAR_MAX] far box ids (global)
    int32_t *cnt;             // [leaves][3] counts (near, far left, far right); -1 = direct
    // Far boxes also separated from the whole target interval (by sep_loc times its width)
    // enter the leaf's local expansion instead of being summed per root and iteration.
    int32_t *far_ld, *far_rd;       // [leaves][FMM_FAR_MAX] the far boxes summed directly
                                    // from the front, those in the expansion from the back
    int32_t *cntd;                  // [leaves][2] counts of the direct ones (left, right)
    double2 *loc_ab;          // [leaves] (centre, half-width) of the target interval
    double *loc;              // [leaves][FMM_LOC] Chebyshev coefficients on that interval
    int nboxes, nleaves;
    const int32_t *box_fmm;   // [nboxes] owning FMM problem of each box
    const int32_t *leaf_fmm;  // [nleaves] owning FMM problem of each leaf
    const int32_t *leaf_box;  // [nleaves] global box id of each leaf
    const int32_t *upper_box; // [nupper] global ids of the boxes above the leaves that hold
                              // poles, the largest (most leaves below) first
    int nupper;
    // the eigenvector-side sources of the upper boxes in parts of at most FMMV_PART_PTS
    // points: items (box, part, parts, partial slot or -1), largest boxes first; the boxes
    // cut into several parts (box, first slot) and their partial weights
    const int4 *upper_item;   // [nupper_item]
    int nupper_item;
    const int2 *split_box;    // [nsplit]
    int nsplit;
    double *vpart;            // [slots][FMM_P][FMMV_MAX_M]
    // targets of the lists: nullptr, the roots of the solver (a target leaf's roots lie in
    // [d_first, d_next]); else the positions of the target points themselves (the poles, for
    // sums over the roots), a leaf spanning [tpos[first], tpos[last]]
    const double *tpos;
};

// Host side: the FMM layout of one batch for one leaf size (device buffers owned here).
struct FmmPlan {
    int leaf = 0;
    int crossover = 0;               // problems with n >= crossover use the FMM
    int nfmm = 0, nboxes = 0, nleaves = 0;
    std::vector<int32_t> fmm_prob_h, fmm_of_h, box_off_h, leaf_off_h;
    int32_t *fmm_prob = nullptr, *fmm_of = nullptr, *box_off = nullptr, *leaf_off = nullptr;
    int32_t *height = nullptr, *box_fmm = nullptr, *leaf_fmm = nullptr;
    int32_t *leaf_box = nullptr, *upper_box = nullptr;
    int nupper = 0;
    int4 *upper_item = nullptr;
    int2 *split_box = nullptr;
    int nupper_item = 0, nsplit = 0;
    double *vpart = nullptr;
    double2 *eq = nullptr;
    int32_t *near_lo = nullptr, *near_hi = nullptr, *far_l = nullptr, *far_r = nullptr;
    int32_t *cnt = nullptr, *near_lf = nullptr;
    int32_t *far_ld = nullptr, *far_rd = nullptr, *cntd = nullptr;
    double2 *loc_ab = nullptr;
    double *loc = nullptr;
    // work items: 64-root pieces of the target leaves (a piece never crosses a leaf)
    int sub = TILE;                    // roots per work item
    int nitems = 0;
    int split = 1;                     // wavefronts per work item (they share its lists)
    std::vector<int32_t> item_off_h;   // FMM problem q owns items [item_off[q], item_off[q+1])
    Tile *leaf_lpt = nullptr;          // work items, longest problems first
    Tile *leaf_nat = nullptr;          // ... in problem order
    // the solver's work items: longer pieces (ssub roots), so a wavefront refills lanes whose
    // roots converged instead of idling until its slowest root is done
    int ssub = 2 * TILE;
    int snitems = 0;
    int ssplit = 1;
    std::vector<int32_t> sitem_off_h;
    Tile *sitem_lpt = nullptr;
    Tile *sitem_nat = nullptr;
    std::vector<Tile *> dir_lpt;       // direct chunks of the other problems, per cut length
    std::vector<int32_t> dir_count;
    int32_t *used = nullptr;           // [nboxes], zeroed at creation
    int gen = 0, t_gen = 0;            // numbers of the last lists built (solver's, roots')
    double *vnode = nullptr, *vw = nullptr;  // eigenvector-side equivalent sources
    double *tail = nullptr;            // [nprob] per-call bound of the last root
    double2 *lgeo = nullptr;           // Loewner far field: box geometry and moments
    double *lmom = nullptr;
    // the lists of the sums over the roots (Y = Qhat X: sources at the roots, targets at the
    // poles), kept apart from the solver's, which later calls on the same poles reuse
    int32_t *t_near_lo = nullptr, *t_near_hi = nullptr, *t_far_l = nullptr, *t_far_r = nullptr;
    int32_t *t_cnt = nullptr, *t_far_ld = nullptr, *t_far_rd = nullptr, *t_cntd = nullptr;
    int32_t *t_near_lf = nullptr;
    int32_t *t_used = nullptr;
    double2 *t_loc_ab = nullptr;
    std::vector<void *> allocs;
};

// Eigenvector-side FMM (Sec. 4.3-4.4 with local shifting): sums over the poles i of a
// problem for every root j, sum_i src_i,c K(d_i - lambda_j), with K = 1/t (the apply
// Y = Qhat^T X: src = zhat_i X_i,c, scaled by b_j) or K = 1/t^2 (b: src = zhat_i^2);
// with trans = 0, sums over the roots j for every pole i, sum_j src_j,c / (d_i - lambda_j)
// (the apply Y = Qhat X: src = b_j X_j,c, scaled by zhat_i), sources at the roots.
struct FmmVec {
    int m;                    // columns of src (<= FMMV_MAX_M)
    int kern;                 // 1: 1/t, 2: 1/t^2
    int trans;                // 1: sums over the poles (targets the roots); 0: over the roots
                              // (source positions lambda_j = d_{K_j} + eta_j, in the .x of
                              // the pairs the pack kernel writes)
    double *src;              // [total][m] pole-major source weights
    double *vnode;            // [boxes][FMM_P] equivalent source nodes
    double *vw;               // [boxes][FMM_P][m] equivalent source weights
    const double *d;          // poles
    const int32_t *origin;    // roots' origins (local indices)
    const double *eta;        // roots' offsets
    const double *post;       // kern 1: per-root scale (b); unused for kern 2
    double *Y;                // kern 1: output columns, ld ldy
    int64_t ldy;
    double *bout;             // kern 2: b_j = (sum)^(-1/2)
    int fuse_b;               // kern 1 on the MFMA: the last of the m weight columns is zhat^2;
                              // the evaluation forms b from it with the kernel 1/t^2, writes
                              // it to bout and scales the other m - 1 columns by it
    const double *zh;         // fuse_b: zhat, for b's near terms (zhat / t)^2
    unsigned long long *work; // kernel timing on: algorithmic flops of the launch (set by
                              // launch_fmmv_eval): (2m + 3) per near pole or far source of a
                              // root for kern 1, 6 for kern 2, plus the output scaling
};
constexpr int FMMV_MAX_M = 16;
constexpr int FMMV_PART_PTS = 512;   // points per part of an upper box's sources (2 chunks)

// Loewner far field (Sec. 4.3, eqs. lowner2 and logv with local shifting): for a far box B
// and a pole x outside it,
//     G_B(x) = sum_{j in B} log((lambda_j - x) / (d_j - x))
//            = sum_{k >= 1} (-1)^(k+1) M_k r^k / k,   r = hw / (c - x),
// with the box's centre c and half-width hw (its span covers its poles and roots) and the
// moments M_k = sum_j ((t_j + D_j)^k - t_j^k), t_j = (d_j - c) / hw, D_j = delta_j / hw,
// delta_j = lambda_j - d_j.  Every moment is a sum of terms proportional to delta_j, so no
// cancellation: P_1 = D, P_{k+1} = (t + D) P_k + D t^k.
constexpr int FMML_K = 28;  // moments per box (|r| <= 1/4 at separation 1.5: 0.25^28 ~ 1e-17)

struct FmmlArgs {
    double2 *pd;              // (d_j, delta_j) per entry (pole and its root's offset)
    double2 *geo;             // [boxes] (c, hw)
    double *mom;              // [boxes][FMML_K] moments M_1 .. M_K
    // pack != 0: the leaves' launch packs its poles itself (when the lists already exist, as
    // the separate packing launch would): (d_j, delta_j) into pd, (d_{K_j}, eta_j) into ke
    // when ke is set, and the last delta of each problem into tail
    int pack;
    const double *d, *eta;
    const int32_t *origin;
    double2 *ke;
    double *tail;
};
hipError_t launch_fmml_moments(const FmmArgs &f, const FmmlArgs &l, hipStream_t s);

// packing of the source weights of the FMM problems (and the list geometry)
struct FmmvPackArgs {
    const int64_t *off;
    const Tile *tiles;   // 64-entry tiles of the FMM problems
    int ntiles;
    const double *d, *zhat, *eta;
    const double *bnorm; // trans 0: b_j, the sources' scale
    const int32_t *origin;
    const double *X;     // kern 1: right-hand sides (column-major, ld ldx), columns c0..c0+m-1
    int64_t ldx;
    int c0;
    double2 *pairs;      // (d_i, zhat_i) for the list geometry; trans 0: (lambda_j, b_j)
    double *tail;        // [nprob] lambda_{n-1} - d_{n-1}
    double2 *ke;         // Loewner packing, when every problem of the batch uses the FMM:
                         // also (d_{K_j}, eta_j) for every root (else nullptr)
};
hipError_t launch_fmmv_pack(const FmmvPackArgs &a, const FmmVec &v, hipStream_t s);
// Loewner far field: (d_j, delta_j) pairs and the last roots' offsets, then the products
hipError_t launch_fmml_pack(const FmmvPackArgs &a, hipStream_t s);
hipError_t launch_loewner_fmm(const VecArgs &a, const FmmArgs &f, const FmmlArgs &l, int split,
                              Queue *q, int grid, hipStream_t s);


hipError_t launch_fmm_build(const FmmArgs &f, hipStream_t s);
// interaction lists only (no secular equivalent sources)
hipError_t launch_fmm_lists(const FmmArgs &f, hipStream_t s);
// pk: when set, the leaves' launch packs the sources itself (pk.pairs non-null; the lists
// must exist already), in place of launch_fmmv_pack
hipError_t launch_fmmv_sources(const FmmArgs &f, const FmmVec &v, const FmmvPackArgs *pk,
                               hipStream_t s);
// grid: persistent (q != nullptr) launches size themselves from num_cu
hipError_t launch_fmmv_eval(const SolveArgs &items, const FmmArgs &f, const FmmVec &v, int split,
                            Queue *q, int num_cu, hipStream_t s);
hipError_t launch_secular_fmm(const SolveArgs &a, const FmmArgs &f, int split, Queue *q,
                              int grid, hipStream_t s);

}  // namespace sdc
