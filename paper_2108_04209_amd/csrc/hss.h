// hss.h -- internal declarations of the HSS conquering pass.
#pragma once

#include "common.h"

namespace sdc {

constexpr int LEAF_MAX = 128;      // largest leaf block (its matrix lives in LDS)
constexpr int LEAF_RANK_MAX = 8;   // largest off-diagonal rank r
constexpr int LEAF_SWEEPS = 16;    // Jacobi sweeps per leaf (the rotation log's capacity)

struct LeafArgs {
    int leaf, r, nleaf, max_sweeps;
    const double *D;  // nleaf x leaf x leaf, row-major
    const double *U;  // nleaf x leaf x r, row-major
    double *Q;        // nleaf x leaf x leaf, eigenvector j contiguous, ascending order
    double *lam;      // nleaf * leaf eigenvalues, ascending per leaf
    double *W;        // Q^T U, column-major with leading dimension ldw
    int64_t ldw;
    double *rot;      // nleaf x max_sweeps x leaf rounds x leaf/2 (cos, signed sin) pairs
    int32_t *rank;    // nleaf x leaf ascending rank of each diagonal entry
    int32_t *sweeps;  // nleaf sweeps logged
    int32_t *status;  // nleaf: 0, or SUPERDC_ST_NOCONV if max_sweeps did not converge
};

struct AssembleArgs {
    int64_t n;             // entries of the level
    int nl, r, level;      // node size, rank, level of the parents
    int with_basis;        // also form the basis columns (not at the root)
    const int32_t *perm;   // merge permutation of the level
    const double *Wprev;   // children's basis columns (n x r, ld n)
    const double *B, *beta, *R;
    double *M;             // output: n x 2r, ld n (Z in columns 0..r-1, V in r..2r-1)
};

// dividing stage (divide.hip)
struct DivideArgs {
    int leaf, r, depth, balanced;
    const double *D, *U, *R, *B;  // original generators (layout of the conquering pass)
    double *D_out, *B_out, *beta_out;
    double *H;                    // [2^(depth+1) - 1][r][r] pending updates, heap order
};
hipError_t launch_divide(const DivideArgs &a, hipStream_t s);

hipError_t launch_leaf_jacobi(const LeafArgs &a, hipStream_t s);
hipError_t launch_merge(const double *lam_children, double *d_out, int32_t *perm, int nc,
                        int64_t n, hipStream_t s);
hipError_t launch_assemble(const AssembleArgs &a, hipStream_t s);
hipError_t launch_permute(const int32_t *perm, int nl, int64_t n, int m, const double *X,
                          int64_t ldx, double *Y, int64_t ldy, int scatter, hipStream_t s);
hipError_t launch_leaf_apply(const double *Q, int L, int64_t n, int m, const double *X,
                             int64_t ldx, double *Y, int64_t ldy, int trans, hipStream_t s);
// ascending sort of every segment of nl keys (ties keep their order); vout[pos] = index
// within the segment of the key placed at pos.  kbuf, vbuf: n-entry work buffers.
hipError_t launch_seg_sort(const double *keys, int nl, int64_t n, double *kout, int32_t *vout,
                           double *kbuf, int32_t *vbuf, hipStream_t s);
hipError_t launch_status_or(const int32_t *st, int cnt, int32_t *out, hipStream_t s);
hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t s);

}  // namespace sdc
