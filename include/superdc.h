/*
 * superdc.h -- C ABI of the MI355X (gfx950) conquering-stage library for SuperDC
 * (Ou & Xia, "SuperDC: Stable superfast divide-and-conquer eigenvalue decomposition").
 *
 * The library solves batches of diagonal-plus-rank-one symmetric eigenproblems
 *
 *     A_p = diag(d_p) + rho_p z_p z_p^T,     p = 0 .. nprob-1,                   (*)
 *
 * the building block of the conquering stage (Sec. 2.2, eqs. rankrupd and rank1upd, with
 * the paper's v = sqrt(rho) z).  For each problem it
 *   1. finds all n_p eigenvalues as roots of the secular equation (eq. seceq) by solving
 *      the shifted equations (eq. shiftedeq) for gaps eta_k relative to a per-root origin
 *      pole d_K ("local shifting", Sec. 4.2.2): lambda_k = d_{K_k} + eta_k (eq. evalnew);
 *   2. recomputes the update vector zhat by Loewner's formula (eq. lowner) and the column
 *      normalisation b (eq. b) of the Cauchy-like eigenvector matrix
 *          Qhat_ij = zhat_i b_j / (d_i - lambda_j)                (eqs. eigvecs, qscale),
 *      with every difference d_i - lambda_j formed as (d_i - d_{K_j}) - eta_j (eq. qk);
 *   3. applies Qhat or Qhat^T to blocks of vectors (Alg. 3 Z-update, Alg. 4);
 *   4. (not in the paper) back-propagates dL/dlambda and dL/d(Qhat^T u) to (d, z, rho).
 * It also runs a whole HSS conquering pass (Alg. 3) on a perfect binary tree.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller unless stated; the
 *     library never frees or keeps it past the call.
 *   - Problems are stored back to back (CSR layout): problem p owns the entries
 *     off[p] .. off[p+1]-1 of every per-entry array (d, z, lam, eta, origin, zhat, ...).
 *     The offsets are given once, on the host, to superdc_batch_create.
 *   - d must be strictly increasing within each problem, z_i != 0, rho_p > 0, all finite
 *     (the paper assumes deflation has already removed the other cases, Sec. 4.1).
 *   - origin[k] is a LOCAL index within its problem: origin[k] in {k, k+1} for k < n_p-1,
 *     origin[n_p-1] = n_p-1.  eta is the gap to that pole, lam = d[origin] + eta rounded.
 *   - Matrices of right-hand sides are column-major over the whole batch: column c of X
 *     starts at X + c*ldx and problem p's rows are off[p] .. off[p+1]-1 (ldx >= total_n).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream).  Calls do
 *     not synchronise with the host.  Host-detectable argument errors return a negative
 *     code synchronously and enqueue nothing.  Data-dependent errors are reported per
 *     problem in the device `status` array written by superdc_secular_solve (bits below);
 *     the later calls skip problems whose status is not 0 or SUPERDC_ST_NOCONV.
 *   - Workspace lives in the context and only grows.  The first call for a batch shape may
 *     allocate; later calls with the same or a smaller shape allocate nothing and issue no
 *     memset, so they may be captured into a hipGraph.
 *   - One context per host thread; calls on one context must not overlap in time.
 */
#ifndef SUPERDC_H
#define SUPERDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define SUPERDC_OK 0
#define SUPERDC_EINVAL -1   /* NULL pointer, bad size, bad option                     */
#define SUPERDC_ENOMEM -2   /* device allocation failed                               */
#define SUPERDC_EHIP -3     /* a HIP runtime call or kernel launch failed             */
#define SUPERDC_ENODEV -4   /* no gfx950 device visible                               */

/* per-problem status bits (device array written by superdc_secular_solve) */
#define SUPERDC_ST_UNSORTED 1   /* d not strictly increasing                          */
#define SUPERDC_ST_ZERO 2       /* some z_i == 0 (would need deflation, Remark 1)     */
#define SUPERDC_ST_NONFINITE 4  /* NaN or Inf in d, z or rho                          */
#define SUPERDC_ST_RHO 8        /* rho <= 0                                           */
#define SUPERDC_ST_NOCONV 16    /* a root hit the iteration cap; it keeps its best     */
                                /* bracketed iterate                                   */

/* per-root iteration record (iters array of superdc_secular_solve): the low 16 bits count
 * the evaluations of the secular sums after the midpoint pass; one of these bits tells how
 * the iteration ended when it did not end on the stopping test (eq. stopcrit) */
#define SUPERDC_ITER_COUNT_MASK 0xffff
#define SUPERDC_ITER_UNMET (1 << 16) /* a step below 2 ulps of the iterate, or a bracket    */
                                     /* collapsed to 2 ulps, ended it before the test held */
#define SUPERDC_ITER_CAP (1 << 17)   /* the iteration cap ended it (status NOCONV)          */
#define SUPERDC_ITER_SKIPPED (1 << 18) /* not solved: the problem's input is invalid        */

typedef struct superdc_ctx superdc_ctx;
typedef struct superdc_batch superdc_batch;

/* Secular-solver options.  superdc_opts_default fills the defaults shown. */
typedef struct {
    double stop_c;       /* c in the stopping test |f| < c n eps (1+|psi|+|phi|)
                            (eq. stopcrit); default 1.0, must be > 0                      */
    int32_t max_iter;    /* iteration cap per root after the midpoint pass; default 40,
                            1..200                                                        */
    int32_t method;      /* 0 auto (direct below the crossover, FMM above), 1 direct sums,
                            2 triangular FMM (Sec. 4.1.2)                                 */
    int32_t fmm_order;   /* Chebyshev nodes per FMM box; 16 (the only supported order)      */
    int32_t fmm_leaf;    /* FMM leaf size; default 64, a multiple of 64, at most 1024     */
    int32_t persistent;  /* 1: one persistent launch per phase for the whole batch;
                            0: one launch per problem per phase (the "plain" baseline)    */
    int32_t apply_kernel;/* Cauchy apply: 0 auto (MFMA for m >= 4), 1 VALU, 2 FP64 MFMA    */
    int32_t fmm_crossover;/* method 0: problems with at least this many roots use the FMM
                            (solver, b, Qhat^T X); 0 = the context's default (1024)       */
    int32_t unshifted;   /* 1: ablation of the local shifting (Sec. 4.2.2): the iterate is
                            kept as lambda itself and every pole difference is formed as
                            d_j - lambda (f evaluated at lambda with no shift); the
                            reciprocals keep the default precision; default 0          */
    int32_t interp;      /* rational interpolation of the iteration (Sec. 4.1.1): 0 the middle
                            way (default); 1 the hybrid of [li93]: the middle way and the
                            fixed-weight scheme (the nearer pole keeps its true weight, the
                            other pole's matches f'), switching scheme after a step that
                            leaves f's sign unchanged and reduces |f| by less than 10x      */
    double hss_tau;      /* superdc_hss_conquer only: deflation tolerance (Remark 1) for every
                            rank-one problem of the pass, finite, >= 0; default 0 (none)  */
} superdc_opts;

void superdc_opts_default(superdc_opts *opts);

/* Create / destroy a context on the current HIP device (must be gfx950). */
int superdc_create(superdc_ctx **ctx);
void superdc_destroy(superdc_ctx *ctx);
const char *superdc_strerror(int code);
/* hipError_t value behind the last SUPERDC_EHIP / SUPERDC_ENOMEM of this host thread */
int superdc_last_hip_error(void);

/*
 * Describe a batch.  off_host[0..nprob] are HOST offsets with off_host[0] = 0 and
 * off_host[p+1] - off_host[p] >= 1; they are copied (to the device as well), so the
 * caller may free them afterwards.  nprob >= 1.  The batch also holds the work lists
 * (root tiles ordered longest-first) that the kernels consume.
 */
int superdc_batch_create(superdc_ctx *ctx, int32_t nprob, const int64_t *off_host,
                         superdc_batch **batch);
void superdc_batch_destroy(superdc_batch *batch);
int64_t superdc_batch_total(const superdc_batch *batch);

/*
 * Autotune the batch's launch shapes on representative data (d, z, rho as for
 * superdc_secular_solve): the secular solver's work-item length (64..512 roots) and split
 * (wavefronts sharing one work item, 1..16), the split of the FMM solver's work items
 * (1..8) when opts select the FMM for some problem, and the splits of the Loewner/b and
 * adjoint kernels, each timed on `stream`.  Synchronises the stream and allocates scratch; call it
 * once, before capturing graphs.  With SUPERDC_TUNE_CACHE set to a file path the choice is
 * read from / appended to that file, keyed by the problem sizes and the CU count.
 * Without tuning a heuristic shape is used.  Results of the solver can differ in the last
 * bits between shapes (the near/far split of some pole-root pairs moves).
 */
int superdc_autotune(superdc_ctx *ctx, superdc_batch *batch, const double *d, const double *z,
                     const double *rho, const superdc_opts *opts, void *stream);
/* Current shapes (out: int32[5]): out[0] solver work-item length, out[1] solver split,
 * out[2] Loewner/b split, out[3] adjoint split, out[4] FMM solver split (0: the heuristic,
 * about 16 wavefronts per CU). */
int superdc_batch_shapes(const superdc_batch *batch, int32_t *out);

/*
 * Eigenvalues of every problem (*) (Alg. 2 with local shifting, Sec. 4.2).
 *   in : d[total], z[total], rho[nprob]
 *   out: lam[total], eta[total], origin[total] (int32, local), iters[total] (int32: the
 *        evaluations of the secular sums after the midpoint pass in the bits
 *        SUPERDC_ITER_COUNT_MASK, plus SUPERDC_ITER_UNMET or SUPERDC_ITER_CAP when the
 *        iteration ended otherwise than on the stopping test, SUPERDC_ITER_SKIPPED for the
 *        roots of a problem with invalid input; may be NULL), status[nprob]
 *        (int32, bits above; always written).
 * opts may be NULL (defaults).
 */
int superdc_secular_solve(superdc_ctx *ctx, const superdc_batch *batch, const double *d,
                          const double *z, const double *rho, double *lam, double *eta,
                          int32_t *origin, int32_t *iters, int32_t *status,
                          const superdc_opts *opts, void *stream);

/*
 * For callers that cannot allocate device memory (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): superdc_secular_solve with the same arguments
 * and outputs, run by the same kernels with direct sums (opts->method 0 or 1; 2 is
 * rejected), whose per-call buffers -- (d_j, rho z_j^2) and (d_K, eta) pairs, 32 bytes per
 * root, and one double per problem -- live in one fixed array in device memory instead of
 * the context's workspace.  The library holds that array on every GPU it runs on until the
 * process ends (SUPERDC_NOALLOC_MAX_TOTAL * 32 + SUPERDC_NOALLOC_MAX_PROBS * 8 bytes,
 * about 123 MiB).  The call allocates nothing, issues no memset and does not synchronise;
 * the batch and the context must have been created beforehand and kernel timing must be
 * off.  Results equal superdc_secular_solve's with opts->method = 1, bit for bit.
 * Errors: SUPERDC_EINVAL for the argument errors of superdc_secular_solve, for
 * opts->method = 2, for total > SUPERDC_NOALLOC_MAX_TOTAL or nprob >
 * SUPERDC_NOALLOC_MAX_PROBS, and when the current device is not the context's.
 * Every call on one GPU uses that GPU's single array: calls that overlap in time on one
 * GPU (other streams, threads or contexts) race and give undefined results; calls ordered
 * on one stream are safe (each call writes every entry it reads before reading it).
 */
#define SUPERDC_NOALLOC_MAX_TOTAL 4000000
#define SUPERDC_NOALLOC_MAX_PROBS 65536
int superdc_secular_solve_noalloc(superdc_ctx *ctx, const superdc_batch *batch,
                                  const double *d, const double *z, const double *rho,
                                  double *lam, double *eta, int32_t *origin, int32_t *iters,
                                  int32_t *status, const superdc_opts *opts, void *stream);

/*
 * Loewner update vector and normalisation (eqs. lowner and b), from the solver's output:
 *   in : d, z (only its signs are used), rho, eta, origin, status
 *   out: zhat[total] with rho zhat_i^2 = prod_j (lambda_j - d_i) / prod_{j!=i} (d_j - d_i)
 *        and sign(zhat_i) = sign(z_i); bnorm[total] with
 *        bnorm_j = (sum_i zhat_i^2 / (d_i - lambda_j)^2)^(-1/2) > 0.
 * Problems that use the FMM (opts.method / opts.fmm_crossover, as for the solver) get b
 * through the eigenvector-side triangular FMM (Sec. 4.3: near poles in the shifted form,
 * far boxes through Chebyshev equivalent sources), the others by direct sums; zhat is
 * always formed by direct products.
 */
int superdc_loewner(superdc_ctx *ctx, const superdc_batch *batch, const double *d,
                    const double *z, const double *rho, const double *eta,
                    const int32_t *origin, const int32_t *status, double *zhat,
                    double *bnorm, const superdc_opts *opts, void *stream);

/*
 * Y = Qhat X (trans = 0) or Y = Qhat^T X (trans = 1) for every problem, with
 * Qhat_ij = zhat_i bnorm_j / ((d_i - d_{K_j}) - eta_j) (eqs. eigvecs, qscale, qk).
 * X and Y are total x m column-major with leading dimensions ldx, ldy >= total; they
 * must not overlap.  m >= 1.  With trans = 1, problems that use the FMM (as for the
 * solver) are applied through the eigenvector-side triangular FMM (Sec. 4.3, Alg. 3
 * Z-update) in passes of 16 columns; the others, and every trans = 0 product, use the
 * FP64 MFMA kernel (m >= 4) or the VALU kernel.
 */
int superdc_cauchy_apply(superdc_ctx *ctx, const superdc_batch *batch, const double *d,
                         const double *zhat, const double *bnorm, const double *eta,
                         const int32_t *origin, const int32_t *status, int trans, int32_t m,
                         const double *X, int64_t ldx, double *Y, int64_t ldy,
                         const superdc_opts *opts, void *stream);

/*
 * Adjoint of the rank-one eigensolver (not in the paper; implicit differentiation of
 * f(lambda_k) = 0).  With r_ik = 1/((d_i - d_{K_k}) - eta_k), q_ik = b_k z_i r_ik,
 * b_k = (sum_i z_i^2 r_ik^2)^(-1/2) and projections p_k = q_k^T u:
 *   in : d, z, rho, eta, origin, status, g_lam[total] = dL/dlambda (may be NULL),
 *        g_proj[total] = dL/dp (may be NULL), u[total] (NULL iff g_proj is NULL)
 *   out: g_d[total] = dL/dd, g_z[total] = dL/dz, g_rho[nprob] = dL/drho.
 */
int superdc_secular_backward(superdc_ctx *ctx, const superdc_batch *batch, const double *d,
                             const double *z, const double *rho, const double *eta,
                             const int32_t *origin, const int32_t *status,
                             const double *g_lam, const double *g_proj, const double *u,
                             double *g_d, double *g_z, double *g_rho,
                             const superdc_opts *opts, void *stream);

/* ------------------------------------------------------------------------------------
 * Deflation (Remark 1) with a user tolerance tau >= 0.
 *
 * For A = diag(d) + v v^T, v = sqrt(rho) z, d non-decreasing (equal poles allowed):
 *   rule 1: pole k deflates if |v_k| < tau; its eigenpair is (d_k, e_k);
 *   rule 2: scanning the remaining poles in increasing order, the current pole a and the
 *           next remaining pole b are rotated together if
 *           |(d_a - d_b) v_a v_b| < (v_a^2 + v_b^2) tau.  With r = |(z_a, z_b)|,
 *           c = z_b / r, s = z_a / r, the rotation G = [c -s; s c] on (a, b) takes
 *           (z_a, z_b) to (0, r); the off-diagonal entry cs (d_a - d_b) it creates is below
 *           tau and is dropped.  Pole a deflates with eigenvalue c^2 d_a + s^2 d_b; pole b
 *           continues into the next test with d_b' = s^2 d_a + c^2 d_b (held in
 *           [d_a, d_b]) and z_b' = r.
 * Decisions are taken in FP64 with the expressions above evaluated as written (no fused
 * multiply-adds), so a plain sequential implementation reaches the same ones.
 * The eigenvector matrix of the deflated problem is Q = G^T P (Qhat (+) I): G the product
 * of the rotations (the first made acting first), P the placement below, Qhat that of the
 * reduced problem.
 *
 *   in : d, z [total] (device), rho [nprob] (device), tau (host scalar, finite, >= 0)
 *   out: per problem p, at its offset, with k = kept[p]:
 *        d_out/z_out[0 .. k)  the reduced problem (strictly increasing poles; solve it with
 *                             the same rho after gathering it into a batch of sizes
 *                             kept[p], superdc_batch_copy_rows);
 *        d_out[k .. n_p)      the deflated eigenvalues in pole order, z_out = 0 there;
 *        perm[j]              the pole (local index) of output position j;
 *        rot_right[i]         for a pole deflated by rule 2, the pole it was rotated into
 *                             (local index), else -1; rot_left[b] = a when rot_right[a] = b,
 *                             else -1;
 *        rot_c[i], rot_s[i]   that rotation's c and s (1 and 0 where there is none);
 *        kept[p] (device int32), status[p] (device int32: SUPERDC_ST_NONFINITE for a
 *        non-finite d, z or rho, SUPERDC_ST_UNSORTED for a decrease in d,
 *        SUPERDC_ST_RHO for rho <= 0; such a problem gets kept = 0 and no other output).
 * tau = 0 deflates nothing (the output is the input and perm the identity).  All
 * arrays are caller-owned device memory; returns SUPERDC_EINVAL for NULL pointers or a
 * bad tau.
 */
int superdc_deflate(superdc_ctx *ctx, const superdc_batch *batch, const double *d,
                    const double *z, const double *rho, double tau, double *d_out,
                    double *z_out, int32_t *perm, int32_t *rot_right, int32_t *rot_left,
                    double *rot_c, double *rot_s, int32_t *kept, int32_t *status, void *stream);

/*
 * The orthogonal factor of a deflation, on total x m column-major blocks (leading
 * dimensions ldx, ldy >= total; every problem on its own rows, as for
 * superdc_cauchy_apply):
 *   trans 0: Y = G^T P X, rows of X indexed by output position (rows [0, k) holding the
 *            reduced problem's Qhat applied to a block, rows [k, n_p) the block's deflated
 *            rows unchanged), so that Y = Q (block);
 *   trans 1: Y = P^T G X, rows of X indexed by pole, so that rows [0, k) of Y are the input
 *            to Qhat^T and rows [k, n_p) are already rows of Q^T X.
 * perm, rot_* as written by superdc_deflate for the same batch.  X and Y must not overlap.
 */
int superdc_deflate_expand(superdc_ctx *ctx, const superdc_batch *batch, const int32_t *perm,
                           const int32_t *rot_right, const int32_t *rot_left,
                           const double *rot_c, const double *rot_s, int trans, int32_t m,
                           const double *X, int64_t ldx, double *Y, int64_t ldy, void *stream);

/*
 * Row copy between two batches with the same number of problems (a batch and its reduced
 * problems), on total x m column-major blocks (leading dimensions lds >= src total,
 * ldd >= dst total): for every problem p, rows [0, k_p) of p's rows in src go to the first
 * k_p rows of p's rows in dst, k_p = min(n_src_p, n_dst_p, rows[p]) (rows: device
 * int32[nprob], or NULL for no third bound).  With fill non-NULL (host pointer) the other
 * rows of dst are set to *fill, else they are left as they are.  src and dst must differ.
 */
int superdc_batch_copy_rows(superdc_ctx *ctx, const superdc_batch *src_batch,
                            const superdc_batch *dst_batch, const int32_t *rows, int32_t m,
                            const double *src, int64_t lds, double *dst, int64_t ldd,
                            const double *fill, void *stream);

/* ------------------------------------------------------------------------------------
 * HSS conquering pass (Alg. 3) on a perfect binary tree.
 *
 * The symmetric HSS matrix is given by its generators (Sec. 2.1, eq. hss) with the leaf
 * blocks already divided (Sec. 3): for a node p with children c1, c2
 *     A_p = blkdiag(A_c1, A_c2) + Z_p Z_p^T,   Z_p = [U_c1 B_p / sqrt(beta_p) ; sqrt(beta_p) U_c2],
 *     U_p = [U_c1 R_c1 ; U_c2 R_c2],  A_leaf = D_leaf      (eqs. du, divnew1; Alg. 1).
 * The conquer computes every A_p's eigenvalues bottom-up: dense leaf eigendecompositions,
 * then per node the merge of the children's spectra (permutation P_p) and r sequential
 * rank-one updates (Sec. 2.2, eq. rankrupd), all nodes of one level in one batched call.
 * The eigenvectors are kept in the structured form of Lemma 2 (eq. eigmat): per node the
 * permutation and r Cauchy-like factors, per leaf a dense block.
 * Levels are numbered as in the paper: root 0, leaves `depth`; node q of level l owns
 * entries [q n_l, (q+1) n_l), n_l = leaf 2^(depth-l), n = leaf 2^depth.
 * ---------------------------------------------------------------------------------- */
typedef struct superdc_hss superdc_hss;

/* Plan a tree: leaf in [2, 128] even, depth in [1, 20], r in [1, 8].  Allocates the
 * level batches, the factor storage and work buffers (O(r n depth) doubles), and the leaf
 * eigensolver's rotation log: room for 16 Jacobi sweeps of (cos, sin) pairs, 16 leaf n
 * doubles (1.07 GB for n = 65536 and leaf 128). */
int superdc_hss_plan_create(superdc_ctx *ctx, int32_t leaf, int32_t depth, int32_t r,
                            superdc_hss **plan);
void superdc_hss_plan_destroy(superdc_hss *plan);

/*
 * Dividing stage (Alg. 1) for the original generators of an HSS matrix (eq. hss: the
 * coupling of node p's children is U_c1 B_p U_c2^T, bases nested by eq. du), in the
 * layout of superdc_hss_conquer.  Top down, each node's pending update H (Lemma genupd,
 * zero at the root) turns its children's coupling into B_p - R_c1 H R_c2^T with
 * beta_p = ||B_p - R_c1 H R_c2^T||_2, and the children inherit R_c H R_c^T plus the
 * balanced division (eq. divnew1): (1/beta_p) B B^T for the left child, beta_p I for the
 * right one; a leaf ends as D - U H U^T.  balanced = 0 uses the earlier division (eq.
 * divide: B B^T and I, beta = 1).  A coupling that vanishes gets beta = 1.
 *   out: leaf_D_out [2^depth][leaf][leaf], B_out [2^depth - 1][r][r], beta_out [2^depth - 1]
 *        -- with leaf_U and R unchanged, exactly the input of superdc_hss_conquer, whose
 *        eigenvalues are then those of the original matrix.
 * Outputs must not alias the inputs.  Device pointers, caller-owned.
 */
int superdc_hss_divide(superdc_ctx *ctx, superdc_hss *plan, const double *leaf_D,
                       const double *leaf_U, const double *R, const double *B, int balanced,
                       double *leaf_D_out, double *B_out, double *beta_out, void *stream);

/*
 * Conquering pass.  Device inputs (row-major small matrices; heap index h = 2^l - 1 + q):
 *   leaf_D [2^depth][leaf][leaf]  symmetric leaf blocks
 *   leaf_U [2^depth][leaf][r]     leaf bases
 *   R      [2^(depth+1) - 1][r][r] transfer matrices (the root's entry is unused)
 *   B      [2^depth - 1][r][r]    coupling generator of each non-leaf node's children
 *   beta   [2^depth - 1]          balancing scalars, > 0
 * Outputs: lam[n] (eigenvalues of A_root, ascending); lam_levels[(depth+1) n] or NULL
 * (row l: eigenvalues of every level-l node, ascending per node); status[1]: OR of the
 * status bits of every rank-one problem solved.  The structured eigenmatrix stays in the
 * plan for superdc_hss_apply until the next conquer on the same plan.
 * opts->hss_tau > 0 deflates every rank-one problem of the pass (Remark 1, as in Alg. 3):
 * per step the host reads the kept counts back (one stream synchronisation; such a pass
 * cannot be captured in a graph), solves the reduced problems as a batch of their sizes and
 * sorts each node's eigenvalues; superdc_hss_apply replays the rotations, placements and
 * sorts.  Without deflation a problem with a vanishing weight or equal poles fails: its
 * node returns NaN eigenvalues and its bits in status (SUPERDC_ST_ZERO, _UNSORTED).
 */
int superdc_hss_conquer(superdc_ctx *ctx, superdc_hss *plan, const double *leaf_D,
                        const double *leaf_U, const double *R, const double *B,
                        const double *beta, double *lam, double *lam_levels, int32_t *status,
                        const superdc_opts *opts, void *stream);

/*
 * Y = Q X (trans = 0) or Q^T X (trans = 1) with the eigenmatrix Q of A_root from the last
 * conquer (Lemma 2, Alg. 4): n x m column-major, leading dimensions >= n, X and Y must not
 * overlap.  Column k of Q is the eigenvector of lam[k].
 */
int superdc_hss_apply(superdc_ctx *ctx, superdc_hss *plan, int trans, int32_t m,
                      const double *X, int64_t ldx, double *Y, int64_t ldy,
                      const superdc_opts *opts, void *stream);

/*
 * Autotune the launch shapes of every level's batch of the plan (superdc_autotune on each
 * level, timed on the level's own first rank-one problems, which one conquer of these
 * generators produces on the way).  Runs that conquer on `stream`, synchronises it and
 * allocates scratch: call it once, before timing or capturing conquers of the plan.  The
 * choice persists in the plan's batches (and in SUPERDC_TUNE_CACHE when set).  Undeflated
 * passes only: opts->hss_tau must be 0 (EINVAL otherwise).
 */
int superdc_hss_autotune(superdc_ctx *ctx, superdc_hss *plan, const double *leaf_D,
                         const double *leaf_U, const double *R, const double *B,
                         const double *beta, const superdc_opts *opts, void *stream);
/* The launch shapes of level `level`'s batch, as superdc_batch_shapes (out: int32[5]). */
int superdc_hss_batch_shapes(const superdc_hss *plan, int32_t level, int32_t *out);

/*
 * Phase timing of superdc_hss_conquer (for measurement).  With timing enabled, each
 * conquer records HIP events on its stream between phases.  superdc_hss_phase_times waits
 * for the last conquer and returns, per phase, the summed milliseconds ms[6] and the
 * number of timed intervals launches[6] (may be NULL): 0 leaf eigendecompositions,
 * 1 merges and assemblies, 2 secular solves (validation + solver), 3 Loewner and b,
 * 4 Cauchy applies, 5 final copies.  Returns SUPERDC_EINVAL if timing was off.
 */
int superdc_hss_set_timing(superdc_hss *plan, int enable);
/* Copy the per-root solver iteration records of the last conquer to dst (device,
 * int32[depth][r][n], level-major; encoded as the iters output of superdc_secular_solve). */
int superdc_hss_iterations(superdc_hss *plan, int32_t *dst, void *stream);
int superdc_hss_phase_times(superdc_hss *plan, double *ms, int32_t *launches);

/*
 * Per-kernel timing (for measurement; process-wide, off by default).  enable: 0 off;
 * 1 HIP events around every launch and the device work counters (superdc_kernel_work,
 * superdc_kernel_counters); 2 the events only; 3 the counters only (their atomic adds cost
 * time, so a pass that times kernels precisely leaves them off).  With events on, every
 * kernel launch of the library is bracketed by two HIP events recorded on the launch's
 * stream.  Do not enable it while a stream is being captured into a graph.
 * superdc_kernel_times waits for every recorded launch, writes the summed milliseconds
 * ms[id] and launch counts launches[id] for the first `count` kernel ids, starts a new
 * collection, and returns the number of kernel ids (negative on error); count = 0 only
 * returns that number.
 * superdc_kernel_name gives the kernel of an id ("unknown" out of range).
 */
int superdc_kernel_timing(int enable);
int superdc_kernel_times(double *ms, int32_t *launches, int32_t count);
/*
 * Work counted on the device while kernel timing was on, per kernel id; kernels without a
 * counter report 0.  The secular solvers (k_secular, k_secular_fmm) count pole-root pair
 * evaluations: each pass of each live root times the poles or equivalent sources it sums.
 * The Cauchy apply kernels (k_apply_mfma, k_apply_valu) and the eigenvector-side FMM
 * evaluations (k_fmmv_eval_mfma, k_fmmv_eval) count algorithmic FP64 flops: (2m + 3) per
 * Cauchy entry (pole or equivalent source against root) for m columns (6 for the b sum
 * alone), plus 2m per output row.  Waits for the device, then clears the counters.
 * Returns the number of kernel ids (negative on error).
 */
int superdc_kernel_work(double *pairs, int32_t count);
/*
 * All device counters of the kernels, as superdc_kernel_work (waits, then clears them):
 * out[4 id + 0] the work above; for the secular solvers out[4 id + 1] the live lanes
 * (roots being iterated) summed over every pass of every wavefront and out[4 id + 2] the
 * lanes of those passes (64 each), whose ratio is the share of lanes doing useful work;
 * out[4 id + 3] is reserved (0).  out holds 4 count doubles.
 */
int superdc_kernel_counters(double *out, int32_t count);
const char *superdc_kernel_name(int32_t id);

#ifdef __cplusplus
}
#endif

#endif /* SUPERDC_H */
