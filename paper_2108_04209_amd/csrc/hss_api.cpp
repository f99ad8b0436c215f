// hss_api.cpp -- host side of the HSS conquering pass (Alg. 3) and of the structured
// eigenmatrix application (Lemma 2, Alg. 4).  Every level is one batch of 2^l equal
// rank-one problems, so each phase of a level is one launch (or one launch per node with
// opts->persistent = 0, the plain baseline).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "fmm.h"
#include "hss.h"

using namespace sdc;

struct superdc_hss {
    superdc_ctx *ctx = nullptr;
    int leaf = 0, depth = 0, r = 0;
    int64_t n = 0;
    std::vector<superdc_batch *> batch;  // levels 0 .. depth-1
    std::vector<void *> allocs;
    double *leafQ = nullptr;   // 2^depth x leaf x leaf
    double *leaf_lam = nullptr;
    double *Wleaf = nullptr;   // n x r
    double *leaf_rot = nullptr;     // Jacobi rotation log: 2^depth x LEAF_SWEEPS x leaf x leaf/2 x 2
    int32_t *leaf_rank = nullptr;   // 2^depth x leaf
    int32_t *leaf_sweeps = nullptr; // 2^depth
    double *M[2] = {nullptr, nullptr};  // n x 2r update / basis columns (ping-pong)
    double *ones = nullptr;    // rho = 1 for every node
    int32_t *iters = nullptr;
    // per level l and step t
    double *poles0 = nullptr;  // [depth][n] merged spectra (poles of step 0)
    double *lam = nullptr;     // [depth][r][n] eigenvalues after step t (poles of step t+1)
    double *eta = nullptr, *zhat = nullptr, *bn = nullptr;  // [depth][r][n]
    int32_t *org = nullptr;    // [depth][r][n]
    int32_t *perm = nullptr;   // [depth][n]
    int32_t *status = nullptr; // [depth][r][2^(depth-1)]
    double *T[2] = {nullptr, nullptr};  // apply work buffers
    double *Hdiv = nullptr;    // dividing stage: pending updates per node (on first use)
    // deflation inside the pass (opts->hss_tau > 0), allocated on first use; per level l and
    // step t ([depth][r][n] unless noted) the factor G^T P of Remark 1, the reduced problem
    // and the sort S of its eigenvalues, so that the step's eigenvector matrix is
    // G^T P (Qhat (+) I) S^T (S^T scatters by dS, S gathers)
    bool defl = false;         // the last conquer deflated
    bool defl_mem = false;
    double *dr = nullptr;      // reduced poles (reduced layout, at most n)
    int32_t *dperm = nullptr, *drr = nullptr, *drl = nullptr, *dS = nullptr;
    double *dc = nullptr, *ds = nullptr;
    int32_t *dkept = nullptr;  // [depth][r][2^(depth-1)]
    std::vector<superdc_batch *> rb;  // [depth][r] reduced batches of the last deflated pass
    // work buffers of the deflated pass
    double *xd = nullptr, *xz = nullptr, *xzr = nullptr, *xlam = nullptr, *xE = nullptr,
           *xk = nullptr;  // n
    int32_t *xv = nullptr; // n
    double2 *xval = nullptr;
    int8_t *xflag = nullptr;
    int4 *xsegi = nullptr;     // deflation scan records: 2^(depth-1) x segments of n
    double2 *xsegd = nullptr;
    double *xY = nullptr, *xR0 = nullptr, *xR1 = nullptr, *xT = nullptr;  // n x 2r
    double *xa[3] = {nullptr, nullptr, nullptr};  // apply work buffers of a deflated pass
    int64_t xcap = 0;
    int64_t tcap = 0;
    bool ready = false;
    bool tune = false;  // the next conquer tunes every level's batch before its first solve
    // optional phase timing: events recorded between phases of the last conquer
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_phase;  // phase that ends at event i (0 leaf, 1 merge/assemble,
                                // 2 secular, 3 loewner/b, 4 apply, 5 copies)
    int nev = 0;

    size_t idx(int l, int t) const { return ((size_t)l * r + t) * (size_t)n; }
    int32_t *st(int l, int t) const {
        return status + ((size_t)l * r + t) * ((size_t)1 << (depth - 1));
    }
    // status words of the deflation pass, after the leaves' words
    size_t nstat() const { return (size_t)depth * r * ((size_t)1 << (depth - 1)) + ((size_t)1 << depth); }
    int32_t *dst(int l, int t) const { return st(l, t) + nstat(); }
    int32_t *kept(int l, int t) const {
        return dkept + ((size_t)l * r + t) * ((size_t)1 << (depth - 1));
    }
    const double *poles(int l, int t) const { return t == 0 ? poles0 + (size_t)l * n : lam + idx(l, t - 1); }
};

namespace {
template <typename T>
hipError_t alloc(superdc_hss *h, T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1));
    if (e == hipSuccess) {
        h->allocs.push_back(q);
        *p = (T *)q;
    }
    return e;
}

int fail(hipError_t e) { return e == hipErrorOutOfMemory ? SUPERDC_ENOMEM : SUPERDC_EHIP; }

// record the end of a phase (no-op unless timing is on)
hipError_t mark(superdc_hss *h, int phase, hipStream_t s) {
    if (!h->timing) return hipSuccess;
    if (h->nev >= (int)h->ev.size()) {
        hipEvent_t e;
        hipError_t rc = hipEventCreate(&e);
        if (rc != hipSuccess) return rc;
        h->ev.push_back(e);
        h->ev_phase.push_back(0);
    }
    h->ev_phase[h->nev] = phase;
    return hipEventRecord(h->ev[h->nev++], s);
}

hipError_t defl_alloc(superdc_hss *h) {
    if (h->defl_mem) return hipSuccess;
    const size_t n = h->n, r = h->r, steps = (size_t)h->depth * r;
    hipError_t e = alloc(h, &h->dr, steps * n);
    if (e == hipSuccess) e = alloc(h, &h->dperm, steps * n);
    if (e == hipSuccess) e = alloc(h, &h->drr, steps * n);
    if (e == hipSuccess) e = alloc(h, &h->drl, steps * n);
    if (e == hipSuccess) e = alloc(h, &h->dS, steps * n);
    if (e == hipSuccess) e = alloc(h, &h->dc, steps * n);
    if (e == hipSuccess) e = alloc(h, &h->ds, steps * n);
    if (e == hipSuccess) e = alloc(h, &h->dkept, steps * ((size_t)1 << (h->depth - 1)));
    for (double **p : {&h->xd, &h->xz, &h->xzr, &h->xlam, &h->xE, &h->xk})
        if (e == hipSuccess) e = alloc(h, p, n);
    if (e == hipSuccess) e = alloc(h, &h->xv, n);
    if (e == hipSuccess) e = alloc(h, &h->xval, n);
    if (e == hipSuccess) e = alloc(h, &h->xflag, n);
    const size_t nrec = ((size_t)1 << (h->depth - 1)) * deflate_segments((int)n);
    if (e == hipSuccess) e = alloc(h, &h->xsegi, nrec);
    if (e == hipSuccess) e = alloc(h, &h->xsegd, nrec);
    for (double **p : {&h->xY, &h->xR0, &h->xR1, &h->xT})
        if (e == hipSuccess) e = alloc(h, p, n * 2 * r);
    if (e == hipSuccess) {
        h->rb.assign(steps, nullptr);
        h->defl_mem = true;
    }
    return e;
}

// One rank-one step of level l with deflation (Remark 1): deflate every node's problem,
// gather the reduced problems into a batch of their sizes (read back from the device),
// solve them, and sort each node's eigenvalues -- the reduced roots and the deflated
// values -- into the poles of the next step.  The remaining update and basis columns
// (cur's columns t+1 .. ncol-1) are taken to the new eigenbasis:
// S ((Qhat^T (+) I) P^T G) X, into the other buffer.
int defl_step(superdc_ctx *ctx, superdc_hss *h, int l, int t, int cur, int ncol,
              const superdc_opts &o, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    superdc_batch *b = h->batch[l];
    const int nprob = b->nprob;
    const int64_t n = h->n;
    const int nl = (int)(n >> l);
    const size_t k = h->idx(l, t);
    const double *poles = h->poles(l, t);
    const double *zc = h->M[cur] + (size_t)t * n;
    int32_t *kept = h->kept(l, t);
    hipError_t e = launch_deflate(b->off_d, nprob, poles, zc, h->ones, o.hss_tau, h->xd, h->xz,
                                  h->dperm + k, h->drr + k, h->drl + k, h->dc + k, h->ds + k,
                                  kept, h->dst(l, t), h->xval, h->xflag, nl, h->xsegi, h->xsegd,
                                  s);
    if (e != hipSuccess) return fail(e);
    std::vector<int32_t> kh(nprob);
    if ((e = hipMemcpyAsync(kh.data(), kept, sizeof(int32_t) * nprob, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e);
    // a node that deflated completely keeps a one-pole stand-in (d = 0, z = 1) whose
    // results are never copied back
    std::vector<int64_t> roff(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) roff[p + 1] = roff[p] + std::max(kh[p], 1);
    // the batch of the same step in the previous pass is kept when the sizes agree (its
    // tile lists and FMM plan depend on nothing else)
    superdc_batch *&rb = h->rb[(size_t)l * h->r + t];
    int rc = SUPERDC_OK;
    if (!rb || rb->off_h != roff) {
        if (rb) superdc_batch_destroy(rb);
        rb = nullptr;
        rc = superdc_batch_create(ctx, nprob, roff.data(), &rb);
        if (rc) return rc;
    }
    const int64_t rt = roff[nprob];
    const double zero = 0.0, one = 1.0;
    double *dr = h->dr + k;
    if ((e = launch_copy_rows(b->off_d, rb->off_d, nprob, rt, 1, kept, h->xd, n, dr, rt, &zero,
                              s)) != hipSuccess ||
        (e = launch_copy_rows(b->off_d, rb->off_d, nprob, rt, 1, kept, h->xz, n, h->xzr, rt, &one,
                              s)) != hipSuccess ||
        (e = mark(h, 1, s)) != hipSuccess)
        return fail(e);
    rc = superdc_secular_solve(ctx, rb, dr, h->xzr, h->ones, h->xlam, h->eta + k, h->org + k,
                               h->iters + k, h->st(l, t), &o, stream);
    if (rc) return rc;
    if ((e = mark(h, 2, s)) != hipSuccess) return fail(e);
    // b of the FMM problems comes with the apply of the remaining columns when there are any
    const int m = ncol - t - 1;
    const bool fuse = m >= 1 && m + 1 <= FMMV_MAX_M;
    rc = loewner_run(ctx, rb, dr, h->xzr, h->ones, h->eta + k, h->org + k, h->st(l, t),
                     h->zhat + k, h->bn + k, &o, stream, true, !fuse);
    if (rc) return rc;
    if ((e = mark(h, 3, s)) != hipSuccess) return fail(e);
    // the step's eigenvalues per node: reduced roots first, deflated values after, sorted
    if ((e = hipMemcpyAsync(h->xE, h->xd, sizeof(double) * n, hipMemcpyDeviceToDevice, s)) !=
            hipSuccess ||
        (e = launch_copy_rows(rb->off_d, b->off_d, nprob, n, 1, kept, h->xlam, rt, h->xE, n,
                              nullptr, s)) != hipSuccess ||
        (e = launch_seg_sort(h->xE, nl, n, h->lam + k, h->dS + k, h->xk, h->xv, s)) != hipSuccess)
        return fail(e);
    if (m > 0) {
        const double *X = h->M[cur] + (size_t)(t + 1) * n;
        if ((e = launch_deflate_expand(b->off_d, nprob, n, m, h->dperm + k, h->drr + k, h->drl + k,
                                       h->dc + k, h->ds + k, 1, X, n, h->xY, n, h->xT, s)) !=
                hipSuccess ||
            (e = launch_copy_rows(b->off_d, rb->off_d, nprob, rt, m, kept, h->xY, n, h->xR0, rt,
                                  &zero, s)) != hipSuccess)
            return fail(e);
        rc = apply_run(ctx, rb, dr, h->zhat + k, h->bn + k, h->eta + k, h->org + k, h->st(l, t), 1,
                       m, h->xR0, rt, h->xR1, rt, &o, stream, true, fuse);
        if (rc) return rc;
        if ((e = launch_copy_rows(rb->off_d, b->off_d, nprob, n, m, kept, h->xR1, rt, h->xY, n,
                                  nullptr, s)) != hipSuccess ||
            (e = launch_permute(h->dS + k, nl, n, m, h->xY, n, h->M[1 - cur] + (size_t)(t + 1) * n,
                                n, 0, s)) != hipSuccess)
            return fail(e);
    }
    if ((e = mark(h, 4, s)) != hipSuccess) return fail(e);
    return SUPERDC_OK;
}
}  // namespace

extern "C" {

void superdc_hss_plan_destroy(superdc_hss *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    for (auto *b : h->rb) superdc_batch_destroy(b);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    for (auto *b : h->batch) superdc_batch_destroy(b);
    for (void *p : h->allocs) (void)hipFree(p);
    delete h;
}

int superdc_hss_plan_create(superdc_ctx *ctx, int32_t leaf, int32_t depth, int32_t r,
                            superdc_hss **out) {
    if (!ctx || !out || leaf < 2 || leaf > LEAF_MAX || (leaf & 1) || depth < 1 || depth > 20 ||
        r < 1 || r > LEAF_RANK_MAX)
        return SUPERDC_EINVAL;
    *out = nullptr;
    superdc_hss *h = new (std::nothrow) superdc_hss();
    if (!h) return SUPERDC_ENOMEM;
    h->ctx = ctx;
    h->leaf = leaf;
    h->depth = depth;
    h->r = r;
    h->n = (int64_t)leaf << depth;
    const int64_t n = h->n;
    for (int l = 0; l < depth; ++l) {
        const int64_t cnt = (int64_t)1 << l, nl = n / cnt;
        std::vector<int64_t> off(cnt + 1);
        for (int64_t q = 0; q <= cnt; ++q) off[q] = q * nl;
        superdc_batch *b = nullptr;
        int rc = superdc_batch_create(ctx, (int32_t)cnt, off.data(), &b);
        if (rc) {
            superdc_hss_plan_destroy(h);
            return rc;
        }
        h->batch.push_back(b);
    }
    const size_t nleaf = (size_t)1 << depth;
    hipError_t e = alloc(h, &h->leafQ, nleaf * leaf * leaf);
    if (e == hipSuccess) e = alloc(h, &h->leaf_lam, n);
    if (e == hipSuccess) e = alloc(h, &h->Wleaf, n * r);
    if (e == hipSuccess)
        e = alloc(h, &h->leaf_rot, nleaf * LEAF_SWEEPS * leaf * (leaf / 2) * 2);
    if (e == hipSuccess) e = alloc(h, &h->leaf_rank, n);
    if (e == hipSuccess) e = alloc(h, &h->leaf_sweeps, nleaf);
    if (e == hipSuccess) e = alloc(h, &h->M[0], n * 2 * r);
    if (e == hipSuccess) e = alloc(h, &h->M[1], n * 2 * r);
    if (e == hipSuccess) e = alloc(h, &h->ones, n);
    if (e == hipSuccess) e = alloc(h, &h->iters, (size_t)depth * r * n);
    if (e == hipSuccess) e = alloc(h, &h->poles0, (size_t)depth * n);
    if (e == hipSuccess) e = alloc(h, &h->lam, (size_t)depth * r * n);
    if (e == hipSuccess) e = alloc(h, &h->eta, (size_t)depth * r * n);
    if (e == hipSuccess) e = alloc(h, &h->zhat, (size_t)depth * r * n);
    if (e == hipSuccess) e = alloc(h, &h->bn, (size_t)depth * r * n);
    if (e == hipSuccess) e = alloc(h, &h->org, (size_t)depth * r * n);
    if (e == hipSuccess) e = alloc(h, &h->perm, (size_t)depth * n);
    // per-node status bits of every rank-one step, then one word per leaf
    // twice the nodes' words: the solves', the leaves', then the deflation pass's
    if (e == hipSuccess)
        e = alloc(h, &h->status, 2 * (size_t)depth * r * ((size_t)1 << (depth - 1)) + nleaf);
    if (e == hipSuccess) e = launch_fill(h->ones, n, 1.0, nullptr);
    if (e == hipSuccess) e = hipMemset(h->perm, 0, sizeof(int32_t) * (size_t)depth * n);
    // level l uses 2^l of the 2^(depth-1) status slots of each step; the rest stay 0
    if (e == hipSuccess)
        e = hipMemset(h->status, 0,
                      sizeof(int32_t) * (2 * (size_t)depth * r * ((size_t)1 << (depth - 1)) + nleaf));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        superdc_hss_plan_destroy(h);
        return fail(e);
    }
    *out = h;
    return SUPERDC_OK;
}

int superdc_hss_divide(superdc_ctx *ctx, superdc_hss *h, const double *leaf_D,
                       const double *leaf_U, const double *R, const double *B, int balanced,
                       double *leaf_D_out, double *B_out, double *beta_out, void *stream) {
    if (!ctx || !h || h->ctx != ctx || !leaf_D || !leaf_U || !R || !B || !leaf_D_out || !B_out ||
        !beta_out || (balanced != 0 && balanced != 1) || leaf_D_out == leaf_D || B_out == B)
        return SUPERDC_EINVAL;
    const size_t nodes = ((size_t)2 << h->depth) - 1;
    if (!h->Hdiv) {
        hipError_t e = alloc(h, &h->Hdiv, nodes * h->r * h->r);
        if (e != hipSuccess) return fail(e);
    }
    DivideArgs a{};
    a.leaf = h->leaf;
    a.r = h->r;
    a.depth = h->depth;
    a.balanced = balanced;
    a.D = leaf_D;
    a.U = leaf_U;
    a.R = R;
    a.B = B;
    a.D_out = leaf_D_out;
    a.B_out = B_out;
    a.beta_out = beta_out;
    a.H = h->Hdiv;
    hipError_t e = launch_divide(a, (hipStream_t)stream);
    return e == hipSuccess ? SUPERDC_OK : fail(e);
}

int superdc_hss_conquer(superdc_ctx *ctx, superdc_hss *h, const double *leaf_D,
                        const double *leaf_U, const double *R, const double *B,
                        const double *beta, double *lam_out, double *lam_levels,
                        int32_t *status_out, const superdc_opts *opts, void *stream) {
    if (!ctx || !h || h->ctx != ctx || !leaf_D || !leaf_U || !R || !B || !beta || !lam_out ||
        !status_out)
        return SUPERDC_EINVAL;
    superdc_opts o;
    if (opts) o = *opts;
    else superdc_opts_default(&o);
    if (!std::isfinite(o.hss_tau) || o.hss_tau < 0.0) return SUPERDC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = h->n;
    const int r = h->r, D = h->depth;
    h->ready = false;
    const bool defl = o.hss_tau > 0.0;
    h->defl = defl;
    if (defl) {
        hipError_t ea = defl_alloc(h);
        if (ea != hipSuccess) return fail(ea);
        // the deflation pass's status words start clear
        ea = hipMemsetAsync(h->dst(0, 0), 0, sizeof(int32_t) * (size_t)D * r * ((size_t)1 << (D - 1)), s);
        if (ea != hipSuccess) return fail(ea);
    }
    h->nev = 0;
    hipError_t e;
    if ((e = mark(h, -1, s)) != hipSuccess) return fail(e);

    // leaves: dense eigendecompositions and W = Q^T U
    LeafArgs la{};
    la.leaf = h->leaf;
    la.r = r;
    la.nleaf = 1 << D;
    la.max_sweeps = LEAF_SWEEPS;
    la.D = leaf_D;
    la.U = leaf_U;
    la.Q = h->leafQ;
    la.lam = h->leaf_lam;
    la.W = h->Wleaf;
    la.ldw = n;
    la.rot = h->leaf_rot;
    la.rank = h->leaf_rank;
    la.sweeps = h->leaf_sweeps;
    la.status = h->status + (size_t)D * r * ((size_t)1 << (D - 1));  // after the nodes' bits
    if ((e = launch_leaf_jacobi(la, s)) != hipSuccess) return fail(e);
    if ((e = mark(h, 0, s)) != hipSuccess) return fail(e);

    const double *child_lam = h->leaf_lam;
    const double *Wprev = h->Wleaf;
    int mbuf = 0;  // buffer the next assembly writes
    for (int l = D - 1; l >= 0; --l) {
        const int nl = (int)(n >> l);
        superdc_batch *b = h->batch[l];
        double *d0 = h->poles0 + (size_t)l * n;
        int32_t *perm = h->perm + (size_t)l * n;
        if ((e = launch_merge(child_lam, d0, perm, nl / 2, n, s)) != hipSuccess) return fail(e);
        AssembleArgs aa{};
        aa.n = n;
        aa.nl = nl;
        aa.r = r;
        aa.level = l;
        aa.with_basis = l > 0;
        aa.perm = perm;
        aa.Wprev = Wprev;
        aa.B = B;
        aa.beta = beta;
        aa.R = R;
        aa.M = h->M[mbuf];
        if ((e = launch_assemble(aa, s)) != hipSuccess) return fail(e);
        if ((e = mark(h, 1, s)) != hipSuccess) return fail(e);
        const int ncol = l > 0 ? 2 * r : r;
        int cur = mbuf;
        for (int t = 0; t < r; ++t) {
            if (defl) {
                int rc = defl_step(ctx, h, l, t, cur, ncol, o, stream);
                if (rc) return rc;
                cur = 1 - cur;
                continue;
            }
            const double *poles = h->poles(l, t);
            const double *zc = h->M[cur] + (size_t)t * n;
            if (h->tune && t == 0) {  // launch shapes of this level, on its own first problem
                const int rc = superdc_autotune(ctx, b, poles, zc, h->ones, &o, stream);
                if (rc) return rc;
            }
            double *lam_t = h->lam + h->idx(l, t);
            double *eta_t = h->eta + h->idx(l, t);
            int32_t *org_t = h->org + h->idx(l, t);
            int32_t *st_t = h->st(l, t);
            int rc = superdc_secular_solve(ctx, b, poles, zc, h->ones, lam_t, eta_t, org_t,
                                           h->iters + h->idx(l, t), st_t, &o, stream);
            if (rc) return rc;
            if ((e = mark(h, 2, s)) != hipSuccess) return fail(e);
            // the solve just built the FMM lists of these poles: Loewner/b and the apply reuse
            // them; b of the FMM problems comes with the apply when columns remain
            const int m = ncol - t - 1;
            const bool fuse = m >= 1 && m + 1 <= FMMV_MAX_M;
            rc = loewner_run(ctx, b, poles, zc, h->ones, eta_t, org_t, st_t,
                             h->zhat + h->idx(l, t), h->bn + h->idx(l, t), &o, stream, true, !fuse);
            if (rc) return rc;
            if ((e = mark(h, 3, s)) != hipSuccess) return fail(e);
            if (m > 0) {
                rc = apply_run(ctx, b, poles, h->zhat + h->idx(l, t), h->bn + h->idx(l, t), eta_t,
                               org_t, st_t, 1, m, h->M[cur] + (size_t)(t + 1) * n, n,
                               h->M[1 - cur] + (size_t)(t + 1) * n, n, &o, stream, true, fuse);
                if (rc) return rc;
                if ((e = mark(h, 4, s)) != hipSuccess) return fail(e);
            }
            cur = 1 - cur;
        }
        child_lam = h->lam + h->idx(l, r - 1);
        Wprev = h->M[cur] + (size_t)r * n;  // basis columns after the last step
        mbuf = 1 - cur;
    }
    e = hipMemcpyAsync(lam_out, h->lam + h->idx(0, r - 1), sizeof(double) * n,
                       hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(e);
    if (lam_levels) {
        for (int l = 0; l < D; ++l) {
            e = hipMemcpyAsync(lam_levels + (size_t)l * n, h->lam + h->idx(l, r - 1),
                               sizeof(double) * n, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return fail(e);
        }
        e = hipMemcpyAsync(lam_levels + (size_t)D * n, h->leaf_lam, sizeof(double) * n,
                           hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(e);
    }
    if ((e = launch_status_or(h->status, (int)(h->nstat() + (defl ? (size_t)D * r * (1 << (D - 1)) : 0)),
                              status_out, s)) != hipSuccess)
        return fail(e);
    if ((e = mark(h, 5, s)) != hipSuccess) return fail(e);
    h->ready = true;
    return SUPERDC_OK;
}

int superdc_hss_autotune(superdc_ctx *ctx, superdc_hss *h, const double *leaf_D,
                         const double *leaf_U, const double *R, const double *B,
                         const double *beta, const superdc_opts *opts, void *stream) {
    if (!ctx || !h || h->ctx != ctx || !leaf_D || !leaf_U || !R || !B || !beta)
        return SUPERDC_EINVAL;
    if (opts && opts->hss_tau != 0.0) return SUPERDC_EINVAL;  // deflated batches vary per pass
    double *lam = nullptr;
    int32_t *st = nullptr;
    hipError_t e = hipMalloc(&lam, sizeof(double) * (size_t)h->n);
    if (e == hipSuccess) e = hipMalloc(&st, sizeof(int32_t));
    int rc = e == hipSuccess ? SUPERDC_OK : fail(e);
    if (rc == SUPERDC_OK) {
        h->tune = true;
        rc = superdc_hss_conquer(ctx, h, leaf_D, leaf_U, R, B, beta, lam, nullptr, st, opts,
                                 stream);
        h->tune = false;
        e = hipStreamSynchronize((hipStream_t)stream);
        if (rc == SUPERDC_OK && e != hipSuccess) rc = fail(e);
    }
    if (lam) (void)hipFree(lam);
    if (st) (void)hipFree(st);
    return rc;
}

int superdc_hss_batch_shapes(const superdc_hss *h, int32_t level, int32_t *out) {
    if (!h || !out || level < 0 || level >= h->depth) return SUPERDC_EINVAL;
    return superdc_batch_shapes(h->batch[level], out);
}

int superdc_hss_iterations(superdc_hss *h, int32_t *dst, void *stream) {
    if (!h || !dst || !h->ready) return SUPERDC_EINVAL;
    const size_t cnt = (size_t)h->depth * h->r * h->n;
    hipError_t e = hipMemcpyAsync(dst, h->iters, sizeof(int32_t) * cnt, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    return e == hipSuccess ? SUPERDC_OK : fail(e);
}

int superdc_hss_set_timing(superdc_hss *h, int enable) {
    if (!h) return SUPERDC_EINVAL;
    h->timing = enable != 0;
    return SUPERDC_OK;
}

int superdc_hss_phase_times(superdc_hss *h, double *ms, int32_t *launches) {
    if (!h || !ms) return SUPERDC_EINVAL;
    for (int i = 0; i < 6; ++i) {
        ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    if (!h->timing || h->nev < 2) return SUPERDC_EINVAL;
    hipError_t e = hipEventSynchronize(h->ev[h->nev - 1]);
    if (e != hipSuccess) return fail(e);
    for (int i = 1; i < h->nev; ++i) {
        float t = 0.f;
        if ((e = hipEventElapsedTime(&t, h->ev[i - 1], h->ev[i])) != hipSuccess) return fail(e);
        const int ph = h->ev_phase[i];
        if (ph >= 0 && ph < 6) {
            ms[ph] += t;
            if (launches) launches[ph] += 1;
        }
    }
    return SUPERDC_OK;
}

int superdc_hss_apply(superdc_ctx *ctx, superdc_hss *h, int trans, int32_t m, const double *X,
                      int64_t ldx, double *Y, int64_t ldy, const superdc_opts *opts,
                      void *stream) {
    if (!ctx || !h || h->ctx != ctx || !X || !Y || m < 1 || (trans != 0 && trans != 1))
        return SUPERDC_EINVAL;
    if (!h->ready || ldx < h->n || ldy < h->n) return SUPERDC_EINVAL;
    superdc_opts o;
    if (opts) o = *opts;
    else superdc_opts_default(&o);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = h->n;
    const int r = h->r, D = h->depth;
    hipError_t e;
    if (h->tcap < n * m) {
        for (int i = 0; i < 2; ++i) {
            if (h->T[i]) {
                (void)hipDeviceSynchronize();
                (void)hipFree(h->T[i]);
                h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void *)h->T[i]));
                h->T[i] = nullptr;
            }
            if ((e = alloc(h, &h->T[i], n * m)) != hipSuccess) return fail(e);
        }
        h->tcap = n * m;
    }
    double *T0 = h->T[0], *T1 = h->T[1];
    if (h->defl) {
        if (h->xcap < n * m) {
            for (double **p : {&h->xa[0], &h->xa[1], &h->xa[2]}) {
                if (*p) {
                    (void)hipDeviceSynchronize();
                    (void)hipFree(*p);
                    h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void *)*p));
                    *p = nullptr;
                }
                if ((e = alloc(h, p, n * m)) != hipSuccess) return fail(e);
            }
            h->xcap = n * m;
        }
    }
    // one step of a deflated pass (see defl_step): trans 1 applies S (Qhat^T (+) I) P^T G
    // to T0, trans 0 G^T P (Qhat (+) I) S^T; the result is left in T0
    auto defl_apply = [&](int l, int t, int tr) -> int {
        superdc_batch *b = h->batch[l], *rb = h->rb[(size_t)l * r + t];
        const int nprob = b->nprob, nl = (int)(n >> l);
        const int64_t rt = rb->total;
        const size_t k = h->idx(l, t);
        const int32_t *kept = h->kept(l, t);
        double *R0 = h->xa[0], *R1 = h->xa[1], *Tx = h->xa[2];
        const double zero = 0.0;
        hipError_t ee;
        if (tr == 1) {
            if ((ee = launch_deflate_expand(b->off_d, nprob, n, m, h->dperm + k, h->drr + k,
                                            h->drl + k, h->dc + k, h->ds + k, 1, T0, n, T1, n, Tx,
                                            s)) != hipSuccess)
                return fail(ee);
        } else if ((ee = launch_permute(h->dS + k, nl, n, m, T0, n, T1, n, 1, s)) != hipSuccess) {
            return fail(ee);
        }
        if ((ee = launch_copy_rows(b->off_d, rb->off_d, nprob, rt, m, kept, T1, n, R0, rt, &zero,
                                   s)) != hipSuccess)
            return fail(ee);
        int rc = superdc_cauchy_apply(ctx, rb, h->dr + k, h->zhat + k, h->bn + k, h->eta + k,
                                      h->org + k, h->st(l, t), tr, m, R0, rt, R1, rt, &o, stream);
        if (rc) return rc;
        if ((ee = launch_copy_rows(rb->off_d, b->off_d, nprob, n, m, kept, R1, rt, T1, n, nullptr,
                                   s)) != hipSuccess)
            return fail(ee);
        if (tr == 1) ee = launch_permute(h->dS + k, nl, n, m, T1, n, T0, n, 0, s);
        else
            ee = launch_deflate_expand(b->off_d, nprob, n, m, h->dperm + k, h->drr + k, h->drl + k,
                                       h->dc + k, h->ds + k, 0, T1, n, T0, n, Tx, s);
        return ee == hipSuccess ? SUPERDC_OK : fail(ee);
    };
    if (trans == 1) {
        // Q^T X: leaves, then per level P and Qhat_1^T .. Qhat_r^T (Alg. 4, transposed)
        if ((e = launch_leaf_apply(h->leafQ, h->leaf, n, m, X, ldx, T0, n, 1, s)) != hipSuccess)
            return fail(e);
        for (int l = D - 1; l >= 0; --l) {
            const int nl = (int)(n >> l);
            if ((e = launch_permute(h->perm + (size_t)l * n, nl, n, m, T0, n, T1, n, 0, s)) !=
                hipSuccess)
                return fail(e);
            std::swap(T0, T1);
            for (int t = 0; t < r; ++t) {
                if (h->defl) {
                    int rc = defl_apply(l, t, 1);
                    if (rc) return rc;
                    continue;
                }
                int rc = superdc_cauchy_apply(ctx, h->batch[l], h->poles(l, t),
                                              h->zhat + h->idx(l, t), h->bn + h->idx(l, t),
                                              h->eta + h->idx(l, t), h->org + h->idx(l, t),
                                              h->st(l, t), 1, m, T0, n, T1, n, &o, stream);
                if (rc) return rc;
                std::swap(T0, T1);
            }
        }
        for (int c = 0; c < m; ++c) {
            e = hipMemcpyAsync(Y + c * ldy, T0 + c * n, sizeof(double) * n,
                               hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return fail(e);
        }
    } else {
        // Q X: per level Qhat_r .. Qhat_1 then P^T, from the root down; leaves last
        for (int c = 0; c < m; ++c) {
            e = hipMemcpyAsync(T0 + c * n, X + c * ldx, sizeof(double) * n,
                               hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return fail(e);
        }
        for (int l = 0; l < D; ++l) {
            const int nl = (int)(n >> l);
            for (int t = r - 1; t >= 0; --t) {
                if (h->defl) {
                    int rc = defl_apply(l, t, 0);
                    if (rc) return rc;
                    continue;
                }
                int rc = superdc_cauchy_apply(ctx, h->batch[l], h->poles(l, t),
                                              h->zhat + h->idx(l, t), h->bn + h->idx(l, t),
                                              h->eta + h->idx(l, t), h->org + h->idx(l, t),
                                              h->st(l, t), 0, m, T0, n, T1, n, &o, stream);
                if (rc) return rc;
                std::swap(T0, T1);
            }
            if ((e = launch_permute(h->perm + (size_t)l * n, nl, n, m, T0, n, T1, n, 1, s)) !=
                hipSuccess)
                return fail(e);
            std::swap(T0, T1);
        }
        if ((e = launch_leaf_apply(h->leafQ, h->leaf, n, m, T0, n, Y, ldy, 0, s)) != hipSuccess)
            return fail(e);
    }
    return SUPERDC_OK;
}

}  // extern "C"
