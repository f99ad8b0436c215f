// api.cpp -- C ABI of the gfx950 conquering-stage library (declared in include/superdc.h).
//
// Host responsibilities only: argument checks, batch plans (work tiles ordered
// longest-problem-first for the persistent launches), grow-only workspace, and the choice
// between one persistent launch per phase and one launch per problem.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "common.h"
#include "fmm.h"

// waves per CU the FMM solver's split aims at (its items times the split)
#ifndef SDC_FMM_WAVES_PER_CU
#define SDC_FMM_WAVES_PER_CU 16
#endif

using namespace sdc;

namespace {

thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    return e == hipErrorOutOfMemory ? SUPERDC_ENOMEM : SUPERDC_EHIP;
}

#define SDC_HIP(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_);     \
    } while (0)

}  // namespace

namespace sdc {
int opts_check(const superdc_opts *o) {
    if (!(o->stop_c > 0.0) || o->max_iter < 1 || o->max_iter > 200) return SUPERDC_EINVAL;
    if (o->method < 0 || o->method > 2) return SUPERDC_EINVAL;
    if (o->fmm_order != FMM_P) return SUPERDC_EINVAL;
    if (o->fmm_leaf < 64 || o->fmm_leaf > 1024 || o->fmm_leaf % 64) return SUPERDC_EINVAL;
    if (o->persistent != 0 && o->persistent != 1) return SUPERDC_EINVAL;
    if (o->apply_kernel < 0 || o->apply_kernel > 2) return SUPERDC_EINVAL;
    if (o->fmm_crossover < 0) return SUPERDC_EINVAL;
    if (o->unshifted != 0 && o->unshifted != 1) return SUPERDC_EINVAL;
    if (o->interp != 0 && o->interp != 1) return SUPERDC_EINVAL;
    if (!std::isfinite(o->hss_tau) || o->hss_tau < 0.0) return SUPERDC_EINVAL;
    return SUPERDC_OK;
}

int fmm_crossover_of(const superdc_ctx *ctx, const superdc_opts &o) {
    return o.method == 1 ? 0x7fffffff
           : o.method == 2 ? 2 * o.fmm_leaf
           : o.fmm_crossover > 0 ? o.fmm_crossover
                                : ctx->fmm_crossover;
}

// persistent grid: enough single-wave workgroups to fill every CU several times
int persistent_grid(const superdc_ctx *ctx, int ntiles, int per_cu) {
    const long g = (long)ctx->num_cu * per_cu;
    return (int)std::max(1L, std::min<long>(g, ntiles));
}

const TileList *tile_list(superdc_batch *b, int chunk) {
    int slot = chunk == 64 ? 0 : chunk == 128 ? 1 : chunk == 256 ? 2 : chunk == 512 ? 3 : -1;
    if (slot < 0) return nullptr;
    TileList &l = b->lists[slot];
    if (l.nat) return &l;
    std::vector<Tile> nat, lpt;
    l.begin.resize(b->nprob + 1);
    for (int p = 0; p < b->nprob; ++p) {
        l.begin[p] = (int32_t)nat.size();
        const int64_t n = b->off_h[p + 1] - b->off_h[p];
        for (int64_t r = 0; r < n; r += chunk) nat.push_back(Tile{p, (int32_t)r});
    }
    l.begin[b->nprob] = (int32_t)nat.size();
    lpt.reserve(nat.size());
    for (int p : b->order)
        for (int32_t t = l.begin[p]; t < l.begin[p + 1]; ++t) lpt.push_back(nat[t]);
    Tile *dn = nullptr, *dl = nullptr;
    if (hipMalloc(&dn, sizeof(Tile) * nat.size()) != hipSuccess) return nullptr;
    if (hipMalloc(&dl, sizeof(Tile) * lpt.size()) != hipSuccess) {
        (void)hipFree(dn);
        return nullptr;
    }
    if (hipMemcpy(dn, nat.data(), sizeof(Tile) * nat.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dl, lpt.data(), sizeof(Tile) * lpt.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dn);
        (void)hipFree(dl);
        return nullptr;
    }
    l.nat = dn;
    l.lpt = dl;
    l.count = (int32_t)nat.size();
    return &l;
}
}  // namespace sdc

namespace {
// Launch shape for problems of the given sizes: the fewest wavefronts per work item
// (split S, a power of two <= 16) and the longest chunk (<= max_chunk) whose work items
// still give every CU 16 wavefronts, keeping >= 256 summed entries per wavefront.
// fewest poles each wavefront of a split sums
#ifndef SDC_MIN_SPLIT_POLES
#define SDC_MIN_SPLIT_POLES 128
#endif

LaunchShape shape_for(const superdc_ctx *ctx, const int64_t *sizes, int count, int max_chunk) {
    const long target = (long)ctx->num_cu * 16;
    int64_t nmax = 0;
    for (int i = 0; i < count; ++i) nmax = std::max(nmax, sizes[i]);
    for (int S = 1; S <= 16; S *= 2) {
        if (S > 1 && nmax / S < SDC_MIN_SPLIT_POLES) break;
        for (int C = max_chunk; C >= TILE; C /= 2) {
            long wg = 0;
            for (int i = 0; i < count; ++i) wg += (sizes[i] + C - 1) / C;
            if (wg * S >= target) return LaunchShape{C, S};
        }
    }
    int S = 1;
    while (S < 16 && nmax / (2 * S) >= SDC_MIN_SPLIT_POLES) S *= 2;
    return LaunchShape{TILE, S};
}

}  // namespace

namespace sdc {
LaunchShape plain_shape(const superdc_ctx *ctx, int64_t n) { return shape_for(ctx, &n, 1, TILE); }
}  // namespace sdc

namespace {
LaunchShape choose_shape(const superdc_ctx *ctx, const superdc_batch *b, int max_chunk) {
    std::vector<int64_t> sizes(b->nprob);
    for (int p = 0; p < b->nprob; ++p) sizes[p] = b->off_h[p + 1] - b->off_h[p];
    return shape_for(ctx, sizes.data(), b->nprob, max_chunk);
}

// far-field separation: a box is far from a target leaf when the gap is >= FMM_SEP times
// the box's width (Chebyshev order 16 then interpolates both kernels to ~1e-14); a source
// enters a target leaf's local expansion when its gap to the target interval is >=
// FMM_SEP_LOC times the interval's width (order 20 then interpolates a source's 1/(s - x)
// to 5e-14 relative and its derivative, which only steers the step, to 2e-12; the stopping
// test's tolerance is n eps (1 + |psi| + |phi|) >= 1.1e-13 relative for the FMM's n >= 1024)
constexpr double FMM_SEP = 1.5;
constexpr double FMM_SEP_LOC = 0.75;

int fmm_dir_slot(int chunk) { return chunk == 64 ? 0 : chunk == 128 ? 1 : chunk == 256 ? 2 : 3; }

void fmm_free(FmmPlan *fp) {
    if (!fp) return;
    for (void *p : fp->allocs) (void)hipFree(p);
    delete fp;
}

template <typename T>
bool fmm_upload(FmmPlan *fp, T **dst, const std::vector<T> &v, size_t count = 0) {
    const size_t n = std::max<size_t>(1, count ? count : v.size());
    if (hipMalloc((void **)dst, sizeof(T) * n) != hipSuccess) return false;
    fp->allocs.push_back(*dst);
    if (!v.empty() &&
        hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
        return false;
    return true;
}

// The FMM layout of a batch: which problems use it, their leaf trees, list buffers and
// work lists.  Rebuilt only when the leaf size or the crossover changes.
FmmPlan *fmm_plan(superdc_batch *b, int leaf, int crossover) {
    if (b->fmm && b->fmm->leaf == leaf && b->fmm->crossover == crossover) return b->fmm;
    (void)hipDeviceSynchronize();
    fmm_free(b->fmm);
    b->fmm = nullptr;
    FmmPlan *fp = new (std::nothrow) FmmPlan();
    if (!fp) return nullptr;
    fp->leaf = leaf;
    fp->crossover = crossover;
    fp->fmm_of_h.assign(b->nprob, -1);
    std::vector<int32_t> height, box_fmm, leaf_fmm;
    fp->box_off_h.push_back(0);
    fp->leaf_off_h.push_back(0);
    for (int p = 0; p < b->nprob; ++p) {
        const int64_t n = b->off_h[p + 1] - b->off_h[p];
        if (n < crossover || n < 2 * leaf) continue;
        const int q = fp->nfmm++;
        fp->fmm_prob_h.push_back(p);
        fp->fmm_of_h[p] = q;
        const int nl = (int)((n + leaf - 1) / leaf);
        int H = 0;
        while ((1 << H) < nl) ++H;
        height.push_back(H);
        const int nb = (2 << H) - 1;
        fp->box_off_h.push_back(fp->box_off_h.back() + nb);
        fp->leaf_off_h.push_back(fp->leaf_off_h.back() + nl);
        box_fmm.insert(box_fmm.end(), nb, q);
        leaf_fmm.insert(leaf_fmm.end(), nl, q);
    }
    fp->nboxes = fp->box_off_h.back();
    fp->nleaves = fp->leaf_off_h.back();
    // the boxes the source kernels visit, so that their grids hold no workgroup without a
    // box: every leaf (all hold poles), and every upper box with poles, largest first
    std::vector<int32_t> leaf_box, upper_box;
    std::vector<int4> upper_item;
    std::vector<int2> split_box;
    int nslot = 0;
    {
        std::vector<std::pair<int, int32_t>> up;  // (leaves below, global box id)
        for (int q = 0; q < fp->nfmm; ++q) {
            const int H = height[q];
            const int nl = fp->leaf_off_h[q + 1] - fp->leaf_off_h[q];
            const int32_t b0 = fp->box_off_h[q];
            for (int l = 0; l < nl; ++l) leaf_box.push_back(b0 + (1 << H) - 1 + l);
            for (int h = 0; h < H; ++h)
                for (int i = 0; i < (1 << h); ++i) {
                    const int first = i << (H - h);
                    if (first < nl)
                        up.emplace_back(std::min(1 << (H - h), nl - first), b0 + (1 << h) - 1 + i);
                }
        }
        std::stable_sort(up.begin(), up.end(),
                         [](const std::pair<int, int32_t> &x, const std::pair<int, int32_t> &y) {
                             return x.first > y.first;
                         });
        for (const auto &e : up) upper_box.push_back(e.second);
        for (const auto &e : up) {
            const int parts = (e.first * FMM_P + FMMV_PART_PTS - 1) / FMMV_PART_PTS;
            if (parts == 1) {
                upper_item.push_back(make_int4(e.second, 0, 1, -1));
                continue;
            }
            split_box.push_back(make_int2(e.second, nslot));
            for (int u = 0; u < parts; ++u)
                upper_item.push_back(make_int4(e.second, u, parts, nslot + u));
            nslot += parts;
        }
    }
    fp->nupper = (int)upper_box.size();
    fp->nupper_item = (int)upper_item.size();
    fp->nsplit = (int)split_box.size();
    // work items (64-root pieces of the target leaves) in problem order and longest-first
    std::vector<Tile> lnat, llpt;
    fp->item_off_h.push_back(0);
    for (int q = 0; q < fp->nfmm; ++q) {
        const int p = fp->fmm_prob_h[q];
        const int64_t n = b->off_h[p + 1] - b->off_h[p];
        for (int64_t r = 0; r < n; r += fp->sub) lnat.push_back(Tile{p, (int32_t)r});
        fp->item_off_h.push_back((int32_t)lnat.size());
    }
    fp->nitems = (int)lnat.size();
    for (int p : b->order) {
        const int q = fp->fmm_of_h[p];
        if (q < 0) continue;
        for (int t = fp->item_off_h[q]; t < fp->item_off_h[q + 1]; ++t) llpt.push_back(lnat[t]);
    }
    // wavefronts per item: enough to give the launch ~16 wavefronts per CU
    fp->split = 1;
    while (fp->split < 8 && (long)fp->nitems * fp->split * 2 <= (long)b->ctx->num_cu * 16)
        fp->split *= 2;
    // the solver's items (pieces of ssub roots that never cross a leaf)
    std::vector<Tile> snat, slpt;
    fp->ssub = leaf % (2 * TILE) == 0 ? 2 * TILE : TILE;  // divides the leaf
    fp->sitem_off_h.push_back(0);
    for (int q = 0; q < fp->nfmm; ++q) {
        const int p = fp->fmm_prob_h[q];
        const int64_t n = b->off_h[p + 1] - b->off_h[p];
        for (int64_t r = 0; r < n; r += fp->ssub) snat.push_back(Tile{p, (int32_t)r});
        fp->sitem_off_h.push_back((int32_t)snat.size());
    }
    fp->snitems = (int)snat.size();
    for (int p : b->order) {
        const int q = fp->fmm_of_h[p];
        if (q < 0) continue;
        for (int t = fp->sitem_off_h[q]; t < fp->sitem_off_h[q + 1]; ++t) slpt.push_back(snat[t]);
    }
    fp->ssplit = 1;
    while (fp->ssplit < 8 &&
           (long)fp->snitems * fp->ssplit * 2 <= (long)b->ctx->num_cu * SDC_FMM_WAVES_PER_CU)
        fp->ssplit *= 2;
    bool ok = fmm_upload(fp, &fp->fmm_prob, fp->fmm_prob_h) &&
              fmm_upload(fp, &fp->fmm_of, fp->fmm_of_h) &&
              fmm_upload(fp, &fp->box_off, fp->box_off_h) &&
              fmm_upload(fp, &fp->leaf_off, fp->leaf_off_h) && fmm_upload(fp, &fp->height, height) &&
              fmm_upload(fp, &fp->box_fmm, box_fmm) && fmm_upload(fp, &fp->leaf_fmm, leaf_fmm) &&
              fmm_upload(fp, &fp->leaf_box, leaf_box) && fmm_upload(fp, &fp->upper_box, upper_box) &&
              fmm_upload(fp, &fp->upper_item, upper_item) && fmm_upload(fp, &fp->split_box, split_box) &&
              fmm_upload(fp, &fp->vpart, std::vector<double>(),
                         (size_t)nslot * FMM_P * FMMV_MAX_M) &&
              fmm_upload(fp, &fp->leaf_nat, lnat) && fmm_upload(fp, &fp->leaf_lpt, llpt) &&
              fmm_upload(fp, &fp->sitem_nat, snat) && fmm_upload(fp, &fp->sitem_lpt, slpt) &&
              fmm_upload(fp, &fp->eq, std::vector<double2>(), (size_t)fp->nboxes * FMM_P) &&
              fmm_upload(fp, &fp->near_lo, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_NEAR_MAX) &&
              fmm_upload(fp, &fp->near_hi, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_NEAR_MAX) &&
              fmm_upload(fp, &fp->far_l, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_FAR_MAX) &&
              fmm_upload(fp, &fp->far_r, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_FAR_MAX) &&
              fmm_upload(fp, &fp->cnt, std::vector<int32_t>(), (size_t)fp->nleaves * 3) &&
              fmm_upload(fp, &fp->near_lf, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_NEAR_MAX) &&
              fmm_upload(fp, &fp->t_near_lf, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_NEAR_MAX) &&
              fmm_upload(fp, &fp->loc_ab, std::vector<double2>(), (size_t)fp->nleaves) &&
              fmm_upload(fp, &fp->far_ld, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_FAR_MAX) &&
              fmm_upload(fp, &fp->far_rd, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_FAR_MAX) &&
              fmm_upload(fp, &fp->cntd, std::vector<int32_t>(), (size_t)fp->nleaves * 2) &&
              fmm_upload(fp, &fp->loc, std::vector<double>(), (size_t)fp->nleaves * FMM_LOC) &&
              fmm_upload(fp, &fp->used, std::vector<int32_t>(), fp->nboxes) &&
              fmm_upload(fp, &fp->vnode, std::vector<double>(), (size_t)fp->nboxes * FMM_P) &&
              fmm_upload(fp, &fp->vw, std::vector<double>(),
                         (size_t)fp->nboxes * FMM_P * FMMV_MAX_M) &&
              fmm_upload(fp, &fp->tail, std::vector<double>(), b->nprob) &&
              fmm_upload(fp, &fp->lgeo, std::vector<double2>(), fp->nboxes) &&
              fmm_upload(fp, &fp->lmom, std::vector<double>(), (size_t)fp->nboxes * FMML_K) &&
              fmm_upload(fp, &fp->t_near_lo, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_NEAR_MAX) &&
              fmm_upload(fp, &fp->t_near_hi, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_NEAR_MAX) &&
              fmm_upload(fp, &fp->t_far_l, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_FAR_MAX) &&
              fmm_upload(fp, &fp->t_far_r, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_FAR_MAX) &&
              fmm_upload(fp, &fp->t_cnt, std::vector<int32_t>(), (size_t)fp->nleaves * 3) &&
              fmm_upload(fp, &fp->t_far_ld, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_FAR_MAX) &&
              fmm_upload(fp, &fp->t_far_rd, std::vector<int32_t>(), (size_t)fp->nleaves * FMM_FAR_MAX) &&
              fmm_upload(fp, &fp->t_cntd, std::vector<int32_t>(), (size_t)fp->nleaves * 2) &&
              fmm_upload(fp, &fp->t_used, std::vector<int32_t>(), fp->nboxes) &&
              fmm_upload(fp, &fp->t_loc_ab, std::vector<double2>(), (size_t)fp->nleaves);
    // direct chunks of the other problems, for each cut length
    fp->dir_lpt.assign(4, nullptr);
    fp->dir_count.assign(4, 0);
    for (int slot = 0; slot < 4 && ok; ++slot) {
        const int C = TILE << slot;
        std::vector<Tile> v;
        for (int p : b->order) {
            if (fp->fmm_of_h[p] >= 0) continue;
            const int64_t n = b->off_h[p + 1] - b->off_h[p];
            for (int64_t r = 0; r < n; r += C) v.push_back(Tile{p, (int32_t)r});
        }
        fp->dir_count[slot] = (int32_t)v.size();
        ok = fmm_upload(fp, &fp->dir_lpt[slot], v);
    }
    // the use flags start below every lists number (the first build is number 1)
    ok = ok && hipMemset(fp->used, 0, sizeof(int32_t) * std::max(1, fp->nboxes)) == hipSuccess &&
         hipMemset(fp->t_used, 0, sizeof(int32_t) * std::max(1, fp->nboxes)) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        fmm_free(fp);
        return nullptr;
    }
    b->fmm = fp;
    return fp;
}

FmmArgs fmm_args(const FmmPlan *fp, const superdc_batch *b, const SolveArgs &a,
                 const superdc_opts &o) {
    FmmArgs f{};
    f.off = b->off_d;
    f.leaf = fp->leaf;
    f.sep = FMM_SEP;
    f.sep_loc = FMM_SEP_LOC;
    f.fmm_prob = fp->fmm_prob;
    f.fmm_of = fp->fmm_of;
    f.box_off = fp->box_off;
    f.leaf_off = fp->leaf_off;
    f.height = fp->height;
    f.dw = a.dw;
    f.tail = a.z2;  // the last root lies below d_{n-1} + sum_j w_j
    f.status = a.status;
    f.used = fp->used;
    f.gen = fp->gen;
    f.eq = fp->eq;
    f.near_lo = fp->near_lo;
    f.near_hi = fp->near_hi;
    f.near_lf = fp->near_lf;
    f.far_l = fp->far_l;
    f.far_r = fp->far_r;
    f.cnt = fp->cnt;
    f.far_ld = fp->far_ld;
    f.far_rd = fp->far_rd;
    f.cntd = fp->cntd;
    f.loc_ab = fp->loc_ab;
    f.loc = fp->loc;
    f.nboxes = fp->nboxes;
    f.nleaves = fp->nleaves;
    f.box_fmm = fp->box_fmm;
    f.leaf_fmm = fp->leaf_fmm;
    f.leaf_box = fp->leaf_box;
    f.upper_box = fp->upper_box;
    f.nupper = fp->nupper;
    f.upper_item = fp->upper_item;
    f.nupper_item = fp->nupper_item;
    f.split_box = fp->split_box;
    f.nsplit = fp->nsplit;
    f.vpart = fp->vpart;
    (void)o;
    return f;
}
// The eigenvector-side FMM of one call: the list geometry comes from `pairs` (written by
// the pack kernel from this call's d) and the last roots' offsets.
FmmArgs fmm_vec_args(const FmmPlan *fp, const superdc_batch *b, const double2 *pairs,
                     const int32_t *status) {
    SolveArgs a{};
    a.dw = const_cast<double2 *>(pairs);
    a.status = const_cast<int32_t *>(status);
    superdc_opts o;
    superdc_opts_default(&o);
    FmmArgs f = fmm_args(fp, b, a, o);
    f.tail = fp->tail;
    return f;
}

// The FMM of the sums over the roots (Y = Qhat X): its own lists and use flags, the
// sources' positions in `pairs` (the roots), the targets at the poles d.
FmmArgs fmm_roots_args(const FmmPlan *fp, const superdc_batch *b, const double2 *pairs,
                       const int32_t *status, const double *d) {
    FmmArgs f = fmm_vec_args(fp, b, pairs, status);
    f.tpos = d;
    f.near_lo = fp->t_near_lo;
    f.near_hi = fp->t_near_hi;
    f.near_lf = fp->t_near_lf;
    f.far_l = fp->t_far_l;
    f.far_r = fp->t_far_r;
    f.cnt = fp->t_cnt;
    f.far_ld = fp->t_far_ld;
    f.far_rd = fp->t_far_rd;
    f.cntd = fp->t_cntd;
    f.used = fp->t_used;
    f.gen = fp->t_gen;
    f.loc_ab = fp->t_loc_ab;
    return f;
}

// the FMM plan that applies to this call, or nullptr (rc = ENOMEM on allocation failure)
FmmPlan *fmm_for(superdc_ctx *ctx, superdc_batch *b, const superdc_opts &o, int &rc) {
    rc = SUPERDC_OK;
    const int crossover = fmm_crossover_of(ctx, o);
    if (b->max_n < crossover) return nullptr;
    FmmPlan *fp = fmm_plan(b, o.fmm_leaf, crossover);
    if (!fp) {
        rc = SUPERDC_ENOMEM;
        return nullptr;
    }
    return fp->nfmm > 0 ? fp : nullptr;
}

// Run the eigenvector-side FMM over every FMM problem of the batch for columns
// [pk.c0, pk.c0 + v.m): pack the sources, build the lists (first pass only), compress the
// used boxes, evaluate at the roots (one persistent launch, or one launch per problem).
hipError_t fmmv_run(superdc_ctx *ctx, const superdc_batch *b, const FmmPlan *fp,
                    const FmmArgs &f, FmmvPackArgs pk, const FmmVec &v, bool lists,
                    bool persistent, hipStream_t s) {
    pk.tiles = fp->leaf_nat;
    pk.ntiles = fp->nitems;
    hipError_t e = hipSuccess;
    if (lists) {  // the lists need the packed positions first
        e = launch_fmmv_pack(pk, v, s);
        if (e == hipSuccess) e = launch_fmm_lists(f, s);
        if (e == hipSuccess) e = launch_fmmv_sources(f, v, nullptr, s);
    } else {  // the leaves' launch packs the sources itself
        e = launch_fmmv_sources(f, v, &pk, s);
    }
    if (e != hipSuccess) return e;
    SolveArgs it{};
    it.off = b->off_d;
    if (persistent) {
        it.tiles = fp->leaf_lpt;
        it.ntiles = fp->nitems;
        return launch_fmmv_eval(it, f, v, fp->split, ctx->queues + Q_FMMV, ctx->num_cu, s);
    }
    for (int q = 0; q < fp->nfmm && e == hipSuccess; ++q) {
        it.tiles = fp->leaf_nat + fp->item_off_h[q];
        it.ntiles = fp->item_off_h[q + 1] - fp->item_off_h[q];
        e = launch_fmmv_eval(it, f, v, fp->split, nullptr, ctx->num_cu, s);
    }
    return e;
}
}  // namespace

namespace sdc {
void *ws_get(superdc_ctx *ctx, int slot, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (ctx->ws_cap[slot] >= bytes) return ctx->ws[slot];
    if (ctx->ws[slot]) {
        if (hipDeviceSynchronize() != hipSuccess) return nullptr;
        (void)hipFree(ctx->ws[slot]);
        ctx->ws[slot] = nullptr;
        ctx->ws_cap[slot] = 0;
    }
    size_t cap = std::max(bytes, ctx->ws_cap[slot] + ctx->ws_cap[slot] / 2);
    void *p = nullptr;
    if (hipMalloc(&p, cap) != hipSuccess) return nullptr;
    ctx->ws[slot] = p;
    ctx->ws_cap[slot] = cap;
    return p;
}
}  // namespace sdc

#define SDC_OPTS(o, opts)                       \
    superdc_opts o;                             \
    if (opts) o = *(opts);                      \
    else superdc_opts_default(&o);              \
    {                                           \
        int rc_ = opts_check(&o);               \
        if (rc_) return rc_;                    \
    }

namespace sdc {
// Loewner/b and the Cauchy apply.  reuse_lists: the batch's FMM interaction lists were
// built by a solve on the same poles d and stay valid (internal callers only).
int loewner_run(superdc_ctx *ctx, const superdc_batch *b, const double *d, const double *z,
                const double *rho, const double *eta, const int32_t *origin,
                const int32_t *status, double *zhat, double *bnorm, const superdc_opts *opts,
                void *stream, bool reuse_lists, bool fmm_b) {
    if (!ctx || !b || b->ctx != ctx || !d || !z || !rho || !eta || !origin || !status || !zhat ||
        !bnorm)
        return SUPERDC_EINVAL;
    SDC_OPTS(o, opts);
    hipStream_t s = (hipStream_t)stream;
    VecArgs a{};
    a.off = b->off_d;
    a.d = d;
    a.z = z;
    a.rho = rho;
    a.eta = eta;
    a.origin = origin;
    a.status = status;
    a.ke = (double2 *)ws_get(ctx, WS_KE, sizeof(double2) * b->total);
    a.dz = (double2 *)ws_get(ctx, WS_DZ, sizeof(double2) * b->total);
    if (!a.ke || !a.dz) return SUPERDC_ENOMEM;
    a.zhat = zhat;
    a.bnorm = bnorm;
    superdc_batch *bm = const_cast<superdc_batch *>(b);
    const TileList *L = tile_list(bm, TILE);
    if (!L) return SUPERDC_ENOMEM;
    // large problems: zhat and b through the FMM (far boxes by moment expansions of the
    // Loewner log-sums and by equivalent sources for b), the others by direct products/sums
    int rc;
    FmmPlan *fp = fmm_for(ctx, bm, o, rc);
    if (rc) return rc;
    FmmvPackArgs pk{};
    FmmVec v{};
    v.trans = 1;
    FmmArgs f{};
    FmmlArgs lf{};
    if (fp) {
        double2 *pairs = (double2 *)ws_get(ctx, WS_VPAIR, sizeof(double2) * b->total);
        double *src = (double *)ws_get(ctx, WS_VSRC, sizeof(double) * b->total);
        if (!pairs || !src) return SUPERDC_ENOMEM;
        pk.off = b->off_d;
        pk.tiles = fp->leaf_nat;
        pk.ntiles = fp->nitems;
        pk.d = d;
        pk.zhat = zhat;
        pk.eta = eta;
        pk.origin = origin;
        pk.pairs = pairs;
        pk.tail = fp->tail;
        // every problem uses the FMM: the Loewner packing writes ke as well
        pk.ke = fp->nfmm == b->nprob ? a.ke : nullptr;
        v.m = 1;
        v.kern = 2;
        v.src = src;
        v.vnode = fp->vnode;
        v.vw = fp->vw;
        v.d = d;
        v.origin = origin;
        v.eta = eta;
        v.bout = bnorm;
        v.zh = zhat;
        f = fmm_vec_args(fp, b, pairs, status);
        lf.pd = pairs;
        lf.geo = fp->lgeo;
        lf.mom = fp->lmom;
        // (d_j, delta_j) pairs, the lists of these poles (unless the solve left them), the
        // Loewner moments of every leaf and used box; with the lists left by the solve the
        // leaves' launch packs the pairs itself
        if (!reuse_lists) {
            SDC_HIP(launch_fmml_pack(pk, s));
            f.gen = ++fp->gen;
            SDC_HIP(launch_fmm_lists(f, s));
        } else {
            lf.pack = 1;
            lf.d = d;
            lf.eta = eta;
            lf.origin = origin;
            lf.ke = pk.ke;
            lf.tail = fp->tail;
        }
        SDC_HIP(launch_fmml_moments(f, lf, s));
    }
    a.tiles = L->lpt;
    a.ntiles = L->count;
    if (!pk.ke) SDC_HIP(launch_pack_ke(a, s));
    if (o.persistent) {
        const int S = b->vec.split;
        if (fp) {
            a.tiles = fp->dir_lpt[0];
            a.ntiles = fp->dir_count[0];
        }
        SDC_HIP(launch_loewner(a, S, ctx->queues + Q_LOEWNER,
                               persistent_grid(ctx, a.ntiles, std::max(1, 32 / S)), s, false));
        if (fp) {
            VecArgs af = a;
            af.tiles = fp->leaf_lpt;
            af.ntiles = fp->nitems;
            SDC_HIP(launch_loewner_fmm(af, f, lf, fp->split, ctx->queues + Q_LOEWNER,
                                       persistent_grid(ctx, af.ntiles, std::max(1, 32 / fp->split)),
                                       s));
        }
        if (fmm_b)
            SDC_HIP(launch_bnorm(a, S, ctx->queues + Q_BNORM,
                                 persistent_grid(ctx, a.ntiles, std::max(1, 32 / S)), s));
        if (fp && fmm_b) SDC_HIP(fmmv_run(ctx, b, fp, f, pk, v, false, true, s));
    } else {
        for (int p = 0; p < b->nprob; ++p) {
            const int64_t np = b->off_h[p + 1] - b->off_h[p];
            const int S = shape_for(ctx, &np, 1, TILE).split;
            if (fp && fp->fmm_of_h[p] >= 0) {
                const int q = fp->fmm_of_h[p];
                VecArgs af = a;
                af.tiles = fp->leaf_nat + fp->item_off_h[q];
                af.ntiles = fp->item_off_h[q + 1] - fp->item_off_h[q];
                SDC_HIP(launch_loewner_fmm(af, f, lf, fp->split, nullptr, 0, s));
                continue;
            }
            a.tiles = L->nat + L->begin[p];
            a.ntiles = L->begin[p + 1] - L->begin[p];
            SDC_HIP(launch_loewner(a, S, nullptr, 0, s, false));
            if (fmm_b) SDC_HIP(launch_bnorm(a, S, nullptr, 0, s));
        }
        if (fp && fmm_b) SDC_HIP(fmmv_run(ctx, b, fp, f, pk, v, false, false, s));
    }
    return SUPERDC_OK;
}

int apply_run(superdc_ctx *ctx, const superdc_batch *b, const double *d, const double *zhat,
              const double *bnorm, const double *eta, const int32_t *origin,
              const int32_t *status, int trans, int32_t m, const double *X, int64_t ldx,
              double *Y, int64_t ldy, const superdc_opts *opts, void *stream, bool reuse_lists,
              bool fuse_b) {
    if (!ctx || !b || b->ctx != ctx || !d || !zhat || !bnorm || !eta || !origin || !status ||
        !X || !Y)
        return SUPERDC_EINVAL;
    if (fuse_b && (trans != 1 || m + 1 > FMMV_MAX_M)) return SUPERDC_EINVAL;
    if ((trans != 0 && trans != 1) || m < 1 || ldx < b->total || ldy < b->total)
        return SUPERDC_EINVAL;
    SDC_OPTS(o, opts);
    // X and Y must not overlap
    const char *x0 = (const char *)X, *x1 = (const char *)(X + (ldx * (m - 1) + b->total));
    const char *y0 = (const char *)Y, *y1 = (const char *)(Y + (ldy * (m - 1) + b->total));
    if (x0 < y1 && y0 < x1) return SUPERDC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    ApplyArgs a{};
    a.off = b->off_d;
    a.d = d;
    a.zhat = zhat;
    a.bnorm = bnorm;
    a.eta = eta;
    a.origin = origin;
    a.status = status;
    a.trans = trans;
    a.m = m;
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.ldy = ldy;
    a.fuse_b = fuse_b ? 1 : 0;
    a.bout = const_cast<double *>(bnorm);  // written only with fuse_b
    const int use_mfma =
        fuse_b ? 1 : (o.apply_kernel == 2 ? 1 : (o.apply_kernel == 1 ? 0 : (m >= 4)));
    superdc_batch *bm = const_cast<superdc_batch *>(b);
    const TileList *L = tile_list(bm, TILE);
    if (!L) return SUPERDC_ENOMEM;
    // Y = Qhat^T X of the large problems by the eigenvector-side FMM (the sums run over the
    // poles for every root, the layout of the solver's lists), Y = Qhat X by the FMM of the
    // sums over the roots (sources at the roots, targets at the poles, lists of their own);
    // the other problems by the direct kernels
    int rc;
    FmmPlan *fp = fmm_for(ctx, bm, o, rc);
    if (rc) return rc;
    if (o.persistent) {
        a.tiles = fp ? fp->dir_lpt[0] : L->lpt;
        a.ntiles = fp ? fp->dir_count[0] : L->count;
        SDC_HIP(launch_apply(a, use_mfma, ctx->queues + Q_APPLY,
                             persistent_grid(ctx, a.ntiles, use_mfma ? 4 : 8), s));
    } else {
        for (int p = 0; p < b->nprob; ++p) {
            if (fp && fp->fmm_of_h[p] >= 0) continue;
            a.tiles = L->nat + L->begin[p];
            a.ntiles = L->begin[p + 1] - L->begin[p];
            SDC_HIP(launch_apply(a, use_mfma, nullptr, 0, s));
        }
    }
    if (fp && trans == 0) {
        const int mc = std::min(m, FMMV_MAX_M);
        double2 *pairs = (double2 *)ws_get(ctx, WS_VPAIR, sizeof(double2) * b->total);
        double *src = (double *)ws_get(ctx, WS_VSRC, sizeof(double) * b->total * mc);
        if (!pairs || !src) return SUPERDC_ENOMEM;
        FmmvPackArgs pk{};
        pk.off = b->off_d;
        pk.d = d;
        pk.zhat = zhat;
        pk.bnorm = bnorm;
        pk.eta = eta;
        pk.origin = origin;
        pk.X = X;
        pk.ldx = ldx;
        pk.pairs = pairs;
        pk.tail = fp->tail;
        FmmVec v{};
        v.trans = 0;
        v.kern = 1;
        v.src = src;
        v.vnode = fp->vnode;
        v.vw = fp->vw;
        v.d = d;
        v.origin = origin;
        v.eta = eta;
        v.post = zhat;
        v.ldy = ldy;
        v.zh = zhat;
        FmmArgs f = fmm_roots_args(fp, b, pairs, status, d);
        f.gen = ++fp->t_gen;  // built with the first columns below
        for (int c0 = 0; c0 < m; c0 += FMMV_MAX_M) {
            pk.c0 = c0;
            v.m = std::min(FMMV_MAX_M, m - c0);
            v.Y = Y + (int64_t)c0 * ldy;
            // the lists depend on the roots' positions, packed with the first columns
            SDC_HIP(fmmv_run(ctx, b, fp, f, pk, v, c0 == 0, o.persistent != 0, s));
        }
    } else if (fp) {
        const int mc = std::min(m + (fuse_b ? 1 : 0), FMMV_MAX_M);
        double2 *pairs = (double2 *)ws_get(ctx, WS_VPAIR, sizeof(double2) * b->total);
        double *src = (double *)ws_get(ctx, WS_VSRC, sizeof(double) * b->total * mc);
        if (!pairs || !src) return SUPERDC_ENOMEM;
        FmmvPackArgs pk{};
        pk.off = b->off_d;
        pk.d = d;
        pk.zhat = zhat;
        pk.eta = eta;
        pk.origin = origin;
        pk.X = X;
        pk.ldx = ldx;
        pk.pairs = pairs;
        pk.tail = fp->tail;
        FmmVec v{};
        v.trans = 1;
        v.kern = 1;
        v.src = src;
        v.vnode = fp->vnode;
        v.vw = fp->vw;
        v.d = d;
        v.origin = origin;
        v.eta = eta;
        v.post = bnorm;
        v.ldy = ldy;
        v.fuse_b = fuse_b ? 1 : 0;
        v.zh = zhat;
        v.bout = const_cast<double *>(bnorm);  // written only with fuse_b
        FmmArgs f = fmm_vec_args(fp, b, pairs, status);
        if (!reuse_lists) f.gen = ++fp->gen;  // built with the first columns below
        for (int c0 = 0; c0 < m; c0 += FMMV_MAX_M) {
            pk.c0 = c0;
            v.m = std::min(FMMV_MAX_M, m - c0) + v.fuse_b;  // one chunk when fused
            v.Y = Y + (int64_t)c0 * ldy;
            SDC_HIP(fmmv_run(ctx, b, fp, f, pk, v, c0 == 0 && !reuse_lists, o.persistent != 0, s));
        }
    }
    return SUPERDC_OK;
}

}  // namespace sdc

extern "C" {

void superdc_opts_default(superdc_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->stop_c = 1.0;
    o->max_iter = 40;
    o->method = 0;
    o->fmm_order = 16;
    o->fmm_leaf = 64;
    o->persistent = 1;
    o->apply_kernel = 0;
}

const char *superdc_strerror(int code) {
    switch (code) {
        case SUPERDC_OK: return "success";
        case SUPERDC_EINVAL: return "invalid argument";
        case SUPERDC_ENOMEM: return "device allocation failed";
        case SUPERDC_EHIP: return "HIP runtime error";
        case SUPERDC_ENODEV: return "no gfx950 device";
        default: return "unknown error";
    }
}

int superdc_last_hip_error(void) { return g_last_hip_error; }

int superdc_create(superdc_ctx **out) {
    if (!out) return SUPERDC_EINVAL;
    *out = nullptr;
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return SUPERDC_ENODEV;
    SDC_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SDC_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SUPERDC_ENODEV;
    superdc_ctx *ctx = new (std::nothrow) superdc_ctx();
    if (!ctx) return SUPERDC_ENOMEM;
    ctx->device = dev;
    ctx->num_cu = prop.multiProcessorCount;
    {
        const int rc = noalloc_init(dev);
        if (rc != SUPERDC_OK) {
            delete ctx;
            return rc;
        }
    }
    hipError_t e = hipMalloc(&ctx->queues, sizeof(Queue) * kNumQueues);
    if (e == hipSuccess) e = hipMemset(ctx->queues, 0, sizeof(Queue) * kNumQueues);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (ctx->queues) (void)hipFree(ctx->queues);
        delete ctx;
        return hip_fail(e);
    }
    *out = ctx;
    return SUPERDC_OK;
}

void superdc_destroy(superdc_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    for (int i = 0; i < kNumWs; ++i)
        if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
    if (ctx->queues) (void)hipFree(ctx->queues);
    delete ctx;
}

int superdc_batch_create(superdc_ctx *ctx, int32_t nprob, const int64_t *off_host,
                         superdc_batch **out) {
    if (!ctx || !off_host || !out || nprob < 1) return SUPERDC_EINVAL;
    *out = nullptr;
    if (off_host[0] != 0) return SUPERDC_EINVAL;
    int32_t max_n = 0;
    for (int p = 0; p < nprob; ++p) {
        const int64_t n = off_host[p + 1] - off_host[p];
        if (n < 1 || n > (int64_t)1 << 30) return SUPERDC_EINVAL;
        max_n = std::max<int32_t>(max_n, (int32_t)n);
    }
    superdc_batch *b = new (std::nothrow) superdc_batch();
    if (!b) return SUPERDC_ENOMEM;
    b->ctx = ctx;
    b->nprob = nprob;
    b->total = off_host[nprob];
    b->max_n = max_n;
    b->off_h.assign(off_host, off_host + nprob + 1);
    b->order.resize(nprob);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return off_host[x + 1] - off_host[x] > off_host[y + 1] - off_host[y];
    });
    hipError_t e = hipMalloc(&b->off_d, sizeof(int64_t) * (nprob + 1));
    if (e == hipSuccess)
        e = hipMemcpy(b->off_d, off_host, sizeof(int64_t) * (nprob + 1), hipMemcpyHostToDevice);
    // problems of 16384 entries and more are validated in slices of about 4096
    b->vsplit = max_n >= 16384 ? std::min(16, max_n / 4096) : 1;
    if (e == hipSuccess && b->vsplit > 1) {
        e = hipMalloc(&b->vsum, sizeof(double) * nprob * b->vsplit);
        if (e == hipSuccess) e = hipMalloc(&b->vst, sizeof(int32_t) * nprob * b->vsplit);
    }
    if (e == hipSuccess && !tile_list(b, TILE)) e = hipErrorOutOfMemory;
    if (e != hipSuccess) {
        superdc_batch_destroy(b);
        return hip_fail(e);
    }
    // launch shapes for the persistent launches (the autotuner may replace them)
    b->sec = choose_shape(ctx, b, SEC_CHUNK);
    // the solver's tile list for that shape is built now, so that a later solve (the
    // allocation-free entry point in particular) finds it ready
    if (!tile_list(b, b->sec.chunk)) {
        superdc_batch_destroy(b);
        return hip_fail(hipErrorOutOfMemory);
    }
    b->vec = choose_shape(ctx, b, TILE);
    b->bwd = b->vec;
    b->app = LaunchShape{TILE, 1};
    *out = b;
    return SUPERDC_OK;
}

void superdc_batch_destroy(superdc_batch *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->off_d) (void)hipFree(b->off_d);
    if (b->vsum) (void)hipFree(b->vsum);
    if (b->vst) (void)hipFree(b->vst);
    fmm_free(b->fmm);
    for (auto &l : b->lists) {
        if (l.nat) (void)hipFree(l.nat);
        if (l.lpt) (void)hipFree(l.lpt);
    }
    delete b;
}

int64_t superdc_batch_total(const superdc_batch *b) { return b ? b->total : -1; }

int superdc_secular_solve(superdc_ctx *ctx, const superdc_batch *b, const double *d,
                          const double *z, const double *rho, double *lam, double *eta,
                          int32_t *origin, int32_t *iters, int32_t *status,
                          const superdc_opts *opts, void *stream) {
    if (!ctx || !b || b->ctx != ctx || !d || !z || !rho || !lam || !eta || !origin || !status)
        return SUPERDC_EINVAL;
    SDC_OPTS(o, opts);
    hipStream_t s = (hipStream_t)stream;
    SolveArgs a{};
    a.off = b->off_d;
    a.d = d;
    a.z = z;
    a.rho = rho;
    a.dw = (double2 *)ws_get(ctx, WS_DW, sizeof(double2) * b->total);
    a.z2 = (double *)ws_get(ctx, WS_Z2, sizeof(double) * b->nprob);
    a.ke = (double2 *)ws_get(ctx, WS_KE, sizeof(double2) * b->total);
    if (!a.dw || !a.z2 || !a.ke) return SUPERDC_ENOMEM;
    a.lam = lam;
    a.eta = eta;
    a.origin = origin;
    a.iters = iters;
    a.status = status;
    a.stop_c = o.stop_c;
    a.max_iter = o.max_iter;
    a.unshifted = o.unshifted;
    a.hybrid = o.interp;
    superdc_batch *bm = const_cast<superdc_batch *>(b);
    // problems at or above the crossover size use the triangular FMM (method 2: every
    // problem large enough to have two leaves; method 1: none)
    const int crossover = fmm_crossover_of(ctx, o);
    FmmPlan *fp = nullptr;
    if (b->max_n >= crossover) {
        fp = fmm_plan(bm, o.fmm_leaf, crossover);
        if (!fp) return SUPERDC_ENOMEM;
        if (fp->nfmm == 0) fp = nullptr;
    }
    FmmArgs f{};
    if (fp) {
        f = fmm_args(fp, b, a, o);
        f.gen = ++fp->gen;  // the lists this solve builds
    }
    if (o.persistent) {
        // one persistent launch over the chunks of the direct problems, longest first,
        // and one over the target leaves of the FMM problems
        const LaunchShape sh = b->sec;
        const TileList *L = tile_list(bm, sh.chunk);
        if (!L) return SUPERDC_ENOMEM;
        a.tiles = L->lpt;
        a.ntiles = L->count;
        a.chunk = sh.chunk;
        if (fp) {
            const int slot = fmm_dir_slot(sh.chunk);
            a.tiles = fp->dir_lpt[slot];
            a.ntiles = fp->dir_count[slot];
        }
        SDC_HIP(launch_validate(a, 0, b->nprob, b->max_n, s, b->vsplit, b->vsum, b->vst));
        if (fp) SDC_HIP(launch_fmm_build(f, s));
        a.work = trace_work(KID_SECULAR);
        SDC_HIP(launch_secular(a, sh.split, ctx->queues + Q_SECULAR,
                               persistent_grid(ctx, a.ntiles, std::max(1, 32 / sh.split)), s));
        if (fp) {
            SolveArgs af = a;
            af.tiles = fp->sitem_lpt;
            af.ntiles = fp->snitems;
            af.chunk = fp->ssub;
            af.work = trace_work(KID_SECULAR_FMM);
            const int ss = b->fmm_ssplit > 0 ? b->fmm_ssplit : fp->ssplit;  // tuned or heuristic
            SDC_HIP(launch_secular_fmm(af, f, ss, ctx->queues + Q_SECULAR_FMM,
                                       persistent_grid(ctx, af.ntiles, std::max(1, 32 / ss)), s));
        }
    } else {
        // one launch per problem, cut into 64-root chunks (split if the problem is large),
        // or its target leaves for an FMM problem
        if (fp) {
            SDC_HIP(launch_validate(a, 0, b->nprob, b->max_n, s, b->vsplit, b->vsum, b->vst));
            SDC_HIP(launch_fmm_build(f, s));
        }
        for (int p = 0; p < b->nprob; ++p) {
            const int64_t np = b->off_h[p + 1] - b->off_h[p];
            if (!fp) SDC_HIP(launch_validate(a, p, 1, (int)np, s));
            if (fp && fp->fmm_of_h[p] >= 0) {
                const int q = fp->fmm_of_h[p];
                SolveArgs af = a;
                af.tiles = fp->sitem_nat + fp->sitem_off_h[q];
                af.ntiles = fp->sitem_off_h[q + 1] - fp->sitem_off_h[q];
                af.chunk = fp->ssub;
                af.work = trace_work(KID_SECULAR_FMM);
                SDC_HIP(launch_secular_fmm(af, f, fp->ssplit, nullptr, 0, s));
                continue;
            }
            const LaunchShape sh = shape_for(ctx, &np, 1, TILE);
            const TileList *L = tile_list(bm, sh.chunk);
            if (!L) return SUPERDC_ENOMEM;
            a.tiles = L->nat + L->begin[p];
            a.ntiles = L->begin[p + 1] - L->begin[p];
            a.chunk = sh.chunk;
            a.work = trace_work(KID_SECULAR);
            SDC_HIP(launch_secular(a, sh.split, nullptr, 0, s));
        }
    }
    return SUPERDC_OK;
}

int superdc_loewner(superdc_ctx *ctx, const superdc_batch *b, const double *d, const double *z,
                    const double *rho, const double *eta, const int32_t *origin,
                    const int32_t *status, double *zhat, double *bnorm,
                    const superdc_opts *opts, void *stream) {
    return loewner_run(ctx, b, d, z, rho, eta, origin, status, zhat, bnorm, opts, stream, false);
}

int superdc_cauchy_apply(superdc_ctx *ctx, const superdc_batch *b, const double *d,
                         const double *zhat, const double *bnorm, const double *eta,
                         const int32_t *origin, const int32_t *status, int trans, int32_t m,
                         const double *X, int64_t ldx, double *Y, int64_t ldy,
                         const superdc_opts *opts, void *stream) {
    return apply_run(ctx, b, d, zhat, bnorm, eta, origin, status, trans, m, X, ldx, Y, ldy, opts,
                     stream, false);
}

int superdc_secular_backward(superdc_ctx *ctx, const superdc_batch *b, const double *d,
                             const double *z, const double *rho, const double *eta,
                             const int32_t *origin, const int32_t *status,
                             const double *g_lam, const double *g_proj, const double *u,
                             double *g_d, double *g_z, double *g_rho,
                             const superdc_opts *opts, void *stream) {
    if (!ctx || !b || b->ctx != ctx || !d || !z || !rho || !eta || !origin || !status || !g_d ||
        !g_z || !g_rho)
        return SUPERDC_EINVAL;
    if ((g_proj == nullptr) != (u == nullptr)) return SUPERDC_EINVAL;
    SDC_OPTS(o, opts);
    hipStream_t s = (hipStream_t)stream;
    BwdArgs a{};
    a.off = b->off_d;
    a.nprob = b->nprob;
    a.d = d;
    a.z = z;
    a.rho = rho;
    a.eta = eta;
    a.origin = origin;
    a.status = status;
    a.g_lam = g_lam;
    a.g_proj = g_proj;
    a.u = u;
    a.g_d = g_d;
    a.g_z = g_z;
    a.g_rho = g_rho;
    a.rk = (double4 *)ws_get(ctx, WS_BK, sizeof(double4) * b->total);
    a.gk = (double *)ws_get(ctx, WS_BP, sizeof(double) * b->total);
    if (!a.rk || !a.gk) return SUPERDC_ENOMEM;
    superdc_batch *bm = const_cast<superdc_batch *>(b);
    const TileList *L = tile_list(bm, TILE);
    if (!L) return SUPERDC_ENOMEM;
    if (o.persistent) {
        a.tiles = L->lpt;
        a.ntiles = L->count;
        const int S = b->bwd.split;
        SDC_HIP(launch_backward(a, S, 0, b->nprob, ctx->queues + Q_BWD1, ctx->queues + Q_BWD2,
                                persistent_grid(ctx, L->count, std::max(1, 32 / S)), s));
    } else {
        for (int p = 0; p < b->nprob; ++p) {
            const int64_t np = b->off_h[p + 1] - b->off_h[p];
            const int S = shape_for(ctx, &np, 1, TILE).split;
            a.tiles = L->nat + L->begin[p];
            a.ntiles = L->begin[p + 1] - L->begin[p];
            SDC_HIP(launch_backward(a, S, p, 1, nullptr, nullptr, 0, s));
        }
    }
    return SUPERDC_OK;
}

}  // extern "C"
