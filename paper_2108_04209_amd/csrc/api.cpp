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

int opts_check(const superdc_opts *o) {
    if (!(o->stop_c > 0.0) || o->max_iter < 1 || o->max_iter > 200) return SUPERDC_EINVAL;
    if (o->method < 0 || o->method > 2) return SUPERDC_EINVAL;
    if (o->fmm_order < 4 || o->fmm_order > 32) return SUPERDC_EINVAL;
    if (o->fmm_leaf < 64 || o->fmm_leaf % 64) return SUPERDC_EINVAL;
    if (o->persistent != 0 && o->persistent != 1) return SUPERDC_EINVAL;
    if (o->apply_kernel < 0 || o->apply_kernel > 2) return SUPERDC_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (o->reserved[i] != 0) return SUPERDC_EINVAL;
    return SUPERDC_OK;
}

// persistent grid: enough single-wave workgroups to fill every CU several times
int persistent_grid(const superdc_ctx *ctx, int ntiles, int per_cu) {
    const long g = (long)ctx->num_cu * per_cu;
    return (int)std::max(1L, std::min<long>(g, ntiles));
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

extern "C" {

void superdc_opts_default(superdc_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->stop_c = 1.0;
    o->max_iter = 40;
    o->method = 0;
    o->fmm_order = 16;
    o->fmm_leaf = 256;
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
    for (int i = 0; i < 8; ++i)
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
    // work items in problem order (plain launches) and longest-problem-first (persistent
    // launches): tiles of TILE entries, and the secular solver's chunks of SEC_CHUNK roots
    std::vector<int> order(nprob);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return off_host[x + 1] - off_host[x] > off_host[y + 1] - off_host[y];
    });
    auto cut = [&](int step, std::vector<Tile> &nat, std::vector<Tile> &lpt,
                   std::vector<int32_t> &begin) {
        begin.resize(nprob + 1);
        for (int p = 0; p < nprob; ++p) {
            begin[p] = (int32_t)nat.size();
            const int64_t n = off_host[p + 1] - off_host[p];
            for (int64_t r = 0; r < n; r += step) nat.push_back(Tile{p, (int32_t)r});
        }
        begin[nprob] = (int32_t)nat.size();
        lpt.reserve(nat.size());
        for (int p : order)
            for (int32_t t = begin[p]; t < begin[p + 1]; ++t) lpt.push_back(nat[t]);
    };
    std::vector<Tile> nat, lpt, cnat, clpt;
    cut(TILE, nat, lpt, b->tile_begin);
    cut(SEC_CHUNK, cnat, clpt, b->chunk_begin);
    b->ntiles = (int32_t)nat.size();
    b->nchunks = (int32_t)cnat.size();
    auto upload = [](Tile **dst, const std::vector<Tile> &v) {
        hipError_t e = hipMalloc(dst, sizeof(Tile) * v.size());
        if (e == hipSuccess)
            e = hipMemcpy(*dst, v.data(), sizeof(Tile) * v.size(), hipMemcpyHostToDevice);
        return e;
    };
    hipError_t e = hipMalloc(&b->off_d, sizeof(int64_t) * (nprob + 1));
    if (e == hipSuccess)
        e = hipMemcpy(b->off_d, off_host, sizeof(int64_t) * (nprob + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = upload(&b->tiles_nat, nat);
    if (e == hipSuccess) e = upload(&b->tiles_lpt, lpt);
    if (e == hipSuccess) e = upload(&b->chunks_nat, cnat);
    if (e == hipSuccess) e = upload(&b->chunks_lpt, clpt);
    if (e != hipSuccess) {
        superdc_batch_destroy(b);
        return hip_fail(e);
    }
    *out = b;
    return SUPERDC_OK;
}

void superdc_batch_destroy(superdc_batch *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->off_d) (void)hipFree(b->off_d);
    if (b->tiles_nat) (void)hipFree(b->tiles_nat);
    if (b->tiles_lpt) (void)hipFree(b->tiles_lpt);
    if (b->chunks_nat) (void)hipFree(b->chunks_nat);
    if (b->chunks_lpt) (void)hipFree(b->chunks_lpt);
    delete b;
}

int64_t superdc_batch_total(const superdc_batch *b) { return b ? b->total : -1; }

#define SDC_OPTS(o, opts)                       \
    superdc_opts o;                             \
    if (opts) o = *(opts);                      \
    else superdc_opts_default(&o);              \
    {                                           \
        int rc_ = opts_check(&o);               \
        if (rc_) return rc_;                    \
    }

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
    if (o.persistent) {
        // one persistent launch over chunks of SEC_CHUNK roots, longest problems first
        a.tiles = b->chunks_lpt;
        a.ntiles = b->nchunks;
        a.chunk = SEC_CHUNK;
        SDC_HIP(launch_validate(a, 0, b->nprob, s));
        SDC_HIP(launch_secular(a, ctx->queues + Q_SECULAR, persistent_grid(ctx, b->nchunks, 24), s));
    } else {
        // one launch per problem, cut into 64-root chunks so each launch spreads its
        // problem over as many wavefronts as it can
        a.chunk = TILE;
        for (int p = 0; p < b->nprob; ++p) {
            a.tiles = b->tiles_nat + b->tile_begin[p];
            a.ntiles = b->tile_begin[p + 1] - b->tile_begin[p];
            SDC_HIP(launch_validate(a, p, 1, s));
            SDC_HIP(launch_secular(a, nullptr, 0, s));
        }
    }
    return SUPERDC_OK;
}

int superdc_loewner(superdc_ctx *ctx, const superdc_batch *b, const double *d, const double *z,
                    const double *rho, const double *eta, const int32_t *origin,
                    const int32_t *status, double *zhat, double *bnorm,
                    const superdc_opts *opts, void *stream) {
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
    if (o.persistent) {
        a.tiles = b->tiles_lpt;
        a.ntiles = b->ntiles;
        const int g = persistent_grid(ctx, b->ntiles, 32);
        SDC_HIP(launch_loewner(a, ctx->queues + Q_LOEWNER, g, s));
        SDC_HIP(launch_bnorm(a, ctx->queues + Q_BNORM, g, s));
    } else {
        for (int p = 0; p < b->nprob; ++p) {
            a.tiles = b->tiles_nat + b->tile_begin[p];
            a.ntiles = b->tile_begin[p + 1] - b->tile_begin[p];
            SDC_HIP(launch_loewner(a, nullptr, 0, s));
            SDC_HIP(launch_bnorm(a, nullptr, 0, s));
        }
    }
    return SUPERDC_OK;
}

int superdc_cauchy_apply(superdc_ctx *ctx, const superdc_batch *b, const double *d,
                         const double *zhat, const double *bnorm, const double *eta,
                         const int32_t *origin, const int32_t *status, int trans, int32_t m,
                         const double *X, int64_t ldx, double *Y, int64_t ldy,
                         const superdc_opts *opts, void *stream) {
    if (!ctx || !b || b->ctx != ctx || !d || !zhat || !bnorm || !eta || !origin || !status ||
        !X || !Y)
        return SUPERDC_EINVAL;
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
    const int use_mfma = o.apply_kernel == 2 ? 1 : (o.apply_kernel == 1 ? 0 : (m >= 4));
    if (o.persistent) {
        a.tiles = b->tiles_lpt;
        a.ntiles = b->ntiles;
        SDC_HIP(launch_apply(a, use_mfma, ctx->queues + Q_APPLY,
                             persistent_grid(ctx, b->ntiles, use_mfma ? 4 : 32), s));
    } else {
        for (int p = 0; p < b->nprob; ++p) {
            a.tiles = b->tiles_nat + b->tile_begin[p];
            a.ntiles = b->tile_begin[p + 1] - b->tile_begin[p];
            SDC_HIP(launch_apply(a, use_mfma, nullptr, 0, s));
        }
    }
    return SUPERDC_OK;
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
    if (o.persistent) {
        a.tiles = b->tiles_lpt;
        a.ntiles = b->ntiles;
        SDC_HIP(launch_backward(a, 0, b->nprob, ctx->queues + Q_BWD1, ctx->queues + Q_BWD2,
                                persistent_grid(ctx, b->ntiles, 32), s));
    } else {
        for (int p = 0; p < b->nprob; ++p) {
            a.tiles = b->tiles_nat + b->tile_begin[p];
            a.ntiles = b->tile_begin[p + 1] - b->tile_begin[p];
            SDC_HIP(launch_backward(a, p, 1, nullptr, nullptr, 0, s));
        }
    }
    return SUPERDC_OK;
}

}  // extern "C"
