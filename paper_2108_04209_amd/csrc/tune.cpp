// tune.cpp -- autotuner for the launch shapes of a batch.
//
// For the secular solver the candidates are the chunk length (64..512 roots per work
// item) times the split (1..16 wavefronts per item sharing the pole range), and for the
// problems that use the triangular FMM the split of its work items (1..8); for the
// Loewner/b and adjoint kernels the split.  Each candidate is run on the caller's data
// and timed with HIP events on the caller's stream; the fastest is kept in the batch.
// Results can be kept across processes in a text cache (environment variable
// SUPERDC_TUNE_CACHE), one line per batch signature.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

using namespace sdc;

namespace {

uint64_t signature(const superdc_batch *b, int num_cu) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the sizes and the CU count
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)num_cu);
    for (int p = 0; p < b->nprob; ++p) mix((uint64_t)(b->off_h[p + 1] - b->off_h[p]));
    return h;
}

// one line per batch: "<key> <chunk> <split> <loewner split> <adjoint split> <fmm split>"
// (fmm split 0: the heuristic); lines in any other form are skipped
bool cache_load(superdc_batch *b, uint64_t key) {
    const char *path = std::getenv("SUPERDC_TUNE_CACHE");
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long k;
        int sc, ss, vs, bs, fs;
        if (std::sscanf(line, "%llx %d %d %d %d %d", &k, &sc, &ss, &vs, &bs, &fs) != 6) continue;
        if (k == key && sc >= 64 && sc <= 512 && ss >= 1 && ss <= 16 && vs >= 1 && vs <= 16 &&
            bs >= 1 && bs <= 16 && fs >= 0 && fs <= 8) {
            b->sec = LaunchShape{sc, ss};
            b->vec = LaunchShape{TILE, vs};
            b->bwd = LaunchShape{TILE, bs};
            b->fmm_ssplit = fs;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const superdc_batch *b, uint64_t key) {
    const char *path = std::getenv("SUPERDC_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%llx %d %d %d %d %d\n", (unsigned long long)key, b->sec.chunk, b->sec.split,
                 b->vec.split, b->bwd.split, b->fmm_ssplit);
    std::fclose(f);
}

// median-free timing: best of `reps` runs after one warm-up
template <typename F>
float time_best(F &&run, hipStream_t s, int reps, bool &ok) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        ok = false;
        return 0.f;
    }
    float best = 1e30f;
    ok = run() == SUPERDC_OK;
    for (int i = 0; i < reps && ok; ++i) {
        (void)hipEventRecord(e0, s);
        ok = run() == SUPERDC_OK;
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) ok = false;
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        best = std::min(best, t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

}  // namespace

extern "C" {

int superdc_autotune(superdc_ctx *ctx, superdc_batch *b, const double *d, const double *z,
                     const double *rho, const superdc_opts *opts, void *stream) {
    if (!ctx || !b || b->ctx != ctx || !d || !z || !rho) return SUPERDC_EINVAL;
    const uint64_t key = signature(b, ctx->num_cu);
    if (cache_load(b, key)) {
        b->tuned = true;
        return SUPERDC_OK;
    }
    superdc_opts o;
    if (opts) o = *opts;
    else superdc_opts_default(&o);
    o.persistent = 1;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = b->total;
    // scratch outputs
    double *lam = nullptr, *eta = nullptr, *zh = nullptr, *bn = nullptr, *gd = nullptr,
           *gz = nullptr, *gr = nullptr;
    int32_t *org = nullptr, *st = nullptr;
    hipError_t e = hipMalloc(&lam, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&eta, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&zh, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&bn, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&gd, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&gz, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&gr, sizeof(double) * b->nprob);
    if (e == hipSuccess) e = hipMalloc(&org, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMalloc(&st, sizeof(int32_t) * b->nprob);
    int rc = e == hipSuccess ? SUPERDC_OK : SUPERDC_ENOMEM;
    const int reps = 2;
    if (rc == SUPERDC_OK) {
        // secular solver: chunk x split
        float best = 1e30f;
        LaunchShape bs = b->sec;
        for (int S = 1; S <= 16; S *= 2) {
            if (S > 1 && b->max_n / S < 128) break;
            for (int C = 512; C >= TILE; C /= 2) {
                long wg = 0;
                for (int p = 0; p < b->nprob; ++p) wg += (b->off_h[p + 1] - b->off_h[p] + C - 1) / C;
                if (wg * S < (long)ctx->num_cu * 2) continue;  // far too few wavefronts
                b->sec = LaunchShape{C, S};
                bool ok = true;
                const float t = time_best([&] {
                    return superdc_secular_solve(ctx, b, d, z, rho, lam, eta, org, nullptr, st,
                                                 &o, stream);
                }, s, reps, ok);
                if (ok && t < best) {
                    best = t;
                    bs = b->sec;
                }
            }
        }
        b->sec = bs;
        // the FMM solver's split, when some problem of the batch uses the FMM
        if (b->max_n >= fmm_crossover_of(ctx, o)) {
            float bestf = 1e30f;
            int bf = 0;
            for (int S = 1; S <= 8; S *= 2) {
                b->fmm_ssplit = S;
                bool ok = true;
                const float t = time_best([&] {
                    return superdc_secular_solve(ctx, b, d, z, rho, lam, eta, org, nullptr, st,
                                                 &o, stream);
                }, s, reps, ok);
                if (ok && t < bestf) {
                    bestf = t;
                    bf = S;
                }
            }
            b->fmm_ssplit = bf;
        }
        // the solution the other phases are tuned on
        rc = superdc_secular_solve(ctx, b, d, z, rho, lam, eta, org, nullptr, st, &o, stream);
    }
    if (rc == SUPERDC_OK) {
        float best = 1e30f;
        int bsplit = b->vec.split;
        for (int S = 1; S <= 16; S *= 2) {
            if (S > 1 && b->max_n / S < 128) break;
            b->vec.split = S;
            bool ok = true;
            const float t = time_best([&] {
                return superdc_loewner(ctx, b, d, z, rho, eta, org, st, zh, bn, &o, stream);
            }, s, reps, ok);
            if (ok && t < best) {
                best = t;
                bsplit = S;
            }
        }
        b->vec.split = bsplit;
        best = 1e30f;
        bsplit = b->bwd.split;
        for (int S = 1; S <= 16; S *= 2) {
            if (S > 1 && b->max_n / S < 128) break;
            b->bwd.split = S;
            bool ok = true;
            const float t = time_best([&] {
                return superdc_secular_backward(ctx, b, d, z, rho, eta, org, st, lam, nullptr,
                                                nullptr, gd, gz, gr, &o, stream);
            }, s, reps, ok);
            if (ok && t < best) {
                best = t;
                bsplit = S;
            }
        }
        b->bwd.split = bsplit;
    }
    (void)hipStreamSynchronize(s);
    for (void *p : {(void *)lam, (void *)eta, (void *)zh, (void *)bn, (void *)gd, (void *)gz,
                    (void *)gr, (void *)org, (void *)st})
        if (p) (void)hipFree(p);
    if (rc == SUPERDC_OK) {
        b->tuned = true;
        cache_store(b, key);
    }
    return rc;
}

int superdc_batch_shapes(const superdc_batch *b, int32_t *out) {
    if (!b || !out) return SUPERDC_EINVAL;
    out[0] = b->sec.chunk;
    out[1] = b->sec.split;
    out[2] = b->vec.split;
    out[3] = b->bwd.split;
    out[4] = b->fmm_ssplit;
    return SUPERDC_OK;
}

}  // extern "C"
