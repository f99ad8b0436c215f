// noalloc.hip -- the allocation-free variant of the secular solve.
//
// superdc_secular_solve keeps its per-call buffers -- the packed (d_j, w_j) pairs, the
// per-problem sum of the weights and the (d_K, eta) pairs of the roots -- in the context's
// grow-only workspace, which the first call of a shape allocates.  Callers that cannot
// allocate at all (code under graph capture, tight serving loops, harnesses that forbid
// hipMalloc) get the same kernels with those buffers in one fixed array in device memory,
// `scratch` below, which every GPU that loads the library holds until the process ends.
//
// In host code `scratch` names a host-side stand-in, not a device address: the device
// address is looked up once per device with hipGetSymbolAddress (at context creation, with
// that device current) and kept in `g_scratch`; only that pointer is ever handed to a
// kernel.
#include <mutex>

#include "common.h"

namespace sdc {
namespace {

// capacity of the scratch array (see superdc.h): SUPERDC_NOALLOC_MAX_TOTAL roots in all and
// SUPERDC_NOALLOC_MAX_PROBS problems
constexpr size_t kPairBytes = sizeof(double2) * (size_t)SUPERDC_NOALLOC_MAX_TOTAL;
constexpr size_t kScratchBytes = 2 * kPairBytes + sizeof(double) * (size_t)SUPERDC_NOALLOC_MAX_PROBS;
static_assert(kPairBytes % 256 == 0, "pair blocks keep 256-byte alignment");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {nullptr};  // device address of `scratch`, per device
std::mutex g_mu;

}  // namespace

int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return SUPERDC_ENODEV;
    std::lock_guard<std::mutex> g(g_mu);
    if (g_scratch[device]) return SUPERDC_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return SUPERDC_EHIP;
    g_scratch[device] = ptr;
    return SUPERDC_OK;
}

}  // namespace sdc

using namespace sdc;

extern "C" int superdc_secular_solve_noalloc(superdc_ctx *ctx, const superdc_batch *b,
                                             const double *d, const double *z,
                                             const double *rho, double *lam, double *eta,
                                             int32_t *origin, int32_t *iters, int32_t *status,
                                             const superdc_opts *opts, void *stream) {
    if (!ctx || !b || b->ctx != ctx || !d || !z || !rho || !lam || !eta || !origin || !status)
        return SUPERDC_EINVAL;
    superdc_opts o;
    if (opts) o = *opts;
    else superdc_opts_default(&o);
    if (opts_check(&o) != SUPERDC_OK) return SUPERDC_EINVAL;
    // direct sums only: the triangular FMM's tree and lists live in the batch, built on
    // the first solve that needs them
    if (o.method == 2) return SUPERDC_EINVAL;
    if (b->total > SUPERDC_NOALLOC_MAX_TOTAL || b->nprob > SUPERDC_NOALLOC_MAX_PROBS)
        return SUPERDC_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device || dev >= kMaxDevices)
        return SUPERDC_EINVAL;
    unsigned char *base = (unsigned char *)g_scratch[dev];
    if (!base) return SUPERDC_EINVAL;  // no context was created on this device
    hipStream_t s = (hipStream_t)stream;
    SolveArgs a{};
    a.off = b->off_d;
    a.d = d;
    a.z = z;
    a.rho = rho;
    a.dw = (double2 *)base;                     // (d_j, w_j), written by k_validate
    a.ke = (double2 *)(base + kPairBytes);      // (d_K, eta), written by the solver
    a.z2 = (double *)(base + 2 * kPairBytes);   // sum_j w_j, written by k_validate
    a.lam = lam;
    a.eta = eta;
    a.origin = origin;
    a.iters = iters;
    a.status = status;
    a.stop_c = o.stop_c;
    a.max_iter = o.max_iter;
    a.unshifted = o.unshifted;
    a.hybrid = o.interp;
    a.work = nullptr;
    // every buffer above is written before it is read within the call, so nothing needs
    // clearing; the work queues in the context reset themselves at the end of each launch
    hipError_t e = hipSuccess;
    if (o.persistent) {
        const LaunchShape sh = b->sec;
        const int slot = sh.chunk == 64 ? 0 : sh.chunk == 128 ? 1 : sh.chunk == 256 ? 2 : 3;
        const TileList &L = b->lists[slot];
        if (!L.lpt) return SUPERDC_EINVAL;  // built with the batch (or by the autotuner)
        a.tiles = L.lpt;
        a.ntiles = L.count;
        a.chunk = sh.chunk;
        e = launch_validate(a, 0, b->nprob, b->max_n, s);
        if (e == hipSuccess)
            e = launch_secular(a, sh.split, ctx->queues + Q_SECULAR,
                               persistent_grid(ctx, a.ntiles, std::max(1, 32 / sh.split)), s);
    } else {
        // one launch per problem on 64-root chunks, as superdc_secular_solve's plain mode
        const TileList &L = b->lists[0];
        if (!L.nat) return SUPERDC_EINVAL;
        for (int p = 0; p < b->nprob && e == hipSuccess; ++p) {
            const int64_t np = b->off_h[p + 1] - b->off_h[p];
            e = launch_validate(a, p, 1, (int)np, s);
            if (e != hipSuccess) break;
            a.tiles = L.nat + L.begin[p];
            a.ntiles = L.begin[p + 1] - L.begin[p];
            a.chunk = TILE;
            int S = 1;  // the split superdc_secular_solve's plain mode picks for this size
            {
                const LaunchShape sh = plain_shape(ctx, np);
                S = sh.split;
            }
            e = launch_secular(a, S, nullptr, 0, s);
        }
    }
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? SUPERDC_ENOMEM : SUPERDC_EHIP;
    return SUPERDC_OK;
}
