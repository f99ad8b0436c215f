// deflate_api.cpp -- C ABI of the deflation pre-pass (Remark 1), its orthogonal factor and
// the row copies between a batch and its reduced problems (declared in include/superdc.h).
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"

using namespace sdc;

namespace {
int fail(hipError_t e) { return e == hipErrorOutOfMemory ? SUPERDC_ENOMEM : SUPERDC_EHIP; }
}  // namespace

extern "C" {

int superdc_deflate(superdc_ctx *ctx, const superdc_batch *b, const double *d, const double *z,
                    const double *rho, double tau, double *d_out, double *z_out, int32_t *perm,
                    int32_t *rot_right, int32_t *rot_left, double *rot_c, double *rot_s,
                    int32_t *kept, int32_t *status, void *stream) {
    if (!ctx || !b || b->ctx != ctx || !d || !z || !rho || !d_out || !z_out || !perm ||
        !rot_right || !rot_left || !rot_c || !rot_s || !kept || !status)
        return SUPERDC_EINVAL;
    if (!std::isfinite(tau) || tau < 0.0) return SUPERDC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double2 *val = (double2 *)ws_get(ctx, WS_DEFL_VAL, sizeof(double2) * b->total);
    int8_t *flag = (int8_t *)ws_get(ctx, WS_DEFL_FLAG, sizeof(int8_t) * b->total);
    const size_t nrec = (size_t)b->nprob * deflate_segments(b->max_n);
    int4 *seg_i = (int4 *)ws_get(ctx, WS_DEFL_SEGI, sizeof(int4) * nrec);
    double2 *seg_d = (double2 *)ws_get(ctx, WS_DEFL_SEGD, sizeof(double2) * nrec);
    if (!val || !flag || !seg_i || !seg_d) return SUPERDC_ENOMEM;
    hipError_t e = launch_deflate(b->off_d, b->nprob, d, z, rho, tau, d_out, z_out, perm,
                                  rot_right, rot_left, rot_c, rot_s, kept, status, val, flag,
                                  b->max_n, seg_i, seg_d, s);
    return e == hipSuccess ? SUPERDC_OK : fail(e);
}

int superdc_deflate_expand(superdc_ctx *ctx, const superdc_batch *b, const int32_t *perm,
                           const int32_t *rot_right, const int32_t *rot_left,
                           const double *rot_c, const double *rot_s, int trans, int32_t m,
                           const double *X, int64_t ldx, double *Y, int64_t ldy, void *stream) {
    if (!ctx || !b || b->ctx != ctx || !perm || !rot_right || !rot_left || !rot_c || !rot_s ||
        !X || !Y || m < 1 || (trans != 0 && trans != 1) || X == Y || ldx < b->total ||
        ldy < b->total)
        return SUPERDC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double *T = nullptr;
    if (trans == 1) {
        T = (double *)ws_get(ctx, WS_DEFL_T, sizeof(double) * b->total * m);
        if (!T) return SUPERDC_ENOMEM;
    }
    hipError_t e = launch_deflate_expand(b->off_d, b->nprob, b->total, m, perm, rot_right,
                                         rot_left, rot_c, rot_s, trans, X, ldx, Y, ldy, T, s);
    return e == hipSuccess ? SUPERDC_OK : fail(e);
}

int superdc_batch_copy_rows(superdc_ctx *ctx, const superdc_batch *src_b,
                            const superdc_batch *dst_b, const int32_t *rows, int32_t m,
                            const double *src, int64_t lds, double *dst, int64_t ldd,
                            const double *fill, void *stream) {
    if (!ctx || !src_b || !dst_b || src_b->ctx != ctx || dst_b->ctx != ctx || !src || !dst ||
        m < 1 || src_b->nprob != dst_b->nprob || src == dst || lds < src_b->total ||
        ldd < dst_b->total)
        return SUPERDC_EINVAL;
    hipError_t e = launch_copy_rows(src_b->off_d, dst_b->off_d, dst_b->nprob, dst_b->total, m,
                                    rows, src, lds, dst, ldd, fill, (hipStream_t)stream);
    return e == hipSuccess ? SUPERDC_OK : fail(e);
}

}  // extern "C"
