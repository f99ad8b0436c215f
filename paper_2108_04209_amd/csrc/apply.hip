// apply.hip -- Y = Qhat X or Qhat^T X for the Cauchy-like eigenvector matrix on gfx950.
//
//   Qhat = diag(zhat) C diag(b),  C_ij = 1/((d_i - d_{K_j}) - eta_j)     (eqs. qscale, qk)
//   Y = Qhat X   : Y_i = zhat_i sum_j C_ij (b_j X_j)       (Alg. 4, untransposed branch)
//   Y = Qhat^T X : Y_j = b_j    sum_i C_ij (zhat_i X_i)    (Alg. 3 Z-update, Alg. 4)
//
// The product is a dense contraction whose left factor is generated, never stored.
// MFMA kernel: a workgroup of 4 wavefronts owns 64 output rows (16 per wavefront) and
// all right-hand sides in blocks of 64 columns.  The reduction runs over 64-entry chunks:
// the scaled right-hand sides (b_s X_s or zhat_s X_s) and the per-entry pole data are
// staged in LDS, then each wavefront generates its 16x4 slice of C with one reciprocal
// per lane and feeds v_mfma_f64_16x16x4f64 against 4x16 slices of the staged block.
// VALU kernel (few right-hand sides): one output row per lane, the same staging, and
// plain FMAs; four wavefronts share a tile's reduction range.
#include "common.h"

namespace sdc {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int AP_ROWS = 64;   // output rows per workgroup
constexpr int AP_K = 64;      // reduction chunk
constexpr int AP_C = 64;      // right-hand sides per pass
constexpr int AP_LD = AP_K + 1;

// per-entry data of the reduction index s
template <int TRANS>
__device__ __forceinline__ void stage_entry(const ApplyArgs &a, int64_t base, int n, int s,
                                            double2 &sd, double &scale) {
    if (s < n) {
        if (TRANS == 0) {  // s runs over roots: (d_{K_s}, eta_s), scale b_s
            sd = make_double2(a.d[base + clamp_idx(a.origin[base + s], n)], a.eta[base + s]);
            scale = a.bnorm[base + s];
        } else {           // s runs over poles: (d_s, zhat_s), scale zhat_s
            sd = make_double2(a.d[base + s], a.zhat[base + s]);
            scale = a.zhat[base + s];
        }
    } else {
        sd = make_double2(0.0, 0.0);
        scale = 0.0;
    }
}

// raw data of one reduction chunk, held in registers while the previous chunk is
// multiplied: threads < 64 hold entry s0 + tid's pole data and scale; every thread holds
// NCT * 4 right-hand-side values, element e = tid + 256 i (row e % 64 of the chunk,
// column e / 64 of the pass)
template <int NCT>
struct ApplyStage {
    double2 sd;
    double sc;
    double x[NCT * 4];
};

template <int TRANS, int NCT>
__device__ __forceinline__ void apply_fetch(const ApplyArgs &a, int64_t base, int n, int s0,
                                            int c0, int ncols, ApplyStage<NCT> &st) {
    const int tid = threadIdx.x;
    if (tid < AP_K) stage_entry<TRANS>(a, base, n, s0 + tid, st.sd, st.sc);
#pragma unroll
    for (int i = 0; i < NCT * 4; ++i) {
        const int e = tid + 256 * i;
        const int sl = e % AP_K, c = e / AP_K;
        const int s = s0 + sl;
        double v = 0.0;
        if (s < n && c < ncols) {
            const double sc = TRANS == 0 ? a.bnorm[base + s] : a.zhat[base + s];
            v = sc * a.X[base + s + (int64_t)(c0 + c) * a.ldx];
        }
        st.x[i] = v;
    }
}

template <int NCT>
__device__ __forceinline__ void apply_store(const ApplyStage<NCT> &st, double *Xs, double2 *Sd) {
    const int tid = threadIdx.x;
    if (tid < AP_K) Sd[tid] = st.sd;
#pragma unroll
    for (int i = 0; i < NCT * 4; ++i) {
        const int e = tid + 256 * i;
        Xs[(e / AP_K) * AP_LD + e % AP_K] = st.x[i];
    }
}

// NCT: 16-column blocks per pass (the pass width is 16 NCT columns)
template <int TRANS, int NCT>
__device__ void apply_tile_mfma(const ApplyArgs &a, Tile t, double *Xs, double2 *Sd) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int o0 = t.row0;
    if (a.status[p] & ~SUPERDC_ST_NOCONV) {
        const double nan = __builtin_nan("");
        for (int e = threadIdx.x; e < AP_ROWS * a.m; e += blockDim.x) {
            const int r = o0 + (e % AP_ROWS), c = e / AP_ROWS;
            if (r < n) a.Y[base + r + (int64_t)c * a.ldy] = nan;
        }
        if (TRANS == 1 && a.fuse_b && threadIdx.x < AP_ROWS && o0 + (int)threadIdx.x < n)
            a.bout[base + o0 + threadIdx.x] = nan;
        return;
    }
    // row data for the entries of C this lane generates: row o = o0 + 16 wv + lane%16
    const int orow = o0 + wv * 16 + (lane & 15);
    const bool ovalid = orow < n;
    const int oc = ovalid ? orow : n - 1;
    double ra, rb = 0.0;
    if (TRANS == 0) {
        ra = a.d[base + oc];
    } else {
        ra = a.d[base + clamp_idx(a.origin[base + oc], n)];
        rb = a.eta[base + oc];
    }
    constexpr int PW = 16 * NCT;  // columns per pass
    for (int c0 = 0; c0 < a.m; c0 += PW) {
        const int ncols = min(PW, a.m - c0);
        const int nct = (ncols + 15) / 16;
        v4d acc[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
        // fuse_b (one pass of at most 15 columns): b = sum (zhat_s / t)^2, each term squared
        // after the division as the b kernel does (zhat^2 and 1/t^2 apart can leave the
        // exponent range); each lane sums the terms of the entries it generates, on the
        // VALU beside the multiply (one column does not need the MFMA)
        const bool fb = TRANS == 1 && NCT == 1 && a.fuse_b;
        double bsum = 0.0;
        ApplyStage<NCT> st;
        apply_fetch<TRANS, NCT>(a, base, n, 0, c0, ncols, st);
        for (int s0 = 0; s0 < n; s0 += AP_K) {
            __syncthreads();  // the previous chunk's reads of Xs/Sd are done
            apply_store<NCT>(st, Xs, Sd);
            __syncthreads();
            // the next chunk's loads are in flight while this one is multiplied
            if (s0 + AP_K < n) apply_fetch<TRANS, NCT>(a, base, n, s0 + AP_K, c0, ncols, st);
            // one slice of 4 sources: this lane's Cauchy entry (one reciprocal with a Newton
            // step) into the MFMA of every column tile; MASK: padding entries past the
            // problem's end are zeroed.  A row past the end (ovalid false) only feeds its own
            // output row, never written.
#define SDC_AP_SLICE(MASK)                                                                 \
    {                                                                                      \
        const int sl = kk + (lane >> 4);                                                   \
        const double2 sd = Sd[sl];                                                         \
        const double tt = TRANS ? (sd.x - ra) - rb : (ra - sd.x) - sd.y;                   \
        const double av = (!(MASK) || s0 + sl < n) ? rcp_nr1(tt) : 0.0;                   \
        _Pragma("unroll") for (int ct = 0; ct < NCT; ++ct) {                               \
            if (ct < nct) {                                                                \
                const double bv = Xs[(ct * 16 + (lane & 15)) * AP_LD + sl];                \
                acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);  \
                if (fb) {                                                                  \
                    const double qv = av * sd.y;                                           \
                    bsum = fma(qv, qv, bsum);                                              \
                }                                                                          \
            }                                                                              \
        }                                                                                  \
    }
#pragma unroll 4
            for (int kk = 0; kk < AP_K; kk += 4) SDC_AP_SLICE(true)
#undef SDC_AP_SLICE
            mfma_drain();  // before any copy of the accumulators between chunks
        }
        if (fb) {  // the four lanes of a Cauchy row (lane % 16) hold its partial sums
            bsum += __shfl_xor(bsum, 16);
            bsum += __shfl_xor(bsum, 32);
        }
        if (a.work && threadIdx.x == 0) {  // kernel timing: this pass's algorithmic flops
            const unsigned long long rows = (unsigned long long)min(AP_ROWS, n - o0);
            const unsigned long long me = (unsigned long long)(ncols + (fb ? 1 : 0));
            atomicAdd(a.work, rows * (unsigned long long)n * (2 * me + 3) + 2 * rows * me);
        }
        mfma_drain();
        // v_mfma_f64_16x16x4f64 returns D[4 v + lane/16][lane % 16] in accumulator v
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = o0 + wv * 16 + 4 * v + (lane >> 4);
            double postb = 0.0;
            if (fb) {  // b's sum of this row is held by the lanes that generated its entries
                postb = 1.0 / sqrt(__shfl(bsum, 4 * v + (lane >> 4)));
                if (row < n && (lane & 15) == 0) a.bout[base + row] = postb;
            }
            if (row < n) {
                const double post = fb ? postb : (TRANS ? a.bnorm[base + row] : a.zhat[base + row]);
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) {
                    const int col = ct * 16 + (lane & 15);
                    if (ct < nct && col < ncols)
                        a.Y[base + row + (int64_t)(c0 + col) * a.ldy] = post * acc[ct][v];
                }
            }
        }
    }
}

template <int TRANS, int NCT>
__global__ __launch_bounds__(256) void k_apply_mfma(ApplyArgs a, Queue *q) {
    __shared__ double Xs[16 * NCT * AP_LD];
    __shared__ double2 Sd[AP_K];
    __shared__ int slot;
    for_each_item(q, a.ntiles, &slot, [&](int item) {
        apply_tile_mfma<TRANS, NCT>(a, a.tiles[item], Xs, Sd);
    });
}

// ---------------------------------------------------------------------------------------
// VALU variant: one output row per lane, up to 8 right-hand sides per pass.  AV_W
// wavefronts share a tile: wavefront w takes the reduction chunks w, w + AV_W, ... (each
// stages its own chunk), and the partial sums are added in wavefront order at the end.
// ---------------------------------------------------------------------------------------
constexpr int AV_C = 8;
constexpr int AV_W = 4;

template <int TRANS>
__device__ void apply_tile_valu(const ApplyArgs &a, Tile t, double *Xs, double2 *Sd,
                                double *red) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int o = t.row0 + lane;
    const bool ovalid = o < n;
    if (a.status[p] & ~SUPERDC_ST_NOCONV) {
        if (ovalid && wv == 0)
            for (int c = 0; c < a.m; ++c) a.Y[base + o + (int64_t)c * a.ldy] = __builtin_nan("");
        return;
    }
    const int oc = ovalid ? o : n - 1;
    double ra, rb = 0.0;
    if (TRANS == 0) {
        ra = a.d[base + oc];
    } else {
        ra = a.d[base + clamp_idx(a.origin[base + oc], n)];
        rb = a.eta[base + oc];
    }
    const double post = TRANS ? a.bnorm[base + oc] : a.zhat[base + oc];
    double *Xw = Xs + wv * WAVE * AV_C;
    double2 *Sw = Sd + wv * WAVE;
    const int nchunk = (n + WAVE - 1) / WAVE;
    const int rounds = (nchunk + AV_W - 1) / AV_W;  // the same count for every wavefront
    for (int c0 = 0; c0 < a.m; c0 += AV_C) {
        const int ncols = min(AV_C, a.m - c0);
        double acc[AV_C];
#pragma unroll
        for (int c = 0; c < AV_C; ++c) acc[c] = 0.0;
        for (int rd = 0; rd < rounds; ++rd) {
            const int s0 = (rd * AV_W + wv) * WAVE;
            __syncthreads();
            {
                double2 sd;
                double sc;
                const int s = s0 + lane;
                stage_entry<TRANS>(a, base, n, s, sd, sc);
                Sw[lane] = sd;
#pragma unroll
                for (int c = 0; c < AV_C; ++c)
                    Xw[lane * AV_C + c] =
                        (s < n && c < ncols) ? sc * a.X[base + s + (int64_t)(c0 + c) * a.ldx] : 0.0;
            }
            __syncthreads();
            const int cnt = max(0, min(WAVE, n - s0));
            for (int sl = 0; sl < cnt; ++sl) {
                const double2 sd = Sw[sl];
                const double tt = TRANS ? (sd.x - ra) - rb : (ra - sd.x) - sd.y;
                const double r = rcp_nr(tt);
#pragma unroll
                for (int c = 0; c < AV_C; ++c)
                    if (c < ncols) acc[c] = __builtin_fma(r, Xw[sl * AV_C + c], acc[c]);
            }
        }
        // partial sums of wavefronts 1.. through LDS, added in wavefront order by wavefront 0
        __syncthreads();
        if (wv > 0)
#pragma unroll
            for (int c = 0; c < AV_C; ++c) red[((wv - 1) * AV_C + c) * WAVE + lane] = acc[c];
        __syncthreads();
        if (wv == 0) {
            for (int w = 1; w < AV_W; ++w)
#pragma unroll
                for (int c = 0; c < AV_C; ++c) acc[c] += red[((w - 1) * AV_C + c) * WAVE + lane];
            if (ovalid)
                for (int c = 0; c < ncols; ++c)
                    a.Y[base + o + (int64_t)(c0 + c) * a.ldy] = post * acc[c];
        }
        if (a.work && threadIdx.x == 0) {  // kernel timing: this pass's algorithmic flops
            const unsigned long long rows = (unsigned long long)min(WAVE, n - t.row0);
            const unsigned long long me = (unsigned long long)ncols;
            atomicAdd(a.work, rows * (unsigned long long)n * (2 * me + 3) + 2 * rows * me);
        }
    }
}

template <int TRANS>
__global__ __launch_bounds__(WAVE * AV_W) void k_apply_valu(ApplyArgs a, Queue *q) {
    // the partial-sum exchange reuses the staging area (it follows a barrier that ends
    // every read of it)
    static_assert((AV_W - 1) * AV_C * WAVE <= AV_W * WAVE * AV_C, "reduction area");
    __shared__ double Xs[AV_W * WAVE * AV_C];
    __shared__ double2 Sd[AV_W * WAVE];
    __shared__ int slot;
    double *red = Xs;
    for_each_item(q, a.ntiles, &slot, [&](int item) {
        apply_tile_valu<TRANS>(a, a.tiles[item], Xs, Sd, red);
    });
}

hipError_t launch_apply(const ApplyArgs &a0, int use_mfma, Queue *q, int grid, hipStream_t s) {
    if (a0.ntiles <= 0) return hipSuccess;
    ApplyArgs a = a0;
    a.work = trace_work(use_mfma ? KID_APPLY_MFMA : KID_APPLY_VALU);
    const dim3 g(q ? grid : a.ntiles);
    if (use_mfma) {
        // the pass width: 16, 32 or 64 columns, the smallest that covers m (64 beyond)
        const int nct = a.m <= 16 ? 1 : (a.m <= 32 ? 2 : 4);
#define SDC_APPLY_MFMA(T, C) \
    SDC_LAUNCH(KID_APPLY_MFMA, (k_apply_mfma<T, C>), g, dim3(256), 0, s, a, q)
        if (a.trans) {
            if (nct == 1) SDC_APPLY_MFMA(1, 1);
            else if (nct == 2) SDC_APPLY_MFMA(1, 2);
            else SDC_APPLY_MFMA(1, 4);
        } else {
            if (nct == 1) SDC_APPLY_MFMA(0, 1);
            else if (nct == 2) SDC_APPLY_MFMA(0, 2);
            else SDC_APPLY_MFMA(0, 4);
        }
#undef SDC_APPLY_MFMA
    } else {
        if (a.trans)
            SDC_LAUNCH(KID_APPLY_VALU, k_apply_valu<1>, g, dim3(WAVE * AV_W), 0, s, a, q);
        else
            SDC_LAUNCH(KID_APPLY_VALU, k_apply_valu<0>, g, dim3(WAVE * AV_W), 0, s, a, q);
    }
    return hipGetLastError();
}

}  // namespace sdc
