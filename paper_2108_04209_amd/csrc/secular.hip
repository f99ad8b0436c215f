// secular.hip -- validation/packing and the secular-equation solver for gfx950.
//
// For every rank-one problem diag(d) + rho z z^T (Sec. 2.2, eq. rank1upd) each root k is
// found on the shifted secular equation g_k(y) = f(d_K + y) (eq. shiftedeq) with its own
// origin pole K in {k, k+1} (Sec. 4.2.1): every pole difference is formed as
// (d_j - d_K) - y, never as d_j - lambda, which is the paper's local shifting (Sec. 4.2.2,
// eq. localshift).  The sums psi_k, phi_k, psi_k', phi_k' (eqs. psiphi1, psiphi, psiphi2)
// are split at k: poles j <= k feed psi, poles j > k feed phi (eq. flu, lower and strictly
// upper triangle), so each partial sum has terms of one sign.
//
// One wavefront owns a tile of 64 consecutive roots of one problem, one root per lane.
// The pole loop index is wave-uniform, so (d_j, w_j) pairs come through the scalar data
// cache and each pair feeds 64 roots.  Pole ranges entirely left of the tile go to psi,
// entirely right to phi; only the 64 poles under the tile are routed per lane.
//
// The iteration (Alg. 2) runs to convergence inside the kernel:
//   pass 0 : sums at the interval midpoint with origin k; the sign of f there picks the
//            origin and the bracket (Sec. 4.2.1);
//   step   : the middle-way rational interpolation of psi and phi by a + b/(d_k - x) and
//            a + b/(d_{k+1} - x) through value and slope (Sec. 4.1.1), solved as a quadratic
//            in the correction s; the last root uses the one-pole model;
//   guard  : a step leaving the bracket is replaced by bisection;
//   stop   : |f| < c n eps (1 + |psi| + |phi|)  (eq. stopcrit), or a step below 2 ulps.
#include "common.h"
#include "fmm.h"

namespace sdc {

// ---------------------------------------------------------------------------------------
// validation and packing: dw_j = (d_j, rho z_j^2), z2 = sum_j w_j, status bits
// ---------------------------------------------------------------------------------------
// status bits of a problem beyond its entries' (those of rho)
__device__ __forceinline__ int rho_status(double rho) {
    if (!isfinite(rho)) return SUPERDC_ST_NONFINITE;
    return rho > 0.0 ? 0 : SUPERDC_ST_RHO;
}

// Workgroup (problem p, slice s): entries [s len, (s + 1) len) of problem p, len = ceil(n /
// gridDim.y).  One slice writes z2 and status itself; several write their partial sum and
// bits to vsum/vst for k_validate_sum.
__global__ __launch_bounds__(1024) void k_validate(SolveArgs a, int prob_first, double *vsum,
                                                   int32_t *vst) {
    const int p = prob_first + blockIdx.x;
    const int S = gridDim.y, sl = blockIdx.y;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int len = (n + S - 1) / S;
    const int j0 = min(n, sl * len), j1 = min(n, j0 + len);
    const double rho = a.rho[p];
    int st = 0;
    double ws = 0.0;
    const double *d = a.d + base, *z = a.z + base;
    const int nt = blockDim.x;
    // four entries per thread per step, all loads issued before any use
    int j = j0 + threadIdx.x;
    for (; j + 3 * nt < j1; j += 4 * nt) {
        double dj[4], dn[4], zj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = j + u * nt;
            dj[u] = d[i];
            zj[u] = z[i];
            dn[u] = i + 1 < n ? d[i + 1] : __builtin_inf();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!isfinite(dj[u]) || !isfinite(zj[u])) st |= SUPERDC_ST_NONFINITE;
            if (zj[u] == 0.0) st |= SUPERDC_ST_ZERO;
            if (!(dj[u] < dn[u])) st |= SUPERDC_ST_UNSORTED;
            const double w = rho * zj[u] * zj[u];
            a.dw[base + j + u * nt] = make_double2(dj[u], w);
            ws += w;
        }
    }
    for (; j < j1; j += nt) {
        const double dj = d[j], zj = z[j];
        if (!isfinite(dj) || !isfinite(zj)) st |= SUPERDC_ST_NONFINITE;
        if (zj == 0.0) st |= SUPERDC_ST_ZERO;
        if (j + 1 < n && !(dj < d[j + 1])) st |= SUPERDC_ST_UNSORTED;
        const double w = rho * zj * zj;
        a.dw[base + j] = make_double2(dj, w);
        ws += w;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        ws += __shfl_xor(ws, o);
        st |= __shfl_xor(st, o);
    }
    __shared__ double sw[1024 / WAVE];
    __shared__ int ss[1024 / WAVE];
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        sw[wv] = ws;
        ss[wv] = st;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        int s = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) {
            t += sw[w];
            s |= ss[w];
        }
        if (S == 1) {
            a.z2[p] = t;
            a.status[p] = s | rho_status(rho);
        } else {
            vsum[(int64_t)p * S + sl] = t;
            vst[(int64_t)p * S + sl] = s;
        }
    }
}

// the slices' partial sums of each problem added in slice order; one thread per problem
__global__ __launch_bounds__(64) void k_validate_sum(SolveArgs a, int prob_first, int nprob,
                                                     int S, const double *vsum,
                                                     const int32_t *vst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nprob) return;
    const int p = prob_first + i;
    double t = 0.0;
    int s = 0;
    for (int sl = 0; sl < S; ++sl) {
        t += vsum[(int64_t)p * S + sl];
        s |= vst[(int64_t)p * S + sl];
    }
    a.z2[p] = t;
    a.status[p] = s | rho_status(a.rho[p]);
}

// ---------------------------------------------------------------------------------------
// the secular sums over a pole range [j0, j1): MODE 0 all psi, 1 all phi, 2 split at k
// ---------------------------------------------------------------------------------------
// LF: the pole difference is formed in lambda-form, d_j - x with x = d_K + y; otherwise in
// the shifted form (d_j - d_K) - y (eq. localshift).  Following the paper's local shifting
// (Sec. 4.2.2), a pole more than one tile away from every root of the wavefront (far) takes
// lambda-form, which is accurate there (eq. farfield); the near poles keep the shifted form.
// The ablation without local shifting takes lambda-form for every pole.  Every reciprocal
// is the hardware estimate refined by one Newton step (relative error <= ~11 ulp,
// measured), so f is evaluated to within 11 eps (|psi| + |phi|) beyond the rounding of the
// sums, the order of the stopping test's own tolerance n eps (1 + |psi| + |phi|).
//
// Outside the window (where every pole of a range lies on one side of every root), poles
// are taken two at a time with one shared reciprocal (the FP64 reciprocal issues at a
// quarter of the FMA rate on gfx950):
//   w0/t0 + w1/t1       = (w0 t1 + w1 t0) / (t0 t1)
//   w0/t0^2 + w1/t1^2   = (w0 t1 t1 + w1 t0 t0) / (t0 t1)^2
// t0 and t1 have the same sign, so neither numerator cancels.  The square of the shared
// reciprocal is applied as (num2 R) R, so no intermediate leaves the exponent range when
// t0 t1 does not.  The products need every |t| of the range inside [2^-300, 2^300]; a range
// outside that (checked once per range for the whole wavefront) takes one reciprocal per
// pole.
template <int MODE, bool LF>
__device__ __forceinline__ void secular_range(const_double2_ptr dw, int j0, int j1,
                                              int k, double dK, double y, double x,
                                              double &psi, double &dpsi, double &phi,
                                              double &dphi) {
#define SDC_SEC_BODY(JJ, PW)                                          \
    {                                                                 \
        const double2 pw = (PW);                                      \
        const double tt = LF ? pw.x - x : (pw.x - dK) - y;            \
        const double r = rcp_nr1(tt);                                 \
        const double wr = pw.y * r;                                   \
        if (MODE == 0) {                                              \
            psi += wr;                                                \
            dpsi = __builtin_fma(wr, r, dpsi);                        \
        } else if (MODE == 1) {                                       \
            phi += wr;                                                \
            dphi = __builtin_fma(wr, r, dphi);                        \
        } else {                                                      \
            /* j <= k exactly when the pole lies left of the iterate: */ \
            /* w_j > 0, so the term's sign routes it (psi < 0 < phi)  */ \
            const double wl = __builtin_fmin(wr, 0.0);                \
            const double wg = __builtin_fmax(wr, 0.0);                \
            psi += wl;                                                \
            dpsi = __builtin_fma(wl, r, dpsi);                        \
            phi += wg;                                                \
            dphi = __builtin_fma(wg, r, dphi);                        \
        }                                                             \
    }
// two poles, one reciprocal (MODE 0 or 1 only)
#define SDC_SEC_PAIR(PA, PB)                                          \
    {                                                                 \
        const double2 pa = (PA), pb = (PB);                           \
        const double t0 = LF ? pa.x - x : (pa.x - dK) - y;            \
        const double t1 = LF ? pb.x - x : (pb.x - dK) - y;            \
        const double R = rcp_nr1(t0 * t1);                            \
        const double u0 = pa.y * t1, u1 = pb.y * t0;                  \
        const double num2 = __builtin_fma(u0, t1, u1 * t0);           \
        if (MODE == 0) {                                              \
            psi = __builtin_fma(u0 + u1, R, psi);                     \
            dpsi = __builtin_fma(num2 * R, R, dpsi);                  \
        } else {                                                      \
            phi = __builtin_fma(u0 + u1, R, phi);                     \
            dphi = __builtin_fma(num2 * R, R, dphi);                  \
        }                                                             \
    }
    // Poles come in blocks of 4 (one 64-byte scalar fetch).  Two register sets A and B
    // alternate, so the next block's fetch is in flight during this block's arithmetic
    // and no register copies are needed between blocks.
#define SDC_SET4(S, Q)                                                  \
    S##0 = make_double2((Q)[0], (Q)[1]);                                \
    S##1 = make_double2((Q)[2], (Q)[3]);                                \
    S##2 = make_double2((Q)[4], (Q)[5]);                                \
    S##3 = make_double2((Q)[6], (Q)[7]);
    int j = j0;
    const_double_ptr q = dw.p + 2 * (int64_t)j0;
    if (MODE != 2 && j + 4 <= j1) {
        // the nearest and farthest pole of the range bound every |t|
        const double dn = MODE == 0 ? dw[j1 - 1].x : dw[j0].x;
        const double df = MODE == 0 ? dw[j0].x : dw[j1 - 1].x;
        const double tn = fabs(LF ? dn - x : (dn - dK) - y);
        const double tf = fabs(LF ? df - x : (df - dK) - y);
        const bool ok = tn >= 0x1p-300 && tf <= 0x1p300;
        if (__ballot(!ok) == 0ull) {
            double2 a0, a1, a2, a3, b0, b1, b2, b3;
            SDC_SET4(a, q)
            for (;;) {
                if (j + 8 > j1) {
                    SDC_SEC_PAIR(a0, a1)
                    SDC_SEC_PAIR(a2, a3)
                    j += 4;
                    q += 8;
                    break;
                }
                SDC_SET4(b, q + 8)
                SDC_SEC_PAIR(a0, a1)
                SDC_SEC_PAIR(a2, a3)
                j += 4;
                q += 8;
                if (j + 8 > j1) {
                    SDC_SEC_PAIR(b0, b1)
                    SDC_SEC_PAIR(b2, b3)
                    j += 4;
                    q += 8;
                    break;
                }
                SDC_SET4(a, q + 8)
                SDC_SEC_PAIR(b0, b1)
                SDC_SEC_PAIR(b2, b3)
                j += 4;
                q += 8;
            }
            for (; j < j1; ++j, q += 2) SDC_SEC_BODY(j, make_double2(q[0], q[1]))
            return;
        }
    }
    if (j + 4 <= j1) {
        double2 a0, a1, a2, a3, b0, b1, b2, b3;
        SDC_SET4(a, q)
        for (;;) {
            if (j + 8 > j1) {
                SDC_SEC_BODY(j, a0)
                SDC_SEC_BODY(j + 1, a1)
                SDC_SEC_BODY(j + 2, a2)
                SDC_SEC_BODY(j + 3, a3)
                j += 4;
                q += 8;
                break;
            }
            SDC_SET4(b, q + 8)
            SDC_SEC_BODY(j, a0)
            SDC_SEC_BODY(j + 1, a1)
            SDC_SEC_BODY(j + 2, a2)
            SDC_SEC_BODY(j + 3, a3)
            j += 4;
            q += 8;
            if (j + 8 > j1) {
                SDC_SEC_BODY(j, b0)
                SDC_SEC_BODY(j + 1, b1)
                SDC_SEC_BODY(j + 2, b2)
                SDC_SEC_BODY(j + 3, b3)
                j += 4;
                q += 8;
                break;
            }
            SDC_SET4(a, q + 8)
            SDC_SEC_BODY(j, b0)
            SDC_SEC_BODY(j + 1, b1)
            SDC_SEC_BODY(j + 2, b2)
            SDC_SEC_BODY(j + 3, b3)
            j += 4;
            q += 8;
        }
    }
    for (; j < j1; ++j, q += 2) SDC_SEC_BODY(j, make_double2(q[0], q[1]))
#undef SDC_SET4
#undef SDC_SEC_PAIR
#undef SDC_SEC_BODY
}

// psi, phi and their derivatives at y (origin K) for root k, when the wavefront's live
// roots all lie in [kmin, kmax]: poles left of the window feed psi, right of it phi, and
// only the window itself is routed per lane.  Poles within one tile of the window use the
// shifted form.
//
// Only the poles [p0, p1) are summed: with S wavefronts sharing a tile (split-K), each
// takes a contiguous 1/S of the poles and the partial sums are combined afterwards.
__device__ __forceinline__ void secular_sums(const double2 *__restrict__ dwg, int n, int p0,
                                             int p1, int kmin, int kmax, int k, double dK,
                                             double y, bool unsh, double &psi, double &dpsi,
                                             double &phi, double &dphi) {
    const_double2_ptr dw = as_const(dwg);
    kmin = wave_uniform(kmin);
    kmax = wave_uniform(kmax);
    n = wave_uniform(n);
    p0 = wave_uniform(p0);
    p1 = wave_uniform(p1);
    psi = dpsi = phi = dphi = 0.0;
    const double x = dK + y;
    const int f0 = max(kmin - TILE, 0), f1 = min(kmax + 1 + TILE, n);
#define SDC_CLIP(A, B) max((A), p0), min((B), p1)
    secular_range<0, true>(dw, SDC_CLIP(0, f0), k, dK, y, x, psi, dpsi, phi, dphi);
    if (unsh) {  // ablation: near poles and the window in lambda-form as well
        secular_range<0, true>(dw, SDC_CLIP(f0, kmin), k, dK, y, x, psi, dpsi, phi, dphi);
        secular_range<2, true>(dw, SDC_CLIP(kmin, kmax + 1), k, dK, y, x, psi, dpsi, phi,
                                      dphi);
        secular_range<1, true>(dw, SDC_CLIP(kmax + 1, f1), k, dK, y, x, psi, dpsi, phi,
                                      dphi);
    } else {
        secular_range<0, false>(dw, SDC_CLIP(f0, kmin), k, dK, y, x, psi, dpsi, phi, dphi);
        secular_range<2, false>(dw, SDC_CLIP(kmin, kmax + 1), k, dK, y, x, psi, dpsi, phi,
                                       dphi);
        secular_range<1, false>(dw, SDC_CLIP(kmax + 1, f1), k, dK, y, x, psi, dpsi, phi,
                                       dphi);
    }
    secular_range<1, true>(dw, SDC_CLIP(f1, n), k, dK, y, x, psi, dpsi, phi, dphi);
#undef SDC_CLIP
}

// The same sums over the poles [p0, p1) as one sign-routed range (every pole in the shifted
// form; lambda-form with LF): the FMM solver's fallback for a leaf whose lists overflowed,
// kept to one loop so that the rare path adds little code to that kernel.
template <bool LF>
__device__ __forceinline__ void sign_routed_sums(const double2 *__restrict__ dwg, int p0, int p1,
                                                 int k, double dK, double y, double &psi,
                                                 double &dpsi, double &phi, double &dphi) {
    psi = dpsi = phi = dphi = 0.0;
    secular_range<2, LF>(as_const(dwg), wave_uniform(p0), wave_uniform(p1), k, dK, y, dK + y,
                         psi, dpsi, phi, dphi);
}

// Combine the partial sums of the S wavefronts of a workgroup through LDS, in wavefront
// order, so every wavefront ends with the same, reproducible totals.
__device__ __forceinline__ void split_reduce4(double *red, int S, double &a, double &b,
                                              double &c, double &d) {
    if (S == 1) return;
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    double4 *r4 = reinterpret_cast<double4 *>(red);
    r4[wv * WAVE + lane] = make_double4(a, b, c, d);
    __syncthreads();
    double4 s = r4[lane];
    for (int w = 1; w < S; ++w) {
        const double4 v = r4[w * WAVE + lane];
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
    }
    __syncthreads();
    a = s.x;
    b = s.y;
    c = s.z;
    d = s.w;
}

// The far field of the boxes in target leaf L's local expansion at x: four Chebyshev series
// on the target interval (psi, psi', phi, phi'), evaluated together by Clenshaw's
// recurrence (four independent chains; one wavefront of a work item adds them).
__device__ __forceinline__ void local_series(const FmmArgs &f, int L, double x, double &psi,
                                             double &dpsi, double &phi, double &dphi) {
    const double2 cw = f.loc_ab[L];
    const double t = cw.y > 0.0 ? fmin(1.0, fmax(-1.0, (x - cw.x) / cw.y)) : 0.0;
    const const_double_ptr c = as_const(f.loc + (int64_t)L * FMM_LOC);
    double r[4];
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
        double b1 = 0.0, b2 = 0.0;
#pragma unroll
        for (int j = FMM_PL - 1; j >= 1; --j) {
            const double b0 = __builtin_fma(2.0 * t, b1, c[fn * FMM_PL + j] - b2);
            b2 = b1;
            b1 = b0;
        }
        r[fn] = __builtin_fma(t, b1, c[fn * FMM_PL] - b2);
    }
    psi += r[0];
    dpsi += r[1];
    phi += r[2];
    dphi += r[3];
}

// The same sums from the triangular FMM lists of target leaf L: near leaves directly
// (routed by the window as above), far boxes through their equivalent
// sources in lambda-form, left boxes into psi and right boxes into phi.  With S wavefronts
// per work item, wavefront wv takes the wv-th of S contiguous parts of every near range
// and the far boxes e = wv (mod S).
__device__ __forceinline__ void fmm_sums(const FmmArgs &f, int L, int nn, int nl, int nr,
                                         const double2 *__restrict__ dwg, int kmin, int kmax,
                                         int k, double dK, double y, int wv, int S, bool unsh,
                                         double &psi, double &dpsi, double &phi, double &dphi) {
    const_double2_ptr dw = as_const(dwg);
    kmin = wave_uniform(kmin);
    kmax = wave_uniform(kmax);
    wv = wave_uniform(wv);
    const int sh = __builtin_ctz((unsigned)S);  // the split is a power of two
    psi = dpsi = phi = dphi = 0.0;
    const double x = dK + y;
    // near leaves: the same window split as the direct sums, so only poles within one tile
    // of the live roots take the shifted form
    const int f0 = kmin - TILE, f1 = kmax + 1 + TILE;
    for (int e = 0; e < nn; ++e) {
        if (wave_uniform(f.near_lf[(int64_t)L * FMM_NEAR_MAX + e])) continue;  // in the expansion
        const int lo0 = wave_uniform(f.near_lo[(int64_t)L * FMM_NEAR_MAX + e]);
        const int hi0 = wave_uniform(f.near_hi[(int64_t)L * FMM_NEAR_MAX + e]);
        const int lo = lo0 + (int)(((int64_t)(hi0 - lo0) * wv) >> sh);  // S = 2^sh
        const int hi = lo0 + (int)(((int64_t)(hi0 - lo0) * (wv + 1)) >> sh);
        secular_range<0, true>(dw, lo, min(hi, f0), k, dK, y, x, psi, dpsi, phi, dphi);
        if (unsh) {  // ablation: near poles and the window in lambda-form as well
            secular_range<0, true>(dw, max(lo, f0), min(hi, kmin), k, dK, y, x, psi, dpsi,
                                          phi, dphi);
            secular_range<2, true>(dw, max(lo, kmin), min(hi, kmax + 1), k, dK, y, x, psi,
                                          dpsi, phi, dphi);
            secular_range<1, true>(dw, max(lo, kmax + 1), min(hi, f1), k, dK, y, x, psi,
                                          dpsi, phi, dphi);
        } else {
            secular_range<0, false>(dw, max(lo, f0), min(hi, kmin), k, dK, y, x, psi, dpsi,
                                           phi, dphi);
            secular_range<2, false>(dw, max(lo, kmin), min(hi, kmax + 1), k, dK, y, x, psi,
                                           dpsi, phi, dphi);
            secular_range<1, false>(dw, max(lo, kmax + 1), min(hi, f1), k, dK, y, x, psi,
                                           dpsi, phi, dphi);
        }
        secular_range<1, true>(dw, max(lo, f1), hi, k, dK, y, x, psi, dpsi, phi, dphi);
    }
    // far boxes outside the leaf's local expansion, through their equivalent sources
    for (int e = wv; e < nl; e += S) {
        const int g = wave_uniform(f.far_ld[(int64_t)L * FMM_FAR_MAX + e]);
        secular_range<0, true>(as_const(f.eq + (int64_t)g * FMM_P), 0, FMM_P, k, dK, y, x, psi,
                               dpsi, phi, dphi);
    }
    for (int e = wv; e < nr; e += S) {
        const int g = wave_uniform(f.far_rd[(int64_t)L * FMM_FAR_MAX + e]);
        secular_range<1, true>(as_const(f.eq + (int64_t)g * FMM_P), 0, FMM_P, k, dK, y, x, psi,
                               dpsi, phi, dphi);
    }
    // the others through the leaf's local expansion (the first wavefront)
    if (wv == 0) local_series(f, L, x, psi, dpsi, phi, dphi);
}

// ---------------------------------------------------------------------------------------
// Teams of lanes for the last roots of a work item.  Once every root of an item has
// started, the lanes of roots that converged would idle until the item's slowest root is
// done; instead, when at most 32 roots are live, the wavefront regroups them so that each
// live root is held by a team of g lanes (the largest power of two with g * live <= 64),
// every lane of a team carrying the root's full state.  Lane `sub` of a team sums every
// g-th pole of each range from sub on (per-lane loads), the team adds its partial sums by
// a butterfly over xor offsets below g, and every lane of the team then takes the same
// step.  The teams of the S wavefronts of a workgroup are formed identically.
// ---------------------------------------------------------------------------------------

// the poles [j0, j1) that lane `sub` of a team of g takes, each with its own reciprocal;
// positive weights, so a term's sign routes it: negative terms (pole left of the iterate)
// to psi, positive ones to phi.  LF: lambda-form differences
template <bool LF>
__device__ __forceinline__ void team_poles(const double2 *__restrict__ dw, int j0, int j1,
                                           int sub, int g, double dK, double y, double x,
                                           double &psi, double &dpsi, double &phi,
                                           double &dphi) {
#pragma unroll 4
    for (int j = j0 + sub; j < j1; j += g) {
        const double2 pw = dw[j];
        const double r = rcp_nr1(LF ? pw.x - x : (pw.x - dK) - y);
        const double wr = pw.y * r;
        const double wl = __builtin_fmin(wr, 0.0), wg = __builtin_fmax(wr, 0.0);
        psi += wl;
        dpsi = __builtin_fma(wl, r, dpsi);
        phi += wg;
        dphi = __builtin_fma(wg, r, dphi);
    }
}

// equivalent sources of one far box (weights of either sign), lambda-form, all into psi
// (LEFT) or all into phi
template <bool LEFT>
__device__ __forceinline__ void team_sources(const double2 *__restrict__ eq, int sub, int g,
                                             double x, double &s0, double &s1) {
    for (int q = sub; q < FMM_P; q += g) {
        const double2 pw = eq[q];
        const double r = rcp_nr1(pw.x - x);
        const double wr = pw.y * r;
        s0 += wr;
        s1 = __builtin_fma(wr, r, s1);
    }
}

// add a team's partial sums (teams are aligned groups of g lanes)
__device__ __forceinline__ void team_reduce(int g, double &a, double &b, double &c, double &d) {
    for (int o = 1; o < g; o <<= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        c += __shfl_xor(c, o);
        d += __shfl_xor(d, o);
    }
}

// lane index of the s-th set bit (from 0) of m, s < popcount(m)
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int s) {
    int pos = 0;
    for (int w = 32; w >= 1; w >>= 1) {
        const unsigned long long low = m & ((1ull << w) - 1ull);
        const int c = __popcll(low);
        if (s >= c) {
            s -= c;
            m >>= w;
            pos += w;
        } else {
            m = low;
        }
    }
    return pos;
}

__device__ __forceinline__ int wave_min(int v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// The sums of secular_sums / fmm_sums for teams of g lanes (see above): lane `sub` of a
// team takes every g-th pole of the wavefront's share of each range, every pole in the
// shifted form (lambda-form in the unshifted ablation); far boxes through their equivalent
// sources; the local expansion by the team's first lane.
__device__ __forceinline__ void team_sums(const FmmArgs *fm, int L, int nn, int nl, int nr,
                                          const double2 *__restrict__ dw, int p0, int p1,
                                          double dK, double y, int wv, int S, int sub, int g,
                                          bool unsh, double &psi, double &dpsi, double &phi,
                                          double &dphi) {
    psi = dpsi = phi = dphi = 0.0;
    const double x = dK + y;
    if (!fm || nn < 0) {  // direct sums over this wavefront's share of the poles
        if (unsh) team_poles<true>(dw, p0, p1, sub, g, dK, y, x, psi, dpsi, phi, dphi);
        else team_poles<false>(dw, p0, p1, sub, g, dK, y, x, psi, dpsi, phi, dphi);
        return;
    }
    const FmmArgs &f = *fm;
    const int sh = __builtin_ctz((unsigned)S);
    for (int e = 0; e < nn; ++e) {
        if (wave_uniform(f.near_lf[(int64_t)L * FMM_NEAR_MAX + e])) continue;  // in the expansion
        const int lo0 = wave_uniform(f.near_lo[(int64_t)L * FMM_NEAR_MAX + e]);
        const int hi0 = wave_uniform(f.near_hi[(int64_t)L * FMM_NEAR_MAX + e]);
        const int lo = lo0 + (int)(((int64_t)(hi0 - lo0) * wv) >> sh);
        const int hi = lo0 + (int)(((int64_t)(hi0 - lo0) * (wv + 1)) >> sh);
        if (unsh) team_poles<true>(dw, lo, hi, sub, g, dK, y, x, psi, dpsi, phi, dphi);
        else team_poles<false>(dw, lo, hi, sub, g, dK, y, x, psi, dpsi, phi, dphi);
    }
    for (int e = wv; e < nl; e += S) {
        const int gb = wave_uniform(f.far_ld[(int64_t)L * FMM_FAR_MAX + e]);
        team_sources<true>(f.eq + (int64_t)gb * FMM_P, sub, g, x, psi, dpsi);
    }
    for (int e = wv; e < nr; e += S) {
        const int gb = wave_uniform(f.far_rd[(int64_t)L * FMM_FAR_MAX + e]);
        team_sources<false>(f.eq + (int64_t)gb * FMM_P, sub, g, x, phi, dphi);
    }
    if (wv == 0 && sub == 0) local_series(f, L, x, psi, dpsi, phi, dphi);  // the team's first lane
}

// One wavefront solves the roots [c0, c1) of one problem.  Each lane holds one live root;
// a lane whose root has converged writes it out and takes the next unsolved root of the
// chunk, so the wavefront does not wait for its slowest root (only the chunk's last
// roots drain with idle lanes).  Every pass evaluates the sums once at each lane's own
// iterate; a fresh root's first pass is its midpoint pass.
//
// With S = blockDim.x / 64 > 1 the S wavefronts of the workgroup carry identical copies of
// the lane states, each sums 1/S of the poles, and the partial sums are combined before
// the (identical) update; wavefront 0 writes the results.
template <bool FMM, bool UNSH>
__device__ void secular_chunk(const SolveArgs &a, Tile t, double *red, const FmmArgs *fm) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int c0 = t.row0, c1 = min(n, t.row0 + a.chunk);
    const int lane = lane_id();
    const int S = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
    const bool writer = wv == 0;
    const int p0 = (int)(((int64_t)n * wv) / S), p1 = (int)(((int64_t)n * (wv + 1)) / S);
    if (a.status[p] & ~SUPERDC_ST_NOCONV) {  // invalid input: outputs are NaN
        const double nan = __builtin_nan("");
        for (int k = c0 + lane; k < c1 && writer; k += WAVE) {
            a.lam[base + k] = nan;
            a.eta[base + k] = nan;
            a.origin[base + k] = k;
            if (a.iters) a.iters[base + k] = SUPERDC_ITER_SKIPPED;
            a.ke[base + k] = make_double2(nan, nan);
        }
        return;
    }
    const double2 *__restrict__ dw = a.dw + base;
    const double z2 = a.z2[p];
    const double eps = 2.220446049250313e-16;
    const double tol = a.stop_c * (double)n * eps;
    const bool unsh = UNSH;  // ablation: the iterate lives in lambda's precision
    // FMM: the target leaf of this chunk and its list sizes (-1: fall back to direct sums)
    int L = 0, nn = -1, nl = 0, nr = 0;
    if (FMM) {
        const int q = fm->fmm_of[p];
        L = wave_uniform(fm->leaf_off[q] + t.row0 / fm->leaf);
        nn = wave_uniform(fm->cnt[3 * (int64_t)L]);
        nl = wave_uniform(fm->cntd[2 * (int64_t)L]);      // far boxes outside the
        nr = wave_uniform(fm->cntd[2 * (int64_t)L + 1]);  // local expansion
    }
    // pair evaluations of this wavefront per pass and live root (kernel timing only)
    int64_t pairs_per_pass = p1 - p0;
    if (a.work && FMM && nn >= 0) {
        pairs_per_pass = 0;
        for (int e = 0; e < nn; ++e) {
            if (fm->near_lf[(int64_t)L * FMM_NEAR_MAX + e]) continue;
            const int lo0 = fm->near_lo[(int64_t)L * FMM_NEAR_MAX + e];
            const int hi0 = fm->near_hi[(int64_t)L * FMM_NEAR_MAX + e];
            pairs_per_pass += (int)(((int64_t)(hi0 - lo0) * (wv + 1)) / S) -
                              (int)(((int64_t)(hi0 - lo0) * wv) / S);
        }
        const int nfar = (nl > wv ? (nl - wv + S - 1) / S : 0) + (nr > wv ? (nr - wv + S - 1) / S : 0);
        pairs_per_pass += (int64_t)FMM_P * nfar;
        // the local expansion (four 20-term Clenshaw series, each 19 steps of a subtraction
        // and an FMA and a last FMA: 240 flops) counts as 34 pairs
        static_assert(FMM_PL == 20, "the local expansion's pair count");
        if (wv == 0) pairs_per_pass += 34;
    }
    unsigned long long work = 0, live = 0, slots = 0;

    int next = c0;  // next unassigned root (wave-uniform)
    bool act = false, last = false, hi_closed = false, noconv = false;
    bool fw = false;     // hybrid: the fixed-weight scheme takes the next step
    double fprev = 0.0;  // hybrid: f at the previous iterate
    int k = c0, K = c0, nev = 0, phase = 0;
    int why = 0;  // how the root stopped: 0 the stopping test, SUPERDC_ITER_* otherwise
    double dk = 0.0, dk1 = 0.0, dK = 0.0, y = 0.0, lo = 0.0, hi = 0.0;
    int g = 1;                 // lanes per live root (a team; see above)
    int pass = 0;
    bool noconv_any = false;   // some root of the wavefront hit the cap (kept across regroups)
    for (;;) {
        // refill idle lanes with the next roots of the chunk, in order
        const unsigned long long freem = __ballot(!act);
        const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(freem >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)freem, 0u));
        if (!act && next + rank < c1) {
            act = true;
            k = next + rank;
            K = k;
            last = k == n - 1;
            dk = dw[k].x;
            dk1 = last ? dk : dw[k + 1].x;
            dK = dk;
            y = last ? 0.5 * z2 : 0.5 * (dk1 - dk);  // midpoint pass
            if (unsh) y = (dK + y) - dK;
            phase = 0;
            nev = 0;
            why = 0;
            hi_closed = false;
            fw = false;
        }
        next = min(c1, next + (int)__popcll(freem));
        if (__ballot(act) == 0ull) break;
        // once every root of the chunk has started, regroup the live roots into teams of
        // lanes when at most half the lanes would otherwise be busy
        if (next >= c1 && g < WAVE) {
            const unsigned long long rep = __ballot(act && (lane & (g - 1)) == 0);
            const int nlive = __popcll(rep);
            int gn = g;
            while (gn < WAVE && nlive * gn * 2 <= WAVE) gn *= 2;
            if (gn > g) {
                noconv_any = noconv_any || __ballot(noconv) != 0ull;
                const int slot = lane / gn;
                const bool keep = slot < nlive;
                const int src = keep ? nth_set_bit(rep, slot) : lane;
                int flags = (act ? 1 : 0) | (last ? 2 : 0) | (hi_closed ? 4 : 0) | (fw ? 8 : 0);
                flags = __shfl(flags, src);
                act = keep && (flags & 1);
                last = (flags & 2) != 0;
                hi_closed = (flags & 4) != 0;
                fw = (flags & 8) != 0;
                k = __shfl(k, src);
                K = __shfl(K, src);
                nev = __shfl(nev, src);
                phase = __shfl(phase, src);
                why = __shfl(why, src);
                fprev = __shfl(fprev, src);
                dk = __shfl(dk, src);
                dk1 = __shfl(dk1, src);
                dK = __shfl(dK, src);
                y = __shfl(y, src);
                lo = __shfl(lo, src);
                hi = __shfl(hi, src);
                noconv = false;
                g = gn;
            }
        }
        const int sub = lane & (g - 1);  // this lane's place in its team

        double psi, dpsi, phi, dphi;
        if (g > 1) {
            team_sums(FMM ? fm : nullptr, L, nn, nl, nr, dw, p0, p1, dK, y, wv, S, sub, g, unsh,
                      psi, dpsi, phi, dphi);
            team_reduce(g, psi, dpsi, phi, dphi);
        } else {
            const int kmin = wave_min(act ? k : 0x7fffffff);
            const int kmax = wave_max(act ? k : -1);
            if (FMM && nn >= 0)
                fmm_sums(*fm, L, nn, nl, nr, dw, kmin, kmax, k, dK, y, wv, S, unsh, psi, dpsi, phi,
                         dphi);
            else if (FMM)  // overflowed lists (rare): every pole, routed by sign, one loop
                sign_routed_sums<UNSH>(dw, p0, p1, k, dK, y, psi, dpsi, phi, dphi);
            else
                secular_sums(dw, n, p0, p1, kmin, kmax, k, dK, y, unsh, psi, dpsi, phi, dphi);
        }
        split_reduce4(red, S, psi, dpsi, phi, dphi);
        // issue priority falls as the item's passes add up: the SIMD serves the items in
        // their first passes (every lane live, the loads of a fresh item) ahead of the
        // long-running ones (measured: 7.2 -> 6.9 ms per conquer step for the FMM solver)
        wave_priority(3 - (++pass >> 1));
        if (a.work) {
            const unsigned long long nroot = (unsigned long long)__popcll(__ballot(act && sub == 0));
            work += (unsigned long long)pairs_per_pass * nroot;
            live += (unsigned long long)__popcll(__ballot(act));
            slots += WAVE;
        }
        if (!act) continue;
        const double f = 1.0 + psi + phi;
        bool done;
        if (phase == 0) {
            // the sign of f at the midpoint fixes the origin and the bracket (Sec. 4.2.1)
            if (!last) {
                if (f >= 0.0) {  // root in (d_k, mid]: origin d_k
                    lo = 0.0;
                    hi = y;
                } else {  // root in (mid, d_{k+1}): origin d_{k+1}
                    K = k + 1;
                    dK = dk1;
                    y = -y;
                    if (unsh) y = (dK + y) - dK;
                    lo = y;
                    hi = 0.0;
                }
            } else if (f < 0.0) {
                lo = y;
                hi = z2;
                hi_closed = true;  // unevaluated bound where f >= 0 is known
            } else {
                lo = 0.0;
                hi = y;
            }
            phase = 1;
        } else {
            ++nev;
            if (f < 0.0) {
                lo = y;
            } else {
                hi = y;
                hi_closed = false;
            }
        }
        done = fabs(f) <= tol * (1.0 + fabs(psi) + fabs(phi));  // eq. stopcrit
        if (!done && nev >= a.max_iter) {
            done = true;
            noconv = true;
            why = SUPERDC_ITER_CAP;
        }
        if (a.hybrid && phase == 1 && nev > 0) {
            // hybrid [li93]: a step that kept f's sign and did not cut |f| tenfold hands the
            // next step to the other scheme
            if ((f < 0.0) == (fprev < 0.0) && fabs(f) > 0.1 * fabs(fprev)) fw = !fw;
        }
        fprev = f;
        if (!done) {
            double yn;
            if (!last) {
                // f ~ C + b1/(d_k - x) + b2/(d_{k+1} - x) through f and f' at the iterate,
                // solved as a quadratic in the step s: the middle way takes b1 = psi' A^2,
                // b2 = phi' B^2; the fixed-weight scheme gives the origin's pole its true
                // weight w_K and the other pole the rest of f'
                const double xl = dK + y;
                const double A = unsh ? dk - xl : (dk - dK) - y;   // < 0
                const double B = unsh ? dk1 - xl : (dk1 - dK) - y;  // > 0
                double C, qa;
                if (!fw) {
                    C = f - dpsi * A - dphi * B;
                    qa = C * (A + B) + dpsi * A * A + dphi * B * B;
                } else {
                    const double wK = dw[K].y, df = dpsi + dphi;
                    double b1, b2;
                    if (K == k) {
                        b1 = wK;
                        b2 = fmax(df - wK / (A * A), 0.0) * B * B;
                    } else {
                        b2 = wK;
                        b1 = fmax(df - wK / (B * B), 0.0) * A * A;
                    }
                    C = f - b1 / A - b2 / B;
                    qa = C * (A + B) + b1 + b2;
                }
                const double qb = A * B * f;
                const double disc = sqrt(fabs(qa * qa - 4.0 * qb * C));
                const double s = qa > 0.0 ? (2.0 * qb) / (qa + disc) : (qa - disc) / (2.0 * C);
                yn = y + s;
            } else {
                // one pole: psi ~ a + b/(d_n - x)
                yn = dpsi * y * y / (1.0 + psi + dpsi * y);
            }
            const bool inside = (yn > lo) && (yn < hi || (hi_closed && yn == hi));
            if (!inside || !isfinite(yn)) yn = 0.5 * (lo + hi);
            // a step below rounding, or a collapsed bracket: accept without re-evaluation
            if (unsh) yn = (dK + yn) - dK;  // lambda = d_K + y rounded, as the iterate itself
            if (fabs(yn - y) <= 2.0 * eps * fabs(yn) ||
                hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi))) {
                done = true;
                why = SUPERDC_ITER_UNMET;
            }
            y = yn;
        }
        if (done) {
            if (writer && sub == 0) {
                a.eta[base + k] = y;
                a.lam[base + k] = dK + y;
                a.origin[base + k] = K;
                if (a.iters) a.iters[base + k] = nev | why;
                a.ke[base + k] = make_double2(dK, y);
            }
            act = false;
        }
    }
    noconv_any = noconv_any || __ballot(noconv) != 0ull;
    if (writer && noconv_any && lane == 0) atomicOr(&a.status[p], SUPERDC_ST_NOCONV);
    if (a.work && lane == 0) {
        atomicAdd(a.work, work);
        atomicAdd(a.work + 1, live);
        atomicAdd(a.work + 2, slots);
    }
}

// blockDim.x = 64 S (S = 1, 2, 4, 8, 16); dynamic LDS: 32 S bytes per lane (S > 1).
// UNSH: the unshifted ablation, a kernel of its own so that its code stays out of the other
template <bool UNSH>
__global__ __launch_bounds__(1024) void k_secular(SolveArgs a, Queue *q) {
    extern __shared__ double red[];
    __shared__ int slot;
    for_each_item(q, a.ntiles, &slot, [&](int item) {
        secular_chunk<false, UNSH>(a, a.tiles[item], red, nullptr);
    });
}

// FMM problems: one work item per 64-root piece of a target leaf; blockDim.x = 64 S with
// the same dynamic LDS as k_secular
template <bool UNSH>
__global__ __launch_bounds__(512) void k_secular_fmm(SolveArgs a, FmmArgs f, Queue *q) {
    extern __shared__ double red[];
    __shared__ int slot;
    for_each_item(q, a.ntiles, &slot, [&](int item) {
        secular_chunk<true, UNSH>(a, a.tiles[item], red, &f);
    });
}

hipError_t launch_secular_fmm(const SolveArgs &a, const FmmArgs &f, int split, Queue *q,
                              int grid, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (split < 1 || split > 8 || (split & (split - 1))) return hipErrorInvalidValue;
    const size_t lds = split > 1 ? sizeof(double4) * WAVE * split : 0;
    if (a.unshifted)
        SDC_LAUNCH(KID_SECULAR_FMM, k_secular_fmm<true>, dim3(q ? grid : a.ntiles),
                   dim3(WAVE * split), lds, s, a, f, q);
    else
        SDC_LAUNCH(KID_SECULAR_FMM, k_secular_fmm<false>, dim3(q ? grid : a.ntiles),
                   dim3(WAVE * split), lds, s, a, f, q);
    return hipGetLastError();
}

hipError_t launch_validate(const SolveArgs &a, int prob_first, int nprob, int max_n, hipStream_t s,
                           int vsplit, double *vsum, int32_t *vst) {
    if (nprob <= 0) return hipSuccess;
    const int S = vsplit > 1 && vsum && vst ? vsplit : 1;
    // one workgroup per slice, sized to the largest slice
    const int per = (max_n + S - 1) / S;
    const int bs = per >= 8192 ? 1024 : (per >= 2048 ? 512 : 256);
    SDC_LAUNCH(KID_VALIDATE, k_validate, dim3(nprob, S), dim3(bs), 0, s, a, prob_first, vsum, vst);
    if (S > 1)
        SDC_LAUNCH(KID_VALIDATE, k_validate_sum, dim3((nprob + 63) / 64), dim3(64), 0, s, a,
                   prob_first, nprob, S, (const double *)vsum, (const int32_t *)vst);
    return hipGetLastError();
}

hipError_t launch_secular(const SolveArgs &a, int split, Queue *q, int grid, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    const size_t lds = split > 1 ? sizeof(double4) * WAVE * split : 0;
    if (a.unshifted)
        SDC_LAUNCH(KID_SECULAR, k_secular<true>, dim3(q ? grid : a.ntiles), dim3(WAVE * split),
                   lds, s, a, q);
    else
        SDC_LAUNCH(KID_SECULAR, k_secular<false>, dim3(q ? grid : a.ntiles), dim3(WAVE * split),
                   lds, s, a, q);
    return hipGetLastError();
}

}  // namespace sdc
