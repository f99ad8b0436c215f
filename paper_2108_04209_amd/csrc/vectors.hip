// vectors.hip -- Loewner update vector and eigenvector normalisation for gfx950.
//
//   rho zhat_i^2 = prod_j (lambda_j - d_i) / prod_{j != i} (d_j - d_i)    (eq. lowner)
//   b_j          = (sum_i zhat_i^2 / (d_i - lambda_j)^2)^(-1/2)             (eq. b)
// Every lambda_j - d_i is formed from the solver's shifted representation as
// (d_{K_j} - d_i) + eta_j (eq. qk), so nearby roots keep their relative accuracy.
//
// The paper evaluates the Loewner products as exponentials of log sums through an FMM
// (eqs. lowner2, logv).  Here each lane keeps the numerator and denominator products of
// one pole as separate running products (two interleaved chains each) and strips their
// binary exponents every 8 factors per chain (frexp), accumulating the exponents in an
// integer; one division and one ldexp finish the pole.  No logarithms, and the 8-factor
// blocks cannot over- or underflow for factors between 2^-120 and 2^120.  Both products are
// homogeneous in the scale of the problem (n factors over n - 1), so a problem whose span
// s = d_{n-1} - d_0 + eta_{n-1} lies outside [2^-32, 2^32] has every factor multiplied by
// 2^-e (e the binary exponent of s, an exact scaling) and e added back at the end: the
// factors are then at most 2 in magnitude, and the result is the same, bit for bit, as for
// the problem scaled into range.  Factors below 2^-120 s (relative gaps or eta_k below
// about 7.5e-37 of the span) can still underflow a block.
#include "common.h"
#include "fmm.h"

namespace sdc {

// ke_j = (d_{K_j}, eta_j) for every root (origin indices are local to the problem)
__global__ __launch_bounds__(64) void k_pack_ke(VecArgs a) {
    const Tile t = a.tiles[blockIdx.x];
    const int64_t base = a.off[t.prob];
    const int n = (int)(a.off[t.prob + 1] - base);
    const int k = t.row0 + lane_id();
    if (k < n) {
        const int K = clamp_idx(a.origin[base + k], n);
        a.ke[base + k] = make_double2(a.d[base + K], a.eta[base + k]);
    }
}

__device__ __forceinline__ void renorm(double &num, double &den, int &E) {
    E += __builtin_amdgcn_frexp_exp(num) - __builtin_amdgcn_frexp_exp(den);
    num = __builtin_amdgcn_frexp_mant(num);
    den = __builtin_amdgcn_frexp_mant(den);
}

// products over roots j in [j0, j1); SKIP drops the denominator factor j == i.
// Two independent product chains (even and odd roots) keep the multiplies from waiting
// on each other; roots are read in pointer-stepped blocks of 4 (one scalar address add per
// block) into two register sets that alternate, so the next block's scalar loads are in
// flight while this block is multiplied; each chain strips its exponents after every 8
// factors.
// SC: every factor is multiplied by sg (a power of two) before it enters its product.
template <bool SKIP, bool SC>
__device__ __forceinline__ void loewner_range(const_double2_ptr ke, const_double_ptr dd,
                                              int j0, int j1,
                                              int i, double di, double &num, double &den,
                                              int &E, double sg) {
#define SDC_SCL(F) (SC ? (F) * sg : (F))
#define SDC_LW_LOAD(S, KP, DP)                                                            \
    S##k0 = (KP)[0]; S##k1 = (KP)[1]; S##k2 = (KP)[2]; S##k3 = (KP)[3];                    \
    S##k4 = (KP)[4]; S##k5 = (KP)[5]; S##k6 = (KP)[6]; S##k7 = (KP)[7];                    \
    S##d0 = (DP)[0]; S##d1 = (DP)[1]; S##d2 = (DP)[2]; S##d3 = (DP)[3];
#define SDC_LW_BLOCK(S, J)                                                                \
    {                                                                                     \
        na *= SDC_SCL((S##k0 - di) + S##k1);                                              \
        nb *= SDC_SCL((S##k2 - di) + S##k3);                                              \
        na *= SDC_SCL((S##k4 - di) + S##k5);                                              \
        nb *= SDC_SCL((S##k6 - di) + S##k7);                                              \
        const double f0 = SDC_SCL(S##d0 - di), f1 = SDC_SCL(S##d1 - di);                  \
        const double f2 = SDC_SCL(S##d2 - di), f3 = SDC_SCL(S##d3 - di);                  \
        da *= (SKIP && (J) == i) ? 1.0 : f0;                                              \
        db *= (SKIP && (J) + 1 == i) ? 1.0 : f1;                                          \
        da *= (SKIP && (J) + 2 == i) ? 1.0 : f2;                                          \
        db *= (SKIP && (J) + 3 == i) ? 1.0 : f3;                                          \
        if (++blk == 4) { /* 8 factors per chain */                                       \
            renorm(na, da, E);                                                            \
            renorm(nb, db, E);                                                            \
            blk = 0;                                                                      \
        }                                                                                 \
    }
    double na = 1.0, da = 1.0, nb = 1.0, db = 1.0;
    int j = j0;
    if (j + 4 <= j1) {
        const_double_ptr kp = ke.p + 2 * (int64_t)j;  // (d_K, eta) pairs
        const_double_ptr dp = dd + j;
        double ak0, ak1, ak2, ak3, ak4, ak5, ak6, ak7, ad0, ad1, ad2, ad3;
        double bk0, bk1, bk2, bk3, bk4, bk5, bk6, bk7, bd0, bd1, bd2, bd3;
        int blk = 0;
        SDC_LW_LOAD(a, kp, dp)
        for (;;) {
            const bool more = j + 8 <= j1;
            if (more) { SDC_LW_LOAD(b, kp + 8, dp + 4) }
            SDC_LW_BLOCK(a, j)
            j += 4;
            kp += 8;
            dp += 4;
            if (!more) break;
            const bool more2 = j + 8 <= j1;
            if (more2) { SDC_LW_LOAD(a, kp + 8, dp + 4) }
            SDC_LW_BLOCK(b, j)
            j += 4;
            kp += 8;
            dp += 4;
            if (!more2) break;
        }
    }
    renorm(na, da, E);  // at most 8 factors per chain since the last strip
    renorm(nb, db, E);
    for (; j < j1; ++j) {  // at most 3 more factors per chain after the strip above
        const double2 kv = ke[j];
        na *= SDC_SCL((kv.x - di) + kv.y);
        da *= (SKIP && j == i) ? 1.0 : SDC_SCL(dd[j] - di);
    }
    num *= na * nb;  // mantissas in [0.5, 1) times at most 3 factors: no over- or underflow
    den *= da * db;
    renorm(num, den, E);
#undef SDC_LW_BLOCK
#undef SDC_LW_LOAD
#undef SDC_SCL
}

// The binary exponent e used to scale a problem's factors (0 when its span is in range):
// the span of poles and roots, d_{n-1} - d_0 + eta_{n-1}, read from the packed pairs.
__device__ __forceinline__ int loewner_scale(const_double2_ptr ke, const_double_ptr dd, int n) {
    const double2 kl = ke[n - 1];
    const double span = (kl.x - dd[0]) + kl.y;
    const int e = __builtin_amdgcn_frexp_exp(span);
    return (e < -32 || e > 32) ? e : 0;
}

// With S = blockDim.x / 64 > 1 wavefronts per tile, wavefront w takes the roots
// [n w / S, n (w+1) / S) and the partial results are combined in wavefront order.
__device__ __forceinline__ void split_range(int n, int &p0, int &p1) {
    const int S = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
    p0 = wave_uniform((int)(((int64_t)n * wv) / S));
    p1 = wave_uniform((int)(((int64_t)n * (wv + 1)) / S));
}

__device__ void loewner_tile(const VecArgs &a, Tile t, double4 *red) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int i = t.row0 + lane_id();
    const bool active = i < n;
    const int S = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
    if (a.status[p] & ~SUPERDC_ST_NOCONV) {
        if (active && wv == 0) {
            const double nan = __builtin_nan("");
            a.zhat[base + i] = nan;
            a.dz[base + i] = make_double2(a.d[base + i], nan);
        }
        return;
    }
    const int ii = active ? i : n - 1;
    const_double2_ptr ke = as_const(a.ke + base);  // written by k_pack_ke
    const_double_ptr dd = as_const(a.d + base);
    const double di = a.d[base + ii];
    double num = 1.0, den = 1.0;
    int E = 0;
    int p0, p1;
    split_range(n, p0, p1);
    const int t1 = wave_uniform(min(t.row0 + TILE, n));
    const int es = wave_uniform(loewner_scale(ke, dd, n));
    if (es == 0) {
        loewner_range<false, false>(ke, dd, p0, min(t.row0, p1), ii, di, num, den, E, 1.0);
        loewner_range<true, false>(ke, dd, max(t.row0, p0), min(t1, p1), ii, di, num, den, E, 1.0);
        loewner_range<false, false>(ke, dd, max(t1, p0), p1, ii, di, num, den, E, 1.0);
    } else {  // every factor scaled by 2^-es; the ratio gains 2^-es, added back below
        const double sg = __builtin_ldexp(1.0, -es);
        loewner_range<false, true>(ke, dd, p0, min(t.row0, p1), ii, di, num, den, E, sg);
        loewner_range<true, true>(ke, dd, max(t.row0, p0), min(t1, p1), ii, di, num, den, E, sg);
        loewner_range<false, true>(ke, dd, max(t1, p0), p1, ii, di, num, den, E, sg);
        if (wv == 0) E += es;
    }
    if (S > 1) {
        red[wv * WAVE + lane_id()] = make_double4(num, den, (double)E, 0.0);
        __syncthreads();
        if (wv == 0) {
            for (int w = 1; w < S; ++w) {
                const double4 v = red[w * WAVE + lane_id()];
                num *= v.x;
                den *= v.y;
                E += (int)v.z;
                renorm(num, den, E);
            }
        }
        __syncthreads();
    }
    if (active && wv == 0) {
        const double R = ldexp(num / den, E);
        const double zi = a.z[base + i];
        const double zh = copysign(sqrt(R / a.rho[p]), zi);
        a.zhat[base + i] = zh;
        a.dz[base + i] = make_double2(di, zh);
    }
}

// ---------------------------------------------------------------------------------------
// Loewner products of the FMM problems: the near leaves of the lists exactly (the same
// renormalised products), the far boxes through their moment expansions
//     sum_{j in B} log((lambda_j - d_i) / (d_j - d_i)) = sum_k (-1)^(k+1) M_k r^k / k,
//     r = hw / (c - d_i),
// with a direct product over the box for the rare pole where |r| > 0.35.  Work items are
// 64-pole pieces of the target leaves; S wavefronts split the lists.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double lw_series(const double *M, double r) {
    // Horner from the top: sum_{k=1}^{K} (-1)^(k+1) M_k r^k / k
    double acc = 0.0;
#pragma unroll
    for (int k = FMML_K; k >= 1; --k) {
        const double ck = ((k & 1) ? 1.0 : -1.0) / (double)k;
        acc = __builtin_fma(acc, r, ck * M[k - 1]);
    }
    return acc * r;
}

// The poles and far boxes of an item are staged through LDS, a round of them at a time
// (every thread loads its share of the round, so a round costs one memory round trip
// instead of one per pole block or per box), and the wavefronts read them from there.
constexpr int LW_CH = 256;  // near poles per round
constexpr int LW_FB = 16;   // far boxes per round
struct LwShared {
    double2 kep[LW_CH];     // (d_K, eta) of the staged poles' roots
    double dd[LW_CH];       // the staged poles
    int jj[LW_CH];          // their indices in the problem
    int rs[FMM_NEAR_MAX + 1];  // start of near range e in the concatenation of the ranges
    int rl[FMM_NEAR_MAX];      // its first pole
    double2 geo[LW_FB];        // (centre, half-width) of the staged far boxes
    double mom[LW_FB][FMML_K];
    int box[LW_FB];
};

__device__ void loewner_fmm_tile(const VecArgs &a, const FmmArgs &f, const FmmlArgs &l, Tile t,
                                 double4 *red, LwShared &sh) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int lane = lane_id();
    const int i = t.row0 + lane;
    const bool active = i < n;
    const int S = blockDim.x / WAVE, wv = wave_uniform((int)(threadIdx.x / WAVE));
    if (a.status[p] & ~SUPERDC_ST_NOCONV) {
        if (active && wv == 0) {
            const double nan = __builtin_nan("");
            a.zhat[base + i] = nan;
            a.dz[base + i] = make_double2(a.d[base + i], nan);
        }
        return;
    }
    const int ii = active ? i : n - 1;
    const_double2_ptr ke = as_const(a.ke + base);  // written by k_pack_ke
    const_double_ptr dd = as_const(a.d + base);
    const double di = a.d[base + ii];
    double num = 1.0, den = 1.0, far = 0.0;
    int E = 0;
    const int qf = f.fmm_of[p];
    const int L = wave_uniform(f.leaf_off[qf] + t.row0 / f.leaf);
    const int nn = wave_uniform(f.cnt[3 * (int64_t)L]);
    const int t0 = t.row0, t1 = wave_uniform(min(t.row0 + TILE, n));
    // exact products over [lo, hi), the poles of this item dropping their own factor;
    // a problem out of range has every factor scaled by sg = 2^-es (added back below)
    const int es = wave_uniform(loewner_scale(ke, dd, n));
    const double sg = __builtin_ldexp(1.0, -es);
    if (nn < 0) {  // overflowed lists (rare): every pole, from global memory
        const int lo = wave_uniform((int)(((int64_t)n * wv) / S));
        const int hi = wave_uniform((int)(((int64_t)n * (wv + 1)) / S));
        if (es == 0) {
            loewner_range<false, false>(ke, dd, lo, min(hi, t0), ii, di, num, den, E, 1.0);
            loewner_range<true, false>(ke, dd, max(lo, t0), min(hi, t1), ii, di, num, den, E, 1.0);
            loewner_range<false, false>(ke, dd, max(lo, t1), hi, ii, di, num, den, E, 1.0);
        } else {
            loewner_range<false, true>(ke, dd, lo, min(hi, t0), ii, di, num, den, E, sg);
            loewner_range<true, true>(ke, dd, max(lo, t0), min(hi, t1), ii, di, num, den, E, sg);
            loewner_range<false, true>(ke, dd, max(lo, t1), hi, ii, di, num, den, E, sg);
        }
    } else {
        __syncthreads();  // the previous item's reads of the staging are done
        // the near ranges' starts in their concatenation (a scan by the first wavefront)
        if (wv == 0) {
            int lo = 0, len = 0;
            if (lane < nn) {
                lo = f.near_lo[(int64_t)L * FMM_NEAR_MAX + lane];
                len = f.near_hi[(int64_t)L * FMM_NEAR_MAX + lane] - lo;
            }
            int incl = len;
            for (int o = 1; o < WAVE; o <<= 1) {
                const int v = __shfl_up(incl, o);
                if (lane >= o) incl += v;
            }
            if (lane < nn) {
                sh.rs[lane + 1] = incl;
                sh.rl[lane] = lo;
            }
            if (lane == 0) sh.rs[0] = 0;
        }
        __syncthreads();
        const int T = sh.rs[nn];
        // near poles, a round of LW_CH at a time: staged by every thread, then wavefront wv
        // multiplies the factors of its contiguous share of the round (two chains, exponents
        // stripped every 8 factors per chain)
        for (int c0 = 0; c0 < T; c0 += LW_CH) {
            const int cnt = min(LW_CH, T - c0);
            for (int u = threadIdx.x; u < cnt; u += blockDim.x) {
                const int pos = c0 + u;
                int e = 0;
                while (sh.rs[e + 1] <= pos) ++e;
                const int j = sh.rl[e] + (pos - sh.rs[e]);
                sh.kep[u] = ke[j];
                sh.dd[u] = dd[j];
                sh.jj[u] = j;
            }
            __syncthreads();
            const int u0 = (int)(((int64_t)cnt * wv) / S), u1 = (int)(((int64_t)cnt * (wv + 1)) / S);
            double na = 1.0, da = 1.0, nb = 1.0, db = 1.0;
            int u = u0, blk = 0;
            for (; u + 2 <= u1; u += 2) {
                const double2 k0 = sh.kep[u], k1 = sh.kep[u + 1];
                const double f0 = (sh.dd[u] - di) * sg, f1 = (sh.dd[u + 1] - di) * sg;
                na *= ((k0.x - di) + k0.y) * sg;
                nb *= ((k1.x - di) + k1.y) * sg;
                da *= sh.jj[u] == ii ? 1.0 : f0;
                db *= sh.jj[u + 1] == ii ? 1.0 : f1;
                if (++blk == 8) {  // 8 factors per chain
                    renorm(na, da, E);
                    renorm(nb, db, E);
                    blk = 0;
                }
            }
            if (u < u1) {
                const double2 k0 = sh.kep[u];
                na *= ((k0.x - di) + k0.y) * sg;
                da *= sh.jj[u] == ii ? 1.0 : (sh.dd[u] - di) * sg;
            }
            renorm(na, da, E);
            renorm(nb, db, E);
            num *= na * nb;
            den *= da * db;
            renorm(num, den, E);
            __syncthreads();  // the round's reads are done before the next is staged
        }
        // far boxes, a round of LW_FB at a time: ids and geometry, then their moments, staged
        // by every thread; wavefront wv takes the round's boxes wv, wv + S, ...
        const int nl = wave_uniform(f.cnt[3 * (int64_t)L + 1]);
        const int nr = wave_uniform(f.cnt[3 * (int64_t)L + 2]);
        for (int c0 = 0; c0 < nl + nr; c0 += LW_FB) {
            const int cnt = min(LW_FB, nl + nr - c0);
            if (threadIdx.x < cnt) {
                const int e = c0 + threadIdx.x;
                const int g = e < nl ? f.far_l[(int64_t)L * FMM_FAR_MAX + e]
                                     : f.far_r[(int64_t)L * FMM_FAR_MAX + e - nl];
                sh.box[threadIdx.x] = g;
                sh.geo[threadIdx.x] = l.geo[g];
            }
            __syncthreads();
            for (int u = threadIdx.x; u < cnt * FMML_K; u += blockDim.x)
                sh.mom[u / FMML_K][u % FMML_K] = l.mom[(int64_t)sh.box[u / FMML_K] * FMML_K + u % FMML_K];
            __syncthreads();
            for (int b = wv; b < cnt; b += S) {
                const double2 gc = sh.geo[b];
                const double r = gc.y / (gc.x - di);
                if (fabs(r) <= 0.35) {
                    far += lw_series(sh.mom[b], r);
                } else {  // too close for the expansion: the box's exact products for this lane
                    const int g = sh.box[b];
                    const int hidx = g - f.box_off[qf];
                    const int H = f.height[qf];
                    int h = 0;
                    while ((2 << h) - 1 <= hidx) ++h;
                    const int bi = hidx - ((1 << h) - 1);
                    const int64_t span = (int64_t)f.leaf << (H - h);
                    const int lo = (int)min((int64_t)n, bi * span);
                    const int hi = (int)min((int64_t)n, (bi + 1) * span);
                    for (int j = lo; j < hi; ++j) {  // j != i: a far box never holds pole i
                        const double2 kv = ke[j];
                        num *= ((kv.x - di) + kv.y) * sg;  // as many factors on both sides
                        den *= (dd[j] - di) * sg;
                        if ((j & 7) == 7) renorm(num, den, E);
                    }
                    renorm(num, den, E);
                }
            }
            __syncthreads();  // the round's reads are done before the next is staged
        }
    }
    if (es != 0 && wv == 0) E += es;
    if (S > 1) {
        red[wv * WAVE + lane_id()] = make_double4(num, den, (double)E, far);
        __syncthreads();
        if (wv == 0) {
            for (int w = 1; w < S; ++w) {
                const double4 v = red[w * WAVE + lane_id()];
                num *= v.x;
                den *= v.y;
                E += (int)v.z;
                far += v.w;
                renorm(num, den, E);
            }
        }
        __syncthreads();
    }
    if (active && wv == 0) {
        const double R = ldexp((num / den) * exp(far), E);
        const double zi = a.z[base + i];
        const double zh = copysign(sqrt(R / a.rho[p]), zi);
        a.zhat[base + i] = zh;
        a.dz[base + i] = make_double2(di, zh);
    }
}

__device__ void bnorm_tile(const VecArgs &a, Tile t, double4 *red) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int j = t.row0 + lane_id();
    const bool active = j < n;
    const int S = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
    if (a.status[p] & ~SUPERDC_ST_NOCONV) {
        if (active && wv == 0) a.bnorm[base + j] = __builtin_nan("");
        return;
    }
    const_double2_ptr dz = as_const(a.dz + base);  // written by k_loewner
    const double2 kv = a.ke[base + (active ? j : n - 1)];
    int p0, p1;
    split_range(n, p0, p1);
    // two poles share one reciprocal (the FP64 reciprocal issues at a quarter of the FMA
    // rate): zhat0^2/t0^2 + zhat1^2/t1^2 = ((zhat0 t1)^2 + (zhat1 t0)^2) / (t0 t1)^2, a sum
    // of two squares over a square, applied as (num R) R.  The products need every |t| inside
    // [2^-300, 2^300] (the range the solver's shared reciprocals use);
    // the smallest |t| of a root is |eta| (its origin is its nearest pole) and the largest
    // is at an end of the pole range.  A wavefront with a root outside takes one
    // reciprocal per pole.
    double s0 = 0.0, s1 = 0.0;
    int i = p0;
    bool paired = false;
    if (p0 < p1) {
        const double tmax = fmax(fabs((dz[p0].x - kv.x) - kv.y), fabs((dz[p1 - 1].x - kv.x) - kv.y));
        const bool ok = fabs(kv.y) >= 0x1p-300 && tmax <= 0x1p300;
        paired = __ballot(!ok) == 0ull;
    }
    if (paired) {
        for (; i + 2 <= p1; i += 2) {
            const double2 q0v = dz[i], q1v = dz[i + 1];
            const double t0 = (q0v.x - kv.x) - kv.y, t1 = (q1v.x - kv.x) - kv.y;
            const double R = rcp_nr(t0 * t1);
            const double u0 = q0v.y * t1, u1 = q1v.y * t0;
            const double num = __builtin_fma(u0, u0, u1 * u1);
            s0 = __builtin_fma(num * R, R, s0);
        }
    }
    for (; i + 2 <= p1; i += 2) {
        const double2 q0v = dz[i], q1v = dz[i + 1];
        const double q0 = q0v.y * rcp_nr((q0v.x - kv.x) - kv.y);
        const double q1 = q1v.y * rcp_nr((q1v.x - kv.x) - kv.y);
        s0 = __builtin_fma(q0, q0, s0);
        s1 = __builtin_fma(q1, q1, s1);
    }
    if (i < p1) {
        const double2 q0v = dz[i];
        const double q0 = q0v.y * rcp_nr((q0v.x - kv.x) - kv.y);
        s0 = __builtin_fma(q0, q0, s0);
    }
    double sum = s0 + s1;
    if (S > 1) {
        red[wv * WAVE + lane_id()] = make_double4(sum, 0.0, 0.0, 0.0);
        __syncthreads();
        if (wv == 0)
            for (int w = 1; w < S; ++w) sum += red[w * WAVE + lane_id()].x;
        __syncthreads();
    }
    if (active && wv == 0) a.bnorm[base + j] = 1.0 / sqrt(sum);
}

// blockDim.x = 64 S; dynamic LDS: one double4 per thread when S > 1
__global__ __launch_bounds__(1024) void k_loewner(VecArgs a, Queue *q) {
    extern __shared__ double4 red4[];
    __shared__ int slot;
    for_each_item(q, a.ntiles, &slot, [&](int item) {
        loewner_tile(a, a.tiles[item], red4);
    });
}

__global__ __launch_bounds__(1024) void k_bnorm(VecArgs a, Queue *q) {
    extern __shared__ double4 red4[];
    __shared__ int slot;
    for_each_item(q, a.ntiles, &slot, [&](int item) {
        bnorm_tile(a, a.tiles[item], red4);
    });
}

__global__ __launch_bounds__(1024) void k_loewner_fmm(VecArgs a, FmmArgs f, FmmlArgs l, Queue *q) {
    extern __shared__ double4 red4[];
    __shared__ LwShared sh;
    __shared__ int slot;
    for_each_item(q, a.ntiles, &slot, [&](int item) {
        loewner_fmm_tile(a, f, l, a.tiles[item], red4, sh);
    });
}

hipError_t launch_pack_ke(const VecArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    SDC_LAUNCH(KID_PACK, k_pack_ke, dim3(a.ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_loewner_fmm(const VecArgs &a, const FmmArgs &f, const FmmlArgs &l, int split,
                              Queue *q, int grid, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    const size_t lds = split > 1 ? sizeof(double4) * WAVE * split : 0;
    SDC_LAUNCH(KID_LOEWNER_FMM, k_loewner_fmm, dim3(q ? grid : a.ntiles), dim3(WAVE * split), lds,
               s, a, f, l, q);
    return hipGetLastError();
}

hipError_t launch_loewner(const VecArgs &a, int split, Queue *q, int grid, hipStream_t s,
                          bool pack) {
    if (a.ntiles <= 0) return hipSuccess;
    const size_t lds = split > 1 ? sizeof(double4) * WAVE * split : 0;
    if (pack) SDC_LAUNCH(KID_PACK, k_pack_ke, dim3(a.ntiles), dim3(64), 0, s, a);
    SDC_LAUNCH(KID_LOEWNER, k_loewner, dim3(q ? grid : a.ntiles), dim3(WAVE * split), lds, s, a, q);
    return hipGetLastError();
}

hipError_t launch_bnorm(const VecArgs &a, int split, Queue *q, int grid, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    const size_t lds = split > 1 ? sizeof(double4) * WAVE * split : 0;
    SDC_LAUNCH(KID_BNORM, k_bnorm, dim3(q ? grid : a.ntiles), dim3(WAVE * split), lds, s, a, q);
    return hipGetLastError();
}

}  // namespace sdc
