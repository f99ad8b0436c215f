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

namespace sdc {

// ---------------------------------------------------------------------------------------
// validation and packing: dw_j = (d_j, rho z_j^2), z2 = sum_j w_j, status bits
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_validate(SolveArgs a, int prob_first) {
    const int p = prob_first + blockIdx.x;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const double rho = a.rho[p];
    int st = 0;
    double ws = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double dj = a.d[base + j], zj = a.z[base + j];
        if (!isfinite(dj) || !isfinite(zj)) st |= SUPERDC_ST_NONFINITE;
        if (zj == 0.0) st |= SUPERDC_ST_ZERO;
        if (j + 1 < n && !(dj < a.d[base + j + 1])) st |= SUPERDC_ST_UNSORTED;
        const double w = rho * zj * zj;
        a.dw[base + j] = make_double2(dj, w);
        ws += w;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        ws += __shfl_xor(ws, o);
        st |= __shfl_xor(st, o);
    }
    __shared__ double sw[4];
    __shared__ int ss[4];
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
        if (!isfinite(rho)) s |= SUPERDC_ST_NONFINITE;
        else if (!(rho > 0.0)) s |= SUPERDC_ST_RHO;
        a.z2[p] = t;
        a.status[p] = s;
    }
}

// ---------------------------------------------------------------------------------------
// the secular sums over a pole range [j0, j1): MODE 0 all psi, 1 all phi, 2 split at k
// ---------------------------------------------------------------------------------------
// FAR: the pole is more than one tile away from every root of the wavefront.  Following
// the paper's local shifting (Sec. 4.2.2), such pairs use lambda directly, d_j - x with
// x = d_K + y, which is accurate there (eq. farfield), and a reciprocal with one Newton
// step (<= 11 ulp, measured); near pairs keep the shifted form (d_j - d_K) - y (eq.
// localshift) and a reciprocal refined twice.
template <int MODE, bool FAR>
__device__ __forceinline__ void secular_range(const_double2_ptr dw, int j0, int j1,
                                              int k, double dK, double y, double x,
                                              double &psi, double &dpsi, double &phi,
                                              double &dphi) {
#define SDC_SEC_BODY(JJ, PW)                                          \
    {                                                                 \
        const double2 pw = (PW);                                      \
        const double r = FAR ? rcp_nr1(pw.x - x) : rcp_nr((pw.x - dK) - y); \
        const double wr = pw.y * r;                                   \
        if (MODE == 0) {                                              \
            psi += wr;                                                \
            dpsi = __builtin_fma(wr, r, dpsi);                        \
        } else if (MODE == 1) {                                       \
            phi += wr;                                                \
            dphi = __builtin_fma(wr, r, dphi);                        \
        } else {                                                      \
            const bool left = (JJ) <= k;                              \
            const double wl = left ? wr : 0.0, wg = left ? 0.0 : wr;  \
            psi += wl;                                                \
            dpsi = __builtin_fma(wl, r, dpsi);                        \
            phi += wg;                                                \
            dphi = __builtin_fma(wg, r, dphi);                        \
        }                                                             \
    }
    // blocks of 4 poles, the next block's scalar fetch issued before this block's math
    int j = j0;
    if (j + 4 <= j1) {
        double2 c0 = dw[j], c1 = dw[j + 1], c2 = dw[j + 2], c3 = dw[j + 3];
        for (; j + 8 <= j1; j += 4) {
            const double2 n0 = dw[j + 4], n1 = dw[j + 5], n2 = dw[j + 6], n3 = dw[j + 7];
            SDC_SEC_BODY(j, c0)
            SDC_SEC_BODY(j + 1, c1)
            SDC_SEC_BODY(j + 2, c2)
            SDC_SEC_BODY(j + 3, c3)
            c0 = n0;
            c1 = n1;
            c2 = n2;
            c3 = n3;
        }
        SDC_SEC_BODY(j, c0)
        SDC_SEC_BODY(j + 1, c1)
        SDC_SEC_BODY(j + 2, c2)
        SDC_SEC_BODY(j + 3, c3)
        j += 4;
    }
    for (; j < j1; ++j) SDC_SEC_BODY(j, dw[j])
#undef SDC_SEC_BODY
}

// psi, phi and their derivatives at y (origin K) for root k, when the wavefront's live
// roots all lie in [kmin, kmax]: poles left of the window feed psi, right of it phi, and
// only the window itself is routed per lane.  Poles within one tile of the window use the
// shifted form.
__device__ __forceinline__ void secular_sums(const double2 *__restrict__ dwg, int n, int kmin,
                                             int kmax, int k, double dK, double y,
                                             double &psi, double &dpsi, double &phi,
                                             double &dphi) {
    const_double2_ptr dw = as_const(dwg);
    kmin = wave_uniform(kmin);
    kmax = wave_uniform(kmax);
    n = wave_uniform(n);
    psi = dpsi = phi = dphi = 0.0;
    const double x = dK + y;
    const int f0 = max(kmin - TILE, 0), f1 = min(kmax + 1 + TILE, n);
    secular_range<0, true>(dw, 0, f0, k, dK, y, x, psi, dpsi, phi, dphi);
    secular_range<0, false>(dw, f0, kmin, k, dK, y, x, psi, dpsi, phi, dphi);
    secular_range<2, false>(dw, kmin, kmax + 1, k, dK, y, x, psi, dpsi, phi, dphi);
    secular_range<1, false>(dw, kmax + 1, f1, k, dK, y, x, psi, dpsi, phi, dphi);
    secular_range<1, true>(dw, f1, n, k, dK, y, x, psi, dpsi, phi, dphi);
}

__device__ __forceinline__ int wave_min(int v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// One wavefront solves the roots [c0, c1) of one problem.  Each lane holds one live root;
// a lane whose root has converged writes it out and takes the next unsolved root of the
// chunk, so the wavefront does not wait for its slowest root (only the chunk's last
// roots drain with idle lanes).  Every pass evaluates the sums once at each lane's own
// iterate; a fresh root's first pass is its midpoint pass.
__device__ void secular_chunk(const SolveArgs &a, Tile t) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int c0 = t.row0, c1 = min(n, t.row0 + a.chunk);
    const int lane = lane_id();
    if (a.status[p] & ~SUPERDC_ST_NOCONV) {  // invalid input: outputs are NaN
        const double nan = __builtin_nan("");
        for (int k = c0 + lane; k < c1; k += WAVE) {
            a.lam[base + k] = nan;
            a.eta[base + k] = nan;
            a.origin[base + k] = k;
            if (a.iters) a.iters[base + k] = 0;
            a.ke[base + k] = make_double2(nan, nan);
        }
        return;
    }
    const double2 *__restrict__ dw = a.dw + base;
    const double z2 = a.z2[p];
    const double eps = 2.220446049250313e-16;
    const double tol = a.stop_c * (double)n * eps;

    int next = c0;  // next unassigned root (wave-uniform)
    bool act = false, last = false, hi_closed = false, noconv = false;
    int k = c0, K = c0, nev = 0, phase = 0;
    double dk = 0.0, dk1 = 0.0, dK = 0.0, y = 0.0, lo = 0.0, hi = 0.0;
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
            phase = 0;
            nev = 0;
            hi_closed = false;
        }
        next = min(c1, next + (int)__popcll(freem));
        if (__ballot(act) == 0ull) break;
        const int kmin = wave_min(act ? k : 0x7fffffff);
        const int kmax = wave_max(act ? k : -1);

        double psi, dpsi, phi, dphi;
        secular_sums(dw, n, kmin, kmax, k, dK, y, psi, dpsi, phi, dphi);
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
        }
        if (!done) {
            double yn;
            if (!last) {
                // middle-way: psi ~ a1 + b1/(d_k - x), phi ~ a2 + b2/(d_{k+1} - x)
                const double A = (dk - dK) - y;   // < 0
                const double B = (dk1 - dK) - y;  // > 0
                const double C = f - dpsi * A - dphi * B;
                const double qa = C * (A + B) + dpsi * A * A + dphi * B * B;
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
            if (fabs(yn - y) <= 2.0 * eps * fabs(yn) ||
                hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)))
                done = true;
            y = yn;
        }
        if (done) {
            a.eta[base + k] = y;
            a.lam[base + k] = dK + y;
            a.origin[base + k] = K;
            if (a.iters) a.iters[base + k] = nev;
            a.ke[base + k] = make_double2(dK, y);
            act = false;
        }
    }
    if (__ballot(noconv) != 0ull && lane == 0) atomicOr(&a.status[p], SUPERDC_ST_NOCONV);
}

__global__ __launch_bounds__(64) void k_secular(SolveArgs a, Queue *q) {
    __shared__ int slot;
    if (q) {
        for (;;) {
            const int item = queue_pull(q, a.ntiles, &slot);
            if (item < 0) break;
            secular_chunk(a, a.tiles[item]);
        }
        queue_leave(q);
    } else if ((int)blockIdx.x < a.ntiles) {
        secular_chunk(a, a.tiles[blockIdx.x]);
    }
}

hipError_t launch_validate(const SolveArgs &a, int prob_first, int nprob, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(nprob), dim3(256), 0, s, a, prob_first);
    return hipGetLastError();
}

hipError_t launch_secular(const SolveArgs &a, Queue *q, int grid, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_secular, dim3(q ? grid : a.ntiles), dim3(64), 0, s, a, q);
    return hipGetLastError();
}

}  // namespace sdc
