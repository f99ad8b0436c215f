// backward.hip -- adjoint of the rank-one eigensolver on gfx950 (not in the paper).
//
// With r_ik = 1/((d_i - d_{K_k}) - eta_k) (the solver's shifted form), S_k = sum_i z_i^2 r_ik^2,
// b_k = S_k^(-1/2), q_ik = b_k z_i r_ik and p_k = q_k^T u = b_k h_k, h_k = sum_i u_i z_i r_ik,
// implicit differentiation of f(lambda_k) = 1 + rho sum_i z_i^2/(d_i - lambda_k) = 0 gives
//   dlambda_k/dd_i = z_i^2 r_ik^2 / S_k, dlambda_k/dz_i = -2 z_i r_ik / S_k,
//   dlambda_k/drho = 1/(rho^2 S_k),
// and the explicit derivatives of p_k follow from those of h_k and b_k.  Collecting terms,
//   lbar_k  = g_lam_k + g_p_k (b_k H2_k - h_k b_k^3 S3_k),  H2 = sum u z r^2, S3 = sum z^2 r^3
//   alpha_k = lbar_k b_k^2,  beta_k = g_p_k b_k,  gamma_k = g_p_k h_k b_k^3
//   g_d_i   = z_i^2 sum_k alpha_k r^2 - u_i z_i sum_k beta_k r^2 + z_i^2 sum_k gamma_k r^3
//   g_z_i   = -2 z_i sum_k alpha_k r + u_i sum_k beta_k r - z_i sum_k gamma_k r^2
//   g_rho   = sum_k alpha_k / rho^2
// Pass 1 (one lane per root) forms the root sums over poles; pass 2 (one lane per pole)
// forms the six Cauchy-like sums over roots; pass 3 reduces g_rho per problem.
#include "common.h"

namespace sdc {

template <bool PROJ>
__device__ void bwd_roots_tile(const BwdArgs &a, Tile t, double4 *red) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int k = t.row0 + lane_id();
    const bool active = k < n;
    const int kk = active ? k : n - 1;
    const bool bad = (a.status[p] & ~SUPERDC_ST_NOCONV) != 0;
    const double dK = a.d[base + clamp_idx(a.origin[base + kk], n)];
    const double eta = a.eta[base + kk];
    const_double_ptr d = as_const(a.d + base);
    const_double_ptr z = as_const(a.z + base);
    const_double_ptr u = as_const(PROJ ? a.u + base : a.z + base);
    double S = 0.0, S3 = 0.0, h = 0.0, H2 = 0.0;
    const int SW = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
    const int i0 = wave_uniform((int)(((int64_t)n * wv) / SW));
    const int i1 = wave_uniform((int)(((int64_t)n * (wv + 1)) / SW));
    if (!bad) {
        for (int i = i0; i < i1; ++i) {
            const double r = rcp_nr((d[i] - dK) - eta);
            const double zr = z[i] * r;
            const double t2 = zr * zr;
            S += t2;
            S3 = __builtin_fma(t2, r, S3);
            if (PROJ) {
                const double uzr = u[i] * zr;
                h += uzr;
                H2 = __builtin_fma(uzr, r, H2);
            }
        }
    }
    if (SW > 1) {  // combine the wavefronts' partial sums in order
        red[wv * WAVE + lane_id()] = make_double4(S, S3, h, H2);
        __syncthreads();
        if (wv == 0)
            for (int w = 1; w < SW; ++w) {
                const double4 v = red[w * WAVE + lane_id()];
                S += v.x;
                S3 += v.y;
                h += v.z;
                H2 += v.w;
            }
        __syncthreads();
    }
    if (!active || wv != 0) return;
    const double nan = __builtin_nan("");
    if (bad) {
        a.rk[base + k] = make_double4(dK, eta, nan, nan);
        a.gk[base + k] = nan;
        return;
    }
    const double b = 1.0 / sqrt(S);
    const double b2 = b * b;
    double lbar = a.g_lam ? a.g_lam[base + k] : 0.0;
    double beta = 0.0, gamma = 0.0;
    if (PROJ) {
        const double gp = a.g_proj[base + k];
        lbar += gp * (b * H2 - h * b2 * b * S3);
        beta = gp * b;
        gamma = gp * h * b2 * b;
    }
    a.rk[base + k] = make_double4(dK, eta, lbar * b2, beta);
    a.gk[base + k] = gamma;
}

template <bool PROJ>
__device__ void bwd_poles_tile(const BwdArgs &a, Tile t, double4 *red) {
    const int p = t.prob;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int i = t.row0 + lane_id();
    const bool active = i < n;
    const int ii = active ? i : n - 1;
    const int SW = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
    if (a.status[p] & ~SUPERDC_ST_NOCONV) {
        if (active && wv == 0) {
            a.g_d[base + i] = __builtin_nan("");
            a.g_z[base + i] = __builtin_nan("");
        }
        return;
    }
    const int k0 = wave_uniform((int)(((int64_t)n * wv) / SW));
    const int k1 = wave_uniform((int)(((int64_t)n * (wv + 1)) / SW));
    const double di = a.d[base + ii];
    const_double4_ptr rk = as_const(a.rk + base);  // written by the roots pass
    const_double_ptr gk = as_const(a.gk + base);
    double A1 = 0.0, A2 = 0.0, A3 = 0.0, B1 = 0.0, B2 = 0.0, B3 = 0.0;
    for (int k = k0; k < k1; ++k) {
        const double4 v = rk[k];
        const double r = rcp_nr((di - v.x) - v.y);
        const double r2 = r * r;
        A1 = __builtin_fma(v.z, r2, A1);
        B1 = __builtin_fma(v.z, r, B1);
        if (PROJ) {
            const double g = gk[k];
            A2 = __builtin_fma(v.w, r2, A2);
            B2 = __builtin_fma(v.w, r, B2);
            A3 = __builtin_fma(g * r2, r, A3);
            B3 = __builtin_fma(g, r2, B3);
        }
    }
    if (SW > 1) {  // combine the wavefronts' partial sums in order
        red[2 * (wv * WAVE + lane_id())] = make_double4(A1, A2, A3, B1);
        red[2 * (wv * WAVE + lane_id()) + 1] = make_double4(B2, B3, 0.0, 0.0);
        __syncthreads();
        if (wv == 0)
            for (int w = 1; w < SW; ++w) {
                const double4 u0 = red[2 * (w * WAVE + lane_id())];
                const double4 u1 = red[2 * (w * WAVE + lane_id()) + 1];
                A1 += u0.x;
                A2 += u0.y;
                A3 += u0.z;
                B1 += u0.w;
                B2 += u1.x;
                B3 += u1.y;
            }
        __syncthreads();
    }
    if (!active || wv != 0) return;
    const double zi = a.z[base + i];
    double gd = zi * zi * (A1 + A3);
    double gz = -2.0 * zi * B1 - zi * B3;
    if (PROJ) {
        const double ui = a.u[base + i];
        gd -= ui * zi * A2;
        gz += ui * B2;
    }
    a.g_d[base + i] = gd;
    a.g_z[base + i] = gz;
}

// blockDim.x = 64 S; dynamic LDS: two double4 per thread when S > 1
template <bool PROJ, int PASS>
__global__ __launch_bounds__(1024) void k_bwd(BwdArgs a, Queue *q) {
    extern __shared__ double4 red4[];
    __shared__ int slot;
    for_each_item(q, a.ntiles, &slot, [&](int item) {
        if (PASS == 1) bwd_roots_tile<PROJ>(a, a.tiles[item], red4);
        else bwd_poles_tile<PROJ>(a, a.tiles[item], red4);
    });
}

// g_rho[p] = sum_k alpha_k / rho_p^2, fixed-order block reduction
__global__ __launch_bounds__(256) void k_bwd_rho(BwdArgs a, int prob_first) {
    const int p = prob_first + blockIdx.x;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) s += a.rk[base + k].z;
    for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double sw[4];
    if (lane_id() == 0) sw[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) t += sw[w];
        const double rho = a.rho[p];
        a.g_rho[p] = (a.status[p] & ~SUPERDC_ST_NOCONV) ? __builtin_nan("") : t / (rho * rho);
    }
}

hipError_t launch_backward(const BwdArgs &a, int split, int prob_first, int nprob, Queue *q1,
                           Queue *q2, int grid, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    const bool proj = a.g_proj != nullptr;
    const dim3 g1(q1 ? grid : a.ntiles), g2(q2 ? grid : a.ntiles), blk(WAVE * split);
    const size_t lds = split > 1 ? 2 * sizeof(double4) * WAVE * split : 0;
    if (proj) {
        SDC_LAUNCH(KID_BWD, (k_bwd<true, 1>), g1, blk, lds, s, a, q1);
        SDC_LAUNCH(KID_BWD, (k_bwd<true, 2>), g2, blk, lds, s, a, q2);
    } else {
        SDC_LAUNCH(KID_BWD, (k_bwd<false, 1>), g1, blk, lds, s, a, q1);
        SDC_LAUNCH(KID_BWD, (k_bwd<false, 2>), g2, blk, lds, s, a, q2);
    }
    SDC_LAUNCH(KID_BWD_RHO, k_bwd_rho, dim3(nprob), dim3(256), 0, s, a, prob_first);
    return hipGetLastError();
}

}  // namespace sdc
