// divide.hip -- the HSS dividing stage (Alg. 1) on gfx950.
//
// Top down over the tree, every node p carries the pending update H_p (r x r, zero at the
// root) that Lemma genupd propagates through the nested bases: the coupling of p's
// children becomes B_p - R_c1 H_p R_c2^T, beta_p is its 2-norm, and the children inherit
// R_c H_p R_c^T plus p's own balanced division (eq. divnew1): (1/beta_p) B B^T for the left
// child and beta_p I for the right one.  A leaf ends as D - U H U^T.  The outputs -- the
// divided leaf blocks, the updated couplings and their norms -- are the input of the
// conquering pass, whose Z_p = [U_c1 B_p / sqrt(beta_p); sqrt(beta_p) U_c2] completes the
// bottom-up half of Alg. 1.  With balanced = 0 the earlier division (eq. divide: B B^T to
// the left child, I to the right, beta = 1) is used instead.
#include "common.h"
#include "hss.h"

namespace sdc {

namespace {
constexpr int RM = LEAF_RANK_MAX;
static_assert(RM * RM == 64, "k_divide_level maps one thread to each entry of an r x r block");

// largest eigenvalue of the symmetric r x r matrix M (row-major in LDS, overwritten) by
// cyclic Jacobi; one thread
__device__ double sym_max_eig(double *M, int r) {
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int p = 0; p < r; ++p) {
            dia += M[p * RM + p] * M[p * RM + p];
            for (int q = p + 1; q < r; ++q) off += M[p * RM + q] * M[p * RM + q];
        }
        if (off <= 1e-34 * dia || off == 0.0) break;
        for (int p = 0; p < r; ++p)
            for (int q = p + 1; q < r; ++q) {
                const double apq = M[p * RM + q];
                if (apq == 0.0) continue;
                const double theta = (M[q * RM + q] - M[p * RM + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < r; ++k) {  // rows p, q
                    const double mp = M[p * RM + k], mq = M[q * RM + k];
                    M[p * RM + k] = c * mp - s * mq;
                    M[q * RM + k] = s * mp + c * mq;
                }
                for (int k = 0; k < r; ++k) {  // columns p, q
                    const double mp = M[k * RM + p], mq = M[k * RM + q];
                    M[k * RM + p] = c * mp - s * mq;
                    M[k * RM + q] = s * mp + c * mq;
                }
            }
    }
    double mx = M[0];
    for (int p = 1; p < r; ++p) mx = fmax(mx, M[p * RM + p]);
    return mx;
}
}  // namespace

// one workgroup (64 threads, thread (i, j) = entry (i, j)) per node of level `lvl`
__global__ __launch_bounds__(64) void k_divide_level(DivideArgs a, int lvl) {
    __shared__ double R1[RM * RM], R2[RM * RM], Hp[RM * RM], Bt[RM * RM], T1[RM * RM],
        T2[RM * RM], M[RM * RM];
    __shared__ double beta_s;
    const int q = blockIdx.x;
    const int h = (1 << lvl) - 1 + q, c1 = 2 * h + 1, c2 = 2 * h + 2;
    const int r = a.r, tid = threadIdx.x, i = tid / RM, j = tid % RM;
    const bool in = i < r && j < r;
    const size_t rr = (size_t)r * r;
    if (in) {
        R1[i * RM + j] = a.R[c1 * rr + i * r + j];
        R2[i * RM + j] = a.R[c2 * rr + i * r + j];
        Hp[i * RM + j] = lvl == 0 ? 0.0 : a.H[h * rr + i * r + j];
    }
    __syncthreads();
    // T1 = Hp R2^T, T2 = Hp R1^T
    if (in) {
        double s1 = 0.0, s2 = 0.0;
        for (int b = 0; b < r; ++b) {
            s1 = __builtin_fma(Hp[i * RM + b], R2[j * RM + b], s1);
            s2 = __builtin_fma(Hp[i * RM + b], R1[j * RM + b], s2);
        }
        T1[i * RM + j] = s1;
        T2[i * RM + j] = s2;
    }
    __syncthreads();
    // the updated coupling B - R1 Hp R2^T (eq. genupd)
    if (in) {
        double s = 0.0;
        for (int b = 0; b < r; ++b) s = __builtin_fma(R1[i * RM + b], T1[b * RM + j], s);
        Bt[i * RM + j] = a.B[h * rr + i * r + j] - s;
    }
    __syncthreads();
    // beta = ||B-tilde||_2 from the largest eigenvalue of B-tilde^T B-tilde
    if (in) {
        double s = 0.0;
        for (int b = 0; b < r; ++b) s = __builtin_fma(Bt[b * RM + i], Bt[b * RM + j], s);
        M[i * RM + j] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double beta = 1.0;
        if (a.balanced) {
            beta = sqrt(fmax(sym_max_eig(M, r), 0.0));
            if (!(beta > 0.0)) beta = 1.0;  // a vanished coupling: Z_p = [0; U_c2]
        }
        beta_s = beta;
        a.beta_out[h] = beta;
    }
    __syncthreads();
    const double beta = beta_s;
    if (in) {
        a.B_out[h * rr + i * r + j] = Bt[i * RM + j];
        // children: R_c Hp R_c^T plus the division's own term
        double h1 = 0.0, h2 = 0.0, bb = 0.0;
        for (int b = 0; b < r; ++b) {
            h1 = __builtin_fma(R1[i * RM + b], T2[b * RM + j], h1);  // R1 (Hp R1^T)
            h2 = __builtin_fma(R2[i * RM + b], T1[b * RM + j], h2);  // R2 (Hp R2^T)
            bb = __builtin_fma(Bt[i * RM + b], Bt[j * RM + b], bb);
        }
        a.H[c1 * rr + i * r + j] = h1 + bb / beta;
        a.H[c2 * rr + i * r + j] = h2 + (i == j ? beta : 0.0);
    }
}

// divided leaf blocks D - U H U^T: one workgroup per leaf, M = U H staged in LDS
__global__ __launch_bounds__(256) void k_divide_leaves(DivideArgs a) {
    __shared__ double UH[LEAF_MAX * RM], Us[LEAF_MAX * RM], Hs[RM * RM];
    const int leafid = blockIdx.x;
    const int L = a.leaf, r = a.r, tid = threadIdx.x;
    const size_t rr = (size_t)r * r;
    const int h = (1 << a.depth) - 1 + leafid;
    const double *U = a.U + (size_t)leafid * L * r;
    for (int e = tid; e < L * r; e += blockDim.x) Us[(e / r) * RM + e % r] = U[e];
    for (int e = tid; e < (int)rr; e += blockDim.x) Hs[(e / r) * RM + e % r] = a.H[h * rr + e];
    __syncthreads();
    for (int e = tid; e < L * r; e += blockDim.x) {
        const int i = e / r, k = e % r;
        double s = 0.0;
        for (int b = 0; b < r; ++b) s = __builtin_fma(Us[i * RM + b], Hs[b * RM + k], s);
        UH[i * RM + k] = s;
    }
    __syncthreads();
    const double *D = a.D + (size_t)leafid * L * L;
    double *Dout = a.D_out + (size_t)leafid * L * L;
    for (int e = tid; e < L * L; e += blockDim.x) {
        const int i = e / L, j = e % L;
        double s = 0.0;
        for (int k = 0; k < r; ++k) s = __builtin_fma(UH[i * RM + k], Us[j * RM + k], s);
        Dout[e] = D[e] - s;
    }
}

hipError_t launch_divide(const DivideArgs &a, hipStream_t s) {
    for (int l = 0; l < a.depth; ++l)
        SDC_LAUNCH(KID_DIVIDE, k_divide_level, dim3(1u << l), dim3(64), 0, s, a, l);
    SDC_LAUNCH(KID_DIVIDE, k_divide_leaves, dim3(1u << a.depth), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sdc
