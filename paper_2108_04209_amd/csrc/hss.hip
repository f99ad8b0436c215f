// hss.hip -- kernels of the HSS conquering pass (Alg. 3) on gfx950, besides the rank-one
// solver: leaf eigendecompositions, merging of the children's spectra (the sort with
// permutation P_p of Sec. 4.4), assembly of the update columns and of the basis
// recursion, and the permutations and leaf products used to apply the structured
// eigenmatrix Q (Lemma 2, Alg. 4).
//
// Layout: one tree level covers all n entries, node q of level l owning rows
// [q n_l, (q+1) n_l), n_l = leaf 2^(depth-l).  Per-level column blocks (update columns Z,
// basis columns W) are column-major with leading dimension n.  Small generators are
// row-major r x r, stored per node in level order (heap index 2^l - 1 + q).
#include "common.h"
#include "hss.h"

namespace sdc {

// ---------------------------------------------------------------------------------------
// leaf eigendecomposition: cyclic Jacobi, one workgroup per leaf, matrix in LDS
// ---------------------------------------------------------------------------------------
constexpr int LJ_LD = LEAF_MAX + 1;

// Round-robin (circle) ordering: in round `rd` every index takes part in exactly one of
// m/2 disjoint pairs, and over m-1 rounds every pair meets once.
__device__ __forceinline__ int rr_player(int pos, int rd, int m) {
    return pos == 0 ? 0 : 1 + (pos - 1 + rd) % (m - 1);
}

__global__ __launch_bounds__(256) void k_leaf_jacobi(LeafArgs a) {
    __shared__ double A[LEAF_MAX * LJ_LD];
    __shared__ double cs[2 * (LEAF_MAX / 2)];
    __shared__ int pq[2 * (LEAF_MAX / 2)];
    __shared__ double red[8];
    __shared__ int nrot;
    __shared__ int rank[LEAF_MAX];
    __shared__ double ev[LEAF_MAX];

    const int leafid = blockIdx.x;
    const int L = a.leaf;
    const int tid = threadIdx.x, nt = blockDim.x;
    const double *D = a.D + (size_t)leafid * L * L;
    double *V = a.Q + (size_t)leafid * L * L;  // column j (an eigenvector) contiguous
    for (int e = tid; e < L * L; e += nt) {
        const int i = e / L, j = e % L;
        A[i * LJ_LD + j] = D[e];
        V[j * L + i] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    // Frobenius norm for the absolute part of the rotation threshold
    double fro = 0.0;
    for (int e = tid; e < L * L; e += nt) {
        const double v = A[(e / L) * LJ_LD + e % L];
        fro += v * v;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) fro += __shfl_xor(fro, o);
    if (lane_id() == 0) red[tid / WAVE] = fro;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < nt / WAVE; ++w) t += red[w];
        red[4] = sqrt(t);
    }
    __syncthreads();
    const double absfloor = 1e-18 * red[4];
    const int m = L;  // even
    const int half = m / 2;
    for (int sweep = 0; sweep < a.max_sweeps; ++sweep) {
        if (tid == 0) nrot = 0;
        __syncthreads();
        for (int rd = 0; rd < m - 1; ++rd) {
            if (tid < half) {
                int p = rr_player(tid, rd, m), q = rr_player(m - 1 - tid, rd, m);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                const double apq = A[p * LJ_LD + q];
                const double app = A[p * LJ_LD + p], aqq = A[q * LJ_LD + q];
                double c = 1.0, s = 0.0;
                if (fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app) * fabs(aqq)) + absfloor) {
                    const double theta = (aqq - app) / (2.0 * apq);
                    double t;
                    if (fabs(theta) > 1e150) t = 0.5 / theta;
                    else t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    s = t * c;
                    atomicAdd(&nrot, 1);
                }
                cs[2 * tid] = c;
                cs[2 * tid + 1] = s;
                pq[2 * tid] = p;
                pq[2 * tid + 1] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int e = tid; e < half * L; e += nt) {
                const int pr = e / L, j = e % L;
                const double c = cs[2 * pr], s = cs[2 * pr + 1];
                if (s == 0.0) continue;
                const int p = pq[2 * pr], q = pq[2 * pr + 1];
                const double ap = A[p * LJ_LD + j], aq = A[q * LJ_LD + j];
                A[p * LJ_LD + j] = c * ap - s * aq;
                A[q * LJ_LD + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, and V <- V J
            for (int e = tid; e < half * L; e += nt) {
                const int pr = e / L, i = e % L;
                const double c = cs[2 * pr], s = cs[2 * pr + 1];
                if (s == 0.0) continue;
                const int p = pq[2 * pr], q = pq[2 * pr + 1];
                const double ap = A[i * LJ_LD + p], aq = A[i * LJ_LD + q];
                A[i * LJ_LD + p] = c * ap - s * aq;
                A[i * LJ_LD + q] = s * ap + c * aq;
                const double vp = V[p * L + i], vq = V[q * L + i];
                V[p * L + i] = c * vp - s * vq;
                V[q * L + i] = s * vp + c * vq;
            }
            __syncthreads();
        }
        if (nrot == 0) break;
        __syncthreads();
    }
    // ascending order of the eigenvalues (ties broken by index)
    if (tid < L) ev[tid] = A[tid * LJ_LD + tid];
    __syncthreads();
    if (tid < L) {
        const double v = ev[tid];
        int r = 0;
        for (int j = 0; j < L; ++j) r += (ev[j] < v) || (ev[j] == v && j < tid);
        rank[tid] = r;
        a.lam[(size_t)leafid * L + r] = v;
    }
    __syncthreads();
    // sorted eigenvectors through LDS (the matrix is no longer needed)
    for (int e = tid; e < L * L; e += nt) {
        const int j = e / L, i = e % L;
        A[rank[j] * LJ_LD + i] = V[j * L + i];
    }
    __syncthreads();
    for (int e = tid; e < L * L; e += nt) {
        const int j = e / L, i = e % L;
        V[j * L + i] = A[j * LJ_LD + i];
    }
    // W = Q^T U (L x r), column-major with leading dimension ldw over the whole level
    const double *U = a.U + (size_t)leafid * L * a.r;
    for (int e = tid; e < L * a.r; e += nt) {
        const int j = e % L, c = e / L;
        double acc = 0.0;
        for (int i = 0; i < L; ++i) acc = __builtin_fma(A[j * LJ_LD + i], U[i * a.r + c], acc);
        a.W[(int64_t)c * a.ldw + (int64_t)leafid * L + j] = acc;
    }
}

// ---------------------------------------------------------------------------------------
// merge of the two sorted child spectra of every node of a level, with the permutation
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int count_less(const double *x, int n, double v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int count_leq(const double *x, int n, double v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_merge(const double *lam_children, double *d_out,
                                               int32_t *perm, int nc, int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t node = e / (2 * nc);
    const int loc = (int)(e % (2 * nc));
    const int64_t base = node * 2 * nc;
    const double *A = lam_children + base, *B = A + nc;
    int pos;
    double v;
    if (loc < nc) {
        v = A[loc];
        pos = loc + count_less(B, nc, v);
    } else {
        v = B[loc - nc];
        pos = (loc - nc) + count_leq(A, nc, v);
    }
    d_out[base + pos] = v;
    perm[base + pos] = loc;
}

// ---------------------------------------------------------------------------------------
// update columns Z = P [W_c1 B_p / sqrt(beta_p) ; sqrt(beta_p) W_c2] and basis columns
// V = P [W_c1 R_c1 ; W_c2 R_c2] of every node of a level
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_assemble(AssembleArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    const int nl = a.nl, nc = nl / 2, r = a.r;
    const int64_t node = e / nl;
    const int64_t base = node * nl;
    const int pos = (int)(e - base);
    const int src = a.perm[e];
    const int child = src < nc ? 0 : 1;
    const int64_t hp = ((int64_t)1 << a.level) - 1 + node;                 // parent heap index
    const int64_t hc = ((int64_t)1 << (a.level + 1)) - 1 + 2 * node + child;  // child heap index
    double w[LEAF_RANK_MAX];
    for (int c = 0; c < r; ++c) w[c] = a.Wprev[(int64_t)c * a.n + base + src];
    const double beta = a.beta[hp];
    const double sb = sqrt(beta);
    const double *B = a.B + hp * r * r;
    for (int c2 = 0; c2 < r; ++c2) {
        double z;
        if (child == 0) {
            double acc = 0.0;
            for (int c = 0; c < r; ++c) acc = __builtin_fma(w[c], B[c * r + c2], acc);
            z = acc / sb;
        } else {
            z = sb * w[c2];
        }
        a.M[(int64_t)c2 * a.n + base + pos] = z;
    }
    if (a.with_basis) {
        const double *R = a.R + hc * r * r;
        for (int c2 = 0; c2 < r; ++c2) {
            double acc = 0.0;
            for (int c = 0; c < r; ++c) acc = __builtin_fma(w[c], R[c * r + c2], acc);
            a.M[(int64_t)(r + c2) * a.n + base + pos] = acc;
        }
    }
}

// ---------------------------------------------------------------------------------------
// applying the structured eigenmatrix: permutations of a level and the leaf products
// ---------------------------------------------------------------------------------------
// scatter (P^T): y[node rows perm[pos]] = x[pos];  gather (P): y[pos] = x[perm[pos]]
__global__ __launch_bounds__(256) void k_permute(const int32_t *perm, int nl, int64_t n, int m,
                                                 const double *X, int64_t ldx, double *Y,
                                                 int64_t ldy, int scatter) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t base = (e / nl) * nl;
    const int64_t src = base + perm[e];
    for (int c = 0; c < m; ++c) {
        if (scatter) Y[src + c * ldy] = X[e + c * ldx];
        else Y[e + c * ldy] = X[src + c * ldx];
    }
}

// Y_leaf = Q_leaf X_leaf (trans 0) or Q_leaf^T X_leaf (trans 1), all leaves of the level
__global__ __launch_bounds__(256) void k_leaf_apply(const double *Q, int L, int64_t n, int m,
                                                    const double *X, int64_t ldx, double *Y,
                                                    int64_t ldy, int trans) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t row = e % n;
    const int c = (int)(e / n);
    const int64_t leafid = row / L;
    const int i = (int)(row % L);
    const double *Ql = Q + leafid * L * L;  // column j contiguous: Ql[j*L + i] = Q_ij
    const double *x = X + c * ldx + leafid * L;
    double acc = 0.0;
    if (trans) {
        for (int k = 0; k < L; ++k) acc = __builtin_fma(Ql[i * L + k], x[k], acc);
    } else {
        for (int k = 0; k < L; ++k) acc = __builtin_fma(Ql[k * L + i], x[k], acc);
    }
    Y[c * ldy + row] = acc;
}

__global__ void k_status_or(const int32_t *st, int cnt, int32_t *out) {
    int v = 0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) v |= st[i];
    for (int o = WAVE / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    __shared__ int red[4];
    if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) t |= red[w];
        out[0] = t;
    }
}

__global__ void k_fill(double *x, int64_t n, double v) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) x[e] = v;
}

static inline dim3 grid_for(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

hipError_t launch_leaf_jacobi(const LeafArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_leaf_jacobi, dim3(a.nleaf), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_merge(const double *lam_children, double *d_out, int32_t *perm, int nc,
                        int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_merge, grid_for(n), dim3(256), 0, s, lam_children, d_out, perm, nc, n);
    return hipGetLastError();
}

hipError_t launch_assemble(const AssembleArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble, grid_for(a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_permute(const int32_t *perm, int nl, int64_t n, int m, const double *X,
                          int64_t ldx, double *Y, int64_t ldy, int scatter, hipStream_t s) {
    hipLaunchKernelGGL(k_permute, grid_for(n), dim3(256), 0, s, perm, nl, n, m, X, ldx, Y, ldy,
                       scatter);
    return hipGetLastError();
}

hipError_t launch_leaf_apply(const double *Q, int L, int64_t n, int m, const double *X,
                             int64_t ldx, double *Y, int64_t ldy, int trans, hipStream_t s) {
    hipLaunchKernelGGL(k_leaf_apply, grid_for(n * m), dim3(256), 0, s, Q, L, n, m, X, ldx, Y, ldy,
                       trans);
    return hipGetLastError();
}

hipError_t launch_status_or(const int32_t *st, int cnt, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_status_or, dim3(1), dim3(256), 0, s, st, cnt, out);
    return hipGetLastError();
}

hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, grid_for(n), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

}  // namespace sdc
