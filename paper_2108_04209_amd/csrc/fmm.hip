// fmm.hip -- triangular FMM of the secular sums on gfx950 (Sec. 4.1.2 with the local
// shifting of Sec. 4.2.2).
//
// The poles of a problem are cut by index into leaves (a tree over the leaves, so boxes
// adapt to clustered poles).  Every box is compressed once per solve into FMM_P
// equivalent sources: the Chebyshev nodes s_q of the box's span and the weights
// W_q = sum_{j in box} w_j L_q(d_j) (L_q the Lagrange basis on those nodes), so that
// sum_j w_j K(x, d_j) ~ sum_q W_q K(x, s_q) for any kernel K smooth over the box -- one
// compression serves both 1/(s-x) and 1/(s-x)^2.  Only boxes that some target lists as far
// field are compressed.  For each target leaf the tree is walked top down: a box separated from the leaf's targets by sep times its width (and by at
// least 64 pole indices) is far field -- entirely left of every target (it feeds psi, the
// lower triangle) or entirely right (phi, the strictly upper triangle), the directional
// interactions of the triangular FMM; zero blocks never appear.  Leaves that are not far
// are near field and are summed directly in shifted form.  The targets move between
// iterations but the poles do not, so only the solver's pass loop runs per iteration.
#include "fmm.h"

namespace sdc {

__device__ __forceinline__ double cheb_node(int q) {
    return cos((2.0 * q + 1.0) * 3.14159265358979323846 / (2.0 * FMM_P));
}

// barycentric weight of Chebyshev node q (first kind): (-1)^q sin((2q+1) pi / 2P)
__device__ __forceinline__ double cheb_bary(int q) {
    return ((q & 1) ? -1.0 : 1.0) * sin((2.0 * q + 1.0) * 3.14159265358979323846 / (2.0 * FMM_P));
}

// pole range [lo, hi) of box g of FMM problem q, and its level h
struct BoxRange {
    int p, lo, hi, n;
    int64_t base;
};

__device__ __forceinline__ BoxRange box_range(const FmmArgs &f, int g) {
    BoxRange r;
    const int q = f.box_fmm[g];
    r.p = f.fmm_prob[q];
    r.base = f.off[r.p];
    r.n = (int)(f.off[r.p + 1] - r.base);
    const int hidx = g - f.box_off[q];
    const int H = f.height[q];
    int h = 0;
    while ((2 << h) - 1 <= hidx) ++h;  // level of the heap index
    const int i = hidx - ((1 << h) - 1);
    const int64_t span = (int64_t)f.leaf << (H - h);
    r.lo = (int)min((int64_t)r.n, i * span);
    r.hi = (int)min((int64_t)r.n, (i + 1) * span);
    return r;
}

// box spans (first and last pole) and cleared use flags: one thread per box
__global__ __launch_bounds__(256) void k_fmm_geom(FmmArgs f) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= f.nboxes) return;
    const BoxRange r = box_range(f, g);
    f.used[g] = 0;
    if (r.lo >= r.hi || (f.status[r.p] & ~SUPERDC_ST_NOCONV))
        f.box_ab[g] = make_double2(__builtin_nan(""), __builtin_nan(""));
    else
        f.box_ab[g] = make_double2(f.dw[r.base + r.lo].x, f.dw[r.base + r.hi - 1].x);
}

// secular equivalent sources of the boxes some target lists as far: one workgroup per box
__global__ __launch_bounds__(256) void k_fmm_boxes(FmmArgs f) {
    __shared__ double part[256][FMM_P + 1];
    const int g = blockIdx.x;
    if (!f.used[g]) return;  // uniform: the whole workgroup leaves
    const BoxRange rg = box_range(f, g);
    const int lo = rg.lo, hi = rg.hi;
    const double2 *dw = f.dw + rg.base;
    const int tid = threadIdx.x;
    const double a = dw[lo].x, b = dw[hi - 1].x;
    const double c = 0.5 * (a + b), hw = 0.5 * (b - a);
    if (hi - lo <= FMM_P) {  // few poles: they are their own equivalent sources
        if (tid < FMM_P)
            f.eq[(int64_t)g * FMM_P + tid] =
                lo + tid < hi ? dw[lo + tid] : make_double2(c, 0.0);
        return;
    }
    double W[FMM_P];
    double tq[FMM_P], lam[FMM_P];
#pragma unroll
    for (int r = 0; r < FMM_P; ++r) {
        W[r] = 0.0;
        tq[r] = cheb_node(r);
        lam[r] = cheb_bary(r);
    }
    for (int j = lo + tid; j < hi; j += blockDim.x) {
        const double2 pw = dw[j];
        const double t = fmin(1.0, fmax(-1.0, (pw.x - c) / hw));
        int hit = -1;
        double inv[FMM_P], den = 0.0;
#pragma unroll
        for (int r = 0; r < FMM_P; ++r) {
            const double dlt = t - tq[r];
            if (dlt == 0.0) hit = r;
            inv[r] = lam[r] / dlt;
            den += inv[r];
        }
        if (hit >= 0) {
            W[hit] += pw.y;  // the pole sits on a node
        } else {
            const double s = pw.y / den;
#pragma unroll
            for (int r = 0; r < FMM_P; ++r) W[r] = __builtin_fma(s, inv[r], W[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < FMM_P; ++r) part[tid][r] = W[r];
    __syncthreads();
    for (int stride = blockDim.x / 2; stride > 0; stride >>= 1) {
        if (tid < stride)
            for (int r = 0; r < FMM_P; ++r) part[tid][r] += part[tid + stride][r];
        __syncthreads();
    }
    if (tid < FMM_P) f.eq[(int64_t)g * FMM_P + tid] = make_double2(c + hw * tq[tid], part[0][tid]);
}

// interaction lists: one thread per target leaf walks its problem's tree; far boxes are
// flagged as used
__global__ __launch_bounds__(64) void k_fmm_lists(FmmArgs f) {
    const int L = blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= f.nleaves) return;
    const int q = f.leaf_fmm[L];
    const int p = f.fmm_prob[q];
    const int64_t base = f.off[p];
    const int n = (int)(f.off[p + 1] - base);
    const int H = f.height[q];
    const int li = L - f.leaf_off[q];
    const int i0 = li * f.leaf, i1 = min(n, i0 + f.leaf);
    int32_t *cnt = f.cnt + 3 * (int64_t)L;
    if (f.status[p] & ~SUPERDC_ST_NOCONV) {
        cnt[0] = -1;
        return;
    }
    const double2 *dw = f.dw + base;
    const double xa = dw[i0].x;
    const double xb = i1 < n ? dw[i1].x : dw[n - 1].x + fmax(f.tail[p], 0.0);
    int stack[64];
    int sp = 0, nn = 0, nl = 0, nr = 0, nleaf = 0;
    bool overflow = false;
    stack[sp++] = 0;
    while (sp > 0 && !overflow) {
        const int hidx = stack[--sp];
        const int g = f.box_off[q] + hidx;
        const double2 ab = f.box_ab[g];
        if (!(ab.x == ab.x)) continue;  // empty box
        int h = 0;
        while ((2 << h) - 1 <= hidx) ++h;
        const int i = hidx - ((1 << h) - 1);
        const int64_t span = (int64_t)f.leaf << (H - h);
        const int lo = (int)min((int64_t)n, i * span), hi = (int)min((int64_t)n, (i + 1) * span);
        const double width = ab.y - ab.x;
        if (ab.y < xa && xa - ab.y >= f.sep * width && hi <= i0 - TILE) {
            if (nl < FMM_FAR_MAX) {
                f.far_l[(int64_t)L * FMM_FAR_MAX + nl++] = g;
                f.used[g] = 1;
            } else {
                overflow = true;
            }
        } else if (ab.x > xb && ab.x - xb >= f.sep * width && lo >= i1 + TILE) {
            if (nr < FMM_FAR_MAX) {
                f.far_r[(int64_t)L * FMM_FAR_MAX + nr++] = g;
                f.used[g] = 1;
            } else {
                overflow = true;
            }
        } else if (h == H) {
            // leaves are visited left to right: a leaf adjacent to the previous near range
            // extends it, so the near field is a few long contiguous ranges (still at most
            // FMM_NEAR_MAX leaves in all)
            if (++nleaf > FMM_NEAR_MAX) {
                overflow = true;
            } else if (nn > 0 && f.near_hi[(int64_t)L * FMM_NEAR_MAX + nn - 1] == lo) {
                f.near_hi[(int64_t)L * FMM_NEAR_MAX + nn - 1] = hi;
            } else if (nn < FMM_NEAR_MAX) {
                f.near_lo[(int64_t)L * FMM_NEAR_MAX + nn] = lo;
                f.near_hi[(int64_t)L * FMM_NEAR_MAX + nn] = hi;
                ++nn;
            } else {
                overflow = true;
            }
        } else {
            if (sp + 2 > 64) {
                overflow = true;
            } else {
                stack[sp++] = 2 * hidx + 2;
                stack[sp++] = 2 * hidx + 1;
            }
        }
    }
    cnt[0] = overflow ? -1 : nn;  // -1: the leaf falls back to direct sums
    cnt[1] = nl;
    cnt[2] = nr;
}

hipError_t launch_fmm_lists(const FmmArgs &f, hipStream_t s) {
    if (f.nboxes <= 0) return hipSuccess;
    SDC_LAUNCH(KID_FMM_GEOM, k_fmm_geom, dim3((f.nboxes + 255) / 256), dim3(256), 0, s, f);
    SDC_LAUNCH(KID_FMM_LISTS, k_fmm_lists, dim3((f.nleaves + 63) / 64), dim3(64), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_fmm_build(const FmmArgs &f, hipStream_t s) {
    if (f.nboxes <= 0) return hipSuccess;
    hipError_t e = launch_fmm_lists(f, s);
    if (e != hipSuccess) return e;
    SDC_LAUNCH(KID_FMM_BOXES, k_fmm_boxes, dim3(f.nboxes), dim3(256), 0, s, f);
    return hipGetLastError();
}

}  // namespace sdc
