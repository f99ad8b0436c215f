// fmm_vec.hip -- eigenvector-side triangular FMM on gfx950 (Sec. 4.3, "Structured
// eigenvectors via FMM with local shifting", and the Z-update of Alg. 3).
//
// For the roots j of a large problem the sums over its poles i
//     apply:  Y_j,c = b_j sum_i r_ij (zhat_i X_i,c)        (Y = Qhat^T X, eqs. eigvecs, qk)
//     b:      b_j   = (sum_i zhat_i^2 r_ij^2)^(-1/2)      (eq. b)
// with r_ij = 1/(d_i - lambda_j) are evaluated on the same pole tree and interaction
// lists as the secular sums: near leaves directly in the shifted form
// (d_i - d_{K_j}) - eta_j, far boxes through equivalent sources in lambda-form.  The
// equivalent sources of a box are its Chebyshev nodes and the weights
// W_q,c = sum_{i in box} src_i,c L_q(d_i), one column per right-hand side.  Plain sums
// need no psi/phi split, but the lists are the directional ones of the solver and the
// near field keeps the local shifting, as the paper prescribes for these products.
#include "fmm.h"

namespace sdc {

typedef double v4d_f __attribute__((ext_vector_type(4)));


// src_i,c = zhat_i X_i,c0+c (kern 1) or zhat_i^2 (kern 2) for pole i of problem p (entries
// from base).  trans 0: src_j,c = b_j X_j,c0+c at the root lambda_j (positions in pairs[j].x)
__device__ __forceinline__ void fmmv_pack_entry(const FmmvPackArgs &a, const FmmVec &v, int p,
                                                int64_t base, int n, int i) {
    if (v.trans == 0) {
        const int K = clamp_idx(a.origin[base + i], n);
        const double bj = a.bnorm[base + i];
        a.pairs[base + i] = make_double2(a.d[base + K] + a.eta[base + i], bj);
        double *src = v.src + (base + i) * v.m;
        for (int c = 0; c < v.m; ++c) src[c] = bj * a.X[base + i + (int64_t)(a.c0 + c) * a.ldx];
        return;
    }
    const double zh = a.zhat[base + i];
    const double di = a.d[base + i];
    a.pairs[base + i] = make_double2(di, zh);
    double *src = v.src + (base + i) * v.m;
    if (v.kern == 1) {
        const int mx = v.m - v.fuse_b;
        for (int c = 0; c < mx; ++c) src[c] = zh * a.X[base + i + (int64_t)(a.c0 + c) * a.ldx];
        if (v.fuse_b) src[mx] = zh * zh;
    } else {
        src[0] = zh * zh;
    }
    if (i == n - 1) {
        const int K = clamp_idx(a.origin[base + i], n);
        a.tail[p] = (a.d[base + K] + a.eta[base + i]) - di;
    }
}

// one lane per pole (per root for trans 0)
__global__ __launch_bounds__(64) void k_fmmv_pack(FmmvPackArgs a, FmmVec v) {
    const Tile t = a.tiles[blockIdx.x];
    const int64_t base = a.off[t.prob];
    const int n = (int)(a.off[t.prob + 1] - base);
    const int i = t.row0 + lane_id();
    if (i < n) fmmv_pack_entry(a, v, t.prob, base, n, i);
}

// Equivalent sources, one workgroup (256 threads) per box, in two launches: LEAVES = true
// compresses every leaf box from its poles; LEAVES = false compresses every used box above
// the leaves from the equivalent sources of its leaves (16 per leaf instead of up to
// n/4 poles: the far field of a leaf's sources equals that of its poles to the
// interpolation accuracy, and the box's nodes interpolate it again).  Points are taken a
// chunk at a time: each of the chunk's threads forms the 16 Lagrange values of one point in
// LDS, then W_q,c += sum_k L_q(x_k) w_k,c over the chunk runs on the FP64 MFMA, its weight
// operands loaded straight from memory (they are point-major: the 4 points x m columns of
// one step are consecutive) before the Lagrange values are formed.
template <bool LEAVES>
__global__ __launch_bounds__(LEAVES ? 64 : 256, LEAVES ? 1 : 4) void k_fmmv_sources(FmmArgs f, FmmVec v,
                                                                              FmmvPackArgs pk) {
    // leaves: one wavefront, 64 points per chunk; upper boxes (up to 16 sources per leaf
    // below): four wavefronts, 256 points per chunk
    constexpr int NW = LEAVES ? 1 : 4;
    constexpr int FV_CHUNK = 64 * NW;
    __shared__ double Lq[FV_CHUNK][FMM_P + 1];
    // leaves in the first launch; in the second the parts of the upper boxes with poles
    // (used ones): (box, part, parts, partial slot)
    const int4 it = LEAVES ? make_int4(f.leaf_box[blockIdx.x], 0, 1, -1) : f.upper_item[blockIdx.x];
    const int g = it.x;
    if (!LEAVES && f.used[g] != f.gen) return;
    const int qf = f.box_fmm[g];
    const int p = f.fmm_prob[qf];
    const int64_t base = f.off[p];
    const int n = (int)(f.off[p + 1] - base);
    const int hidx = g - f.box_off[qf];
    const int H = f.height[qf];
    int h = 0;
    while ((2 << h) - 1 <= hidx) ++h;
    if (f.status[p] & ~SUPERDC_ST_NOCONV) return;
    const int bi = hidx - ((1 << h) - 1);
    const int64_t span = (int64_t)f.leaf << (H - h);
    const int lo = (int)min((int64_t)n, bi * span), hi = (int)min((int64_t)n, (bi + 1) * span);
    if (lo >= hi) return;  // empty box (never listed)
    const int tid = threadIdx.x;
    if (LEAVES && pk.pairs) {  // the leaf's poles packed here, as k_fmmv_pack would
        for (int i = lo + tid; i < hi; i += blockDim.x) fmmv_pack_entry(pk, v, p, base, n, i);
        __syncthreads();
    }
    const int m = v.m;
    const double2 *d2 = f.dw + base;  // the points' positions in .x (poles, or roots)
    auto d = [&](int i) { return d2[i].x; };
    const double *src = v.src + base * m;
    const double a = d(lo), b = d(hi - 1);
    const double cc = 0.5 * (a + b), hw = 0.5 * (b - a);
    double *node = v.vnode + (int64_t)g * FMM_P;
    double *w = v.vw + (int64_t)g * FMM_P * m;
    if (LEAVES && hi - lo <= FMM_P) {  // few poles: they are their own equivalent sources
        if (tid < FMM_P) {
            const bool in = lo + tid < hi;
            node[tid] = in ? d(lo + tid) : cc;
            for (int c = 0; c < m; ++c) w[tid * m + c] = in ? src[(int64_t)(lo + tid) * m + c] : 0.0;
        }
        return;
    }
    // the points: poles of a leaf, or the sources of the box's leaves
    const int leaf0 = (1 << H) - 1 + bi * (1 << (H - h));      // heap index of the first leaf
    const int nleaf = (int)((hi - lo + f.leaf - 1) / f.leaf);  // leaves with poles
    const int npts = LEAVES ? hi - lo : nleaf * FMM_P;
    // this part's points [pk0, pk1)
    const int pk0 = LEAVES ? 0 : min(npts, it.y * FMMV_PART_PTS);
    const int pk1 = LEAVES ? npts : (it.z == 1 ? npts : min(npts, pk0 + FMMV_PART_PTS));
    const int lane = tid & (WAVE - 1), wv = tid / WAVE;
    double tq[FMM_P], lam[FMM_P];
#pragma unroll
    for (int r = 0; r < FMM_P; ++r) {
        tq[r] = cheb_node(r);
        lam[r] = cheb_bary(r);
    }
    const double ihw = 1.0 / hw;
    v4d_f acc = v4d_f{0.0, 0.0, 0.0, 0.0};
    // the points' weights, m per point: the leaf's poles in src, or the sources of the
    // box's leaves
    const double *wsrc = LEAVES ? src + (int64_t)lo * m
                                : v.vw + (int64_t)(f.box_off[qf] + leaf0) * FMM_P * m;
    for (int k0 = pk0; k0 < pk1; k0 += FV_CHUNK) {
        // W (16 nodes x 16 columns) += L (16 x chunk) S (chunk x 16) on the FP64 MFMA: each
        // wavefront takes 64 points of the chunk, 4 per step
        // (A lane l = L[l % 16][k + l / 16], B lane l = S[k + l / 16][l % 16])
        double bs[16];
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int pt = k0 + wv * 64 + 4 * st + (lane >> 4), c = lane & 15;
            bs[st] = pt < pk1 && c < m ? wsrc[(int64_t)pt * m + c] : 0.0;
        }
        const int k = k0 + tid;
        if (k < pk1) {
            const double x = LEAVES ? d(lo + k)
                                    : v.vnode[(int64_t)(f.box_off[qf] + leaf0) * FMM_P + k];
            const double t = fmin(1.0, fmax(-1.0, (x - cc) * ihw));
            int hit = -1;
            double inv[FMM_P], den = 0.0;
#pragma unroll
            for (int r = 0; r < FMM_P; ++r) {
                const double dlt = t - tq[r];
                if (dlt == 0.0) hit = r;
                inv[r] = lam[r] * rcp_nr(dlt);
                den += inv[r];
            }
            const double iden = 1.0 / den;
#pragma unroll
            for (int r = 0; r < FMM_P; ++r)
                Lq[tid][r] = hit >= 0 ? (r == hit ? 1.0 : 0.0) : inv[r] * iden;
        } else {
#pragma unroll
            for (int r = 0; r < FMM_P; ++r) Lq[tid][r] = 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int kk = wv * 64 + 4 * st + (lane >> 4);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Lq[kk][lane & 15], bs[st], acc, 0, 0, 0);
        }
        __syncthreads();
    }
    mfma_drain();
    // the four wavefronts' partial W added in wavefront order (through the staging LDS);
    // accumulator r of lane l holds W[4 r + l / 16][l % 16]
    double *red = &Lq[0][0];
    if (NW > 1 && wv > 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) red[((wv - 1) * 4 + r) * WAVE + lane] = acc[r];
    }
    if (NW > 1) __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double s2 = acc[r];
            for (int u = 0; u < NW - 1; ++u) s2 += red[(u * 4 + r) * WAVE + lane];
            const int qn = 4 * r + (lane >> 4), cn = lane & 15;
            if (it.w >= 0)  // one part of several: its partial weights, summed afterwards
                f.vpart[((int64_t)it.w * FMM_P + qn) * FMMV_MAX_M + cn] = s2;
            else if (cn < m)
                w[qn * m + cn] = s2;
        }
    }
    if (it.y == 0 && tid < FMM_P) node[tid] = cc + hw * tq[tid];
}

// The weights of the upper boxes computed in several parts: the parts' partial weights
// added in part order.  One workgroup per such box, thread (node q, column c).
__global__ __launch_bounds__(FMM_P * FMMV_MAX_M) void k_fmmv_sources_sum(FmmArgs f, FmmVec v) {
    const int2 sb = f.split_box[blockIdx.x];
    const int g = sb.x;
    if (f.used[g] != f.gen) return;
    const int qf = f.box_fmm[g];
    const int p = f.fmm_prob[qf];
    if (f.status[p] & ~SUPERDC_ST_NOCONV) return;
    const int n = (int)(f.off[p + 1] - f.off[p]);
    const int hidx = g - f.box_off[qf];
    const int H = f.height[qf];
    int h = 0;
    while ((2 << h) - 1 <= hidx) ++h;
    const int bi = hidx - ((1 << h) - 1);
    const int64_t span = (int64_t)f.leaf << (H - h);
    const int lo = (int)min((int64_t)n, bi * span), hi = (int)min((int64_t)n, (bi + 1) * span);
    const int nleaf = (hi - lo + f.leaf - 1) / f.leaf;
    const int parts = (nleaf * FMM_P + FMMV_PART_PTS - 1) / FMMV_PART_PTS;
    const int q = threadIdx.x / FMMV_MAX_M, c = threadIdx.x % FMMV_MAX_M;
    if (c >= v.m) return;
    double s = 0.0;
    for (int u = 0; u < parts; ++u) s += f.vpart[((int64_t)(sb.y + u) * FMM_P + q) * FMMV_MAX_M + c];
    v.vw[((int64_t)g * FMM_P + q) * v.m + c] = s;
}

// Evaluation at the roots: work items are 64-root pieces of the target leaves; S
// wavefronts per item split the near ranges and the far boxes, and their partial sums are
// added in wavefront order.  NC >= m accumulators per lane.
template <int KERN, int NC>
__device__ void fmmv_item(const SolveArgs &it, const FmmArgs &f, const FmmVec &v, Tile t,
                          double *red) {
    const int p = t.prob;
    const int64_t base = it.off[p];
    const int n = (int)(it.off[p + 1] - base);
    const int lane = lane_id();
    const int S = blockDim.x / WAVE, wv = wave_uniform((int)(threadIdx.x / WAVE));
    const int j = t.row0 + lane;
    const bool active = j < n;
    const int m = v.m;
    if (f.status[p] & ~SUPERDC_ST_NOCONV) {
        if (active && wv == 0) {
            const double nan = __builtin_nan("");
            if (KERN == 1)
                for (int c = 0; c < m; ++c) v.Y[base + j + (int64_t)c * v.ldy] = nan;
            else
                v.bout[base + j] = nan;
        }
        return;
    }
    const int jj = active ? j : n - 1;
    const double dK = v.d[base + clamp_idx(v.origin[base + jj], n)];
    const double eta = v.eta[base + jj];
    const double x = dK + eta;
    const int qf = f.fmm_of[p];
    const int L = wave_uniform(f.leaf_off[qf] + t.row0 / f.leaf);
    int nn = wave_uniform(f.cnt[3 * (int64_t)L]);
    const int nl = wave_uniform(f.cnt[3 * (int64_t)L + 1]);
    const int nr = wave_uniform(f.cnt[3 * (int64_t)L + 2]);
    const const_double_ptr dd = as_const(v.d + base);
    const const_double_ptr src = as_const(v.src + base * m);
    const const_double_ptr zhv = as_const((KERN == 2 ? v.zh : v.d) + base);
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    int64_t ent = 0;  // pole or source entries this wavefront sums per root (kernel timing)
    // one near range [lo, hi) of poles, shifted form, two Newton steps
    auto near = [&](int lo, int hi) {
        ent += hi > lo ? hi - lo : 0;
        for (int i = lo; i < hi; ++i) {
            const double r = rcp_nr((dd[i] - dK) - eta);
            if (KERN == 1) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    if (c < m) acc[c] = __builtin_fma(r, src[(int64_t)i * m + c], acc[c]);
            } else {  // (zhat / t)^2, squared after the division (r^2 zhat^2 can leave range)
                const double qv = r * zhv[i];
                acc[0] = __builtin_fma(qv, qv, acc[0]);
            }
        }
    };
    if (nn < 0) {  // lists overflowed: every pole directly, split over the wavefronts
        near(wave_uniform((int)(((int64_t)n * wv) / S)), wave_uniform((int)(((int64_t)n * (wv + 1)) / S)));
    } else {
        for (int e = 0; e < nn; ++e) {
            const int lo0 = wave_uniform(f.near_lo[(int64_t)L * FMM_NEAR_MAX + e]);
            const int hi0 = wave_uniform(f.near_hi[(int64_t)L * FMM_NEAR_MAX + e]);
            near(lo0 + (int)(((int64_t)(hi0 - lo0) * wv) / S),
                 lo0 + (int)(((int64_t)(hi0 - lo0) * (wv + 1)) / S));
        }
        // far boxes of both sides, lambda-form, one Newton step
        for (int e = wv; e < nl + nr; e += S) {
            const int g = wave_uniform(e < nl ? f.far_l[(int64_t)L * FMM_FAR_MAX + e]
                                              : f.far_r[(int64_t)L * FMM_FAR_MAX + e - nl]);
            const const_double_ptr nd = as_const(v.vnode + (int64_t)g * FMM_P);
            const const_double_ptr ww = as_const(v.vw + (int64_t)g * FMM_P * m);
            ent += FMM_P;
#pragma unroll 4
            for (int q = 0; q < FMM_P; ++q) {
                const double r = rcp_nr1(nd[q] - x);
                if (KERN == 1) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (c < m) acc[c] = __builtin_fma(r, ww[q * m + c], acc[c]);
                } else {
                    acc[0] = __builtin_fma(r * r, ww[q], acc[0]);
                }
            }
        }
    }
    const unsigned long long rows = (unsigned long long)__popcll(__ballot(active));
    if (v.work && lane == 0) {  // kernel timing: algorithmic flops of this wavefront's share
        const unsigned long long per = KERN == 1 ? 2 * (unsigned long long)m + 3 : 6;
        atomicAdd(v.work, rows * (unsigned long long)ent * per +
                              (wv == 0 && KERN == 1 ? rows * (unsigned long long)m : 0));
    }
    if (S > 1) {
        if (wv > 0)
#pragma unroll
            for (int c = 0; c < NC; ++c) red[((wv - 1) * NC + c) * WAVE + lane] = acc[c];
        __syncthreads();
        if (wv == 0)
            for (int w = 1; w < S; ++w)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] += red[((w - 1) * NC + c) * WAVE + lane];
        __syncthreads();
    }
    if (active && wv == 0) {
        if (KERN == 1) {
            const double post = v.post[base + j];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < m) v.Y[base + j + (int64_t)c * v.ldy] = post * acc[c];
        } else {
            v.bout[base + j] = 1.0 / sqrt(acc[0]);
        }
    }
}

// blockDim.x = 64 S; dynamic LDS: (S - 1) NC doubles per lane
template <int KERN, int NC>
__global__ __launch_bounds__(512) void k_fmmv_eval(SolveArgs it, FmmArgs f, FmmVec v, Queue *q) {
    extern __shared__ double red[];
    __shared__ int slot;
    for_each_item(q, it.ntiles, &slot, [&](int item) {
        fmmv_item<KERN, NC>(it, f, v, it.tiles[item], red);
    });
}

// ---------------------------------------------------------------------------------------
// Y = Qhat^T X through the FMM on MFMA: for a 64-root work item the near poles and the far
// boxes' equivalent sources form one gathered reduction dimension, and the product
//     Y_j,c = b_j sum_k 1/((s_k - d_{K_j}) - eta_j) W_k,c
// (s_k a pole or a Chebyshev node, W_k,c its weight) is the dense contraction of the
// direct apply: 64-source chunks are staged through LDS (the next chunk's data in
// registers while the current one is multiplied), each wavefront generates its 16 x 4
// slices of the Cauchy block and feeds v_mfma_f64_16x16x4f64.  Every source uses the
// shifted difference, never less accurate than the lambda-form.
// ---------------------------------------------------------------------------------------
constexpr int FV_K = 64;            // sources per chunk
constexpr int FV_LD = FV_K + 1;

// The chunks of an item (built once per item in LDS): near ranges in 64-pole chunks, then
// the far boxes 4 at a time (64 equivalent sources).  kind 0: poles [a, a + cnt); kind 1:
// far boxes fbox[a .. a + cnt).
// (at most FMM_NEAR_MAX near leaves of at most 1024 poles, the largest leaf the options
// allow; a run of adjacent leaves has no more chunks than its leaves, since every leaf but
// a problem's last holds a multiple of 64 poles)
constexpr int FV_MAXCH = FMM_NEAR_MAX * (1024 / FV_K) + (2 * FMM_FAR_MAX + 3) / 4;

static_assert(FV_K * 16 == 4 * 256, "a chunk's 64 sources x 16 columns: four per thread");

struct FvStage {
    double2 sd;    // source position and, with fuse_b, zhat (near poles) or the weight of
                   // zhat^2 (far equivalent sources) (threads < 64)
    double w[4];   // weights: element e = tid + 256 i -> source e / 16, column e % 16 (the
                   // weights are stored source-major, so 16 threads read a source's row)
};

// TRANS 0 (sums over the roots): a near source is root j, staged as (d_{K_j}, eta_j) for
// the shifted difference (d_i - d_{K_j}) - eta_j; a far one as (node, 0)
template <int TRANS>
__device__ __forceinline__ void fv_fetch(const FmmVec &v, int64_t base, int n, const int *fbox,
                                         int4 ch, FvStage &st) {
    const int tid = threadIdx.x;
    const int m = v.m;
    // weight element i of this thread: source r16 + 16 i of the chunk, column c
    const int c = tid & 15, r16 = tid >> 4;
    if (ch.x == 0) {
        if (tid < FV_K) {
            const int j = ch.y + tid;
            if (tid >= ch.z) st.sd = make_double2(0.0, 0.0);
            else if (TRANS == 0)
                st.sd = make_double2(v.d[base + clamp_idx(v.origin[base + j], n)], v.eta[base + j]);
            else
                st.sd = make_double2(v.d[base + j], v.fuse_b ? v.zh[base + j] : 0.0);
        }
        const double *srow = v.src + (base + ch.y + r16) * m + c;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            st.w[i] = (r16 + 16 * i < ch.z && c < m) ? srow[(int64_t)16 * i * m] : 0.0;
    } else {
        // far chunk: box i of the chunk holds its FMM_P = 16 sources r16
        if (tid < FV_K) {
            const int bx = tid / FMM_P, qn = tid % FMM_P;
            const int64_t sq = bx < ch.z ? (int64_t)fbox[ch.y + bx] * FMM_P + qn : -1;
            st.sd = sq >= 0 ? make_double2(v.vnode[sq], v.fuse_b ? v.vw[sq * m + m - 1] : 0.0)
                            : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            st.w[i] = (i < ch.z && c < m)
                          ? v.vw[((int64_t)fbox[ch.y + i] * FMM_P + r16) * m + c]
                          : 0.0;
    }
}

struct FvShared {
    double Xs[16 * FV_LD];
    double2 Sd[FV_K];
    int4 ctab[FV_MAXCH];
    int fbox[2 * FMM_FAR_MAX];
    int nch;
};

template <int TRANS>
__device__ void fmmv_item_mfma(const SolveArgs &it, const FmmArgs &f, const FmmVec &v, Tile t,
                               FvShared &sh) {
    const int p = t.prob;
    const int64_t base = it.off[p];
    const int n = (int)(it.off[p + 1] - base);
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int o0 = t.row0;
    const int m = v.m;
    const int mo = m - v.fuse_b;  // output columns
    if (f.status[p] & ~SUPERDC_ST_NOCONV) {
        const double nan = __builtin_nan("");
        for (int e = threadIdx.x; e < FV_K * mo; e += blockDim.x) {
            const int r = o0 + (e % FV_K), c = e / FV_K;
            if (r < n) v.Y[base + r + (int64_t)c * v.ldy] = nan;
        }
        if (v.fuse_b && threadIdx.x < FV_K && o0 + (int)threadIdx.x < n)
            v.bout[base + o0 + threadIdx.x] = nan;
        return;
    }
    const int qf = f.fmm_of[p];
    const int L = wave_uniform(f.leaf_off[qf] + t.row0 / f.leaf);
    const int nn = wave_uniform(f.cnt[3 * (int64_t)L]);
    const bool direct = nn < 0;  // overflowed lists: every pole, 64 at a time
    __syncthreads();  // the previous item's reads of the tables are done
    if (!direct) {
        const int nl = f.cnt[3 * (int64_t)L + 1], nr = f.cnt[3 * (int64_t)L + 2];
        for (int e = threadIdx.x; e < nl + nr; e += blockDim.x)
            sh.fbox[e] = e < nl ? f.far_l[(int64_t)L * FMM_FAR_MAX + e]
                                : f.far_r[(int64_t)L * FMM_FAR_MAX + e - nl];
        if (threadIdx.x == 0) {
            int c = 0;
            for (int e = 0; e < nn; ++e) {
                const int lo = f.near_lo[(int64_t)L * FMM_NEAR_MAX + e];
                const int hi = f.near_hi[(int64_t)L * FMM_NEAR_MAX + e];
                for (int a = lo; a < hi; a += FV_K) sh.ctab[c++] = make_int4(0, a, min(FV_K, hi - a), 0);
            }
            for (int a = 0; a < nl + nr; a += 4) sh.ctab[c++] = make_int4(1, a, min(4, nl + nr - a), 0);
            sh.nch = c;
        }
    } else if (threadIdx.x == 0) {
        sh.nch = (n + FV_K - 1) / FV_K;
    }
    __syncthreads();
    const int nch = wave_uniform(sh.nch);
    auto chunk = [&](int ci) -> int4 {
        return direct ? make_int4(0, ci * FV_K, min(FV_K, n - ci * FV_K), 0) : sh.ctab[ci];
    };
    // the root of the Cauchy rows this lane generates: row o0 + 16 wv + lane%16
    const int orow = o0 + wv * 16 + (lane & 15);
    const bool ovalid = orow < n;
    const int oc = ovalid ? orow : n - 1;
    // the target of the Cauchy row: root (d_K, eta), or (TRANS 0) pole d_i
    const double ra = TRANS ? v.d[base + clamp_idx(v.origin[base + oc], n)] : v.d[base + oc];
    const double rb = TRANS ? v.eta[base + oc] : 0.0;
    v4d_f acc = v4d_f{0.0, 0.0, 0.0, 0.0};
    // fuse_b: this lane's share of b's sum for its Cauchy row (the sources it generates
    // entries for), on the VALU beside the multiply: one column does not need the MFMA
    double bsum = 0.0;
    const bool fb = v.fuse_b != 0;
    FvStage st;
    int4 cur = chunk(0);
    fv_fetch<TRANS>(v, base, n, sh.fbox, cur, st);
    int64_t ent = 0;  // near poles and far sources summed per root (kernel timing)
    for (int ci = 0; ci < nch; ++ci) {
        __syncthreads();  // the previous chunk's reads of Xs/Sd are done
        if (threadIdx.x < FV_K) sh.Sd[threadIdx.x] = st.sd;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = threadIdx.x + 256 * i;
            sh.Xs[(e & 15) * FV_LD + (e >> 4)] = st.w[i];
        }
        __syncthreads();
        const int nvalid = wave_uniform(cur.x == 0 ? cur.z : cur.z * FMM_P);
        const bool cur_near = cur.x == 0;
        ent += nvalid;
        if (ci + 1 < nch) {
            cur = chunk(ci + 1);
            fv_fetch<TRANS>(v, base, n, sh.fbox, cur, st);  // in flight during the multiply
        }
        // one slice of 4 sources: the Cauchy entries of this lane's row (one reciprocal
        // with a Newton step each) into the MFMA; MASK: a partial chunk, whose padding
        // entries are zeroed (a padding source may sit on a row's target).  A row past the
        // problem's end (ovalid false) only feeds its own output row, never written.
#define SDC_FV_SLICE(MASK)                                                              \
    {                                                                                   \
        const int sl = kk + (lane >> 4);                                                \
        const double2 sdv = sh.Sd[sl];                                                  \
        const double tt = TRANS ? (sdv.x - ra) - rb : (ra - sdv.x) - sdv.y;             \
        const double av = (!(MASK) || sl < nvalid) ? rcp_nr1(tt) : 0.0;                 \
        const double bv = sh.Xs[(lane & 15) * FV_LD + sl];                              \
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);               \
        if (fb) {                                                                       \
            if (cur_near) { /* (zhat / t)^2: squared after the division */              \
                const double qv = av * sdv.y;                                           \
                bsum = fma(qv, qv, bsum);                                               \
            } else { /* far sources: weights of zhat^2, t bounded away from 0 */        \
                bsum = fma(av * av, sdv.y, bsum);                                       \
            }                                                                           \
        }                                                                               \
    }
        if (nvalid == FV_K) {
#pragma unroll 4
            for (int kk = 0; kk < FV_K; kk += 4) SDC_FV_SLICE(false)
        } else {
#pragma unroll 4
            for (int kk = 0; kk < FV_K; kk += 4) SDC_FV_SLICE(true)
        }
#undef SDC_FV_SLICE
        mfma_drain();  // before any copy of the accumulators between chunks
    }
    if (fb) {  // the four lanes of a Cauchy row (lane % 16) hold its partial sums
        bsum += __shfl_xor(bsum, 16);
        bsum += __shfl_xor(bsum, 32);
    }
    if (v.work && threadIdx.x == 0) {  // kernel timing: the item's algorithmic flops
        const unsigned long long rows = (unsigned long long)min(FV_K, n - o0);
        atomicAdd(v.work, rows * (unsigned long long)ent * (2 * (unsigned long long)m + 3) +
                              2 * rows * (unsigned long long)mo);
    }
    mfma_drain();
    // v_mfma_f64_16x16x4f64 returns D[4 r + lane/16][lane % 16] in accumulator r
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = o0 + wv * 16 + 4 * r + (lane >> 4);
        const int col = lane & 15;
        double post;
        if (fb) {  // b's sum of this row is held by the lanes that generated its entries
            post = 1.0 / sqrt(__shfl(bsum, 4 * r + (lane >> 4)));
            if (row < n && col == 0) v.bout[base + row] = post;
        } else {
            post = row < n ? v.post[base + row] : 0.0;
        }
        if (row < n && col < mo) v.Y[base + row + (int64_t)col * v.ldy] = post * acc[r];
    }
}

template <int TRANS>
__global__ __launch_bounds__(256) void k_fmmv_eval_mfma(SolveArgs it, FmmArgs f, FmmVec v,
                                                        Queue *q) {
    __shared__ FvShared sh;
    __shared__ int slot;
    for_each_item(q, it.ntiles, &slot, [&](int item) {
        fmmv_item_mfma<TRANS>(it, f, v, it.tiles[item], sh);
    });
}

// ---------------------------------------------------------------------------------------
// Loewner far field: box moments.  LEAVES = true: every leaf from its poles and roots;
// LEAVES = false: every used box above the leaves from its leaves' moments, translated to
// the box's centre and half-width (t_box = alpha + beta t_leaf):
//     M_k = sum_m C(k, m) alpha^(k-m) beta^m M_m(leaf)
// (M_0 = 0: each pole-root pair carries opposite unit charges).  One workgroup per box; the
// per-thread partial moments are added in a fixed order through LDS.

// binomial coefficient C(k, m) for k <= FMML_K (integers below 2^53: exact in double); used
// with constant arguments only, so every coefficient is a literal of the unrolled loops
__host__ __device__ constexpr double binom(int k, int m) {
    double c = 1.0;
    for (int j = 1; j <= m; ++j) c = c * (k - m + j) / j;
    return c;
}
// ---------------------------------------------------------------------------------------
template <bool LEAVES>
__global__ __launch_bounds__(LEAVES ? 64 : 256, LEAVES ? 1 : 4) void k_fmml_moments(FmmArgs f, FmmlArgs l) {
    __shared__ double part[64][FMML_K + 1];
    __shared__ double part2[LEAVES ? 1 : 64][FMML_K + 1];
    const int g = LEAVES ? f.leaf_box[blockIdx.x] : f.upper_box[blockIdx.x];
    if (!LEAVES && f.used[g] != f.gen) return;
    const int qf = f.box_fmm[g];
    const int p = f.fmm_prob[qf];
    const int64_t base = f.off[p];
    const int n = (int)(f.off[p + 1] - base);
    const int hidx = g - f.box_off[qf];
    const int H = f.height[qf];
    int h = 0;
    while ((2 << h) - 1 <= hidx) ++h;
    if (f.status[p] & ~SUPERDC_ST_NOCONV) return;
    const int bi = hidx - ((1 << h) - 1);
    const int64_t span = (int64_t)f.leaf << (H - h);
    const int lo = (int)min((int64_t)n, bi * span), hi = (int)min((int64_t)n, (bi + 1) * span);
    if (lo >= hi) return;
    if (LEAVES && l.pack) {  // the leaf's poles packed here (the same arithmetic as k_fmml_pack)
        for (int j = lo + (int)threadIdx.x; j < hi; j += blockDim.x) {
            const double dj = l.d[base + j];
            const double dK = l.d[base + clamp_idx(l.origin[base + j], n)];
            const double ej = l.eta[base + j];
            const double delta = (dK - dj) + ej;
            l.pd[base + j] = make_double2(dj, delta);
            if (l.ke) l.ke[base + j] = make_double2(dK, ej);
            if (j == n - 1) l.tail[p] = delta;
        }
        __syncthreads();
    }
    const double2 *pd = l.pd + base;
    const double a = pd[lo].x, b = pd[hi - 1].x + pd[hi - 1].y;  // poles and roots of the box
    const double c = 0.5 * (a + b), hw = 0.5 * (b - a), ihw = 1.0 / hw;
    const int tid = threadIdx.x;
    double M[FMML_K];
#pragma unroll
    for (int k = 0; k < FMML_K; ++k) M[k] = 0.0;
    if (LEAVES) {
        for (int j = lo + tid; j < hi; j += blockDim.x) {
            const double t = (pd[j].x - c) * ihw, D = pd[j].y * ihw, tD = t + D;
            double P = D, tk = 1.0;
#pragma unroll
            for (int k = 0; k < FMML_K; ++k) {
                M[k] += P;  // P = (t + D)^(k+1) - t^(k+1)
                tk *= t;
                P = __builtin_fma(tD, P, D * tk);
            }
        }
    } else {
        const int leaf0 = (1 << H) - 1 + bi * (1 << (H - h));
        const int nleaf = (int)((hi - lo + f.leaf - 1) / f.leaf);
        for (int e = tid; e < nleaf; e += blockDim.x) {
            const int gl = f.box_off[qf] + leaf0 + e;
            const double2 gc = l.geo[gl];
            const double al = (gc.x - c) * ihw, be = gc.y * ihw;
            const double *Ml = l.mom + (int64_t)gl * FMML_K;
            // moment m of the leaf spread over k >= m: C(k, m) alpha^(k-m) beta^m M_m, the
            // power of alpha built up along k (no row of coefficients kept: few registers)
            double bm = 1.0;
#pragma unroll
            for (int m = 1; m <= FMML_K; ++m) {
                bm *= be;
                double q = Ml[m - 1] * bm;  // alpha^(k-m) beta^m M_m
#pragma unroll
                for (int k = m; k <= FMML_K; ++k) {
                    M[k - 1] = __builtin_fma(binom(k, m), q, M[k - 1]);
                    q *= al;
                }
            }
        }
    }
    if (LEAVES) {  // one wavefront: lane k adds column k over the 64 lanes in order
#pragma unroll
        for (int k = 0; k < FMML_K; ++k) part[tid][k] = M[k];
        __syncthreads();
        if (tid < FMML_K) {
            double sk = 0.0;
            for (int u = 0; u < 64; ++u) sk += part[u][tid];
            l.mom[(int64_t)g * FMML_K + tid] = sk;
        }
    } else {
        // only the first nleaf threads hold moments.  Beyond 64 leaves the four wavefronts
        // are folded onto the first, (w0 + w2) + (w1 + w3), through two 64-row buffers; then
        // lane k adds column k over the rows in use, in order (one pass, no barrier per level
        // of a tree)
        const int nleaf = (int)((hi - lo + f.leaf - 1) / f.leaf);
        const int wv = tid / WAVE, ln = tid % WAVE;
        if (nleaf > WAVE) {
            if (wv >= 2) {
#pragma unroll
                for (int k = 0; k < FMML_K; ++k) (wv == 2 ? part : part2)[ln][k] = M[k];
            }
            __syncthreads();
            if (wv < 2) {
#pragma unroll
                for (int k = 0; k < FMML_K; ++k) M[k] += (wv == 0 ? part : part2)[ln][k];
            }
            __syncthreads();
            if (wv == 1) {
#pragma unroll
                for (int k = 0; k < FMML_K; ++k) part[ln][k] = M[k];
            }
            __syncthreads();
            if (wv == 0) {
#pragma unroll
                for (int k = 0; k < FMML_K; ++k) M[k] += part[ln][k];
            }
            __syncthreads();
        }
        if (wv == 0) {
#pragma unroll
            for (int k = 0; k < FMML_K; ++k) part[ln][k] = M[k];
        }
        __syncthreads();
        if (tid < FMML_K) {
            double sk = 0.0;
            for (int u = 0; u < min(nleaf, WAVE); ++u) sk += part[u][tid];
            l.mom[(int64_t)g * FMML_K + tid] = sk;
        }
    }
    if (tid == 0) l.geo[g] = make_double2(c, hw);
}

hipError_t launch_fmml_moments(const FmmArgs &f, const FmmlArgs &l, hipStream_t s) {
    if (f.nboxes <= 0) return hipSuccess;
    SDC_LAUNCH(KID_FMML_MOMENTS, k_fmml_moments<true>, dim3(f.nleaves), dim3(64), 0, s, f, l);
    if (f.nupper > 0)
        SDC_LAUNCH(KID_FMML_MOMENTS, k_fmml_moments<false>, dim3(f.nupper), dim3(256), 0, s, f,
                   l);
    return hipGetLastError();
}

// (d_j, delta_j) with delta_j = lambda_j - d_j = (d_{K_j} - d_j) + eta_j; one lane per entry
__global__ __launch_bounds__(64) void k_fmml_pack(FmmvPackArgs a) {
    const Tile t = a.tiles[blockIdx.x];
    const int64_t base = a.off[t.prob];
    const int n = (int)(a.off[t.prob + 1] - base);
    const int j = t.row0 + lane_id();
    if (j >= n) return;
    const double dj = a.d[base + j];
    const double dK = a.d[base + clamp_idx(a.origin[base + j], n)];
    const double ej = a.eta[base + j];
    const double delta = (dK - dj) + ej;
    a.pairs[base + j] = make_double2(dj, delta);
    if (a.ke) a.ke[base + j] = make_double2(dK, ej);
    if (j == n - 1) a.tail[t.prob] = delta;
}

hipError_t launch_fmml_pack(const FmmvPackArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    SDC_LAUNCH(KID_FMML_PACK, k_fmml_pack, dim3(a.ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fmmv_pack(const FmmvPackArgs &a, const FmmVec &v, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    SDC_LAUNCH(KID_FMMV_PACK, k_fmmv_pack, dim3(a.ntiles), dim3(64), 0, s, a, v);
    return hipGetLastError();
}

hipError_t launch_fmmv_sources(const FmmArgs &f, const FmmVec &v, const FmmvPackArgs *pk,
                               hipStream_t s) {
    if (f.nboxes <= 0) return hipSuccess;
    FmmvPackArgs none{};
    SDC_LAUNCH(KID_FMMV_SOURCES, k_fmmv_sources<true>, dim3(f.nleaves), dim3(64), 0, s, f, v,
               pk ? *pk : none);
    if (f.nupper_item > 0)
        SDC_LAUNCH(KID_FMMV_SOURCES, k_fmmv_sources<false>, dim3(f.nupper_item), dim3(256), 0, s,
                   f, v, none);
    if (f.nsplit > 0)
        SDC_LAUNCH(KID_FMMV_SOURCES, k_fmmv_sources_sum, dim3(f.nsplit), dim3(FMM_P * FMMV_MAX_M),
                   0, s, f, v);
    return hipGetLastError();
}

hipError_t launch_fmmv_eval(const SolveArgs &it, const FmmArgs &f, const FmmVec &v0, int split,
                            Queue *q, int num_cu, hipStream_t s) {
    if (it.ntiles <= 0) return hipSuccess;
    FmmVec v = v0;
    // the MFMA for a dense enough block of columns, and for every sum over the roots
    const bool mfma = v.kern == 1 && (v.m >= 4 || v.fuse_b || v.trans == 0);
    v.work = trace_work(mfma ? KID_FMMV_EVAL_MFMA : KID_FMMV_EVAL);
    if (mfma) {
        const dim3 g(q ? min(it.ntiles, num_cu * 4) : it.ntiles);
        if (v.trans == 0)
            SDC_LAUNCH(KID_FMMV_EVAL_MFMA, k_fmmv_eval_mfma<0>, g, dim3(256), 0, s, it, f, v, q);
        else
            SDC_LAUNCH(KID_FMMV_EVAL_MFMA, k_fmmv_eval_mfma<1>, g, dim3(256), 0, s, it, f, v, q);
        return hipGetLastError();
    }
    if (v.trans == 0) return hipErrorInvalidValue;
    const dim3 g(q ? min(it.ntiles, num_cu * max(1, 32 / split)) : it.ntiles), blk(WAVE * split);
    if (v.kern == 2) {
        const size_t lds = sizeof(double) * WAVE * (split - 1) * 1;
        SDC_LAUNCH(KID_FMMV_EVAL, (k_fmmv_eval<2, 1>), g, blk, lds, s, it, f, v, q);
    } else {
        const size_t lds = sizeof(double) * WAVE * (split - 1) * 8;
        SDC_LAUNCH(KID_FMMV_EVAL, (k_fmmv_eval<1, 8>), g, blk, lds, s, it, f, v, q);
    }
    return hipGetLastError();
}

}  // namespace sdc
