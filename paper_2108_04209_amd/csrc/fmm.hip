// fmm.hip -- triangular FMM of the secular sums on gfx950 (Sec. 4.1.2 with the local
// shifting of Sec. 4.2.2).
//
// The poles of a problem are cut by index into leaves (a tree over the leaves, so boxes
// adapt to clustered poles).  Every box is compressed once per solve into FMM_P
// equivalent sources: the Chebyshev nodes s_q of the box's span and the weights
// W_q = sum_{j in box} w_j L_q(d_j) (L_q the Lagrange basis on those nodes), so that
// sum_j w_j K(x, d_j) ~ sum_q W_q K(x, s_q) for any kernel K smooth over the box -- one
// compression serves both 1/(s-x) and 1/(s-x)^2.  Every leaf is compressed from its
// poles; above the leaves only boxes that some target lists as far field are compressed,
// from their leaves' sources.  For each target leaf the tree is walked top down: a box separated from the leaf's targets by sep times its width (and by at
// least 64 pole indices) is far field -- entirely left of every target (it feeds psi, the
// lower triangle) or entirely right (phi, the strictly upper triangle), the directional
// interactions of the triangular FMM; zero blocks never appear.  Leaves that are not far
// are near field and are summed directly in shifted form.  The targets move between
// iterations but the poles do not, so only the solver's pass loop runs per iteration.
#include "fmm.h"

namespace sdc {


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

// Secular equivalent sources of box g.  LEAVES: a leaf from its poles, one wavefront (beside
// the one that builds the leaf's lists).  Upper boxes: a box some target lists as far, four
// wavefronts, from the equivalent sources of its leaves (16 per leaf instead of every pole
// below: the far field of a leaf's sources equals that of its poles to the interpolation
// accuracy, and the box's nodes interpolate it again).  part holds 64 or 256 rows of
// FMM_P + 1 doubles, red 16 of them (upper boxes); tid is the thread's index among the box's
// nt threads (one wavefront for a leaf, which syncs only itself).
template <bool LEAVES>
__device__ __forceinline__ void box_sources(const FmmArgs &f, int g, double *part, double *red,
                                            int tid, int nt) {
    static_assert(FMM_P == 16, "the upper boxes' sum maps 256 threads to 16 x 16");
    const int qf = f.box_fmm[g];
    const int hidx = g - f.box_off[qf];
    const int H = f.height[qf];
    int h = 0;
    while ((2 << h) - 1 <= hidx) ++h;
    const BoxRange rg = box_range(f, g);
    const int lo = rg.lo, hi = rg.hi;
    if (lo >= hi || (f.status[rg.p] & ~SUPERDC_ST_NOCONV)) return;
    const double2 *dw = f.dw + rg.base;
    const double a = dw[lo].x, b = dw[hi - 1].x;
    const double c = 0.5 * (a + b), hw = 0.5 * (b - a);
    if (LEAVES && hi - lo <= FMM_P) {  // few poles: they are their own equivalent sources
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
    const double ihw = 1.0 / hw;
    // the points: the leaf's poles, or the sources of the box's leaves
    const int bi = hidx - ((1 << h) - 1);
    const int leaf0 = f.box_off[qf] + (1 << H) - 1 + bi * (1 << (H - h));
    const int npts = LEAVES ? hi - lo : ((hi - lo + f.leaf - 1) / f.leaf) * FMM_P;
    for (int k = tid; k < npts; k += nt) {
        const double2 pw = LEAVES ? dw[lo + k] : f.eq[(int64_t)leaf0 * FMM_P + k];
        const double t = fmin(1.0, fmax(-1.0, (pw.x - c) * ihw));
        int hit = -1;
        double inv[FMM_P], den = 0.0;
#pragma unroll
        for (int r = 0; r < FMM_P; ++r) {
            const double dlt = t - tq[r];
            if (dlt == 0.0) hit = r;
            inv[r] = lam[r] * rcp_nr(dlt);
            den += inv[r];
        }
        if (hit >= 0) {
            W[hit] += pw.y;  // the point sits on a node
        } else {
            const double s = pw.y * rcp_nr(den);
#pragma unroll
            for (int r = 0; r < FMM_P; ++r) W[r] = __builtin_fma(s, inv[r], W[r]);
        }
    }
    // the threads' partial weights added in a fixed order through LDS (shuffle trees cost
    // several microseconds here): one wavefront, lane q adds column q over the 64 lanes;
    // four, thread (s, q) adds column q over threads 16 s .. 16 s + 15, then lane q the 16
    double wq = 0.0;
#pragma unroll
    for (int r = 0; r < FMM_P; ++r) part[tid * (FMM_P + 1) + r] = W[r];
    if (LEAVES)
        wave_sync();
    else
        __syncthreads();
    if (LEAVES) {
        if (tid < FMM_P)
            for (int u = 0; u < 64; ++u) wq += part[u * (FMM_P + 1) + tid];
    } else {
        const int q = tid & (FMM_P - 1), s0 = tid >> 4;
        double ps = 0.0;
        for (int u = 16 * s0; u < 16 * s0 + 16; ++u) ps += part[u * (FMM_P + 1) + q];
        red[s0 * (FMM_P + 1) + q] = ps;
        __syncthreads();
        if (tid < FMM_P)
            for (int u = 0; u < 16; ++u) wq += red[u * (FMM_P + 1) + tid];
    }
    if (tid < FMM_P) f.eq[(int64_t)g * FMM_P + tid] = make_double2(c + hw * tq[tid], wq);
}

// the used upper boxes (the leaves are compressed by the lists launch of the solver)
__global__ __launch_bounds__(256) void k_fmm_boxes(FmmArgs f) {
    __shared__ double part[256 * (FMM_P + 1)];
    __shared__ double red[16 * (FMM_P + 1)];
    const int g = f.upper_box[blockIdx.x];
    if (f.used[g] != f.gen) return;
    box_sources<false>(f, g, part, red, threadIdx.x, blockDim.x);
}

// interaction lists: one wavefront per target leaf walks its problem's tree level by level.
// Lane i holds the i-th candidate box of the level (children of the previous level's open
// boxes, left to right).  A candidate separated from the leaf is far (flagged as used), a
// leaf that is not is near, any other box opens its two children for the next level.  More
// than 64 candidates on a level, or full lists, make the leaf fall back to direct sums.
template <bool EQ>
__global__ __launch_bounds__(EQ ? 2 * WAVE : WAVE) void k_fmm_lists(FmmArgs f) {
    __shared__ int slot[WAVE];
    __shared__ double part[EQ ? WAVE * (FMM_P + 1) : 1];
    const int L = blockIdx.x;
    // EQ (the solver's lists): a second wavefront compresses the leaf itself meanwhile
    if (EQ && threadIdx.x >= WAVE) {
        box_sources<true>(f, f.leaf_box[L], part, nullptr, threadIdx.x - WAVE, WAVE);
        return;
    }
    const int lane = threadIdx.x;
    const int q = f.leaf_fmm[L];
    const int p = f.fmm_prob[q];
    const int64_t base = f.off[p];
    const int n = (int)(f.off[p + 1] - base);
    const int H = f.height[q];
    const int li = L - f.leaf_off[q];
    const int i0 = li * f.leaf, i1 = min(n, i0 + f.leaf);
    int32_t *cnt = f.cnt + 3 * (int64_t)L;
    if (f.status[p] & ~SUPERDC_ST_NOCONV) {
        if (lane == 0) cnt[0] = -1;
        return;
    }
    const double2 *dw = f.dw + base;
    // the target leaf's span: its roots lie in [d_first, d_next] (the solver's targets), or
    // the target points themselves (poles, for the sums over the roots)
    const double xa = f.tpos ? f.tpos[base + i0] : dw[i0].x;
    const double xb = f.tpos ? f.tpos[base + i1 - 1]
                             : (i1 < n ? dw[i1].x : dw[n - 1].x + fmax(f.tail[p], 0.0));
    int32_t *far_l = f.far_l + (int64_t)L * FMM_FAR_MAX;
    int32_t *far_r = f.far_r + (int64_t)L * FMM_FAR_MAX;
    int32_t *near_lo = f.near_lo + (int64_t)L * FMM_NEAR_MAX;
    int32_t *near_hi = f.near_hi + (int64_t)L * FMM_NEAR_MAX;
    int hidx = 0, ncand = 1;  // the root
    int nn = 0, nl = 0, nr = 0, ndl = 0, ndr = 0, nel = 0, ner = 0;
    bool overflow = false;
    for (int h = 0; h <= H && ncand > 0 && !overflow; ++h) {
        const bool valid = lane < ncand;
        const int g = f.box_off[q] + hidx;
        const int i = hidx - ((1 << h) - 1);
        const int64_t span = (int64_t)f.leaf << (H - h);
        const int lo = (int)min((int64_t)n, i * span), hi = (int)min((int64_t)n, (i + 1) * span);
        const bool live = valid && lo < hi;  // empty boxes are dropped
        // the box's span: its first and last point
        const double2 ab = live ? make_double2(dw[lo].x, dw[hi - 1].x) : make_double2(0.0, 0.0);
        const double width = ab.y - ab.x;
        const bool fl = live && ab.y < xa && xa - ab.y >= f.sep * width && hi <= i0 - TILE;
        const bool fr = live && !fl && ab.x > xb && ab.x - xb >= f.sep * width && lo >= i1 + TILE;
        // also separated from the whole target interval: into the leaf's local expansion
        const double wloc = f.sep_loc * (xb - xa);
        const bool loc = (fl && xa - ab.y >= wloc) || (fr && ab.x - xb >= wloc);
        const bool nr_leaf = live && !fl && !fr && h == H;
        // a near leaf that is that far from the target interval (and a tile of indices
        // away) enters the local expansion with its poles
        const bool nloc = nr_leaf && ((ab.y < xa && xa - ab.y >= wloc && hi <= i0 - TILE) ||
                                      (ab.x > xb && ab.x - xb >= wloc && lo >= i1 + TILE));
        const bool open = live && !fl && !fr && h < H;
        // far boxes, appended in lane order
        const unsigned long long ml = __ballot(fl), mr = __ballot(fr);
        const int rl = __builtin_amdgcn_mbcnt_hi((unsigned)(ml >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)ml, 0u));
        const int rr = __builtin_amdgcn_mbcnt_hi((unsigned)(mr >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mr, 0u));
        if (nl + __popcll(ml) > FMM_FAR_MAX || nr + __popcll(mr) > FMM_FAR_MAX) {
            overflow = true;
            break;
        }
        if (fl) {
            far_l[nl + rl] = g;
            f.used[g] = f.gen;
        }
        if (fr) {
            far_r[nr + rr] = g;
            f.used[g] = f.gen;
        }
        nl += __popcll(ml);
        nr += __popcll(mr);
        // split for the solver: the far boxes summed directly from the front of far_ld/far_rd,
        // those in the expansion from the back (both together fit, as the lists did)
        {
            const unsigned long long mdl = __ballot(fl && !loc), mdr = __ballot(fr && !loc);
            const unsigned long long mel = __ballot(fl && loc), mer = __ballot(fr && loc);
            auto rank = [&](unsigned long long mk) {
                return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
            };
            int32_t *ld = f.far_ld + (int64_t)L * FMM_FAR_MAX, *rd = f.far_rd + (int64_t)L * FMM_FAR_MAX;
            if (fl) {
                if (loc) ld[FMM_FAR_MAX - 1 - (nel + rank(mel))] = g;
                else ld[ndl + rank(mdl)] = g;
            }
            if (fr) {
                if (loc) rd[FMM_FAR_MAX - 1 - (ner + rank(mer))] = g;
                else rd[ndr + rank(mdr)] = g;
            }
            ndl += __popcll(mdl);
            ndr += __popcll(mdr);
            nel += __popcll(mel);
            ner += __popcll(mer);
        }
        // near leaves (ascending), adjacent ones of the same kind (direct or into the local
        // expansion) merged into one range
        const unsigned long long mn = __ballot(nr_leaf);
        if (mn) {
            if (__popcll(mn) > FMM_NEAR_MAX) {
                overflow = true;
                break;
            }
            const unsigned long long below = lane ? (mn & ((1ull << lane) - 1)) : 0ull;
            const int prev = below ? 63 - __builtin_clzll(below) : -1;
            const int hprev = __shfl(hi, prev < 0 ? 0 : prev);
            const bool lprev = __shfl((int)nloc, prev < 0 ? 0 : prev) != 0;
            const bool start = nr_leaf && (prev < 0 || hprev != lo || lprev != nloc);
            const unsigned long long ms = __ballot(start);
            const int rs = __builtin_amdgcn_mbcnt_hi((unsigned)(ms >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)ms, 0u));
            // the run of a start lane ends at the last near lane before the next start
            const unsigned long long after = lane < 63 ? (ms & ~((2ull << lane) - 1)) : 0ull;
            const int nxt = after ? __builtin_ctzll(after) : 64;
            const unsigned long long upto = nxt < 64 ? (mn & ((1ull << nxt) - 1)) : mn;
            const int last = upto ? 63 - __builtin_clzll(upto) : 0;
            const int hend = __shfl(hi, last);
            if (start) {
                near_lo[nn + rs] = lo;
                near_hi[nn + rs] = hend;
                f.near_lf[(int64_t)L * FMM_NEAR_MAX + nn + rs] = nloc ? 1 : 0;
            }
            nn += __popcll(ms);
        }
        // the children of the open boxes, in order, are the next level's candidates
        const unsigned long long mo = __ballot(open);
        const int no = __popcll(mo);
        if (2 * no > WAVE) {
            overflow = true;
            break;
        }
        const int ro = __builtin_amdgcn_mbcnt_hi((unsigned)(mo >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mo, 0u));
        wave_sync();
        if (open) slot[ro] = hidx;
        wave_sync();
        ncand = 2 * no;
        hidx = lane < ncand ? 2 * slot[lane >> 1] + 1 + (lane & 1) : 0;
    }
    if (lane == 0) {
        cnt[0] = overflow ? -1 : nn;  // -1: the leaf falls back to direct sums
        cnt[1] = nl;
        cnt[2] = nr;
        f.cntd[2 * (int64_t)L] = ndl;
        f.cntd[2 * (int64_t)L + 1] = ndr;
        f.loc_ab[L] = make_double2(0.5 * (xa + xb), 0.5 * (xb - xa));
    }
}

// Local expansion of a target leaf (one workgroup per leaf): the far field of the boxes
// listed for it in the expansion and of the near ranges flagged for it (their poles
// themselves), psi_far(x) = sum W_q / (s_q - x) over the sources left of the leaf and
// phi_far over those right of it, with their derivatives, sampled at the FMM_PL Chebyshev
// nodes of the target interval [xa, xb] (which holds every iterate of the leaf's roots) and
// turned into Chebyshev coefficients, so that the solver evaluates four short series per
// root and iteration instead of the sources one by one.  Every source is at least sep_loc
// interval widths from the interval.  Thread (node m, part u) sums the boxes e = u (mod
// LOC_PARTS), two sources per reciprocal (all on one side of the node), and every
// LOC_PARTS-th pole of the flagged ranges; the parts are added in order.
constexpr int LOC_PARTS = 16;
__global__ __launch_bounds__(FMM_PL * LOC_PARTS) void k_fmm_local(FmmArgs f) {
    __shared__ double part[LOC_PARTS][4][FMM_PL];  // [part][function][node]
    __shared__ double val[4][FMM_PL];              // [function][node]
    __shared__ double Tkm[FMM_PL][FMM_PL];         // T_k(t_m) = cos(k (2m + 1) pi / 2P)
    const int L = blockIdx.x;
    const int tid = threadIdx.x;
    for (int e = tid; e < FMM_PL * FMM_PL; e += blockDim.x)
        Tkm[e / FMM_PL][e % FMM_PL] =
            cos((double)((e / FMM_PL) * (2 * (e % FMM_PL) + 1)) * 3.14159265358979323846 /
                (2.0 * FMM_PL));
    const int q = f.leaf_fmm[L];
    const int p = f.fmm_prob[q];
    if (f.status[p] & ~SUPERDC_ST_NOCONV) return;
    const int nn = f.cnt[3 * (int64_t)L];
    if (nn < 0) return;  // the leaf sums every pole directly
    const int nel = f.cnt[3 * (int64_t)L + 1] - f.cntd[2 * (int64_t)L];
    const int ner = f.cnt[3 * (int64_t)L + 2] - f.cntd[2 * (int64_t)L + 1];
    const double2 cw = f.loc_ab[L];
    const int m = tid % FMM_PL, u = tid / FMM_PL;
    const double tm = cheb_node(m, FMM_PL);
    const double x = cw.x + cw.y * tm;
    double ps = 0.0, dps = 0.0, ph = 0.0, dph = 0.0;
    for (int e = u; e < nel + ner; e += LOC_PARTS) {
        const bool left = e < nel;
        const int k = left ? e : e - nel;
        const int g = (left ? f.far_ld : f.far_rd)[(int64_t)L * FMM_FAR_MAX + FMM_FAR_MAX - 1 - k];
        const double2 *eq = f.eq + (int64_t)g * FMM_P;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll 2
        for (int r = 0; r < FMM_P; r += 2) {
            // w0/t0 + w1/t1 = (w0 t1 + w1 t0)/(t0 t1), and the squares likewise
            const double2 a = eq[r], b = eq[r + 1];
            const double t0 = a.x - x, t1 = b.x - x;
            const double pr = fabs(t0 * t1);
            if (pr > 0x1p-900 && pr < 0x1p900) {
                const double R = rcp_nr(t0 * t1);
                const double u0 = a.y * t1, u1 = b.y * t0;
                s0 = __builtin_fma(u0 + u1, R, s0);
                s1 = __builtin_fma(__builtin_fma(u0, t1, u1 * t0) * R, R, s1);
            } else {  // the product would leave the exponent range: one source at a time
                const double r0 = rcp_nr(t0), r1 = rcp_nr(t1);
                s0 += a.y * r0 + b.y * r1;
                s1 += a.y * r0 * r0 + b.y * r1 * r1;
            }
        }
        if (left) {
            ps += s0;
            dps += s1;
        } else {
            ph += s0;
            dph += s1;
        }
    }
    // flagged near ranges: their poles, left of the leaf into psi, right of it into phi
    {
        const int64_t base = f.off[p];
        const int i0 = (L - f.leaf_off[q]) * f.leaf;
        const double2 *dw = f.dw + base;
        for (int e = 0; e < nn; ++e) {
            if (!f.near_lf[(int64_t)L * FMM_NEAR_MAX + e]) continue;
            const int lo = f.near_lo[(int64_t)L * FMM_NEAR_MAX + e];
            const int hi = f.near_hi[(int64_t)L * FMM_NEAR_MAX + e];
            double s0 = 0.0, s1 = 0.0;
            for (int j = lo + u; j < hi; j += LOC_PARTS) {
                const double2 pw = dw[j];
                const double r = rcp_nr(pw.x - x);
                const double wr = pw.y * r;
                s0 += wr;
                s1 = __builtin_fma(wr, r, s1);
            }
            if (hi <= i0) {
                ps += s0;
                dps += s1;
            } else {
                ph += s0;
                dph += s1;
            }
        }
    }
    part[u][0][m] = ps;
    part[u][1][m] = dps;
    part[u][2][m] = ph;
    part[u][3][m] = dph;
    __syncthreads();
    if (tid < 4 * FMM_PL) {
        const int fn = tid / FMM_PL, mm = tid % FMM_PL;  // (function, node): parts in order
        double sv = 0.0;
        for (int w = 0; w < LOC_PARTS; ++w) sv += part[w][fn][mm];
        val[fn][mm] = sv;
    }
    __syncthreads();
    if (tid >= 4 * FMM_PL) return;
    // c_k = (2 - [k = 0]) / P * sum_m f(t_m) T_k(t_m), thread (function fn, degree k)
    const int fn = tid / FMM_PL, k = tid % FMM_PL;
    double ck = 0.0;
#pragma unroll 4
    for (int mm = 0; mm < FMM_PL; ++mm) ck = __builtin_fma(val[fn][mm], Tkm[k][mm], ck);
    f.loc[(int64_t)L * FMM_LOC + fn * FMM_PL + k] = ck * ((k == 0 ? 1.0 : 2.0) / FMM_PL);
}

hipError_t launch_fmm_lists(const FmmArgs &f, hipStream_t s) {
    if (f.nboxes <= 0) return hipSuccess;
    SDC_LAUNCH(KID_FMM_LISTS, k_fmm_lists<false>, dim3(f.nleaves), dim3(WAVE), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_fmm_build(const FmmArgs &f, hipStream_t s) {
    if (f.nboxes <= 0) return hipSuccess;
    // the lists and every leaf's equivalent sources in one launch, then the used upper boxes
    SDC_LAUNCH(KID_FMM_LISTS, k_fmm_lists<true>, dim3(f.nleaves), dim3(2 * WAVE), 0, s, f);
    if (f.nupper > 0)
        SDC_LAUNCH(KID_FMM_BOXES, k_fmm_boxes, dim3(f.nupper), dim3(256), 0, s, f);
    SDC_LAUNCH(KID_FMM_LOCAL, k_fmm_local, dim3(f.nleaves), dim3(FMM_PL * LOC_PARTS), 0, s, f);
    return hipGetLastError();
}

}  // namespace sdc
