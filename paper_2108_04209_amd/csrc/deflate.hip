// deflate.hip -- deflation of the rank-one problems of a batch (Remark 1) on gfx950, and
// the orthogonal factor it leaves in the eigenvector matrix.
//
// For A = diag(d) + v v^T, v = sqrt(rho) z, d non-decreasing, and a user tolerance tau:
//   rule 1: pole k deflates if |v_k| < tau (eigenpair (d_k, e_k));
//   rule 2: scanning the other poles left to right, the current pole a and the next pole b
//           rotate together if |(d_a - d_b) v_a v_b| < (v_a^2 + v_b^2) tau (z can stand
//           for v: both sides scale by rho).  G = [c -s; s c] with c = z_b / r,
//           s = z_a / r, r = |(z_a, z_b)| takes (z_a, z_b) to (0, r); the off-diagonal
//           entry cs (d_a - d_b) of G diag(d_a, d_b) G^T is below tau and is dropped.  Pole a
//           deflates with eigenvalue c^2 d_a + s^2 d_b; pole b goes on with
//           d_b' = s^2 d_a + c^2 d_b (held in [d_a, d_b]) and z_b' = r.
// A = G^T (diag(d') + v' v'^T) G up to the dropped entries, so the eigenvector matrix is
// Q = G^T P (Qhat (+) I), with P placing the reduced problem's eigenvectors and the deflated
// unit vectors at their poles.
//
// The scan is sequential only through runs of rotations.  One wavefront owns a problem and
// takes its poles 64 at a time: the poles that survive rule 1 are packed into lanes, every
// lane tests its pair (left neighbour, itself) at once, and only the lane after a rotation
// is re-tested with the rotated values.  A window of 64 poles costs one pass plus one per
// rotation in it.
//
// Decisions are taken with the same expressions in the same order as a plain sequential
// implementation, without contraction into fused multiply-adds, so they do not depend on
// how the lanes split the work.
#include "common.h"

namespace sdc {

constexpr int DEFL_SEG = 2048;  // poles per segment of the parallel scan (a multiple of 64)

struct DeflArgs {
    const int64_t *off;
    const double *d, *z, *rho;
    double tau;
    double *dout, *zout;
    int32_t *perm, *rright, *rleft;
    double *rc, *rs;
    int32_t *kept, *status;
    double2 *val;    // workspace: final (d, z) of each pole by pole index
    int8_t *flag;    // workspace: 1 kept, 0 deflated
    int4 *seg_i;     // workspace [nprob][maxseg]: current pole, first survivor, status, kept
    double2 *seg_d;  // workspace [nprob][maxseg]: the current pole's (d, z)
    int maxseg;
};

// the rule-2 test and the rotation (evaluated exactly as written)
__device__ __forceinline__ bool defl_test(double da, double za, double db, double zb,
                                          double tau) {
#pragma clang fp contract(off)
    const double r2 = za * za + zb * zb;
    const double lhs = fabs(((da - db) * za) * zb);
    return lhs < r2 * tau;
}

__device__ __forceinline__ void defl_rotate(double da, double za, double db, double zb,
                                            double &c, double &s, double &dl, double &dr,
                                            double &r) {
#pragma clang fp contract(off)
    const double r2 = za * za + zb * zb;
    r = sqrt(r2);
    c = zb / r;
    s = za / r;
    const double cc = c * c, ss = s * s;
    dl = cc * da + ss * db;
    dr = ss * da + cc * db;
    if (dr < da) dr = da;
    if (dr > db) dr = db;
}

// read a double / int from lane l (l wave-uniform)
__device__ __forceinline__ double lane_get(double v, int l) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ int lane_get(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// The scan over poles [lo, hi) of a problem, a window of 64 at a time, with the incoming
// current pole (ca, cd, cz) (ca < 0: none yet): rule 1, the packing of the survivors into
// lanes and the rule-2 tests, writing the outcome of every pole of the range and of the
// incoming pole once it is decided.  On return (ca, cd, cz) is the current pole, still
// undecided; `first` is the range's first pole that survives rule 1 (-1: none).  Returns
// the number of poles decided kept.
__device__ int defl_scan(const DeflArgs &a, int64_t base, int lo, int hi, double sv, int &ca,
                         double &cd, double &cz, int &first, double *sd, double *sz, int *si) {
    const int lane = threadIdx.x;
    const double tau = a.tau;
    const double *d = a.d + base, *z = a.z + base;
    double2 *val = a.val + base;
    int8_t *flag = a.flag + base;
    int32_t *rright = a.rright + base, *rleft = a.rleft + base;
    double *rc = a.rc + base, *rs = a.rs + base;
    int nkept = 0;
    first = -1;
    // the next window's loads are issued before this one is worked on
    double ndi = lo + lane < hi ? d[lo + lane] : 0.0, nzi = lo + lane < hi ? z[lo + lane] : 0.0;
    for (int c0 = lo; c0 < hi; c0 += WAVE) {
        const int i = c0 + lane;
        const bool valid = i < hi;
        const double di = ndi, zi = nzi;
        if (i + WAVE < hi) {
            ndi = d[i + WAVE];
            nzi = z[i + WAVE];
        }
        const bool r1 = valid && fabs(sv * zi) < tau;  // rule 1
        if (valid) {
            rright[i] = -1;
            rleft[i] = -1;
            rc[i] = 1.0;
            rs[i] = 0.0;
            if (r1) {
                val[i] = make_double2(di, 0.0);
                flag[i] = 0;
            }
        }
        // pack the poles that survive rule 1 into lanes 0 .. cnt-1, in order
        const unsigned long long cm = __ballot(valid && !r1);
        const int cnt = __popcll(cm);
        const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(cm >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)cm, 0u));
        if (valid && !r1) {
            sd[rank] = di;
            sz[rank] = zi;
            si[rank] = i;
        }
        __syncthreads();
        const bool live = lane < cnt;
        const double bd = live ? sd[lane] : 0.0, bz = live ? sz[lane] : 0.0;
        const int bi = live ? si[lane] : -1;
        __syncthreads();
        if (cnt == 0) continue;
        if (first < 0) first = lane_get(bi, 0);
        // left neighbour of every lane's pair: the previous lane's pole, the current pole
        // of the scan for lane 0
        double ld = __shfl_up(bd, 1), lz = __shfl_up(bz, 1);
        int li = __shfl_up(bi, 1);
        int start = 0;
        if (lane == 0) {
            ld = cd;
            lz = cz;
            li = ca;
        }
        if (ca < 0) start = 1;  // the first surviving pole has no left neighbour
        int rot_lane = -1;      // lane of the last rotation in this window
        double md = 0.0, mz = 0.0;
        for (;;) {
            const bool test = live && lane >= start;
            const bool F = test && defl_test(ld, lz, bd, bz, tau);
            const unsigned long long fm = __ballot(F);
            const int j = fm ? (int)__builtin_ctzll(fm) : cnt;
            // pairs start .. j-1 do not rotate: their left poles are kept as they stand
            if (lane >= start && lane < j && live) {
                val[li] = make_double2(ld, lz);
                flag[li] = 1;
            }
            nkept += max(0, j - start);
            if (!fm) break;
            // pair j rotates: its left pole deflates, its right pole goes on rotated
            double c = 0.0, s = 0.0, dl = 0.0, dr = 0.0, r = 0.0;
            if (lane == j) {
                defl_rotate(ld, lz, bd, bz, c, s, dl, dr, r);
                val[li] = make_double2(dl, 0.0);
                flag[li] = 0;
                rright[li] = bi;
                rleft[bi] = li;
                rc[li] = c;
                rs[li] = s;
            }
            md = lane_get(dr, j);
            mz = lane_get(r, j);
            rot_lane = j;
            if (lane == j + 1) {
                ld = md;
                lz = mz;
            }
            start = j + 1;
            if (start >= cnt) break;
        }
        // the window's last pole becomes the current pole of the scan
        if (rot_lane == cnt - 1) {
            cd = md;
            cz = mz;
        } else {
            cd = lane_get(bd, cnt - 1);
            cz = lane_get(bz, cnt - 1);
        }
        ca = lane_get(bi, cnt - 1);
    }
    return nkept;
}

// validation of poles [lo, hi) of problem p: finite, non-decreasing (across the range's
// end as well), rho > 0
__device__ int defl_check(const DeflArgs &a, int p, int64_t base, int lo, int hi, int n) {
    const int lane = threadIdx.x;
    const double *d = a.d + base, *z = a.z + base;
    int st = 0;
    for (int i = lo + lane; i < hi; i += WAVE) {
        const double di = d[i], zi = z[i];
        if (!isfinite(di) || !isfinite(zi)) st |= SUPERDC_ST_NONFINITE;
        if (i + 1 < n && d[i + 1] < di) st |= SUPERDC_ST_UNSORTED;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) st |= __shfl_xor(st, o);
    const double rho = a.rho[p];
    if (!isfinite(rho)) st |= SUPERDC_ST_NONFINITE;
    else if (!(rho > 0.0)) st |= SUPERDC_ST_RHO;
    return st;
}

// Segments of DEFL_SEG poles are scanned in parallel (blockIdx.y), each as if no pole came
// before it; their records keep the undecided current pole at the end, the first pole that
// survives rule 1, the status bits and the number of poles decided kept.
__global__ __launch_bounds__(WAVE) void k_deflate(DeflArgs a) {
    __shared__ double sd[WAVE], sz[WAVE];
    __shared__ int si[WAVE];
    const int p = blockIdx.x, sg = blockIdx.y;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int lo = sg * DEFL_SEG;
    if (lo >= n) return;
    const int hi = min(n, lo + DEFL_SEG);
    const int64_t r = (int64_t)p * a.maxseg + sg;
    const int st = defl_check(a, p, base, lo, hi, n);
    if (st) {
        if (threadIdx.x == 0) {
            a.seg_i[r] = make_int4(-1, -1, st, 0);
            a.seg_d[r] = make_double2(0.0, 0.0);
        }
        return;
    }
    int ca = -1, first = -1;
    double cd = 0.0, cz = 0.0;
    const int nk = defl_scan(a, base, lo, hi, sqrt(a.rho[p]), ca, cd, cz, first, sd, sz, si);
    if (threadIdx.x == 0) {
        a.seg_i[r] = make_int4(ca, first, 0, nk);
        a.seg_d[r] = make_double2(cd, cz);
    }
}

// The joins, in order, one wavefront per problem.  The scan entering segment s holds the
// current pole of everything before it.  If that pole and the segment's first survivor do
// not rotate, the pole is kept and the segment's own scan stands exactly (it started from
// that survivor); if they do, the segment is scanned again from the incoming pole.
__global__ __launch_bounds__(WAVE) void k_deflate_join(DeflArgs a) {
    __shared__ double sd[WAVE], sz[WAVE];
    __shared__ int si[WAVE];
    const int p = blockIdx.x;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int nseg = (n + DEFL_SEG - 1) / DEFL_SEG;
    const int64_t r0 = (int64_t)p * a.maxseg;
    int st = 0;
    for (int sg = 0; sg < nseg; ++sg) st |= a.seg_i[r0 + sg].z;
    if (st) {
        if (threadIdx.x == 0) {
            a.status[p] = st;
            a.kept[p] = 0;
        }
        return;
    }
    const double sv = sqrt(a.rho[p]);
    int4 ri = a.seg_i[r0];
    double2 rd = a.seg_d[r0];
    int ca = ri.x, nk = ri.w;
    double cd = rd.x, cz = rd.y;
    for (int sg = 1; sg < nseg; ++sg) {
        ri = a.seg_i[r0 + sg];
        rd = a.seg_d[r0 + sg];
        const int f = ri.y;
        if (f < 0) continue;  // nothing survives rule 1 here: the current pole passes on
        if (ca >= 0 && defl_test(cd, cz, a.d[base + f], a.z[base + f], a.tau)) {
            int first;
            const int lo = sg * DEFL_SEG;
            nk += defl_scan(a, base, lo, min(n, lo + DEFL_SEG), sv, ca, cd, cz, first, sd, sz, si);
            continue;
        }
        if (ca >= 0) {  // the incoming pole is kept; the segment's scan stands
            if (threadIdx.x == 0) {
                a.val[base + ca] = make_double2(cd, cz);
                a.flag[base + ca] = 1;
            }
            ++nk;
        }
        ca = ri.x;
        cd = rd.x;
        cz = rd.y;
        nk += ri.w;
    }
    if (ca >= 0) {
        if (threadIdx.x == 0) {
            a.val[base + ca] = make_double2(cd, cz);
            a.flag[base + ca] = 1;
        }
        ++nk;
    }
    if (threadIdx.x == 0) {
        a.kept[p] = nk;
        a.status[p] = 0;
    }
}

// kept poles per segment, for the placement
__global__ __launch_bounds__(WAVE) void k_deflate_count(DeflArgs a) {
    const int p = blockIdx.x, sg = blockIdx.y;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int lo = sg * DEFL_SEG;
    if (lo >= n || a.status[p]) return;
    const int hi = min(n, lo + DEFL_SEG);
    int c = 0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += WAVE) c += a.flag[base + i] != 0;
    for (int o = WAVE / 2; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (threadIdx.x == 0) a.seg_i[(int64_t)p * a.maxseg + sg].w = c;
}

// placement: kept poles first, deflated ones after, each in pole order
__global__ __launch_bounds__(WAVE) void k_deflate_place(DeflArgs a) {
    const int p = blockIdx.x, sg = blockIdx.y;
    const int64_t base = a.off[p];
    const int n = (int)(a.off[p + 1] - base);
    const int lo = sg * DEFL_SEG;
    if (lo >= n || a.status[p]) return;
    const int hi = min(n, lo + DEFL_SEG);
    const int lane = threadIdx.x;
    int pk = 0;  // kept poles before this segment
    for (int u = 0; u < sg; ++u) pk += a.seg_i[(int64_t)p * a.maxseg + u].w;
    int pd = a.kept[p] + (lo - pk);
    const double2 *val = a.val + base;
    const int8_t *flag = a.flag + base;
    int8_t nfl = lo + lane < hi ? flag[lo + lane] : 0;
    double2 nv = lo + lane < hi ? val[lo + lane] : make_double2(0.0, 0.0);
    for (int c0 = lo; c0 < hi; c0 += WAVE) {
        const int i = c0 + lane;
        const bool valid = i < hi;
        const int8_t fl = nfl;
        const double2 v = nv;
        if (i + WAVE < hi) {  // the next window's loads in flight
            nfl = flag[i + WAVE];
            nv = val[i + WAVE];
        }
        const bool k = valid && fl != 0;
        const unsigned long long km = __ballot(k), dm = __ballot(valid && !k);
        const unsigned long long mm = k ? km : dm;
        const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mm >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)mm, 0u));
        if (valid) {
            const int j = (k ? pk : pd) + rank;
            a.dout[base + j] = v.x;
            a.zout[base + j] = k ? v.y : 0.0;
            a.perm[base + j] = i;
        }
        pk += __popcll(km);
        pd += __popcll(dm);
    }
}

// ---------------------------------------------------------------------------------------
// the orthogonal factor: Y = G^T P U (trans 0) or Y = P^T G X (trans 1) on total x m
// column-major blocks (leading dimensions ldx, ldy), each problem on its own rows
// ---------------------------------------------------------------------------------------
struct ExpandArgs {
    const int64_t *off;
    int nprob, m;
    const int32_t *perm, *rright, *rleft;
    const double *rc, *rs;
    const double *X;
    int64_t ldx;
    double *Y;
    int64_t ldy;
    double *T;  // workspace for trans 1 (total x m, leading dimension total)
};

__device__ __forceinline__ int find_prob(const int64_t *off, int nprob, int64_t e) {
    int lo = 0, hi = nprob;  // off[lo] <= e < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

// trans 0: Y[perm[j]] = X[j]; trans 1: Y[j] = T[perm[j]]  (one thread per row and column)
__global__ __launch_bounds__(256) void k_defl_place(ExpandArgs a, int trans, int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total * a.m) return;
    const int64_t row = e % total;
    const int c = (int)(e / total);
    const int p = find_prob(a.off, a.nprob, row);
    const int64_t base = a.off[p];
    const int pj = a.perm[row];
    if (pj < 0 || pj >= a.off[p + 1] - base) return;  // not a placement of this problem
    const int64_t prow = base + pj;
    if (trans == 0) a.Y[c * a.ldy + prow] = a.X[c * a.ldx + row];
    else a.Y[c * a.ldy + row] = a.T[c * total + prow];
}

// rotations along their chains (one thread per chain and column) on V (leading dimension
// ldv): trans 0 applies G^T = G_1^T ... G_R^T, walking each chain back from its last pole;
// trans 1 applies G = G_R ... G_1, walking forward from its first pole.  Chains are
// disjoint.
__global__ __launch_bounds__(256) void k_defl_rotate(ExpandArgs a, int trans, int64_t total,
                                                     double *V, int64_t ldv) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total * a.m) return;
    const int64_t row = e % total;
    const int c = (int)(e / total);
    const bool end = a.rleft[row] >= 0 && a.rright[row] < 0;
    const bool beg = a.rright[row] >= 0 && a.rleft[row] < 0;
    if (!(trans == 0 ? end : beg)) return;
    const int p = find_prob(a.off, a.nprob, row);
    const int64_t base = a.off[p];
    double *v = V + c * ldv + base;
    const int32_t *rr = a.rright + base, *rl = a.rleft + base;
    const double *rc = a.rc + base, *rs = a.rs + base;
    const int i = (int)(row - base);
    // a chain runs through strictly increasing poles; a link that does not is not
    // followed, so every walk ends within n_p steps
    if (trans == 0) {
        int bb = i;
        for (int aa = rl[bb]; aa >= 0 && aa < bb; bb = aa, aa = rl[aa]) {
            const double cc = rc[aa], ss = rs[aa];
            const double ya = v[aa], yb = v[bb];
            v[aa] = cc * ya + ss * yb;
            v[bb] = -ss * ya + cc * yb;
        }
    } else {
        const int n = (int)(a.off[p + 1] - base);
        int aa = i;
        for (int bb = rr[aa]; bb > aa && bb < n; aa = bb, bb = rr[bb]) {
            const double cc = rc[aa], ss = rs[aa];
            const double ya = v[aa], yb = v[bb];
            v[aa] = cc * ya - ss * yb;
            v[bb] = ss * ya + cc * yb;
        }
    }
}

__global__ __launch_bounds__(256) void k_defl_copy(const double *X, int64_t ldx, double *T,
                                                   int64_t total, int m) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total * m) return;
    const int64_t row = e % total;
    const int c = (int)(e / total);
    T[c * total + row] = X[c * ldx + row];
}

// ---------------------------------------------------------------------------------------
// row copies between two batch layouts (total x m column-major each): rows [0, cnt_p) of
// problem p, cnt_p = min(rows ? rows[p] : n_src, n_src, n_dst); the other rows of dst get
// `fill` when has_fill
// ---------------------------------------------------------------------------------------
struct CopyRowsArgs {
    const int64_t *soff, *doff;
    int nprob, m;
    const int32_t *rows;
    const double *src;
    int64_t lds;
    double *dst;
    int64_t ldd;
    int has_fill;
    double fill;
};

__global__ __launch_bounds__(256) void k_copy_rows(CopyRowsArgs a, int64_t dtotal) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= dtotal * a.m) return;
    const int64_t row = e % dtotal;
    const int c = (int)(e / dtotal);
    const int p = find_prob(a.doff, a.nprob, row);
    const int64_t db = a.doff[p], nd = a.doff[p + 1] - db;
    const int64_t sb = a.soff[p], ns = a.soff[p + 1] - sb;
    int64_t cnt = ns < nd ? ns : nd;
    if (a.rows) {
        const int64_t r = a.rows[p] < 0 ? 0 : a.rows[p];
        if (r < cnt) cnt = r;
    }
    const int64_t j = row - db;
    double *out = a.dst + c * a.ldd + row;
    if (j < cnt) *out = a.src[c * a.lds + sb + j];
    else if (a.has_fill) *out = a.fill;
}

// ---------------------------------------------------------------------------------------
int deflate_segments(int max_n) {
    const int s = (max_n + DEFL_SEG - 1) / DEFL_SEG;
    return s > 1 ? s : 1;
}

hipError_t launch_deflate(const int64_t *off, int nprob, const double *d, const double *z,
                          const double *rho, double tau, double *dout, double *zout,
                          int32_t *perm, int32_t *rright, int32_t *rleft, double *rc, double *rs,
                          int32_t *kept, int32_t *status, double2 *val, int8_t *flag,
                          int max_n, int4 *seg_i, double2 *seg_d, hipStream_t s) {
    DeflArgs a{off,  d,      z,      rho,  tau,  dout,  zout,  perm,   rright,
               rleft, rc,    rs,     kept, status, val, flag, seg_i, seg_d, deflate_segments(max_n)};
    const dim3 g2(nprob, a.maxseg);
    SDC_LAUNCH(KID_DEFLATE, k_deflate, g2, dim3(WAVE), 0, s, a);
    SDC_LAUNCH(KID_DEFLATE, k_deflate_join, dim3(nprob), dim3(WAVE), 0, s, a);
    SDC_LAUNCH(KID_DEFLATE, k_deflate_count, g2, dim3(WAVE), 0, s, a);
    SDC_LAUNCH(KID_DEFLATE, k_deflate_place, g2, dim3(WAVE), 0, s, a);
    return hipGetLastError();
}

static dim3 grid_of(int64_t cnt) { return dim3((unsigned)((cnt + 255) / 256)); }

hipError_t launch_deflate_expand(const int64_t *off, int nprob, int64_t total, int m,
                                 const int32_t *perm, const int32_t *rright,
                                 const int32_t *rleft, const double *rc, const double *rs,
                                 int trans, const double *X, int64_t ldx, double *Y,
                                 int64_t ldy, double *T, hipStream_t s) {
    ExpandArgs a{off, nprob, m, perm, rright, rleft, rc, rs, X, ldx, Y, ldy, T};
    const int64_t cnt = total * m;
    if (cnt == 0) return hipSuccess;
    if (trans == 0) {
        SDC_LAUNCH(KID_DEFL_PLACE, k_defl_place, grid_of(cnt), dim3(256), 0, s, a, 0, total);
        SDC_LAUNCH(KID_DEFL_ROTATE, k_defl_rotate, grid_of(cnt), dim3(256), 0, s, a, 0, total, Y,
                   ldy);
    } else {
        SDC_LAUNCH(KID_DEFL_PLACE, k_defl_copy, grid_of(cnt), dim3(256), 0, s, X, ldx, T, total, m);
        SDC_LAUNCH(KID_DEFL_ROTATE, k_defl_rotate, grid_of(cnt), dim3(256), 0, s, a, 1, total, T,
                   total);
        SDC_LAUNCH(KID_DEFL_PLACE, k_defl_place, grid_of(cnt), dim3(256), 0, s, a, 1, total);
    }
    return hipGetLastError();
}

hipError_t launch_copy_rows(const int64_t *soff, const int64_t *doff, int nprob,
                            int64_t dtotal, int m, const int32_t *rows, const double *src,
                            int64_t lds, double *dst, int64_t ldd, const double *fill,
                            hipStream_t s) {
    CopyRowsArgs a{soff, doff, nprob, m, rows, src, lds, dst, ldd, fill ? 1 : 0, fill ? *fill : 0.0};
    const int64_t cnt = dtotal * m;
    if (cnt == 0) return hipSuccess;
    SDC_LAUNCH(KID_COPY_ROWS, k_copy_rows, grid_of(cnt), dim3(256), 0, s, a, dtotal);
    return hipGetLastError();
}

}  // namespace sdc
