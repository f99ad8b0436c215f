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
// leaf eigendecomposition: cyclic Jacobi in three kernels:
//   k_leaf_jacobi  rotates A -- kept by position, its upper triangle packed by rows
//                  (66 KB for a leaf of 128) -- in LDS, two leaves to a CU (the rounds are
//                  short and end in a barrier: a second leaf's waves fill the first one's
//                  waits), and logs every round's rotations to HBM as (cos, signed sin) by
//                  position;
//   k_leaf_vectors replays the log on V = I with V in registers: a lane holds 16
//                  consecutive positions of 4 rows, so a round is static register code;
//   k_leaf_w       W = Q^T U from the stored eigenvectors.
// The pairs follow the odd-even ordering over positions: round A pairs positions
// (2k, 2k+1), round B pairs (2k+1, 2k+2), and after every round the two indices of a pair
// trade positions.  Over L rounds every pair of indices meets once (the network ends on
// the reversed order, so a sweep reverses the positions), and a pair's rotation only ever
// touches two neighbouring positions.
// ---------------------------------------------------------------------------------------
constexpr int LJ_THREADS = 1024;
constexpr int LJ_PACKED = LEAF_MAX * (LEAF_MAX + 1) / 2;
// slots of the folded block triangle per thread: (h/2)(h+1) blocks, h = LEAF_MAX/2 rounded
// up to even, over the threads past the first wavefront
constexpr int LJ_BLK =
    ((LEAF_MAX / 4) * (LEAF_MAX / 2 + 1) + LJ_THREADS - WAVE - 1) / (LJ_THREADS - WAVE);
constexpr int LV_SEG = 16;                          // positions a lane holds
constexpr int LV_NSEG = LEAF_MAX / LV_SEG;          // segments of a row (8)
constexpr int LV_RPL = 4;                           // rows a lane holds
constexpr int LV_WROWS = WAVE / LV_NSEG * LV_RPL;   // rows per wavefront (32)
constexpr int LV_PAIRS = LEAF_MAX / 2;              // log entries a round is staged with
constexpr int LV_SP = LV_SEG / 2;                   // pairs of a segment in round A (8)
constexpr int LV_CLD = LV_PAIRS + LV_NSEG;          // staged entry k sits at k + k / LV_SP,
                                                    // so the segments' reads hit distinct banks
constexpr int LV_RB = 4;                            // rounds per staged block
static_assert(LEAF_MAX / 2 <= WAVE, "a round's pairs must fit one wavefront");
static_assert(LJ_PACKED < (1 << 15), "addresses in the packed triangle fit 15 bits");
static_assert(LV_PAIRS == WAVE, "one staged log entry per lane");
static_assert(LV_NSEG * LV_SEG == LEAF_MAX && LV_NSEG <= 16 && 16 % LV_NSEG == 0,
              "a row's segments are neighbouring lanes of one 16-lane DPP row");
static_assert(LV_RB == 4, "a staged block starts on a round A, and two padding rounds negate\n"
              "every position but the first");

// entry (i, j), i <= j, of the upper triangle of an m x m matrix (m even) packed by rows,
// each row holding its even columns first and then its odd ones: a round's blocks take a
// column of one parity from every pair, so lanes with neighbouring column pairs read
// neighbouring words of a row instead of every other one (which halved the LDS bank
// throughput)
__device__ __forceinline__ int ut(int i, int j, int m) {
    const int start = (i * (2 * m - i + 1)) >> 1;  // where row i starts
    const int odd = i & 1;
    const int neven = (m - i - odd) >> 1;           // even columns in [i, m)
    return start + ((j & 1) ? neven + ((j - i - 1 + odd) >> 1) : ((j - i - odd) >> 1));
}

// cos and sin of the rotation with tangent t
__device__ __forceinline__ double2 rot_cs(double t) {
    const double c = rcp_nr(sqrt(t * t + 1.0));
    return make_double2(c, t * c);
}

// The matrix is kept by position: entry (i, j) of the packed upper triangle is the entry
// of the two indices at positions i and j.  A round's rotation of pair k then acts on the
// positions (l, r) of the pair by the reflection [[sigma, c], [c, -sigma]] -- the rotation
// followed by the trade of positions -- with theta = (A(r,r) - A(l,l)) / (2 A(l,r)) taken
// at the positions (the sign of sigma then comes out right whichever of the two indices is
// the smaller), and the round is A <- R A R with R the direct sum of the reflections (the
// identity on the two positions that sit out round B).  Every 2 x 2 block (rows of pair P1,
// columns of pair P2) depends only on its own four entries, so a round is a single pass over
// the blocks P1 <= P2 at addresses fixed for each round type.  Diagonal blocks take
// (x, w; w, y) to (y + t w, 0; 0, x - t w), or to (y, w; w, x) when there is no rotation.
//
// The first wavefront owns the blocks that the next round's rotations read: the diagonal
// blocks, the blocks (k, k+1) of neighbouring pairs and the block (0, m/2 - 1).  A pair of
// the next round joins one position of pair k and one of pair k+1 of this round (or a
// position that sits the round out), so its three entries all lie in those blocks.  That
// wavefront therefore computes the next round's rotations right after its own blocks,
// while the other wavefronts still update theirs, and a round ends in a single barrier;
// the rotation data is double-buffered by round parity.
__global__ __launch_bounds__(LJ_THREADS, 2 * LJ_THREADS / WAVE / 4) void k_leaf_jacobi(LeafArgs a) {
    __shared__ double A[LJ_PACKED];         // upper triangle by position, packed by rows
    __shared__ double2 cs[2][LEAF_MAX / 2];  // (c, sigma) of each pair
    __shared__ double tt[2][LEAF_MAX / 2];   // tangent of each pair's rotation (0: none)
    __shared__ double red[LJ_THREADS / WAVE];
    __shared__ int swept[2];       // per sweep parity: the sweep rotated something
    __shared__ int swbig[2];       // per sweep parity: some tangent was at least 1e-6

    const int leafid = blockIdx.x;
    const int L = a.leaf;
    const int tid = threadIdx.x, nt = blockDim.x;
    const double *D = a.D + (size_t)leafid * L * L;
    // Frobenius norm (of the whole block) for the absolute part of the rotation threshold
    double fro = 0.0;
    for (int e = tid; e < L * L; e += nt) {
        const int i = e / L, j = e - i * L;
        const double v = D[e];
        if (i <= j) A[ut(i, j, L)] = v;
        fro += v * v;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) fro += __shfl_xor(fro, o);
    if (lane_id() == 0) red[tid / WAVE] = fro;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < nt / WAVE; ++w) tot += red[w];
    const double absfloor = 1e-18 * sqrt(tot);
    const int m = L;  // even
    const int half = m / 2;
    const int hh = (half + 1) & ~1;          // half rounded up to even, for the folding
    const int nfold = (hh / 2) * (hh + 1);  // blocks of the folded triangle
    const int total = a.max_sweeps * m;     // rounds the log has room for
    double2 *log = reinterpret_cast<double2 *>(a.rot) + (size_t)leafid * total * half;
    const bool first = tid < WAVE;
    // addresses of the block of row pair (r0, r1) and column pair (c0, c1), r1 < c0: a
    // column pair (m-1, 0) is the pair that sits round B out, whose entries (r, 0) are kept
    // at (0, r)
    auto block_addr = [&](int r0, int r1, int c0, int c1, int4 &ad) {
        if (c1 != 0) ad = make_int4(ut(r0, c0, m), ut(r0, c1, m), ut(r1, c0, m), ut(r1, c1, m));
        else ad = make_int4(ut(r0, m - 1, m), ut(0, r0, m), ut(r1, m - 1, m), ut(0, r1, m));
    };
    // the other wavefronts' blocks, the same in every round: the folded triangle dealt out
    // over their threads, without the first wavefront's blocks.  A slot keeps P1 | P2 << 8
    // and, per round type, the addresses of the two rows' entries in the column pair's
    // first column (16 bits each); the second column's follow from the row's parity, so
    // that the kernel keeps to 64 registers and two leaves share a CU
    int bP[LJ_BLK];  // < 0: no block
    int adA[LJ_BLK], adB[LJ_BLK];
#pragma unroll
    for (int u = 0; u < LJ_BLK; ++u) {
        bP[u] = -1;
        adA[u] = adB[u] = 0;
        const int blk = (tid - WAVE) + u * (nt - WAVE);
        if (first || blk >= nfold) continue;
        const int r = blk / (hh + 1), e = blk - r * (hh + 1);
        int P1, P2;
        if (e < hh - r) {
            P1 = r;
            P2 = r + e;
        } else {
            P1 = hh - 1 - r;
            P2 = e - 1;
        }
        if (P2 >= half) continue;  // padding of an odd half
        if (P2 - P1 <= 1 || (P1 == 0 && P2 == half - 1)) continue;  // the first wavefront's
        bP[u] = P1 | P2 << 8;
        int4 ad;
        block_addr(2 * P1, 2 * P1 + 1, 2 * P2, 2 * P2 + 1, ad);
        adA[u] = ad.x | ad.z << 16;
        if (P2 < half - 1) block_addr(2 * P1 + 1, 2 * P1 + 2, 2 * P2 + 1, 2 * P2 + 2, ad);
        else block_addr(2 * P1 + 1, 2 * P1 + 2, m - 1, 0, ad);
        adB[u] = ad.x | ad.z << 16;
    }
    // the four addresses of slot block (P1, P2) in a round of type b from the packed pair:
    // in row r the column pair's second column lies neven(r) + odd(r) words after its first
    // in round A (even, odd), and 1 - odd(r) - neven(r) words in round B (odd, even); when
    // the column pair (m-1, 0) sits out, rows r0 = 2 P1 + 1 and r1 = r0 + 1 keep column 0
    // at (0, r), which is m/2 + P1 and P1 + 1
    auto slot_addr = [&](int pk, int P1, int b, bool cols_idle) {
        const int ax = pk & 0xffff, az = pk >> 16;
        if (cols_idle) return make_int4(ax, half + P1, az, P1 + 1);
        auto step = [&](int r) {
            const int odd = r & 1, neven = (m - r - odd) >> 1;
            return b ? 1 - odd - neven : neven + odd;
        };
        const int r0 = 2 * P1 + b;
        return make_int4(ax, ax + step(r0), az, az + step(r0 + 1));
    };

    // off-diagonal block of pairs P1 < P2 at addresses ad, with the reflections of buffer b
    // (cols_idle: the column pair sits the round out)
    auto update_block = [&](int P1, int P2, const int4 &ad, int b, bool cols_idle) {
        const double2 r1 = cs[b][P1];
        const double x00 = A[ad.x], x01 = A[ad.y], x10 = A[ad.z], x11 = A[ad.w];
        // rows: R1 X
        const double y00 = fma(r1.x, x10, r1.y * x00), y10 = fma(r1.x, x00, -(r1.y * x10));
        const double y01 = fma(r1.x, x11, r1.y * x01), y11 = fma(r1.x, x01, -(r1.y * x11));
        if (cols_idle) {
            A[ad.x] = y00;
            A[ad.y] = y01;
            A[ad.z] = y10;
            A[ad.w] = y11;
            return;
        }
        // columns: (R1 X) R2
        const double2 r2 = cs[b][P2];
        A[ad.x] = fma(r2.x, y01, r2.y * y00);
        A[ad.y] = fma(r2.x, y00, -(r2.y * y01));
        A[ad.z] = fma(r2.x, y11, r2.y * y10);
        A[ad.w] = fma(r2.x, y10, -(r2.y * y11));
    };

    // rotations of round g (first wavefront, lane k: pair k) into buffer g & 1, with the
    // log entry; returns the lane's tangent (0: no rotation)
    auto rotations = [&](int g) -> double {
        const int k = tid;
        const int B = g & 1;  // m is even: round A pairs positions (2k, 2k+1), B (2k+1, 2k+2)
        double t = 0.0;
        if (k < half) {
            // in round B, positions m-1 and 0 sit out
            const bool idle = B && k == half - 1;
            const int lp = idle ? 0 : 2 * k + B, rp = lp + 1;
            const double w = A[ut(lp, rp, m)];
            const double x = A[ut(lp, lp, m)], y = A[ut(rp, rp, m)];
            if (!idle && fabs(w) > 2.220446049250313e-16 * sqrt(fabs(x) * fabs(y)) + absfloor) {
                // the rotation only has to annihilate w to rounding, so reciprocals by
                // Newton-refined estimates stand in for the divisions
                const double theta = (y - x) * (0.5 * rcp_nr(w));
                if (fabs(theta) > 1e150) t = 0.5 * rcp_nr(theta);
                else t = (theta >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(theta) + sqrt(theta * theta + 1.0));
            }
            const double2 r = t != 0.0 ? rot_cs(t) : make_double2(1.0, 0.0);
            cs[B][k] = r;
            tt[B][k] = t;
            // the left position's new column is c y + sigma x and the right one's
            // c x - sigma y, for the columns x, y at the two positions before the round
            if (!idle) {
                // the lane's offset through an empty asm, so that the per-lane log address is
                // formed here rather than held in registers through the rounds
                int kk = k;
                asm volatile("" : "+v"(kk));
                log[(size_t)g * half + kk] = r;
            }
        }
        return t;
    };
    // whether some pair (i, j) of the matrix as it stands would pass the rotation test, over
    // all threads (ends in a barrier).  A sweep that rotates nothing leaves the matrix as it
    // is, so when no pair passes, the next sweep would be empty.  It runs about once per
    // leaf: the thread index goes through an empty asm so that none of its index
    // arithmetic is hoisted out of the rounds and held in registers through them.
    auto any_pair_rotates = [&]() -> bool {
        int t = tid;
        asm volatile("" : "+v"(t));
        const int tpr = nt / m;  // threads per row
        const int i = t / tpr;
        bool any = false;
        if (i < m) {
            const double x = fabs(A[ut(i, i, m)]);
            for (int j = i + 1 + t % tpr; j < m; j += tpr)
                any |= fabs(A[ut(i, j, m)]) > 2.220446049250313e-16 * sqrt(x * fabs(A[ut(j, j, m)])) + absfloor;
        }
        return __syncthreads_or(any);
    };

    // first wavefront: whether the current sweep has rotated anything so far, and anything
    // by a tangent of at least 1e-6
    bool rot_acc = false, big_acc = false;
    if (first) {
        const double t = rotations(0);
        rot_acc = __any(t != 0.0);
        big_acc = __any(fabs(t) >= 1e-6);
    }
    __syncthreads();
    int sweep = 0;
    bool converged = false, reversed = false;  // reversed: an empty sweep ran
    for (int g = 0;; ++g) {
        const int b = g & 1;  // rotation buffer, and round B when set
        if (first) {
            const int k = tid;
            if (k < half && !(b && k == half - 1)) {
                // diagonal block of pair k at positions (l, l+1)
                const int l = 2 * k + b;
                const int ixx = ut(l, l, m), ixw = ut(l, l + 1, m), iyy = ut(l + 1, l + 1, m);
                const double t = tt[b][k];
                const double x = A[ixx], w = A[ixw], y = A[iyy];
                A[ixx] = fma(t, w, y);
                A[iyy] = fma(-t, w, x);
                A[ixw] = t != 0.0 ? 0.0 : w;
            }
            int4 ad;
            if (!b && k + 1 < half) {  // round A: block (k, k+1)
                block_addr(2 * k, 2 * k + 1, 2 * k + 2, 2 * k + 3, ad);
                update_block(k, k + 1, ad, b, false);
            }
            if (b && k >= 1 && k < half) {  // round B: block (k-1, k)
                const bool idle = k == half - 1;
                block_addr(2 * k - 1, 2 * k, idle ? m - 1 : 2 * k + 1, idle ? 0 : 2 * k + 2, ad);
                update_block(k - 1, k, ad, b, idle);
            }
            if (k == 0 && half >= 3) {  // block (0, m/2 - 1)
                if (!b) block_addr(0, 1, m - 2, m - 1, ad);
                else block_addr(1, 2, m - 1, 0, ad);
                update_block(0, half - 1, ad, b, b);
            }
            if (g + 1 < total) {
                wave_sync();
                const double t = rotations(g + 1);
                rot_acc |= __any(t != 0.0);
                big_acc |= __any(fabs(t) >= 1e-6);
                if ((g + 1) % m == m - 1) {  // the sweep's last round is decided
                    if (tid == 0) {
                        swept[((g + 1) / m) & 1] = rot_acc;
                        swbig[((g + 1) / m) & 1] = big_acc;
                    }
                    rot_acc = big_acc = false;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < LJ_BLK; ++u) {
                if (bP[u] < 0) continue;
                const int P1 = bP[u] & 0xff, P2 = bP[u] >> 8;
                const bool idle = b && P2 == half - 1;
                update_block(P1, P2, slot_addr(b ? adB[u] : adA[u], P1, b, idle), b, idle);
            }
        }
        __syncthreads();
        if (g % m == m - 1) {  // the end of sweep g / m
            if (!swept[(g / m) & 1]) {  // a sweep without rotations: nothing of it needs replaying
                converged = reversed = true;
                break;
            }
            ++sweep;
            // once the sweep's rotations are all tiny, the next one may well be empty: test
            // every pair now instead of running it to find out (the same decision)
            if (!swbig[(g / m) & 1] && !any_pair_rotates()) {
                converged = true;
                break;
            }
            if (sweep == a.max_sweeps) break;
        }
    }
    // ascending order of the eigenvalues (ties broken by position).  A sweep reverses the
    // positions, and the replay stops short of a last sweep without rotations, so position j
    // here is position m-1-j of the replayed vectors when that sweep ran
    if (tid < L) {
        const double v = A[ut(tid, tid, L)];
        int r = 0;
        for (int j = 0; j < L; ++j) {
            const double w = A[ut(j, j, L)];
            r += (w < v) || (w == v && j < tid);
        }
        a.rank[(size_t)leafid * L + (reversed ? L - 1 - tid : tid)] = r;
        a.lam[(size_t)leafid * L + r] = v;
    }
    if (tid == 0) {
        a.sweeps[leafid] = sweep;
        a.status[leafid] = converged ? 0 : SUPERDC_ST_NOCONV;
    }
}

// value of the neighbouring lane (lane + 1 for UP, lane - 1 otherwise) within a row of 16
// lanes; the lanes at a row's end get their own value back
template <bool UP>
__device__ __forceinline__ double lane_shift(double x) {
    constexpr int ctrl = UP ? 0x101 : 0x111;  // DPP row_shl:1 / row_shr:1
    const long long b = __double_as_longlong(x);
    const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    const int l2 = __builtin_amdgcn_update_dpp(lo, lo, ctrl, 0xf, 0xf, false);
    const int h2 = __builtin_amdgcn_update_dpp(hi, hi, ctrl, 0xf, 0xf, false);
    return __longlong_as_double(((long long)h2 << 32) | (unsigned int)l2);
}

// the LV_RB rounds of a staged block, whose first round is a round A (static code with no
// exit between the rounds, so V keeps its registers through the block)
__device__ __forceinline__ void replay_block(double (&v)[LV_RPL][LV_SEG], const double2 (*c)[LV_CLD],
                                             int sg, bool has_left) {
#pragma unroll
    for (int u = 0; u < LV_RB; ++u) {
        const double2 *cu = c[u] + sg * (LV_SP + 1);  // entries 8 sg .. 8 sg + 7
        if ((u & 1) == 0) {
            // round A: pairs (2j, 2j+1) of the segment
#pragma unroll
            for (int j = 0; j < LV_SP; ++j) {
                const double2 e = cu[j];
#pragma unroll
                for (int r = 0; r < LV_RPL; ++r) {
                    const double x = v[r][2 * j], y = v[r][2 * j + 1];
                    v[r][2 * j] = fma(e.x, y, e.y * x);
                    v[r][2 * j + 1] = fma(e.x, x, -(e.y * y));
                }
            }
        } else {
            // round B: pairs (2j+1, 2j+2) inside the segment, and the pairs across its
            // ends: (16 sg + 15, 16 sg + 16) with entry 8 sg + 7 on the right, and
            // (16 sg - 1, 16 sg) with entry 8 sg - 1 on the left
            // the last segment's entry 8 sg + 7 is past the round's pairs, so (0, 1) keeps
            // its last position; the first segment has no left pair, and (0, -1) keeps
            // its first position (the neighbours' values are finite either way)
            const double2 er = cu[LV_SP - 1];
            double2 el = cu[has_left ? -2 : 0];
            if (!has_left) el = make_double2(0.0, -1.0);
#pragma unroll
            for (int r = 0; r < LV_RPL; ++r) {
                const double y = lane_shift<true>(v[r][0]);             // right neighbour's first
                const double x = lane_shift<false>(v[r][LV_SEG - 1]);  // left neighbour's last
                const double xs = v[r][LV_SEG - 1], ys = v[r][0];
                v[r][LV_SEG - 1] = fma(er.x, y, er.y * xs);
                v[r][0] = fma(el.x, x, -(el.y * ys));
            }
#pragma unroll
            for (int j = 0; j < LV_SP - 1; ++j) {
                const double2 e = cu[j];
#pragma unroll
                for (int r = 0; r < LV_RPL; ++r) {
                    const double x = v[r][2 * j + 1], y = v[r][2 * j + 2];
                    v[r][2 * j + 1] = fma(e.x, y, e.y * x);
                    v[r][2 * j + 2] = fma(e.x, x, -(e.y * y));
                }
            }
        }
    }
}

// Replay of the rotation log on V = I.  Rows of V J are independent and a round's
// rotations touch neighbouring positions only, so V stays in registers: wavefront w of a
// leaf owns rows [32 w, 32 w + 32); lane 8 g + s holds rows 32 w + 4 g .. + 3 at positions
// [16 s, 16 s + 16) (positions past the leaf are zero padding).  Each round is static code:
// pairs inside a segment from registers, the pairs across segments (round B) with the
// neighbouring lane's value.  The log streams through LDS a block of rounds at a time, the
// next block's loads in flight; only this wavefront touches its LDS, so no barrier is
// needed.  A log entry (c, sigma) takes the columns x, y at the pair's positions to
// (c y + sigma x, c x - sigma y); entries past a round's real pairs are (0, 1), which keeps
// x in place and only negates the padding.
__global__ __launch_bounds__(WAVE, 2) void k_leaf_vectors(LeafArgs a) {
    __shared__ double2 cf[2][LV_RB][LV_CLD];
    const int L = a.leaf, half = L / 2;
    const int nwl = (L + LV_WROWS - 1) / LV_WROWS;
    const int leafid = blockIdx.x / nwl, w = blockIdx.x - leafid * nwl;
    const int lane = threadIdx.x;
    const int sg = lane % LV_NSEG;
    const int row0 = w * LV_WROWS + (lane / LV_NSEG) * LV_RPL, pos0 = sg * LV_SEG;
    const bool has_left = sg > 0;
    double v[LV_RPL][LV_SEG];
#pragma unroll
    for (int r = 0; r < LV_RPL; ++r)
#pragma unroll
        for (int j = 0; j < LV_SEG; ++j) v[r][j] = (row0 + r == pos0 + j) ? 1.0 : 0.0;

    const double2 *log = reinterpret_cast<const double2 *>(a.rot) + (size_t)leafid * a.max_sweeps * L * half;
    const int nsw = a.sweeps[leafid];
    const int rounds = nsw * L;  // L is even: round rd is a round A when rd is even
    // whole blocks only: when the rounds end half-way through a block, its last two rounds
    // run on (0, 1) entries, which keep x and negate y -- over a round A and a round B that
    // negates every position but 0, undone when the vectors are written
    const int nblk = (rounds + LV_RB - 1) / LV_RB;
    const bool padded = rounds % LV_RB != 0;
    const int slot = lane + lane / LV_SP;  // where this lane stages its entry
    double2 nx[LV_RB];
#pragma unroll
    for (int u = 0; u < LV_RB; ++u)
        nx[u] = (u < rounds && lane < half - (u & 1)) ? log[(size_t)u * half + lane] : make_double2(0.0, 1.0);
    for (int b = 0; b < nblk; ++b) {
        double2(*c)[LV_CLD] = cf[b & 1];
#pragma unroll
        for (int u = 0; u < LV_RB; ++u) c[u][slot] = nx[u];
        wave_sync();
#pragma unroll
        for (int u = 0; u < LV_RB; ++u) {
            const int rr = (b + 1) * LV_RB + u;
            nx[u] = (rr < rounds && lane < half - (u & 1)) ? log[(size_t)rr * half + lane]
                                                          : make_double2(0.0, 1.0);
        }
        replay_block(v, c, sg, has_left);
        wave_sync();
    }
    // the column at position pos is the eigenvector whose ascending rank the Jacobi kernel
    // stored for that position
    const int32_t *rank = a.rank + (size_t)leafid * L;
    double *Q = a.Q + (size_t)leafid * L * L;  // eigenvector k contiguous
#pragma unroll
    for (int j = 0; j < LV_SEG; ++j) {
        const int pos = pos0 + j;
        if (pos >= L) continue;
        const size_t k = (size_t)rank[pos];
        const bool flip = padded && pos != 0;
#pragma unroll
        for (int r = 0; r < LV_RPL; ++r)
            if (row0 + r < L) Q[k * L + row0 + r] = flip ? -v[r][j] : v[r][j];
    }
}

// W = Q^T U (L x r) per leaf, column-major with leading dimension ldw over the whole level
__global__ __launch_bounds__(256) void k_leaf_w(LeafArgs a) {
    __shared__ double Us[LEAF_MAX * LEAF_RANK_MAX];
    const int leafid = blockIdx.x;
    const int L = a.leaf, r = a.r, tid = threadIdx.x;
    const double *U = a.U + (size_t)leafid * L * r;
    for (int e = tid; e < L * r; e += blockDim.x) Us[e] = U[e];
    __syncthreads();
    const double *Q = a.Q + (size_t)leafid * L * L;
    for (int e = tid; e < L * r; e += blockDim.x) {
        const int k = e % L, c = e / L;
        const double *q = Q + (size_t)k * L;
        double acc = 0.0;
        for (int i = 0; i < L; ++i) acc = __builtin_fma(q[i], Us[i * r + c], acc);
        a.W[(int64_t)c * a.ldw + (int64_t)leafid * L + k] = acc;
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

// One pass of a bottom-up merge sort inside every segment of nl keys: runs of w (the last
// one ragged) are merged pairwise.  An element's place is its index in its run plus the
// number of keys of the partner run that go before it (strictly smaller for the left run,
// smaller or equal for the right one), so equal keys keep their order and every place lies
// inside the pair of runs whatever the keys hold.
__global__ __launch_bounds__(256) void k_sort_pass(const double *kin, const int32_t *vin,
                                                   double *kout, int32_t *vout, int nl, int w,
                                                   int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t base = (e / nl) * nl;
    const int i = (int)(e - base);
    const int ps = (i / (2 * w)) * (2 * w);
    const int mid = min(ps + w, nl), end = min(ps + 2 * w, nl);
    const double v = kin[e];
    const int32_t idx = vin ? vin[e] : i;
    int pos;
    if (i < mid) pos = (i - ps) + count_less(kin + base + mid, end - mid, v);
    else pos = (i - mid) + count_leq(kin + base + ps, mid - ps, v);
    kout[base + ps + pos] = v;
    vout[base + ps + pos] = idx;
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
    // the merge writes a permutation only when the children's spectra are sorted and free of
    // NaN (a failed child solve returns NaN): clamp, so that such a node stays in bounds and
    // only its status reports it
    const int src = min(max(a.perm[e], 0), nl - 1);
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
    const int64_t src = base + min(max(perm[e], 0), nl - 1);  // in bounds for any perm (k_assemble)
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
    SDC_LAUNCH(KID_LEAF, k_leaf_jacobi, dim3(a.nleaf), dim3(LJ_THREADS), 0, s, a);
    SDC_LAUNCH(KID_LEAF_VECTORS, k_leaf_vectors, dim3(a.nleaf * ((a.leaf + LV_WROWS - 1) / LV_WROWS)),
               dim3(WAVE), 0, s, a);
    SDC_LAUNCH(KID_LEAF_VECTORS, k_leaf_w, dim3(a.nleaf), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_merge(const double *lam_children, double *d_out, int32_t *perm, int nc,
                        int64_t n, hipStream_t s) {
    SDC_LAUNCH(KID_MERGE, k_merge, grid_for(n), dim3(256), 0, s, lam_children, d_out, perm, nc, n);
    return hipGetLastError();
}

hipError_t launch_seg_sort(const double *keys, int nl, int64_t n, double *kout, int32_t *vout,
                           double *kbuf, int32_t *vbuf, hipStream_t s) {
    int passes = 0;
    while ((1 << passes) < nl) ++passes;
    if (passes == 0) {  // segments of one key
        SDC_LAUNCH(KID_SORT, k_sort_pass, grid_for(n), dim3(256), 0, s, keys, nullptr, kout, vout,
                   1, 1, n);
        return hipGetLastError();
    }
    const double *kin = keys;
    const int32_t *vin = nullptr;
    for (int q = 0; q < passes; ++q) {
        // the last pass writes the outputs
        const bool to_out = ((passes - 1 - q) & 1) == 0;
        double *ko = to_out ? kout : kbuf;
        int32_t *vo = to_out ? vout : vbuf;
        SDC_LAUNCH(KID_SORT, k_sort_pass, grid_for(n), dim3(256), 0, s, kin, vin, ko, vo, nl,
                   1 << q, n);
        kin = ko;
        vin = vo;
    }
    return hipGetLastError();
}

hipError_t launch_assemble(const AssembleArgs &a, hipStream_t s) {
    SDC_LAUNCH(KID_ASSEMBLE, k_assemble, grid_for(a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_permute(const int32_t *perm, int nl, int64_t n, int m, const double *X,
                          int64_t ldx, double *Y, int64_t ldy, int scatter, hipStream_t s) {
    SDC_LAUNCH(KID_PERMUTE, k_permute, grid_for(n), dim3(256), 0, s, perm, nl, n, m, X, ldx, Y, ldy,
                       scatter);
    return hipGetLastError();
}

hipError_t launch_leaf_apply(const double *Q, int L, int64_t n, int m, const double *X,
                             int64_t ldx, double *Y, int64_t ldy, int trans, hipStream_t s) {
    SDC_LAUNCH(KID_LEAF_APPLY, k_leaf_apply, grid_for(n * m), dim3(256), 0, s, Q, L, n, m, X, ldx, Y, ldy,
                       trans);
    return hipGetLastError();
}

hipError_t launch_status_or(const int32_t *st, int cnt, int32_t *out, hipStream_t s) {
    SDC_LAUNCH(KID_STATUS_OR, k_status_or, dim3(1), dim3(256), 0, s, st, cnt, out);
    return hipGetLastError();
}

hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t s) {
    SDC_LAUNCH(KID_FILL, k_fill, grid_for(n), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

}  // namespace sdc
