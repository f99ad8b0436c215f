/*
 * superdc_oracle.c -- plain, slow FP64 CPU oracle for the conquering-stage rank-one
 * problem of SuperDC (Ou & Xia, "SuperDC: Stable superfast divide-and-conquer
 * eigenvalue decomposition").
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load this library.  The HIP library shares no code with it.
 *
 * The problem (Sec. 2.2, eq. rank1upd with v = sqrt(rho) z) is the eigendecomposition
 *     A = diag(d) + rho z z^T,   d strictly increasing, z_i != 0, rho > 0.
 * Every quantity below has a plain definition, and this file writes that definition out:
 *   - eigenvalues: roots of the secular equation f(x) = 1 + sum_j w_j/(d_j - x),
 *     w_j = rho z_j^2 (eq. seceq), one per interval (d_k, d_{k+1}) and one above d_n
 *     (interlacing, eq. interlace).  Each root is found on the shifted equation
 *     g(y) = f(d_K + y) = 1 + sum_j w_j/(delta_j - y), delta_j = d_j - d_K (eq. shiftedeq,
 *     eq. deltajk), with the origin K chosen by the sign of f at the interval midpoint
 *     (Sec. 4.2.1).  The iteration here is plain bisection-safeguarded Newton with
 *     compensated sums -- deliberately not the paper's modified Newton.
 *   - zhat: Loewner's formula (eq. lowner), evaluated as a product of ratios that each
 *     lie in (0,1) by interlacing, so the running product never overflows.
 *   - b: normalisation of the Cauchy-like eigenvector matrix (eq. b).
 *   - Qhat X and Qhat^T X with Qhat_ij = zhat_i b_j / (d_i - lambda_j) (eq. eigvecs,
 *     eq. qscale), every d_i - lambda_j formed as (d_i - d_{K_j}) - eta_j (eq. qk).
 *   - the adjoint of lambda and of projections p_k = q_k^T u with respect to (d, z, rho),
 *     from implicit differentiation of f(lambda_k) = 0 (not in the paper).
 *   - deflation with a user tolerance tau (Remark 1): the two rules taken in the paper's
 *     order, the second as a left-to-right scan in which a pole that survives a rotation
 *     carries its rotated values on to the next comparison.
 *
 * Status bits returned by the validating entry points:
 *   1 d not strictly increasing, 2 some z_i == 0, 4 non-finite input, 8 rho <= 0,
 *   16 a root did not converge within the iteration cap.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EUNSORTED 1
#define OR_EZERO 2
#define OR_ENONFINITE 4
#define OR_ERHO 8
#define OR_ENOCONV 16

#define OR_MAXIT 1000

/* ---------------------------------------------------------------------------------- */
/* Neumaier's compensated summation                                                   */
/* ---------------------------------------------------------------------------------- */
typedef struct {
    double s, c;
} csum;

static inline void cs_add(csum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double cs_val(const csum *a) { return a->s + a->c; }

/* ---------------------------------------------------------------------------------- */
/* validation (Sec. 2.2: sorted poles; Sec. 4.1 assumes no deflation is needed)       */
/* ---------------------------------------------------------------------------------- */
int oracle_validate(int64_t n, const double *d, const double *z, double rho)
{
    int st = 0;
    if (!isfinite(rho)) st |= OR_ENONFINITE;
    else if (!(rho > 0.0)) st |= OR_ERHO;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(d[i]) || !isfinite(z[i])) st |= OR_ENONFINITE;
        if (z[i] == 0.0) st |= OR_EZERO;
        if (i + 1 < n && !(d[i] < d[i + 1])) st |= OR_EUNSORTED;
    }
    return st;
}

/* g(y) = 1 + sum_j w_j / ((d_j - d_K) - y) and g'(y) = sum_j w_j / ((d_j - d_K) - y)^2 */
static double shifted_eval(int64_t n, const double *d, const double *w, int64_t K, double y,
                           double *gprime)
{
    csum g = {1.0, 0.0}, gp = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
        double t = (d[j] - d[K]) - y;
        double term = w[j] / t;
        cs_add(&g, term);
        cs_add(&gp, term / t);
    }
    if (gprime) *gprime = cs_val(&gp);
    return cs_val(&g);
}

/*
 * One root k (0-based) of the secular equation.  Origin and bracket (Sec. 4.2.1):
 *   k < n-1: h = d_{k+1} - d_k; if f(d_k + h/2) >= 0 the root lies in (d_k, d_k + h/2] and
 *            the origin is K = k with y in (0, h/2]; otherwise the origin is K = k+1 and
 *            y in (-h/2, 0).
 *   k = n-1: origin n-1, y in (0, sum_j w_j] because f(d_n + sum w) >= 0.
 * Then bisection-safeguarded Newton on g (g increases on the bracket).
 */
static int solve_root(int64_t n, const double *d, const double *w, double wsum, int64_t k,
                      double *eta, int32_t *origin, int32_t *iters)
{
    int64_t K;
    double lo, hi;
    int hi_closed; /* the upper end is a point where g >= 0, not a pole */
    if (k < n - 1) {
        double h = d[k + 1] - d[k];
        double fmid = shifted_eval(n, d, w, k, 0.5 * h, NULL);
        if (fmid >= 0.0) {
            K = k;
            lo = 0.0;
            hi = 0.5 * h;
            hi_closed = 1;
        } else {
            K = k + 1;
            lo = -0.5 * h;
            hi = 0.0;
            hi_closed = 0;
        }
    } else {
        K = n - 1;
        lo = 0.0;
        hi = wsum;
        hi_closed = 1;
    }
    double y = 0.5 * (lo + hi);
    int it, ok = 0;
    for (it = 1; it <= OR_MAXIT; ++it) {
        double gp;
        double g = shifted_eval(n, d, w, K, y, &gp);
        if (g == 0.0) {
            ok = 1;
            break;
        }
        if (g < 0.0) {
            lo = y;
        } else {
            hi = y;
            hi_closed = 0;
        }
        double yn = y - g / gp;
        int inside = (yn > lo) && (yn < hi || (hi_closed && yn == hi));
        if (!inside || !isfinite(yn)) yn = 0.5 * (lo + hi);
        if (fabs(yn - y) <= 2.0 * DBL_EPSILON * fabs(yn)) {
            y = yn;
            ok = 1;
            break;
        }
        y = yn;
        if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) {
            ok = 1;
            break;
        }
    }
    *eta = y;
    *origin = (int32_t)K;
    if (iters) *iters = it;
    return ok ? 0 : OR_ENOCONV;
}

/*
 * Eigenvalues of diag(d) + rho z z^T.  roots == NULL solves all n roots (nroots must be n);
 * otherwise output slot t holds root roots[t].  lam_t = d_{origin_t} + eta_t.
 */
int oracle_secular(int64_t n, const double *d, const double *z, double rho,
                   const int64_t *roots, int64_t nroots, double *lam, double *eta,
                   int32_t *origin, int32_t *iters)
{
    int st = oracle_validate(n, d, z, rho);
    if (st) return st;
    double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    csum ws = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
        w[j] = rho * z[j] * z[j];
        cs_add(&ws, w[j]);
    }
    double wsum = cs_val(&ws);
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : fail)
    for (int64_t t = 0; t < nroots; ++t) {
        int64_t k = roots ? roots[t] : t;
        int32_t K, itc;
        double e;
        fail |= solve_root(n, d, w, wsum, k, &e, &K, &itc);
        eta[t] = e;
        origin[t] = K;
        lam[t] = d[K] + e;
        if (iters) iters[t] = itc;
    }
    free(w);
    return fail;
}

/*
 * Loewner's formula (eq. lowner): rho zhat_i^2 = prod_j (lambda_j - d_i) / prod_{j != i} (d_j - d_i),
 * with lambda_j - d_i = (d_{K_j} - d_i) + eta_j.  The factors are paired as
 *   (lambda_{n-1} - d_i) * prod_{j<i} (lambda_j - d_i)/(d_j - d_i)
 *                        * prod_{i<=j<n-1} (lambda_j - d_i)/(d_{j+1} - d_i),
 * every ratio in (0,1) by interlacing.  Sign of zhat_i is that of z_i.
 * poles == NULL computes every i (npoles must be n); else slot t holds pole poles[t].
 */
void oracle_loewner(int64_t n, const double *d, const double *z, double rho,
                    const double *eta, const int32_t *origin, const int64_t *poles,
                    int64_t npoles, double *zhat)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < npoles; ++t) {
        int64_t i = poles ? poles[t] : t;
        double R = (d[origin[n - 1]] - d[i]) + eta[n - 1];
        for (int64_t j = 0; j < i; ++j) R *= ((d[origin[j]] - d[i]) + eta[j]) / (d[j] - d[i]);
        for (int64_t j = i; j < n - 1; ++j)
            R *= ((d[origin[j]] - d[i]) + eta[j]) / (d[j + 1] - d[i]);
        zhat[t] = copysign(sqrt(R / rho), z[i]);
    }
}

/* b_j = (sum_i zhat_i^2 / (d_i - lambda_j)^2)^(-1/2)   (eq. b) */
void oracle_bnorm(int64_t n, const double *d, const double *zhat, const double *eta,
                  const int32_t *origin, const int64_t *roots, int64_t nroots, double *b)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nroots; ++t) {
        int64_t j = roots ? roots[t] : t;
        csum s = {0.0, 0.0};
        for (int64_t i = 0; i < n; ++i) {
            double q = zhat[i] / ((d[i] - d[origin[j]]) - eta[j]);
            cs_add(&s, q * q);
        }
        b[t] = 1.0 / sqrt(cs_val(&s));
    }
}

/* one entry of the Cauchy-like eigenvector matrix (eq. eigvecs with eq. qk) */
static inline double qhat(const double *d, const double *zhat, const double *b,
                          const double *eta, const int32_t *origin, int64_t i, int64_t j)
{
    return zhat[i] * b[j] / ((d[i] - d[origin[j]]) - eta[j]);
}

/*
 * Y = Qhat X (trans = 0) or Y = Qhat^T X (trans = 1).  X is n x m column-major with leading
 * dimension ldx, Y likewise with ldy.  rows == NULL computes every output row (nrows = n);
 * else output row t of Y (Y[t + c*ldy]) holds row rows[t] of the product.
 */
void oracle_cauchy_apply(int64_t n, const double *d, const double *zhat, const double *b,
                         const double *eta, const int32_t *origin, int trans, int64_t m,
                         const double *X, int64_t ldx, const int64_t *rows, int64_t nrows,
                         double *Y, int64_t ldy)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t r = rows ? rows[t] : t;
        for (int64_t c = 0; c < m; ++c) {
            double acc = 0.0;
            for (int64_t s = 0; s < n; ++s) {
                double q = trans ? qhat(d, zhat, b, eta, origin, s, r)
                                 : qhat(d, zhat, b, eta, origin, r, s);
                acc += q * X[s + c * ldx];
            }
            Y[t + c * ldy] = acc;
        }
    }
}

/*
 * Adjoint of the rank-one eigensolver.  With r_ik = 1/(d_i - lambda_k) (shifted form),
 * S_k = sum_i z_i^2 r_ik^2, b_k = S_k^(-1/2), eigenvectors q_ik = b_k z_i r_ik, and the
 * projections p_k = q_k^T u, implicit differentiation of f(lambda_k; d, z, rho) = 0 gives
 *   d lambda_k / d d_i = z_i^2 r_ik^2 / S_k,  d lambda_k / d z_i = -2 z_i r_ik / S_k,
 *   d lambda_k / d rho = 1 / (rho^2 S_k),
 * and p_k = b_k h_k with h_k = sum_i u_i z_i r_ik depends on (d, z) directly and through
 * lambda_k.  Given g_lam = dL/dlambda and g_proj = dL/dp (either may be NULL), this
 * accumulates dL/dd, dL/dz, dL/drho by the chain rule written out term by term.
 */
void oracle_backward(int64_t n, const double *d, const double *z, double rho,
                     const double *eta, const int32_t *origin, const double *g_lam,
                     const double *g_proj, const double *u, double *g_d, double *g_z,
                     double *g_rho)
{
    double *lbar = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *Sk = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *hk = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *bk = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));

    /* per root: S_k, h_k, dh/dlambda, dS/dlambda, and the total derivative weight */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) {
        csum S = {0, 0}, h = {0, 0}, H2 = {0, 0}, S3 = {0, 0};
        for (int64_t i = 0; i < n; ++i) {
            double r = 1.0 / ((d[i] - d[origin[k]]) - eta[k]);
            cs_add(&S, z[i] * z[i] * r * r);
            cs_add(&S3, z[i] * z[i] * r * r * r);
            if (g_proj) {
                cs_add(&h, u[i] * z[i] * r);
                cs_add(&H2, u[i] * z[i] * r * r);
            }
        }
        double s = cs_val(&S), b = 1.0 / sqrt(s);
        double lb = g_lam ? g_lam[k] : 0.0;
        if (g_proj) {
            /* dp_k/dlambda_k = b_k dh/dlambda + h_k db/dlambda,
               dh/dlambda = sum u z r^2, db/dlambda = -b^3 sum z^2 r^3 */
            double hv = cs_val(&h);
            lb += g_proj[k] * (b * cs_val(&H2) - hv * b * b * b * cs_val(&S3));
            hk[k] = hv;
        }
        lbar[k] = lb;
        Sk[k] = s;
        bk[k] = b;
    }

    /* per pole: chain rule through lambda (all k) and the direct dependence of p_k */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        csum gd = {0, 0}, gz = {0, 0};
        for (int64_t k = 0; k < n; ++k) {
            double r = 1.0 / ((d[i] - d[origin[k]]) - eta[k]);
            /* through lambda_k */
            cs_add(&gd, lbar[k] * z[i] * z[i] * r * r / Sk[k]);
            cs_add(&gz, lbar[k] * (-2.0) * z[i] * r / Sk[k]);
            if (g_proj) {
                double b = bk[k], gp = g_proj[k];
                /* dp_k/dd_i at fixed lambda: b dh/dd_i + h db/dd_i,
                   dh/dd_i = -u_i z_i r^2, db/dd_i = b^3 z_i^2 r^3 */
                cs_add(&gd, gp * (-b * u[i] * z[i] * r * r + hk[k] * b * b * b * z[i] * z[i] * r * r * r));
                /* dp_k/dz_i at fixed lambda: dh/dz_i = u_i r, db/dz_i = -b^3 z_i r^2 */
                cs_add(&gz, gp * (b * u[i] * r - hk[k] * b * b * b * z[i] * r * r));
            }
        }
        g_d[i] = cs_val(&gd);
        g_z[i] = cs_val(&gz);
    }

    csum gr = {0, 0};
    for (int64_t k = 0; k < n; ++k) cs_add(&gr, lbar[k] / (rho * rho * Sk[k]));
    *g_rho = cs_val(&gr);

    free(lbar);
    free(Sk);
    free(hk);
    free(bk);
}

/* ---------------------------------------------------------------------------------- */
/* deflation (Remark 1)                                                               */
/* ---------------------------------------------------------------------------------- */
/*
 * A = diag(d) + v v^T with v = sqrt(rho) z, d non-decreasing, tau >= 0.
 *   rule 1: pole k is deflated if |v_k| < tau; its eigenpair is (d_k, e_k).
 *   rule 2: over the remaining poles in increasing order, the current pole a and the next
 *           remaining pole b are rotated together if |(d_a - d_b) v_a v_b| < (v_a^2 + v_b^2)
 *           tau (both sides scale by rho, so z takes the place of v).  With r =
 *           sqrt(z_a^2 + z_b^2), c = z_b / r, s = z_a / r the rotation G = [c -s; s c] on
 *           (a, b) maps (z_a, z_b) to (0, r) and diag(d_a, d_b) to
 *           [c^2 d_a + s^2 d_b, cs (d_a - d_b); cs (d_a - d_b), s^2 d_a + c^2 d_b]; the
 *           off-diagonal entry is below tau and is dropped.  Pole a is deflated with the
 *           eigenvalue c^2 d_a + s^2 d_b; pole b continues with d_b' = s^2 d_a + c^2 d_b
 *           (held inside [d_a, d_b]) and z_b' = r and is compared with the next pole.
 *           Otherwise pole a is kept.
 * Every expression is evaluated exactly as written (this file is built without FP
 * contraction), so another implementation that evaluates the same expressions in the
 * same order reaches the same decisions.
 *
 * Outputs (all of length n):
 *   dout/zout[0 .. kept)  the reduced problem, strictly increasing poles;
 *   dout[kept .. n)       the deflated eigenvalues in order of their pole's index, zout = 0;
 *   perm[j]               the pole index of output position j;
 *   rright[i]             for a pole deflated by rule 2, the pole it was rotated with
 *                         (-1 otherwise); rleft[b] = a whenever rright[a] = b (-1 otherwise);
 *   rc[i], rs[i]          that rotation's c and s (1 and 0 where there is none).
 * Returns kept.
 */
int64_t oracle_deflate(int64_t n, const double *d, const double *z, double rho, double tau,
                       double *dout, double *zout, int32_t *perm, int32_t *rright,
                       int32_t *rleft, double *rc, double *rs)
{
    const double sv = sqrt(rho);
    /* per pole: its final value and whether it is kept */
    double *dv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *zv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    char *keep = (char *)malloc((size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        rright[i] = -1;
        rleft[i] = -1;
        rc[i] = 1.0;
        rs[i] = 0.0;
        dv[i] = d[i];
        zv[i] = 0.0;
        keep[i] = 0;
    }
    int64_t a = -1;     /* the current pole of the scan */
    double da = 0.0, za = 0.0;
    for (int64_t b = 0; b < n; ++b) {
        if (fabs(sv * z[b]) < tau) continue; /* rule 1 */
        if (a < 0) {
            a = b;
            da = d[b];
            za = z[b];
            continue;
        }
        const double db = d[b], zb = z[b];
        const double r2 = za * za + zb * zb;
        const double lhs = fabs(((da - db) * za) * zb);
        if (lhs < r2 * tau) { /* rule 2: rotate a into b */
            const double r = sqrt(r2);
            const double c = zb / r, s = za / r;
            const double cc = c * c, ss = s * s;
            const double dl = cc * da + ss * db;
            double dr = ss * da + cc * db;
            if (dr < da) dr = da;
            if (dr > db) dr = db;
            dv[a] = dl;
            rright[a] = (int32_t)b;
            rleft[b] = (int32_t)a;
            rc[a] = c;
            rs[a] = s;
            a = b;
            da = dr;
            za = r;
        } else { /* a is kept with its current values */
            keep[a] = 1;
            dv[a] = da;
            zv[a] = za;
            a = b;
            da = db;
            za = zb;
        }
    }
    if (a >= 0) {
        keep[a] = 1;
        dv[a] = da;
        zv[a] = za;
    }
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) kept += keep[i];
    int64_t pk = 0, pd = kept;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t j = keep[i] ? pk++ : pd++;
        dout[j] = dv[i];
        zout[j] = keep[i] ? zv[i] : 0.0;
        perm[j] = (int32_t)i;
    }
    free(dv);
    free(zv);
    free(keep);
    return kept;
}
