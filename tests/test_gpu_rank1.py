"""GPU parity of the rank-one path against the CPU oracle, through the C ABI.

Each kernel is checked in isolation on the oracle's own outputs (oracle -> GPU is the only
direction data flows), plus end-to-end properties of the GPU pipeline.

Tolerances, derived from the arithmetic:
  eigenvalues   max_k |lambda_k - lambda_k^or| <= 1e-12 ||A||_2  (||A||_2 = max |lambda|)
  origins       identical: both sides decide K from the sign of f at the interval midpoint
                in FP64; the workloads keep f(mid) far from 0
  zhat, b       (from the oracle's eta) relative 1e-12: n-term products / sums of
                same-sign terms, each to ~0.5 ulp, so n eps = 1e-13 at n = 1024
  apply         (from the oracle's zhat, b, eta) |dY| <= 1e-12 * sum_j |Q_ij X_j|
  end to end    ||Qhat^T Qhat - I||_max <= 1e-12 with the GPU's own zhat, b, eta;
                zhat against the oracle's within the first-order effect of the two
                solvers' gap differences: 0.5 sum_j |d eta_j| / |lambda_j - d_i|
"""
import numpy as np
import pytest

from paper_2108_04209_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def oracle_of(orc, batch):
    return orc.solve_batch(batch)


def check_eigs(res, ref, batch):
    for p in range(batch.nprob):
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        assert res["status"][p] == 0, (p, res["status"][p])
        nA = np.abs(ref["lam"][a:e]).max()
        err = np.abs(res["lam"][a:e] - ref["lam"][a:e]).max()
        assert err <= 1e-12 * nA, (p, err / nA)
        bad = np.flatnonzero(res["origin"][a:e] != ref["origin"][a:e])
        assert bad.size == 0, (p, bad[:5])


def apply_tol(batch, ref, X):
    """1e-12 * sum_j |Qhat_ij X_jc| per output entry, for both orientations."""
    tol = {0: np.zeros_like(X), 1: np.zeros_like(X)}
    for p in range(batch.nprob):
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        d = batch.d[a:e]
        K = ref["origin"][a:e]
        C = 1.0 / ((d[:, None] - d[K][None, :]) - ref["eta"][a:e][None, :])
        Q = np.abs(ref["zhat"][a:e][:, None] * C * ref["b"][a:e][None, :])
        tol[0][a:e] = 1e-12 * (Q @ np.abs(X[a:e]))
        tol[1][a:e] = 1e-12 * (Q.T @ np.abs(X[a:e]))
    return tol


# -------------------------------------------------------------------- secular solve
@pytest.mark.parametrize("kind", ["cfg0", "uniform", "clustered", "tinyrho"])
@pytest.mark.parametrize("persistent", [1, 0])
def test_secular_solve(orc, kind, persistent):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    if kind == "cfg0":
        batch = gen.concat([gen.cfg0()[0]])
    else:
        sizes = [1, 2, 3, 5, 63, 64, 65, 127, 128, 129, 200, 511, 1000]
        if kind == "clustered":
            sizes = [s for s in sizes if s >= 16]
        batch = gen.small_batch(sizes, seed=21, kind=kind)
    ref = oracle_of(orc, batch)
    res = gp.run(batch, opts=native.default_opts(persistent=persistent), vectors=False)
    check_eigs(res, ref, batch)
    if kind == "tinyrho":  # gaps ~1e-20: only the shifted representation resolves them
        assert np.max(np.abs(res["eta"] - ref["eta"]) / np.abs(ref["eta"])) <= 1e-12


def test_noconv_flag():
    """max_iter = 1 cannot meet the stopping test for every root: the problem is flagged
    and every iterate still lies inside its bracket."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    batch = gen.small_batch([500], seed=2)
    res = gp.run(batch, opts=native.default_opts(max_iter=1), vectors=False)
    assert res["status"][0] & native.ST_NOCONV
    k = np.arange(500)
    org, eta = res["origin"], res["eta"]
    assert np.all(eta[org == k] > 0) and np.all(eta[org == k + 1] < 0)


def test_status_bits():
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    good = gen.small_batch([40], seed=1).problem(0)
    probs = []
    for kind in range(5):
        d, z, rho = good.d.copy(), good.z.copy(), good.rho
        if kind == 1:
            d[10], d[11] = d[11], d[10]
        elif kind == 2:
            z[5] = 0.0
        elif kind == 3:
            d[3] = np.nan
        elif kind == 4:
            rho = -1.0
        probs.append(gen.RankOne(d, z, rho))
    batch = gen.concat(probs)
    X = np.ones((batch.total_n, 4))
    res = gp.run(batch, X=X, trans=(0, 1))
    st = res["status"]
    assert st[0] == 0
    assert st[1] & native.ST_UNSORTED
    assert st[2] & native.ST_ZERO
    assert st[3] & native.ST_NONFINITE
    assert st[4] & native.ST_RHO
    for k in ("lam", "zhat", "b", "Y0", "Y1"):
        assert np.all(np.isnan(res[k][40:])), k
        assert np.all(np.isfinite(res[k][:40])), k


def test_status_bits_sliced():
    """Problems of 16384 entries and more are validated in slices, one workgroup each, with
    the slices' sums and status bits combined by a second launch: a defect in a late slice,
    an unsorted pair across a slice boundary (the last entry of a slice is compared with the
    first of the next), and a valid problem whose eigenvalues keep the trace identity
    sum(lambda) = sum(d) + rho |z|^2 and interlace with the poles."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    n = 20000  # four slices of 5000
    good = gen.small_batch([n], seed=3).problem(0)
    probs = []
    for kind in range(4):
        d, z, rho = good.d.copy(), good.z.copy(), good.rho
        if kind == 1:
            d[4999], d[5000] = d[5000], d[4999]  # across the first slice boundary
        elif kind == 2:
            z[17000] = 0.0
        elif kind == 3:
            d[19999] = np.inf
        probs.append(gen.RankOne(d, z, rho))
    batch = gen.concat(probs)
    res = gp.run(batch, vectors=False)
    st = res["status"]
    assert st[0] == 0, st
    assert st[1] & native.ST_UNSORTED and not st[1] & (native.ST_ZERO | native.ST_NONFINITE)
    assert st[2] & native.ST_ZERO and not st[2] & (native.ST_UNSORTED | native.ST_NONFINITE)
    assert st[3] & native.ST_NONFINITE
    lam = res["lam"][:n]
    assert np.all(np.isnan(res["lam"][n:]))
    # interlacing, up to the rounding of d_K + eta (eta can lie below half an ulp of d_K)
    assert np.all(lam[:-1] >= good.d[:-1]) and np.all(lam[:-1] <= good.d[1:])
    assert lam[-1] >= good.d[-1]
    k = np.arange(n)
    org, eta = res["origin"][:n], res["eta"][:n]
    assert np.all((org == k) | (org == k + 1))
    assert np.all(eta[org == k] > 0) and np.all(eta[org == k + 1] < 0)
    tr = good.d.sum() + good.rho * np.dot(good.z, good.z)
    assert abs(lam.sum() - tr) <= 1e-12 * n * np.abs(lam).max()


# -------------------------------------------------------------------- Loewner and b
@pytest.mark.parametrize("kind", ["cfg0", "uniform", "clustered"])
def test_loewner_kernel(orc, kind):
    from tests import gpu_pipeline as gp
    if kind == "cfg0":
        batch = gen.concat([gen.cfg0()[0]])
    else:
        batch = gen.small_batch([1, 2, 7, 64, 65, 130, 700, 2100], seed=5,
                                kind="uniform" if kind == "uniform" else "clustered") \
            if kind == "uniform" else gen.small_batch([16, 64, 65, 130, 700, 2100], seed=5, kind="clustered")
    ref = oracle_of(orc, batch)
    zh, bn = gp.loewner_from(batch, ref["eta"], ref["origin"])
    assert np.all(np.abs(zh - ref["zhat"]) <= 1e-12 * np.abs(ref["zhat"])), \
        np.max(np.abs(zh - ref["zhat"]) / np.abs(ref["zhat"]))
    assert np.all(np.abs(bn - ref["b"]) <= 1e-12 * np.abs(ref["b"])), \
        np.max(np.abs(bn - ref["b"]) / np.abs(ref["b"]))


# -------------------------------------------------------------------- Cauchy apply
@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("m", [1, 3, 16, 17, 64, 70])
def test_apply_kernel(orc, kernel, m):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    batch, X = gen.small_batch([1, 17, 64, 100, 260], seed=31, m=m)
    ref = oracle_of(orc, batch)
    tol = apply_tol(batch, ref, X)
    for t in (0, 1):
        Y = gp.apply_from(batch, ref["zhat"], ref["b"], ref["eta"], ref["origin"], X, t,
                          opts=native.default_opts(apply_kernel=kernel))
        Yo = np.concatenate([orc.cauchy_apply(batch.problem(p).d, ref["zhat"][a:e], ref["b"][a:e],
                                              ref["eta"][a:e], ref["origin"][a:e], X[a:e], trans=t)
                             for p, (a, e) in enumerate(zip(batch.off[:-1], batch.off[1:]))])
        assert np.all(np.abs(Y - Yo) <= tol[t] + 1e-300), (t, np.max(np.abs(Y - Yo) - tol[t]))


# -------------------------------------------------------------------- end to end
@pytest.mark.parametrize("persistent", [1, 0])
def test_end_to_end_cfg0(orc, persistent):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    pr, X = gen.cfg0()
    batch = gen.concat([pr])
    n = pr.n
    ref = oracle_of(orc, batch)
    res = gp.run(batch, X=np.eye(n), trans=(0, 1), opts=native.default_opts(persistent=persistent))
    check_eigs(res, ref, batch)
    Q = res["Y0"]
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-12
    assert np.abs(res["Y1"] - Q.T).max() <= 1e-13
    # zhat within the first-order effect of the gap differences between the two solvers
    d, K = pr.d, ref["origin"]
    gap = np.abs((d[K][None, :] - d[:, None]) + ref["eta"][None, :])   # |lambda_j - d_i|
    deta = np.abs(res["eta"] - ref["eta"])
    tol = 4 * (0.5 * (deta[None, :] / gap).sum(axis=1)) + 1e-13
    rel = np.abs(res["zhat"] - ref["zhat"]) / np.abs(ref["zhat"])
    assert np.all(rel <= tol), np.max(rel - tol)


def test_persistent_vs_plain_and_determinism():
    """The batched persistent launches are bitwise reproducible from run to run (each work
    item is solved by one wavefront whatever the queue order); the plain per-problem
    launches cut problems into smaller chunks, which moves the near/far split of some
    pole-root pairs, so they agree to rounding level only."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    batch, X = gen.small_batch([70, 300, 64, 1025, 9, 2000], seed=4, m=17)
    r1 = gp.run(batch, X=X, trans=(0, 1), opts=native.default_opts(persistent=1))
    r2 = gp.run(batch, X=X, trans=(0, 1), opts=native.default_opts(persistent=1))
    r0 = gp.run(batch, X=X, trans=(0, 1), opts=native.default_opts(persistent=0))
    for k in ("lam", "eta", "origin", "iters", "zhat", "b", "Y0", "Y1"):
        assert np.array_equal(r1[k], r2[k]), k
    np.testing.assert_array_equal(r1["origin"], r0["origin"])
    assert np.abs(r1["lam"] - r0["lam"]).max() <= 1e-14 * np.abs(r1["lam"]).max()
    assert np.abs(r1["Y1"] - r0["Y1"]).max() <= 1e-11 * np.abs(X).max()


def test_cfg2_sampled(orc):
    """The full batched level (4096 problems, n log-uniform in [64, 8192]) in one
    persistent pass; a seeded sample of problems, always including the largest and the
    smallest, is checked against the oracle; every problem's Qhat passes a sampled
    orthogonality check through the GPU apply."""
    from tests import gpu_pipeline as gp
    batch, X = gen.cfg2()
    res = gp.run(batch, X=X[:, :4], trans=(0, 1))
    assert np.all(res["status"] == 0)
    sizes = batch.sizes()
    rng = np.random.default_rng(0)
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes))}
                  | set(rng.choice(batch.nprob, 4, replace=False).tolist()))
    for p in pick:
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        lam, eta, org, its, st = orc.secular(pr.d, pr.z, pr.rho)
        assert np.abs(res["lam"][a:e] - lam).max() <= 1e-12 * np.abs(lam).max()
        assert np.array_equal(res["origin"][a:e], org)
    # Qhat^T (Qhat X) = X for every problem at once
    Y0 = res["Y0"]
    r2 = gp.run(batch, X=Y0, trans=(1,))
    assert np.abs(r2["Y1"] - X[:, :4]).max() <= 1e-11 * np.abs(X[:, :4]).max()


# -------------------------------------------------------------------- adjoint
@pytest.mark.parametrize("proj", [False, True])
def test_backward_kernel(orc, proj):
    from tests import gpu_pipeline as gp
    batch = gen.small_batch([1, 2, 33, 64, 65, 300, 1000], seed=8)
    ref = oracle_of(orc, batch)
    g = np.random.default_rng(3)
    gl = g.standard_normal(batch.total_n)
    gp_ = g.standard_normal(batch.total_n) if proj else None
    u = g.standard_normal(batch.total_n) if proj else None
    gd, gz, gr = gp.backward_from(batch, ref["eta"], ref["origin"], g_lam=gl, g_proj=gp_, u=u)
    for p in range(batch.nprob):
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        eta, K = ref["eta"][a:e], ref["origin"][a:e]
        od, oz, orr = orc.backward(pr.d, pr.z, pr.rho, eta, K, g_lam=gl[a:e],
                                   g_proj=None if gp_ is None else gp_[a:e],
                                   u=None if u is None else u[a:e])
        bd, bz, br = adjoint_abs_bound(pr.d, pr.z, pr.rho, eta, K, gl[a:e],
                                       None if gp_ is None else gp_[a:e],
                                       None if u is None else u[a:e])
        tol = 64 * (e - a + 8) * np.finfo(float).eps
        assert np.all(np.abs(gd[a:e] - od) <= tol * bd), (p, np.max(np.abs(gd[a:e] - od) / bd))
        assert np.all(np.abs(gz[a:e] - oz) <= tol * bz), (p, np.max(np.abs(gz[a:e] - oz) / bz))
        assert abs(gr[p] - orr) <= tol * br, p


def adjoint_abs_bound(d, z, rho, eta, K, gl, gpj, u):
    """The adjoint's sums with every term replaced by its absolute value: the scale
    against which floating-point summation error is measured (condition of the sums)."""
    r = 1.0 / ((d[:, None] - d[K][None, :]) - eta[None, :])     # r[i, k]
    ar = np.abs(r)
    z2 = z * z
    S = (z2[:, None] * r * r).sum(0)
    b = 1.0 / np.sqrt(S)
    S3a = (z2[:, None] * ar ** 3).sum(0)
    lb = np.abs(gl).copy()
    B = np.zeros_like(b)
    G = np.zeros_like(b)
    if gpj is not None:
        ha = (np.abs(u * z)[:, None] * ar).sum(0)
        H2a = (np.abs(u * z)[:, None] * ar ** 2).sum(0)
        lb += np.abs(gpj) * (b * H2a + ha * b ** 3 * S3a)
        B = np.abs(gpj) * b
        G = np.abs(gpj) * ha * b ** 3
    A = lb * b * b
    bd = z2 * (ar ** 2 @ A) + z2 * (ar ** 3 @ G)
    bz = 2 * np.abs(z) * (ar @ A) + np.abs(z) * (ar ** 2 @ G)
    if gpj is not None:
        bd += np.abs(u * z) * (ar ** 2 @ B)
        bz += np.abs(u) * (ar @ B)
    br = A.sum() / rho ** 2
    return bd, bz, br


# -------------------------------------------------------------------- scale invariance
@pytest.mark.parametrize("e", [-250, 250])
@pytest.mark.parametrize("method", [1, 2])
def test_power_of_two_scaling(e, method):
    """diag(s d) + (s rho) z z^T = s A for s = 2^e: eigenvalues and gaps scale by s, the
    origins, zhat (rho zhat^2 scales by s) and the eigenvector matrix do not change, b scales
    by s.  Scaling by a power of two is exact, so every quantity must come out as the
    unscaled one times its power of s to rounding -- in particular no intermediate of the
    shared reciprocals (t0 t1, its reciprocal squared) and no block of the Loewner products
    may leave the exponent range (s = 2^-250 puts pole gaps near 2^-270)."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    batch, X = gen.small_batch([1024, 300, 2048], seed=61, m=8)
    s = 2.0 ** e
    sb = gen.Batch(off=batch.off, d=batch.d * s, z=batch.z.copy(), rho=batch.rho * s)
    o = native.default_opts(method=method)
    print(f"scaling 2^{e}, method {method}", flush=True)
    r0 = gp.run(batch, X=X, trans=(1,), opts=o)
    r1 = gp.run(sb, X=X, trans=(1,), opts=o)
    assert np.all(r0["status"] == 0) and np.all(r1["status"] == 0)
    np.testing.assert_array_equal(r1["origin"], r0["origin"])
    np.testing.assert_array_equal(r1["iters"], r0["iters"])
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    assert rel(r1["lam"] / s, r0["lam"]) <= 4e-16
    assert np.all(np.abs(r1["eta"] / s - r0["eta"]) <= 4e-16 * np.abs(r0["eta"]))
    assert np.all(np.abs(r1["zhat"] - r0["zhat"]) <= 1e-15 * np.abs(r0["zhat"]))
    assert np.all(np.abs(r1["b"] / s - r0["b"]) <= 1e-15 * np.abs(r0["b"]))
    assert rel(r1["Y1"], r0["Y1"]) <= 1e-14
