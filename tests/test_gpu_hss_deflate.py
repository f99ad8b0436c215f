"""GPU: the HSS conquering pass with deflation (Remark 1) inside every rank-one step,
after the dividing stage, on the paper's first example and on matrices like it.

Deflation drops, per step, couplings below tau (rule 1: |z_k| < tau, a perturbation of
norm below 2 tau ||z||; rule 2: a rotated off-diagonal entry below tau), so by Weyl every
eigenvalue moves by at most the sum of what the steps drop: the bounds below are that sum
for the number of deflations a pass can make, not a fit to the results.

  - tridiagonal matrix with 3 on the diagonal and -1 beside it (HSS rank 2): eigenvalues
    against the closed form 3 - 2 cos(k pi / (n + 1)); sampled eigenvectors from the
    structured eigenmatrix: orthonormal, and T q = lambda q with T applied directly;
  - the whole eigenmatrix of a small case (n = 1024): Q^T Q = I, T Q = Q Lambda, and the
    two directions of the structured product transposes of each other;
  - the paper's residual, relative error and orthogonality measures on the whole
    eigenmatrix at n = 8192;
  - random tridiagonal matrices (localised eigenvectors) against LAPACK's tridiagonal
    solver;
  - a dense-generator HSS matrix, where almost nothing deflates, against the pass without
    deflation.
"""
import numpy as np
import pytest

from paper_2108_04209_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def run(tree, tau, balanced=True):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    ctx = gp.context()
    plan = native.HSSPlan(ctx, tree.leaf, tree.depth, tree.r)
    g = {k: gp.to_dev(v) for k, v in native.pack_hss(tree).items()}
    dv = native.hss_divide(ctx, plan, g, balanced=balanced)
    out = native.hss_conquer(ctx, plan, dv, opts=native.default_opts(hss_tau=tau))
    torch.cuda.synchronize()
    return plan, out["lam"].cpu().numpy(), int(out["status"].cpu().numpy()[0])


def tmatvec(d, e, X):
    Y = d[:, None] * X
    Y[:-1] += e[:, None] * X[1:]
    Y[1:] += e[:, None] * X[:-1]
    return Y


def columns(plan, ks, n):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    E = np.zeros((len(ks), n))
    E[np.arange(len(ks)), ks] = 1.0
    return native.hss_apply(gp.context(), plan, gp.to_dev(E), trans=0).cpu().numpy().T


@pytest.mark.parametrize("n,leaf,tau,bound", [(8192, 64, 1e-10, 1e-9), (8192, 64, 1e-13, 1e-12),
                                              (65536, 128, 1e-10, 1e-9)])
def test_tridiagonal_example(n, leaf, tau, bound):
    plan, lam, st = run(gen.tridiag_hss(n, leaf), tau)
    assert st == 0
    exact = np.sort(3.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    assert np.abs(lam - exact).max() <= bound * 5.0
    rng = np.random.default_rng(7)
    ks = np.sort(np.r_[0, n - 1, rng.choice(n, 30, replace=False)])
    Qs = columns(plan, ks, n)
    res = np.linalg.norm(tmatvec(np.full(n, 3.0), np.full(n - 1, -1.0), Qs) - Qs * lam[ks], axis=0)
    assert res.max() <= max(bound, 1e-11) * 5.0
    assert np.abs(Qs.T @ Qs - np.eye(len(ks))).max() <= 1e-11


def test_tridiagonal_accuracy_measures():
    """The paper's three accuracy measures for its first example (its table for Ex. 1) on the
    whole eigenmatrix at n = 8192 with tau = 1e-10: residual gamma = max_k ||T q_k - lambda_k
    q_k|| / (n ||T||), relative error delta = ||lambda* - lambda|| / (n ||lambda*||) against the
    closed form, loss of orthogonality theta = max_k ||Q^T q_k - e_k|| / n.  The bounds are
    those of the sampled test above (per-root residual and eigenvalue error at most
    5 x 1e-9, orthogonality 1e-11) in the paper's normalisation, not a fit to the results."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    n = 8192
    plan, lam, st = run(gen.tridiag_hss(n, 64), 1e-10)
    assert st == 0
    Q = torch.empty((n, n), dtype=torch.float64, device="cuda")  # row c: column c of Q
    for c0 in range(0, n, 2048):
        E = torch.zeros((2048, n), dtype=torch.float64, device="cuda")
        E[torch.arange(2048), torch.arange(c0, c0 + 2048)] = 1.0
        Q[c0:c0 + 2048] = native.hss_apply(gp.context(), plan, E, trans=0)
    torch.cuda.synchronize()
    exact = np.sort(3.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    nA = exact.max()
    TQ = 3.0 * Q
    TQ[:, :-1] -= Q[:, 1:]
    TQ[:, 1:] -= Q[:, :-1]
    lam_d = torch.from_numpy(lam).to("cuda")
    gamma = float((TQ - Q * lam_d[:, None]).norm(dim=1).max()) / (n * nA)
    del TQ
    G = Q @ Q.T
    G.diagonal().sub_(1.0)
    theta = float(G.norm(dim=1).max()) / n
    delta = float(np.linalg.norm(lam - exact) / (n * np.linalg.norm(exact)))
    assert gamma <= 5e-9 / (n * nA)
    assert theta <= 1e-11 / n
    assert delta <= 5e-9 * np.sqrt(n) / (n * np.linalg.norm(exact))


def test_tridiagonal_eigenmatrix_small():
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    n = 1024
    plan, lam, st = run(gen.tridiag_hss(n, 32), 1e-12)
    assert st == 0
    I = gp.to_dev(np.eye(n))
    Q = native.hss_apply(gp.context(), plan, I, trans=0).cpu().numpy().T
    QT = native.hss_apply(gp.context(), plan, I, trans=1).cpu().numpy().T
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-12
    assert np.abs(QT - Q.T).max() <= 1e-13
    T = tmatvec(np.full(n, 3.0), np.full(n - 1, -1.0), np.eye(n))
    assert np.abs(T @ Q - Q * lam).max() <= 1e-11 * 5.0


@pytest.mark.parametrize("seed", [0, 1])
def test_tridiagonal_random(seed):
    from scipy.linalg import eigvalsh_tridiagonal
    n = 4096
    g = np.random.default_rng(41 + seed)
    d, e = g.uniform(1, 5, n), g.uniform(-1, 1, n - 1)
    plan, lam, st = run(gen.tridiag_hss(n, 128, diag=d, off=e), 1e-12)
    assert st == 0
    ev = eigvalsh_tridiagonal(d, e)
    nA = np.abs(ev).max()
    assert np.abs(lam - ev).max() <= 1e-11 * nA
    ks = np.sort(g.choice(n, 24, replace=False))
    Qs = columns(plan, ks, n)
    res = np.linalg.norm(tmatvec(d, e, Qs) - Qs * lam[ks], axis=0)
    assert res.max() <= 1e-11 * nA
    assert np.abs(Qs.T @ Qs - np.eye(len(ks))).max() <= 1e-11


def test_dense_generators_unchanged():
    tree = gen.hss_original(n=4096, leaf=64, r=4, cfg=44)
    _, lam0, st0 = run(tree, 0.0)
    _, lam1, st1 = run(tree, 1e-15)
    assert st0 == 0 and st1 == 0
    assert np.abs(lam1 - lam0).max() <= 1e-13 * np.abs(lam0).max()


def test_vanished_couplings_and_fully_deflated_nodes():
    """Couplings that vanish (B_p = 0: the dividing stage takes beta_p = 1 and the update
    column of the left child is zero, so rule 1 takes all of its poles) and leaf bases that
    are zero (every update column vanishes, every node deflates completely and its reduced
    problem is a one-pole stand-in whose results are never used): the spectrum is still
    LAPACK's of the assembled matrix, and the structured eigenmatrix stays orthogonal."""
    import copy
    from oracle import hss as ohss
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    base = gen.hss_original(n=1024, leaf=32, r=4, cfg=45)
    t1 = copy.deepcopy(base)
    for l in (0, 2):
        t1.B[l][:] = 0.0
    t2 = copy.deepcopy(base)
    t2.leaf_U[:] = 0.0
    for t in (t1, t2):
        plan, lam, st = run(t, 1e-13)
        assert st == 0
        ev = np.linalg.eigvalsh(ohss.dense_original(t))
        assert np.abs(lam - ev).max() <= 1e-12 * np.abs(ev).max()
        n = t.n
        Q = native.hss_apply(gp.context(), plan, gp.to_dev(np.eye(n)), trans=0).cpu().numpy().T
        assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-12
