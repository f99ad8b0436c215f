"""Pins of the oracle's dividing stage (Alg. 1 with Lemma genupd and the balanced update
of eq. divnew1), against facts fixed by the mathematics:
  - dividing is exact algebra: the divided form blkdiag(D-hat) + sum_p Z_p Z_p^T assembled
    densely equals the HSS matrix of the original generators (eq. hss) to rounding, so its
    spectrum equals LAPACK's on the original matrix;
  - the tridiagonal matrix of the paper's first example, written as an HSS form of rank 2,
    assembles to the tridiagonal matrix exactly, and tridiag(-1, 3, -1) has the closed-form
    spectrum 3 - 2 cos(k pi / (n + 1));
  - with orthonormal nested bases, the assembled matrix has trace sum tr D_leaf and squared
    Frobenius norm sum ||D_leaf||_F^2 + 2 sum_p ||B_p||_F^2 (each coupling block appears
    twice, and orthonormal bases keep its norm);
  - Prop. prop:b: with the balanced update, ||B-tilde|| at level l is at most 2^l beta;
    the unbalanced update (eq. divide) lets it grow far beyond that on the same tree.
"""
import numpy as np
import pytest

from paper_2108_04209_amd import gen


@pytest.mark.parametrize("n,leaf,r,cfg", [(512, 32, 4, 7), (1024, 16, 8, 8), (256, 64, 2, 9)])
def test_divided_form_is_the_matrix(n, leaf, r, cfg):
    from oracle import hss as oh
    t = gen.hss_original(n=n, leaf=leaf, r=r, cfg=cfg)
    A = oh.dense_original(t)
    Ad = oh.dense_nodes(oh.divide(t))[(0, 0)]
    nrm = np.abs(np.linalg.eigvalsh(A)).max()
    assert np.abs(A - Ad).max() <= 1e-14 * nrm * np.sqrt(n)
    assert np.abs(np.linalg.eigvalsh(A) - np.linalg.eigvalsh(Ad)).max() <= 1e-13 * nrm


def test_tridiagonal_example():
    from oracle import hss as oh
    n = 512
    t = gen.tridiag_hss(n, 32)
    A = oh.dense_original(t)
    T = np.diag(np.full(n, 3.0)) + np.diag(np.full(n - 1, -1.0), 1) + np.diag(np.full(n - 1, -1.0), -1)
    assert np.array_equal(A, T)
    ev = np.sort(np.linalg.eigvalsh(oh.dense_nodes(oh.divide(t))[(0, 0)]))
    exact = np.sort(3.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    assert np.abs(ev - exact).max() <= 16 * np.finfo(float).eps * 5.0
    # random entries, against LAPACK on the tridiagonal matrix itself
    g = np.random.default_rng(3)
    d, e = g.uniform(1, 5, n), g.uniform(-1, 1, n - 1)
    t2 = gen.tridiag_hss(n, 32, diag=d, off=e)
    T2 = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.array_equal(oh.dense_original(t2), T2)
    ev2 = np.linalg.eigvalsh(oh.dense_nodes(oh.divide(t2))[(0, 0)])
    assert np.abs(ev2 - np.linalg.eigvalsh(T2)).max() <= 1e-13 * np.abs(ev2).max()


def test_balanced_norm_bound_and_unbalanced_growth():
    from oracle import hss as oh
    t = gen.hss_original(n=2048, leaf=16, r=4, cfg=10)
    bmax = max(np.linalg.norm(t.B[l][q], 2) for l in t.B for q in range(len(t.B[l])))
    bal = oh.divide(t, balanced=True)
    unb = oh.divide(t, balanced=False)
    for l in range(t.depth):
        nb = max(np.linalg.norm(bal.B[l][q], 2) for q in range(1 << l))
        assert nb <= (1 << l) * bmax * (1 + 1e-12), l
    deep = t.depth - 1
    g_bal = max(np.linalg.norm(bal.B[deep][q], 2) for q in range(1 << deep))
    g_unb = max(np.linalg.norm(unb.B[deep][q], 2) for q in range(1 << deep))
    assert g_unb > 100 * g_bal
    # both are exact divisions of the same matrix (small tree)
    s = gen.hss_original(n=256, leaf=16, r=4, cfg=11)
    A = oh.dense_original(s)
    for bl in (True, False):
        Ad = oh.dense_nodes(oh.divide(s, balanced=bl))[(0, 0)]
        assert np.abs(A - Ad).max() <= 1e-10 * np.abs(A).max() * (1 if bl else 1e6)


def test_trace_and_frobenius_of_the_assembly():
    from oracle import hss as oh
    t = gen.hss_original(n=1024, leaf=32, r=4, cfg=12)
    A = oh.dense_original(t)
    assert np.abs(A - A.T).max() == 0.0
    fro = float(np.sum(t.leaf_D ** 2)) + 2.0 * sum(float(np.sum(t.B[l] ** 2)) for l in t.B)
    assert np.sum(A ** 2) == pytest.approx(fro, rel=1e-13)
    assert np.trace(A) == pytest.approx(sum(np.trace(x) for x in t.leaf_D), rel=1e-13, abs=1e-13)
    # the divided form has the same invariants of its spectrum
    ev = np.linalg.eigvalsh(oh.dense_nodes(oh.divide(t))[(0, 0)])
    assert np.sum(ev ** 2) == pytest.approx(fro, rel=1e-12)


def test_vanished_coupling_takes_unit_beta():
    """A coupling that vanishes has no norm to balance by: beta = 1, and the division is
    still exact (the left child's update column is zero)."""
    import copy
    from oracle import hss as oh
    t = copy.deepcopy(gen.hss_original(n=256, leaf=16, r=4, cfg=13))
    t.B[0][:] = 0.0
    d = oh.divide(t)
    assert d.beta[0][0] == 1.0 and np.all(d.B[0][0] == 0.0)
    A = oh.dense_original(t)
    Ad = oh.dense_nodes(d)[(0, 0)]
    assert np.abs(A - Ad).max() <= 1e-13 * np.abs(A).max()
