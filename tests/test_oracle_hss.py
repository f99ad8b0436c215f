"""Pins of the HSS-conquer oracle (oracle/hss.py) against the definition of an HSS matrix.

- The off-diagonal block of every A_p equals U_c1 B_p U_c2^T (eq. du), whatever the
  balancing scalar beta_p: this pins the update Z_p = [U_c1 B_p/sqrt(beta_p); sqrt(beta_p) U_c2].
- The structured O(n r log n) product equals the dense assembled matrix's product.
- trace(A_root) from the generators equals the trace of the assembled matrix, and the sum
  of its LAPACK eigenvalues.
- Orthonormal bases make the nested U_p orthonormal.
"""
import numpy as np
import pytest

from oracle import hss as ohss
from paper_2108_04209_amd import gen


@pytest.fixture(scope="module", params=[(16, 3, 4), (32, 4, 8)])
def tree(request):
    leaf, depth, r = request.param
    return gen.hss_tree(n=leaf << depth, leaf=leaf, r=r, cfg=300 + leaf)


def test_offdiagonal_blocks(tree):
    A = ohss.dense_nodes(tree)
    U = ohss.bases(tree)
    for lvl in range(tree.depth):
        for q in range(1 << lvl):
            Ap = A[(lvl, q)]
            h = Ap.shape[0] // 2
            Ua, Ub = U[(lvl + 1, 2 * q)], U[(lvl + 1, 2 * q + 1)]
            np.testing.assert_allclose(Ap[:h, h:], Ua @ tree.B[lvl][q] @ Ub.T, atol=1e-13)
            np.testing.assert_array_equal(Ap, Ap.T)


def test_structured_matvec(tree):
    A = ohss.dense_nodes(tree)[(0, 0)]
    X = np.random.default_rng(0).standard_normal((tree.n, 3))
    np.testing.assert_allclose(ohss.matvec(tree, X), A @ X, atol=1e-12 * np.abs(A).sum(1).max())


def test_trace_and_eigenvalues(tree):
    A = ohss.dense_nodes(tree)[(0, 0)]
    t = ohss.trace(tree)
    assert t == pytest.approx(np.trace(A), rel=1e-13)
    lev = ohss.level_eigenvalues(tree)
    assert lev[0].sum() == pytest.approx(t, rel=1e-12)
    # leaf row: eigenvalues of the leaf blocks themselves
    for q in range(1 << tree.depth):
        np.testing.assert_allclose(lev[tree.depth, q * tree.leaf:(q + 1) * tree.leaf],
                                   np.linalg.eigvalsh(tree.leaf_D[q]), atol=1e-13)


def test_nested_bases_orthonormal(tree):
    U = ohss.bases(tree)
    for (lvl, q), u in U.items():
        np.testing.assert_allclose(u.T @ u, np.eye(tree.r), atol=1e-13)
