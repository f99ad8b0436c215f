"""Oracle for the HSS dividing and conquering passes (test infrastructure only).

The conquering stage (Alg. 3) computes the eigendecomposition of the symmetric HSS
matrix defined by its generators (Sec. 2.1, eq. hss).  With the leaf blocks taken as
already divided and the balanced update of Sec. 3 (Alg. 1, bottom-up part), the matrix
of a node p with children c1, c2 is

    A_p = blkdiag(A_c1, A_c2) + Z_p Z_p^T,   Z_p = [U_c1 B_p / sqrt(beta_p) ; sqrt(beta_p) U_c2],
    A_leaf = D_leaf,   U_p = [U_c1 R_c1 ; U_c2 R_c2]   (eq. du),

and the conquer returns the eigenvalues of A_root (and of every A_p on the way).  This
module writes that definition out: dense assembly plus LAPACK eigenvalues (a library
routine) for small trees, and a structured O(n r log n) matrix-vector product for
residual checks at full size.  It shares nothing with the HIP path.
"""
from __future__ import annotations

import numpy as np


def _children(lvl, q):
    return (lvl + 1, 2 * q), (lvl + 1, 2 * q + 1)


def node_size(tree, lvl):
    return tree.leaf << (tree.depth - lvl)


def bases(tree):
    """U of every node: leaves from the generators, parents by the nested relation."""
    U = {(tree.depth, q): tree.leaf_U[q] for q in range(1 << tree.depth)}
    for lvl in range(tree.depth - 1, 0, -1):
        for q in range(1 << lvl):
            (l1, a), (_, b) = _children(lvl, q)
            U[(lvl, q)] = np.vstack([U[(l1, a)] @ tree.R[l1][a], U[(l1, b)] @ tree.R[l1][b]])
    return U


def zmat(tree, U, lvl, q):
    (l1, a), (_, b) = _children(lvl, q)
    s = np.sqrt(tree.beta[lvl][q])
    return np.vstack([U[(l1, a)] @ tree.B[lvl][q] / s, s * U[(l1, b)]])


def dense_nodes(tree):
    """Dense A_p for every node (small trees only)."""
    U = bases(tree)
    A = {(tree.depth, q): tree.leaf_D[q].copy() for q in range(1 << tree.depth)}
    for lvl in range(tree.depth - 1, -1, -1):
        for q in range(1 << lvl):
            (l1, a), (_, b) = _children(lvl, q)
            Z = zmat(tree, U, lvl, q)
            na = A[(l1, a)].shape[0]
            M = np.zeros((2 * na, 2 * na))
            M[:na, :na] = A[(l1, a)]
            M[na:, na:] = A[(l1, b)]
            A[(lvl, q)] = M + Z @ Z.T
    return A


def level_eigenvalues(tree, dense=None):
    """Eigenvalues of every node, ascending per node, concatenated per level:
    returns array (depth+1, n); row l holds the nodes of level l left to right.
    dense: the output of dense_nodes(tree), if the caller has it already."""
    A = dense_nodes(tree) if dense is None else dense
    out = np.empty((tree.depth + 1, tree.n))
    for lvl in range(tree.depth + 1):
        sz = node_size(tree, lvl)
        for q in range(1 << lvl):
            out[lvl, q * sz:(q + 1) * sz] = np.linalg.eigvalsh(A[(lvl, q)])
    return out


def trace(tree):
    """trace(A_root) from the generators: sum of leaf traces plus sum_p ||Z_p||_F^2."""
    U = bases(tree)
    t = sum(np.trace(tree.leaf_D[q]) for q in range(1 << tree.depth))
    for lvl in range(tree.depth):
        for q in range(1 << lvl):
            t += np.sum(zmat(tree, U, lvl, q) ** 2)
    return float(t)


def matvec(tree, X):
    """A_root @ X in O(n r log n) by the tree recursion (X: n x m)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    D = tree.depth
    leaf = tree.leaf
    # upward pass: g[(l,q)] = U_(l,q)^T X_(l,q)
    g = {}
    for q in range(1 << D):
        g[(D, q)] = tree.leaf_U[q].T @ X[q * leaf:(q + 1) * leaf]
    for lvl in range(D - 1, 0, -1):
        for q in range(1 << lvl):
            (l1, a), (_, b) = _children(lvl, q)
            g[(lvl, q)] = tree.R[l1][a].T @ g[(l1, a)] + tree.R[l1][b].T @ g[(l1, b)]
    # coefficients f[(l,q)] such that the node's rows receive U_(l,q) f
    f = {}
    for lvl in range(0, D):
        for q in range(1 << lvl):
            (l1, a), (_, b) = _children(lvl, q)
            s = np.sqrt(tree.beta[lvl][q])
            Bs = tree.B[lvl][q] / s
            v = Bs.T @ g[(l1, a)] + s * g[(l1, b)]          # Z_p^T X_p
            fa, fb = Bs @ v, s * v                           # Z_p v = [U_a fa ; U_b fb]
            f[(l1, a)] = f.get((l1, a), 0) + fa
            f[(l1, b)] = f.get((l1, b), 0) + fb
    # downward pass: push coefficients to the leaves through the transfer matrices
    for lvl in range(1, D):
        for q in range(1 << lvl):
            if (lvl, q) not in f:
                continue
            (l1, a), (_, b) = _children(lvl, q)
            f[(l1, a)] = f.get((l1, a), 0) + tree.R[l1][a] @ f[(lvl, q)]
            f[(l1, b)] = f.get((l1, b), 0) + tree.R[l1][b] @ f[(lvl, q)]
    Y = np.empty_like(X)
    for q in range(1 << D):
        rows = slice(q * leaf, (q + 1) * leaf)
        Y[rows] = tree.leaf_D[q] @ X[rows] + tree.leaf_U[q] @ f[(D, q)]
    return Y


# ------------------------------------------------------------------------ dividing stage
def dense_original(tree):
    """The HSS matrix of undivided generators, written out (eq. hss): D_p = [[D_c1,
    U_c1 B_p U_c2^T], [U_c2 B_p^T U_c1^T, D_c2]] with the nested bases."""
    U = bases(tree)
    A = {(tree.depth, q): tree.leaf_D[q].copy() for q in range(1 << tree.depth)}
    for lvl in range(tree.depth - 1, -1, -1):
        for q in range(1 << lvl):
            (l1, a), (_, b) = _children(lvl, q)
            na = A[(l1, a)].shape[0]
            M = np.zeros((2 * na, 2 * na))
            M[:na, :na] = A[(l1, a)]
            M[na:, na:] = A[(l1, b)]
            C = U[(l1, a)] @ tree.B[lvl][q] @ U[(l1, b)].T
            M[:na, na:] = C
            M[na:, :na] = C.T
            A[(lvl, q)] = M
    return A[(0, 0)]


def divide(tree, balanced=True):
    """The balanced dividing stage (Alg. 1, top-down part) for square couplings.

    Top down, every node p carries the pending update H_p of Lemma genupd (zero at the
    root): its children's coupling becomes B_p - R_c1 H_p R_c2^T (eq. genupd), beta_p is
    that coupling's 2-norm, and the children inherit R_c H_p R_c^T plus p's own division
    (eq. divnew1): (1/beta_p) B B^T for the left child, beta_p I for the right.  A leaf ends
    as D - U H U^T.  Returns a tree of the same shape with the divided leaf blocks, the
    updated couplings and their norms, i.e. the input of the conquering pass.
    balanced=False gives the earlier dividing (eq. divide: B B^T to the left child, I to the
    right, beta = 1), whose generators can grow exponentially down the tree."""
    import copy
    D, r = tree.depth, tree.r
    out = copy.deepcopy(tree)
    H = {(0, 0): np.zeros((r, r))}
    for lvl in range(D):
        for q in range(1 << lvl):
            (l1, a), (_, b) = _children(lvl, q)
            R1, R2 = tree.R[l1][a], tree.R[l1][b]
            Hp = H[(lvl, q)]
            Bt = tree.B[lvl][q] - R1 @ Hp @ R2.T
            beta = np.linalg.norm(Bt, 2) if balanced else 1.0
            if not beta > 0.0:
                beta = 1.0  # a vanished coupling: nothing to balance, Z_p = [0; U_c2]
            out.B[lvl][q] = Bt
            out.beta[lvl][q] = beta
            H[(l1, a)] = R1 @ Hp @ R1.T + (Bt @ Bt.T) / beta
            H[(l1, b)] = R2 @ Hp @ R2.T + beta * np.eye(r)
    for q in range(1 << D):
        U = tree.leaf_U[q]
        out.leaf_D[q] = tree.leaf_D[q] - U @ H[(D, q)] @ U.T
    return out
