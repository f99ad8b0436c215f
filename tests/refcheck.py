"""Independent reference routines used only by tests to pin the oracle.

Nothing here shares code with the oracle or the HIP path:
  - cyclic (round-robin ordered) Jacobi eigendecomposition of a dense symmetric matrix,
  - brute-force bisection of the secular equation in 50-digit arithmetic (mpmath),
  - dense assembly of diag(d) + rho z z^T.
"""
from __future__ import annotations

import mpmath
import numpy as np


def dense(d, z, rho):
    return np.diag(d) + rho * np.outer(z, z)


def jacobi_eigh(A, tol=1e-17, max_sweeps=60):
    """Cyclic Jacobi with round-robin pair ordering; every round rotates n/2 disjoint pairs.

    Returns ascending eigenvalues and the matching orthonormal eigenvectors (columns).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    if n == 1:
        return A.diagonal().copy(), V
    m = n + (n % 2)
    players = list(range(m))
    fro = np.linalg.norm(A)
    for _ in range(max_sweeps):
        off = np.linalg.norm(A - np.diag(np.diag(A)))
        if off <= tol * fro:
            break
        for _r in range(m - 1):
            pairs = [(players[i], players[m - 1 - i]) for i in range(m // 2)]
            pairs = [(min(a, b), max(a, b)) for a, b in pairs if a < n and b < n]
            P = np.array([a for a, _ in pairs])
            Q = np.array([b for _, b in pairs])
            apq = A[P, Q]
            app = A[P, P]
            aqq = A[Q, Q]
            nz = apq != 0.0
            with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
                theta = np.where(nz, (aqq - app) / (2.0 * np.where(nz, apq, 1.0)), 0.0)
                t = np.where(nz, np.sign(theta) / (np.abs(theta) + np.sqrt(theta * theta + 1.0)), 0.0)
                # |theta| so large that theta^2 overflows: t = 1/(2 theta)
                t = np.where(nz & ~np.isfinite(theta * theta), 0.5 / theta, t)
            t = np.where(nz & (theta == 0.0), 1.0, t)
            c = 1.0 / np.sqrt(t * t + 1.0)
            s = t * c
            # rows then columns: A <- J^T A J with J[p,p]=c, J[p,q]=s, J[q,p]=-s, J[q,q]=c
            Ap, Aq = A[P, :].copy(), A[Q, :].copy()
            A[P, :] = c[:, None] * Ap - s[:, None] * Aq
            A[Q, :] = s[:, None] * Ap + c[:, None] * Aq
            Ap, Aq = A[:, P].copy(), A[:, Q].copy()
            A[:, P] = Ap * c[None, :] - Aq * s[None, :]
            A[:, Q] = Ap * s[None, :] + Aq * c[None, :]
            Vp, Vq = V[:, P].copy(), V[:, Q].copy()
            V[:, P] = Vp * c[None, :] - Vq * s[None, :]
            V[:, Q] = Vp * s[None, :] + Vq * c[None, :]
            # rotate the tournament (player 0 fixed)
            players = [players[0]] + [players[-1]] + players[1:-1]
    w = np.diag(A).copy()
    order = np.argsort(w)
    return w[order], V[:, order]


def mp_roots(d, z, rho, dps=50, steps=220):
    """All n roots of f(x) = 1 + sum rho z_j^2 / (d_j - x) by plain bisection in mpmath,
    using the interval (d_k, d_{k+1}) and, for the last root, (d_n, d_n + rho ||z||^2]."""
    with mpmath.workdps(dps):
        D = [mpmath.mpf(float(x)) for x in d]
        W = [mpmath.mpf(float(rho)) * mpmath.mpf(float(x)) ** 2 for x in z]
        n = len(D)

        def f(x):
            return 1 + mpmath.fsum(W[j] / (D[j] - x) for j in range(n))

        out = []
        for k in range(n):
            lo = D[k]
            hi = D[k + 1] if k + 1 < n else D[k] + mpmath.fsum(W)
            for _ in range(steps):
                mid = (lo + hi) / 2
                if f(mid) < 0:
                    lo = mid
                else:
                    hi = mid
            out.append((lo + hi) / 2)
        return out
