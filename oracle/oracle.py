"""ctypes front end of the plain C oracle (superdc_oracle.c).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU-baseline leg
use it.  Every function takes and returns numpy float64 / int arrays on the host.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "superdc_oracle.c")
LIB = os.path.join(HERE, "libsuperdc_oracle.so")

ST_UNSORTED, ST_ZERO, ST_NONFINITE, ST_RHO, ST_NOCONV = 1, 2, 4, 8, 16

_lib = None

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_P = C.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        i64, dbl = C.c_int64, C.c_double
        lib.oracle_validate.argtypes = [i64, _P, _P, dbl]
        lib.oracle_validate.restype = C.c_int
        lib.oracle_secular.argtypes = [i64, _P, _P, dbl, _P, i64, _P, _P, _P, _P]
        lib.oracle_secular.restype = C.c_int
        lib.oracle_loewner.argtypes = [i64, _P, _P, dbl, _P, _P, _P, i64, _P]
        lib.oracle_loewner.restype = None
        lib.oracle_bnorm.argtypes = [i64, _P, _P, _P, _P, _P, i64, _P]
        lib.oracle_bnorm.restype = None
        lib.oracle_cauchy_apply.argtypes = [i64, _P, _P, _P, _P, _P, C.c_int, i64, _P, i64,
                                            _P, i64, _P, i64]
        lib.oracle_cauchy_apply.restype = None
        lib.oracle_backward.argtypes = [i64, _P, _P, dbl, _P, _P, _P, _P, _P, _P, _P, _P]
        lib.oracle_backward.restype = None
        lib.oracle_deflate.argtypes = [i64, _P, _P, dbl, dbl, _P, _P, _P, _P, _P, _P, _P]
        lib.oracle_deflate.restype = i64
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def validate(d, z, rho) -> int:
    d, z = _f64(d), _f64(z)
    return int(load().oracle_validate(d.size, _ptr(d), _ptr(z), float(rho)))


def secular(d, z, rho, roots=None):
    """All (or the listed) roots.  Returns (lam, eta, origin, iters, status)."""
    d, z = _f64(d), _f64(z)
    n = d.size
    if roots is None:
        cnt, rp = n, None
    else:
        rp = np.ascontiguousarray(roots, dtype=np.int64)
        cnt = rp.size
    lam = np.empty(cnt)
    eta = np.empty(cnt)
    org = np.empty(cnt, dtype=np.int32)
    its = np.empty(cnt, dtype=np.int32)
    st = load().oracle_secular(n, _ptr(d), _ptr(z), float(rho), _ptr(rp), cnt, _ptr(lam),
                               _ptr(eta), _ptr(org), _ptr(its))
    return lam, eta, org, its, int(st)


def loewner(d, z, rho, eta, origin, poles=None):
    d, z, eta = _f64(d), _f64(z), _f64(eta)
    origin = np.ascontiguousarray(origin, dtype=np.int32)
    n = d.size
    if poles is None:
        cnt, pp = n, None
    else:
        pp = np.ascontiguousarray(poles, dtype=np.int64)
        cnt = pp.size
    out = np.empty(cnt)
    load().oracle_loewner(n, _ptr(d), _ptr(z), float(rho), _ptr(eta), _ptr(origin), _ptr(pp),
                          cnt, _ptr(out))
    return out


def bnorm(d, zhat, eta, origin, roots=None):
    d, zhat, eta = _f64(d), _f64(zhat), _f64(eta)
    origin = np.ascontiguousarray(origin, dtype=np.int32)
    n = d.size
    if roots is None:
        cnt, rp = n, None
    else:
        rp = np.ascontiguousarray(roots, dtype=np.int64)
        cnt = rp.size
    out = np.empty(cnt)
    load().oracle_bnorm(n, _ptr(d), _ptr(zhat), _ptr(eta), _ptr(origin), _ptr(rp), cnt,
                        _ptr(out))
    return out


def cauchy_apply(d, zhat, b, eta, origin, X, trans=0, rows=None):
    """Y = Qhat X (trans 0) or Qhat^T X (trans 1); X is n x m (any layout)."""
    d, zhat, b, eta = _f64(d), _f64(zhat), _f64(b), _f64(eta)
    origin = np.ascontiguousarray(origin, dtype=np.int32)
    X = np.asfortranarray(np.asarray(X, dtype=np.float64).reshape(d.size, -1))
    n, m = X.shape
    if rows is None:
        cnt, rp = n, None
    else:
        rp = np.ascontiguousarray(rows, dtype=np.int64)
        cnt = rp.size
    Y = np.zeros((cnt, m), order="F")
    load().oracle_cauchy_apply(n, _ptr(d), _ptr(zhat), _ptr(b), _ptr(eta), _ptr(origin),
                               int(trans), m, X.ctypes.data_as(C.c_void_p), n, _ptr(rp), cnt,
                               Y.ctypes.data_as(C.c_void_p), cnt)
    return Y


def backward(d, z, rho, eta, origin, g_lam=None, g_proj=None, u=None):
    d, z, eta = _f64(d), _f64(z), _f64(eta)
    origin = np.ascontiguousarray(origin, dtype=np.int32)
    n = d.size
    gl = None if g_lam is None else _f64(g_lam)
    gp = None if g_proj is None else _f64(g_proj)
    uu = None if u is None else _f64(u)
    if (gp is None) != (uu is None):
        raise ValueError("g_proj and u go together")
    g_d = np.empty(n)
    g_z = np.empty(n)
    g_r = np.empty(1)
    load().oracle_backward(n, _ptr(d), _ptr(z), float(rho), _ptr(eta), _ptr(origin), _ptr(gl),
                           _ptr(gp), _ptr(uu), _ptr(g_d), _ptr(g_z), _ptr(g_r))
    return g_d, g_z, float(g_r[0])


def solve_batch(batch, with_vectors=True):
    """Run the full rank-one pipeline problem by problem on a gen.Batch.
    Returns dict of concatenated lam, eta, origin, zhat, b, status[P]."""
    tot = batch.total_n
    out = {k: np.empty(tot) for k in ("lam", "eta", "zhat", "b")}
    out["origin"] = np.empty(tot, dtype=np.int32)   # local (per-problem) origin index
    out["iters"] = np.empty(tot, dtype=np.int32)
    out["status"] = np.zeros(batch.nprob, dtype=np.int32)
    for p in range(batch.nprob):
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        lam, eta, org, its, st = secular(pr.d, pr.z, pr.rho)
        out["status"][p] = st
        if st & ~ST_NOCONV:
            continue
        out["lam"][a:e], out["eta"][a:e], out["origin"][a:e], out["iters"][a:e] = lam, eta, org, its
        if with_vectors:
            zh = loewner(pr.d, pr.z, pr.rho, eta, org)
            out["zhat"][a:e] = zh
            out["b"][a:e] = bnorm(pr.d, zh, eta, org)
    return out


def deflate(d, z, rho, tau):
    """Deflation of diag(d) + rho z z^T with tolerance tau (Remark 1).  Returns a dict with
    kept, d, z (reduced problem first, then the deflated eigenvalues with z = 0), perm (pole
    index of each output position), rright, rleft, c, s (the rotations, by pole index)."""
    d, z = _f64(d), _f64(z)
    n = d.size
    out = {"d": np.empty(n), "z": np.empty(n), "perm": np.empty(n, dtype=np.int32),
           "rright": np.empty(n, dtype=np.int32), "rleft": np.empty(n, dtype=np.int32),
           "c": np.empty(n), "s": np.empty(n)}
    out["kept"] = int(load().oracle_deflate(n, _ptr(d), _ptr(z), float(rho), float(tau),
                                            _ptr(out["d"]), _ptr(out["z"]), _ptr(out["perm"]),
                                            _ptr(out["rright"]), _ptr(out["rleft"]),
                                            _ptr(out["c"]), _ptr(out["s"])))
    return out


def deflate_expand(df, U, trans=0):
    """The orthogonal factor of the deflation applied to a block.

    With G the product of the rotations (the first made acting first) and P the
    placement of output position j at pole perm[j], the full eigenvector matrix is
    Q = G^T P (Qhat (+) I).  trans 0: returns G^T P U for U whose rows are output positions;
    trans 1: returns P^T G X for X whose rows are pole indices."""
    U = np.array(np.asarray(U, dtype=np.float64).reshape(df["d"].size, -1), copy=True)
    n = U.shape[0]
    rot = [a for a in range(n) if df["rright"][a] >= 0]  # creation order: increasing a
    if trans == 0:
        Y = np.empty_like(U)
        Y[df["perm"]] = U
        for a in reversed(rot):  # G^T = G_1^T ... G_R^T: the last rotation first
            b, c, s = df["rright"][a], df["c"][a], df["s"][a]
            ya, yb = Y[a].copy(), Y[b].copy()
            Y[a] = c * ya + s * yb
            Y[b] = -s * ya + c * yb
        return Y
    Y = U
    for a in rot:  # G = G_R ... G_1: the first rotation first
        b, c, s = df["rright"][a], df["c"][a], df["s"][a]
        ya, yb = Y[a].copy(), Y[b].copy()
        Y[a] = c * ya - s * yb
        Y[b] = s * ya + c * yb
    return Y[df["perm"]]


def deflated_eig(d, z, rho, tau, vectors=True):
    """Eigenvalues (and, for small n, the dense eigenvector matrix) of diag(d) + rho z z^T
    through deflation: the reduced problem by the secular oracle, the deflated eigenvalues
    as they come.  Eigenvalue j belongs to output position j of deflate()."""
    df = deflate(d, z, rho, tau)
    k = df["kept"]
    n = df["d"].size
    lam = df["d"].copy()
    res = {"deflate": df, "status": 0}
    if k > 0:
        dr, zr = df["d"][:k], df["z"][:k]
        lr, eta, org, its, st = secular(dr, zr, rho)
        res["status"] = st
        lam[:k] = lr
        res["eta"], res["origin"] = eta, org
        if vectors:
            zh = loewner(dr, zr, rho, eta, org)
            b = bnorm(dr, zh, eta, org)
            res["zhat"], res["b"] = zh, b
            Qh = cauchy_apply(dr, zh, b, eta, org, np.eye(k), 0)
            U = np.zeros((n, n))
            U[:k, :k] = Qh
            U[k:, k:] = np.eye(n - k)
            res["Q"] = deflate_expand(df, U, 0)
    elif vectors:
        res["Q"] = deflate_expand(df, np.eye(n), 0)
    res["lam"] = lam
    return res
