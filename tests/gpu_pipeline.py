"""Helpers for GPU tests: upload a gen.Batch, run the C-ABI pipeline, fetch results."""
from __future__ import annotations

import numpy as np
import torch

from paper_2108_04209_amd import native


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev())


_CTX = None


def context():
    global _CTX
    if _CTX is None:
        _CTX = native.Context()
    return _CTX


def run(batch, X=None, trans=(0,), opts=None, vectors=True):
    """Solve every problem of a gen.Batch on the GPU.  X: host (total, m) array or None."""
    ctx = context()
    b = native.Batch(ctx, batch.off)
    d, z, rho = to_dev(batch.d), to_dev(batch.z), to_dev(batch.rho)
    o = opts if opts is not None else native.default_opts()
    s = native.secular_solve(ctx, b, d, z, rho, opts=o)
    out = {k: v for k, v in s.items()}
    if vectors:
        zh, bn = native.loewner(ctx, b, d, z, rho, s["eta"], s["origin"], s["status"], opts=o)
        out["zhat"], out["b"] = zh, bn
        if X is not None:
            Xt = to_dev(np.asarray(X).T)  # (m, total) rows = right-hand sides
            for t in trans:
                Y = native.cauchy_apply(ctx, b, d, zh, bn, s["eta"], s["origin"], s["status"],
                                        Xt, trans=t, opts=o)
                out[f"Y{t}"] = Y
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    for t in trans:
        if f"Y{t}" in res:
            res[f"Y{t}"] = res[f"Y{t}"].T  # back to (total, m)
    res["_batch"] = b
    return res


def _stage_inputs(batch, eta, origin):
    return (to_dev(batch.d), to_dev(batch.z), to_dev(batch.rho), to_dev(eta),
            to_dev(origin, torch.int32), torch.zeros(batch.nprob, dtype=torch.int32, device=dev()))


def loewner_from(batch, eta, origin, opts=None):
    """GPU Loewner/b fed with given (eta, origin) (e.g. the oracle's)."""
    ctx = context()
    b = native.Batch(ctx, batch.off)
    d, z, rho, e, o, st = _stage_inputs(batch, eta, origin)
    zh, bn = native.loewner(ctx, b, d, z, rho, e, o, st, opts=opts)
    torch.cuda.synchronize()
    return zh.cpu().numpy(), bn.cpu().numpy()


def apply_from(batch, zhat, bnorm, eta, origin, X, trans, opts=None):
    """GPU Cauchy apply fed with given (zhat, b, eta, origin); X host (total, m)."""
    ctx = context()
    b = native.Batch(ctx, batch.off)
    d, z, rho, e, o, st = _stage_inputs(batch, eta, origin)
    Xt = to_dev(np.asarray(X).T)
    Y = native.cauchy_apply(ctx, b, d, to_dev(zhat), to_dev(bnorm), e, o, st, Xt, trans=trans,
                            opts=opts)
    torch.cuda.synchronize()
    return Y.cpu().numpy().T


def backward_from(batch, eta, origin, g_lam=None, g_proj=None, u=None, opts=None):
    """GPU adjoint fed with given (eta, origin)."""
    ctx = context()
    b = native.Batch(ctx, batch.off)
    d, z, rho, e, o, st = _stage_inputs(batch, eta, origin)
    f = lambda a: None if a is None else to_dev(a)
    gd, gz, gr = native.secular_backward(ctx, b, d, z, rho, e, o, st, g_lam=f(g_lam),
                                         g_proj=f(g_proj), u=f(u), opts=opts)
    torch.cuda.synchronize()
    return gd.cpu().numpy(), gz.cpu().numpy(), gr.cpu().numpy()


def deflated_run(batch, tau, X=None, opts=None):
    """Deflate every problem of a gen.Batch on the GPU, solve the reduced problems, and
    (with X: host (total, m)) apply the full eigenvector matrix Q = G^T P (Qhat (+) I) and its
    transpose.  Eigenvalue j of problem p belongs to output position j."""
    ctx = context()
    b = native.Batch(ctx, batch.off)
    d, z, rho = to_dev(batch.d), to_dev(batch.z), to_dev(batch.rho)
    df = native.deflate(ctx, b, d, z, rho, tau)
    kept = df["kept"].cpu().numpy()
    # the reduced batch: problems of kept[p] poles (one dummy pole where nothing is kept)
    roff = np.concatenate([[0], np.cumsum(np.maximum(kept, 1))]).astype(np.int64)
    rb = native.Batch(ctx, roff)
    dr = native.batch_copy_rows(ctx, b, rb, df["d"], rows=df["kept"], fill=0.0).view(-1)
    zr = native.batch_copy_rows(ctx, b, rb, df["z"], rows=df["kept"], fill=1.0).view(-1)
    o = opts if opts is not None else native.default_opts()
    s = native.secular_solve(ctx, rb, dr, zr, rho, opts=o)
    lam = df["d"].clone()
    native.batch_copy_rows(ctx, rb, b, s["lam"], rows=df["kept"], dst=lam.view(1, -1))
    out = {"lam": lam, "kept": df["kept"], "dstatus": df["status"], "rstatus": s["status"],
           "dfl": df}
    if X is not None:
        zh, bn = native.loewner(ctx, rb, dr, zr, rho, s["eta"], s["origin"], s["status"], opts=o)
        Xt = to_dev(np.asarray(X).T)
        # Q X: Qhat on the leading rows, the deflated rows as they are, then G^T P
        Xr = native.batch_copy_rows(ctx, b, rb, Xt, rows=df["kept"], fill=0.0)
        Yr = native.cauchy_apply(ctx, rb, dr, zh, bn, s["eta"], s["origin"], s["status"], Xr,
                                 trans=0, opts=o)
        U = Xt.clone()
        native.batch_copy_rows(ctx, rb, b, Yr, rows=df["kept"], dst=U)
        out["Y0"] = native.deflate_expand(ctx, b, df, U, trans=0)
        # Q^T X: P^T G, then Qhat^T on the leading rows
        V = native.deflate_expand(ctx, b, df, Xt, trans=1)
        Vr = native.batch_copy_rows(ctx, b, rb, V, rows=df["kept"], fill=0.0)
        Wr = native.cauchy_apply(ctx, rb, dr, zh, bn, s["eta"], s["origin"], s["status"], Vr,
                                 trans=1, opts=o)
        native.batch_copy_rows(ctx, rb, b, Wr, rows=df["kept"], dst=V)
        out["Y1"] = V
    torch.cuda.synchronize()
    res = {}
    for k, v in out.items():
        if k == "dfl":
            res[k] = {kk: vv.cpu().numpy() for kk, vv in v.items()}
        else:
            res[k] = v.cpu().numpy()
    for t in (0, 1):
        if f"Y{t}" in res:
            res[f"Y{t}"] = res[f"Y{t}"].T
    return res
