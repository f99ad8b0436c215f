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
