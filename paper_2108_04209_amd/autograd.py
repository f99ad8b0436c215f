"""torch.autograd binding of the batched rank-one eigensolver.

`secular_eig(batch, d, z, rho, u=None)` returns the eigenvalues lam of every problem
diag(d_p) + rho_p z_p z_p^T and, when u is given, the projections p_k = q_k^T u of the
eigenvectors q_k = b_k (z_i / (d_i - lambda_k))_i on u.  The backward pass is the library's
hand-written adjoint (superdc_secular_backward): implicit differentiation of the secular
equation f(lambda_k) = 0 through Cauchy-like sums, never a dense eigendecomposition.
All work runs in libsuperdc.so; this module only wires tensors.

Nothing here waits for the device: like the C ABI, the binding leaves data-dependent
errors on the device.  A problem with invalid input (d not strictly increasing, z_i = 0,
rho <= 0, non-finite values) gets NaN eigenvalues, projections and gradients; pass an
int32 tensor `status` of shape (nprob,) to receive the per-problem status bits
(native.ST_*) by a device-side copy and check them whenever the caller synchronises.
"""
from __future__ import annotations

import torch

from . import native


class _SecularEig(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d, z, rho, u, batch, opts, status):
        lib_ctx = batch.ctx
        s = native.secular_solve(lib_ctx, batch, d, z, rho, opts=opts)
        if status is not None:
            status.copy_(s["status"])  # enqueued on the stream: no host synchronisation
        outs = [s["lam"]]
        if u is not None:
            zh, bn = native.loewner(lib_ctx, batch, d, z, rho, s["eta"], s["origin"], s["status"],
                                    opts=opts)
            p = native.cauchy_apply(lib_ctx, batch, d, zh, bn, s["eta"], s["origin"], s["status"],
                                    u.contiguous().view(1, -1), trans=1, opts=opts).view(-1)
            outs.append(p)
        ctx.save_for_backward(d, z, rho, s["eta"], s["origin"], s["status"],
                              u if u is not None else torch.empty(0, device=d.device))
        ctx.batch, ctx.opts, ctx.has_u = batch, opts, u is not None
        return tuple(outs) if len(outs) > 1 else outs[0]

    @staticmethod
    def backward(ctx, *grads):
        d, z, rho, eta, origin, status, u = ctx.saved_tensors
        g_lam = grads[0]
        g_proj = grads[1] if ctx.has_u else None
        g_lam = None if g_lam is None else g_lam.contiguous()
        if g_proj is not None:
            g_proj = g_proj.contiguous()
        gd, gz, gr = native.secular_backward(ctx.batch.ctx, ctx.batch, d, z, rho, eta, origin,
                                             status, g_lam=g_lam, g_proj=g_proj,
                                             u=u if g_proj is not None else None, opts=ctx.opts)
        gu = None
        if ctx.has_u and ctx.needs_input_grad[3]:
            raise NotImplementedError("gradient with respect to u is not provided")
        return gd, gz, gr, gu, None, None, None


def secular_eig(batch, d, z, rho, u=None, opts=None, status=None):
    """Differentiable eigenvalues (and projections on u) of a batch of rank-one problems.
    batch: native.Batch; d, z: (total,) float64 CUDA tensors; rho: (nprob,).
    status: optional int32 CUDA tensor (nprob,) that receives the status bits."""
    o = opts if opts is not None else native.default_opts()
    if status is not None and (status.dtype != torch.int32 or status.numel() != batch.nprob
                               or not status.is_cuda):
        raise ValueError("status must be an int32 CUDA tensor with one entry per problem")
    return _SecularEig.apply(d.contiguous(), z.contiguous(), rho.contiguous(),
                             None if u is None else u.contiguous(), batch, o, status)
