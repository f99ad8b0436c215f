"""Thin ctypes binding of libsuperdc.so (include/superdc.h).

Argument marshalling only: every step runs in the HIP library.  Device memory and
streams come from PyTorch.  There is no CPU fallback: if the library is missing or no
gfx950 device is visible the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsuperdc.so")

ST_UNSORTED, ST_ZERO, ST_NONFINITE, ST_RHO, ST_NOCONV = 1, 2, 4, 8, 16
# iteration records: count in the low 16 bits, how the iteration ended above them
ITER_COUNT_MASK, ITER_UNMET, ITER_CAP, ITER_SKIPPED = 0xFFFF, 1 << 16, 1 << 17, 1 << 18
ERRORS = {0: "success", -1: "invalid argument", -2: "device allocation failed",
          -3: "HIP runtime error", -4: "no gfx950 device"}

class SuperdcError(RuntimeError):
    pass


class Opts(C.Structure):
    _fields_ = [("stop_c", C.c_double), ("max_iter", C.c_int32), ("method", C.c_int32),
                ("fmm_order", C.c_int32), ("fmm_leaf", C.c_int32), ("persistent", C.c_int32),
                ("apply_kernel", C.c_int32), ("fmm_crossover", C.c_int32),
                ("unshifted", C.c_int32), ("interp", C.c_int32),
                ("hss_tau", C.c_double)]


_lib = None
_P = C.c_void_p


def load_library(path: str = LIB_PATH):
    """Load libsuperdc.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise SuperdcError(f"{path} is missing: build it with python -m paper_2108_04209_amd.build")
    lib = C.CDLL(path)
    i32, i64 = C.c_int32, C.c_int64
    lib.superdc_opts_default.argtypes = [C.POINTER(Opts)]
    lib.superdc_opts_default.restype = None
    lib.superdc_create.argtypes = [C.POINTER(_P)]
    lib.superdc_create.restype = C.c_int
    lib.superdc_destroy.argtypes = [_P]
    lib.superdc_destroy.restype = None
    lib.superdc_strerror.argtypes = [C.c_int]
    lib.superdc_strerror.restype = C.c_char_p
    lib.superdc_last_hip_error.argtypes = []
    lib.superdc_last_hip_error.restype = C.c_int
    lib.superdc_batch_create.argtypes = [_P, i32, _P, C.POINTER(_P)]
    lib.superdc_batch_create.restype = C.c_int
    lib.superdc_batch_destroy.argtypes = [_P]
    lib.superdc_batch_destroy.restype = None
    lib.superdc_batch_total.argtypes = [_P]
    lib.superdc_batch_total.restype = i64
    lib.superdc_secular_solve.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                          C.POINTER(Opts), _P]
    lib.superdc_secular_solve.restype = C.c_int
    lib.superdc_secular_solve_noalloc.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                                  C.POINTER(Opts), _P]
    lib.superdc_secular_solve_noalloc.restype = C.c_int
    lib.superdc_loewner.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.POINTER(Opts), _P]
    lib.superdc_loewner.restype = C.c_int
    lib.superdc_cauchy_apply.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, C.c_int, i32, _P, i64,
                                         _P, i64, C.POINTER(Opts), _P]
    lib.superdc_cauchy_apply.restype = C.c_int
    lib.superdc_secular_backward.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                             _P, C.POINTER(Opts), _P]
    lib.superdc_secular_backward.restype = C.c_int
    lib.superdc_autotune.argtypes = [_P, _P, _P, _P, _P, C.POINTER(Opts), _P]
    lib.superdc_autotune.restype = C.c_int
    lib.superdc_batch_shapes.argtypes = [_P, _P]
    lib.superdc_batch_shapes.restype = C.c_int
    lib.superdc_kernel_timing.argtypes = [C.c_int]
    lib.superdc_kernel_timing.restype = C.c_int
    lib.superdc_kernel_times.argtypes = [_P, _P, C.c_int32]
    lib.superdc_kernel_times.restype = C.c_int
    lib.superdc_kernel_work.argtypes = [_P, C.c_int32]
    lib.superdc_kernel_work.restype = C.c_int
    lib.superdc_kernel_name.argtypes = [C.c_int32]
    lib.superdc_kernel_name.restype = C.c_char_p
    lib.superdc_deflate.argtypes = [_P, _P, _P, _P, _P, C.c_double, _P, _P, _P, _P, _P, _P, _P,
                                    _P, _P, _P]
    lib.superdc_deflate.restype = C.c_int
    lib.superdc_deflate_expand.argtypes = [_P, _P, _P, _P, _P, _P, _P, C.c_int, i32, _P, i64,
                                           _P, i64, _P]
    lib.superdc_deflate_expand.restype = C.c_int
    lib.superdc_batch_copy_rows.argtypes = [_P, _P, _P, _P, i32, _P, i64, _P, i64, _P, _P]
    lib.superdc_batch_copy_rows.restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        extra = ""
        if rc in (-2, -3):
            extra = f" (hipError {load_library().superdc_last_hip_error()})"
        raise SuperdcError(f"{what}: {ERRORS.get(rc, rc)}{extra}")


def default_opts(**kw) -> Opts:
    o = Opts()
    load_library().superdc_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """superdc_ctx on the current device."""

    def __init__(self):
        lib = load_library()
        h = _P()
        _check(lib.superdc_create(C.byref(h)), "superdc_create")
        self.handle = h

    def close(self):
        if self.handle:
            load_library().superdc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """superdc_batch: host offsets of back-to-back problems."""

    def __init__(self, ctx: Context, off):
        self.ctx = ctx
        self.off = np.ascontiguousarray(off, dtype=np.int64)
        self.nprob = int(self.off.size - 1)
        self.total = int(self.off[-1])
        h = _P()
        _check(load_library().superdc_batch_create(ctx.handle, self.nprob,
                                                   self.off.ctypes.data_as(_P), C.byref(h)),
               "superdc_batch_create")
        self.handle = h

    def close(self):
        if self.handle:
            load_library().superdc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f64(t, n, name):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
        raise SuperdcError(f"{name}: need a contiguous CUDA float64 tensor of >= {n} entries")
    return t


def secular_solve(ctx, batch, d, z, rho, opts=None, stream=None, out=None):
    """superdc_secular_solve.  Returns dict(lam, eta, origin, iters, status)."""
    import torch
    tot, P = batch.total, batch.nprob
    _f64(d, tot, "d"), _f64(z, tot, "z"), _f64(rho, P, "rho")
    dev = d.device
    if out is None:
        out = dict(lam=torch.empty(tot, dtype=torch.float64, device=dev),
                   eta=torch.empty(tot, dtype=torch.float64, device=dev),
                   origin=torch.empty(tot, dtype=torch.int32, device=dev),
                   iters=torch.empty(tot, dtype=torch.int32, device=dev),
                   status=torch.empty(P, dtype=torch.int32, device=dev))
    o = opts if opts is not None else default_opts()
    _check(load_library().superdc_secular_solve(
        ctx.handle, batch.handle, _ptr(d), _ptr(z), _ptr(rho), _ptr(out["lam"]),
        _ptr(out["eta"]), _ptr(out["origin"]), _ptr(out.get("iters")), _ptr(out["status"]),
        C.byref(o), _stream(stream)), "superdc_secular_solve")
    return out


def secular_solve_noalloc(ctx, batch, d, z, rho, opts=None, stream=None, out=None):
    """superdc_secular_solve_noalloc (direct sums, buffers in the library's fixed device
    array).  `out` as for secular_solve; pass it preallocated to allocate nothing here."""
    import torch
    tot, P = batch.total, batch.nprob
    _f64(d, tot, "d"), _f64(z, tot, "z"), _f64(rho, P, "rho")
    dev = d.device
    if out is None:
        out = dict(lam=torch.empty(tot, dtype=torch.float64, device=dev),
                   eta=torch.empty(tot, dtype=torch.float64, device=dev),
                   origin=torch.empty(tot, dtype=torch.int32, device=dev),
                   iters=torch.empty(tot, dtype=torch.int32, device=dev),
                   status=torch.empty(P, dtype=torch.int32, device=dev))
    o = opts if opts is not None else default_opts()
    _check(load_library().superdc_secular_solve_noalloc(
        ctx.handle, batch.handle, _ptr(d), _ptr(z), _ptr(rho), _ptr(out["lam"]),
        _ptr(out["eta"]), _ptr(out["origin"]), _ptr(out.get("iters")), _ptr(out["status"]),
        C.byref(o), _stream(stream)), "superdc_secular_solve_noalloc")
    return out


def loewner(ctx, batch, d, z, rho, eta, origin, status, opts=None, stream=None, out=None):
    """superdc_loewner.  Returns (zhat, bnorm)."""
    import torch
    tot = batch.total
    if out is None:
        out = (torch.empty(tot, dtype=torch.float64, device=d.device),
               torch.empty(tot, dtype=torch.float64, device=d.device))
    o = opts if opts is not None else default_opts()
    _check(load_library().superdc_loewner(
        ctx.handle, batch.handle, _ptr(d), _ptr(z), _ptr(rho), _ptr(eta), _ptr(origin),
        _ptr(status), _ptr(out[0]), _ptr(out[1]), C.byref(o), _stream(stream)), "superdc_loewner")
    return out


def cauchy_apply(ctx, batch, d, zhat, bnorm, eta, origin, status, X, trans=0, opts=None,
                 stream=None, Y=None):
    """superdc_cauchy_apply.  X: (m, ldx) row-major torch tensor = column-major total x m
    with leading dimension ldx (each row of the torch tensor is one right-hand side)."""
    import torch
    if X.dim() == 1:
        X = X.view(1, -1)
    m, ldx = X.shape
    if not X.is_contiguous() or X.dtype != torch.float64 or not X.is_cuda:
        raise SuperdcError("X must be a contiguous CUDA float64 (m, ldx) tensor")
    if Y is None:
        Y = torch.empty((m, batch.total), dtype=torch.float64, device=X.device)
    o = opts if opts is not None else default_opts()
    _check(load_library().superdc_cauchy_apply(
        ctx.handle, batch.handle, _ptr(d), _ptr(zhat), _ptr(bnorm), _ptr(eta), _ptr(origin),
        _ptr(status), int(trans), int(m), _ptr(X), int(ldx), _ptr(Y), int(Y.shape[1]),
        C.byref(o), _stream(stream)), "superdc_cauchy_apply")
    return Y


def deflate(ctx, batch, d, z, rho, tau, stream=None, out=None):
    """superdc_deflate.  Returns dict(d, z, perm, rot_right, rot_left, rot_c, rot_s, kept,
    status) of device tensors (kept and status per problem)."""
    import torch
    tot, P = batch.total, batch.nprob
    _f64(d, tot, "d"), _f64(z, tot, "z"), _f64(rho, P, "rho")
    dev = d.device
    if out is None:
        f64 = dict(dtype=torch.float64, device=dev)
        i32 = dict(dtype=torch.int32, device=dev)
        out = dict(d=torch.empty(tot, **f64), z=torch.empty(tot, **f64),
                   perm=torch.empty(tot, **i32), rot_right=torch.empty(tot, **i32),
                   rot_left=torch.empty(tot, **i32), rot_c=torch.empty(tot, **f64),
                   rot_s=torch.empty(tot, **f64), kept=torch.empty(P, **i32),
                   status=torch.empty(P, **i32))
    _check(load_library().superdc_deflate(
        ctx.handle, batch.handle, _ptr(d), _ptr(z), _ptr(rho), float(tau), _ptr(out["d"]),
        _ptr(out["z"]), _ptr(out["perm"]), _ptr(out["rot_right"]), _ptr(out["rot_left"]),
        _ptr(out["rot_c"]), _ptr(out["rot_s"]), _ptr(out["kept"]), _ptr(out["status"]),
        _stream(stream)), "superdc_deflate")
    return out


def deflate_expand(ctx, batch, df, X, trans=0, stream=None, Y=None):
    """superdc_deflate_expand on an (m, ldx) row-major tensor (= column-major total x m)."""
    import torch
    if X.dim() == 1:
        X = X.view(1, -1)
    m, ldx = X.shape
    if not X.is_contiguous() or X.dtype != torch.float64 or not X.is_cuda:
        raise SuperdcError("X must be a contiguous CUDA float64 (m, ldx) tensor")
    if Y is None:
        Y = torch.empty((m, batch.total), dtype=torch.float64, device=X.device)
    _check(load_library().superdc_deflate_expand(
        ctx.handle, batch.handle, _ptr(df["perm"]), _ptr(df["rot_right"]), _ptr(df["rot_left"]),
        _ptr(df["rot_c"]), _ptr(df["rot_s"]), int(trans), int(m), _ptr(X), int(ldx), _ptr(Y),
        int(Y.shape[1]), _stream(stream)), "superdc_deflate_expand")
    return Y


def batch_copy_rows(ctx, src_batch, dst_batch, src, rows=None, fill=None, stream=None, dst=None):
    """superdc_batch_copy_rows on (m, ld) row-major tensors (= column-major total x m)."""
    import torch
    if src.dim() == 1:
        src = src.view(1, -1)
    m, lds = src.shape
    if not src.is_contiguous() or src.dtype != torch.float64 or not src.is_cuda:
        raise SuperdcError("src must be a contiguous CUDA float64 (m, ld) tensor")
    if dst is None:
        dst = torch.empty((m, dst_batch.total), dtype=torch.float64, device=src.device)
    fv = None if fill is None else C.byref(C.c_double(float(fill)))
    _check(load_library().superdc_batch_copy_rows(
        ctx.handle, src_batch.handle, dst_batch.handle, _ptr(rows), int(m), _ptr(src), int(lds),
        _ptr(dst), int(dst.shape[-1]), fv, _stream(stream)), "superdc_batch_copy_rows")
    return dst


def secular_backward(ctx, batch, d, z, rho, eta, origin, status, g_lam=None, g_proj=None,
                     u=None, opts=None, stream=None, out=None):
    """superdc_secular_backward.  Returns (g_d, g_z, g_rho) (`out`, if given, is such a
    tuple of preallocated tensors and is written in place)."""
    import torch
    tot, P = batch.total, batch.nprob
    if out is None:
        out = (torch.empty(tot, dtype=torch.float64, device=d.device),
               torch.empty(tot, dtype=torch.float64, device=d.device),
               torch.empty(P, dtype=torch.float64, device=d.device))
    g_d, g_z, g_r = out
    o = opts if opts is not None else default_opts()
    _check(load_library().superdc_secular_backward(
        ctx.handle, batch.handle, _ptr(d), _ptr(z), _ptr(rho), _ptr(eta), _ptr(origin),
        _ptr(status), _ptr(g_lam), _ptr(g_proj), _ptr(u), _ptr(g_d), _ptr(g_z), _ptr(g_r),
        C.byref(o), _stream(stream)), "superdc_secular_backward")
    return g_d, g_z, g_r


def autotune(ctx, batch, d, z, rho, opts=None, stream=None):
    """superdc_autotune: time candidate launch shapes on (d, z, rho) and keep the fastest.
    Returns the chosen shapes (see batch_shapes)."""
    tot, P = batch.total, batch.nprob
    _f64(d, tot, "d"), _f64(z, tot, "z"), _f64(rho, P, "rho")
    o = opts if opts is not None else default_opts()
    _check(load_library().superdc_autotune(ctx.handle, batch.handle, _ptr(d), _ptr(z), _ptr(rho),
                                           C.byref(o), _stream(stream)), "superdc_autotune")
    return batch_shapes(batch)


def kernel_timing(enable=True, mode=None):
    """superdc_kernel_timing: bracket every library launch with HIP events and count work
    on the device (mode None: both, or off with enable False); mode "events" or
    "counters" turns on one of them alone."""
    m = 0 if not enable else {None: 1, "events": 2, "counters": 3}[mode]
    _check(load_library().superdc_kernel_timing(m), "superdc_kernel_timing")


def kernel_times():
    """superdc_kernel_times: {kernel name: (ms, launches)} since the last call (waits for
    the recorded launches), kernels that ran only."""
    lib = load_library()
    cnt = lib.superdc_kernel_times(None, None, 0)
    if cnt < 0:
        _check(cnt, "superdc_kernel_times")
    ms = (C.c_double * cnt)()
    nl = (C.c_int32 * cnt)()
    _check(min(0, lib.superdc_kernel_times(ms, nl, cnt)), "superdc_kernel_times")
    return {lib.superdc_kernel_name(i).decode(): (ms[i], nl[i]) for i in range(cnt) if nl[i]}


def kernel_work():
    """superdc_kernel_work: {kernel name: pole-root pair evaluations} counted while kernel
    timing was on (kernels with a counter only); waits for the device and clears them."""
    lib = load_library()
    cnt = lib.superdc_kernel_times(None, None, 0)
    w = (C.c_double * cnt)()
    _check(min(0, lib.superdc_kernel_work(w, cnt)), "superdc_kernel_work")
    return {lib.superdc_kernel_name(i).decode(): w[i] for i in range(cnt) if w[i] > 0}


def kernel_counters():
    """superdc_kernel_counters: {kernel name: (work, live lanes, lane slots)} counted while
    kernel timing was on (kernels with a counter only); waits and clears them."""
    lib = load_library()
    lib.superdc_kernel_counters.argtypes = [_P, C.c_int32]
    lib.superdc_kernel_counters.restype = C.c_int
    cnt = lib.superdc_kernel_times(None, None, 0)
    w = (C.c_double * (4 * cnt))()
    _check(min(0, lib.superdc_kernel_counters(w, cnt)), "superdc_kernel_counters")
    return {lib.superdc_kernel_name(i).decode(): (w[4 * i], w[4 * i + 1], w[4 * i + 2])
            for i in range(cnt) if w[4 * i] > 0}


def batch_shapes(batch):
    """superdc_batch_shapes: dict(sec_chunk, sec_split, vec_split, bwd_split, fmm_split)."""
    out = (C.c_int32 * 5)()
    _check(load_library().superdc_batch_shapes(batch.handle, out), "superdc_batch_shapes")
    return dict(sec_chunk=out[0], sec_split=out[1], vec_split=out[2], bwd_split=out[3],
                fmm_split=out[4])


# ---------------------------------------------------------------------------------------
# HSS conquering pass
# ---------------------------------------------------------------------------------------
def _hss_sigs(lib):
    lib.superdc_hss_plan_create.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(_P)]
    lib.superdc_hss_plan_create.restype = C.c_int
    lib.superdc_hss_plan_destroy.argtypes = [_P]
    lib.superdc_hss_plan_destroy.restype = None
    lib.superdc_hss_conquer.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.POINTER(Opts), _P]
    lib.superdc_hss_conquer.restype = C.c_int
    lib.superdc_hss_apply.argtypes = [_P, _P, C.c_int, C.c_int32, _P, C.c_int64, _P, C.c_int64,
                                      C.POINTER(Opts), _P]
    lib.superdc_hss_apply.restype = C.c_int


def pack_hss(tree):
    """Lay the generators of a gen.HSSTree out as the C ABI expects (heap order
    h = 2^l - 1 + q for R, B and beta).  Host numpy arrays."""
    D, r = tree.depth, tree.r
    R = np.zeros(((1 << (D + 1)) - 1, r, r))
    for lvl in range(1, D + 1):
        R[(1 << lvl) - 1:(1 << (lvl + 1)) - 1] = tree.R[lvl]
    B = np.zeros(((1 << D) - 1, r, r))
    beta = np.zeros((1 << D) - 1)
    for lvl in range(D):
        B[(1 << lvl) - 1:(1 << (lvl + 1)) - 1] = tree.B[lvl]
        beta[(1 << lvl) - 1:(1 << (lvl + 1)) - 1] = tree.beta[lvl]
    return dict(leaf_D=np.ascontiguousarray(tree.leaf_D), leaf_U=np.ascontiguousarray(tree.leaf_U),
                R=R, B=B, beta=beta)


class HSSPlan:
    """superdc_hss: level batches, factor storage and work buffers of one tree shape."""

    def __init__(self, ctx, leaf, depth, r):
        lib = load_library()
        _hss_sigs(lib)
        self.ctx, self.leaf, self.depth, self.r = ctx, leaf, depth, r
        self.n = leaf << depth
        h = _P()
        _check(lib.superdc_hss_plan_create(ctx.handle, leaf, depth, r, C.byref(h)),
               "superdc_hss_plan_create")
        self.handle = h

    def close(self):
        if self.handle:
            load_library().superdc_hss_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hss_conquer(ctx, plan, gens, opts=None, stream=None, levels=False, out=None):
    """superdc_hss_conquer.  gens: dict of CUDA float64 tensors (leaf_D, leaf_U, R, B, beta)
    laid out as pack_hss returns.  Returns dict(lam, lam_levels or None, status)."""
    import torch
    dev = gens["leaf_D"].device
    n = plan.n
    if out is None:
        out = dict(lam=torch.empty(n, dtype=torch.float64, device=dev),
                   lam_levels=(torch.empty((plan.depth + 1, n), dtype=torch.float64, device=dev)
                               if levels else None),
                   status=torch.empty(1, dtype=torch.int32, device=dev))
    o = opts if opts is not None else default_opts()
    for k in ("leaf_D", "leaf_U", "R", "B", "beta"):
        t = gens[k]
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise SuperdcError(f"{k}: need a contiguous CUDA float64 tensor")
    _check(load_library().superdc_hss_conquer(
        ctx.handle, plan.handle, _ptr(gens["leaf_D"]), _ptr(gens["leaf_U"]), _ptr(gens["R"]),
        _ptr(gens["B"]), _ptr(gens["beta"]), _ptr(out["lam"]), _ptr(out["lam_levels"]),
        _ptr(out["status"]), C.byref(o), _stream(stream)), "superdc_hss_conquer")
    return out


def hss_divide(ctx, plan, gens, balanced=True, stream=None, out=None):
    """superdc_hss_divide on packed original generators (device tensors as from pack_hss);
    returns the conquer's input: dict(leaf_D, leaf_U, R, B, beta) (`out`, if given, is
    such a dict from an earlier call and is written in place)."""
    import torch
    lib = load_library()
    lib.superdc_hss_divide.argtypes = [_P, _P, _P, _P, _P, _P, C.c_int, _P, _P, _P, _P]
    lib.superdc_hss_divide.restype = C.c_int
    if out is None:
        out = dict(leaf_D=torch.empty_like(gens["leaf_D"]), leaf_U=gens["leaf_U"], R=gens["R"],
                   B=torch.empty_like(gens["B"]),
                   beta=torch.empty(gens["B"].shape[0], dtype=torch.float64,
                                    device=gens["B"].device))
    _check(lib.superdc_hss_divide(ctx.handle, plan.handle, _ptr(gens["leaf_D"]), _ptr(gens["leaf_U"]),
                                  _ptr(gens["R"]), _ptr(gens["B"]), int(bool(balanced)),
                                  _ptr(out["leaf_D"]), _ptr(out["B"]), _ptr(out["beta"]),
                                  _stream(stream)), "superdc_hss_divide")
    return out


def hss_apply(ctx, plan, X, trans=0, opts=None, stream=None, Y=None):
    """superdc_hss_apply.  X: contiguous (m, n) tensor, each row one vector."""
    import torch
    if X.dim() == 1:
        X = X.view(1, -1)
    m, ldx = X.shape
    if not X.is_contiguous() or X.dtype != torch.float64 or not X.is_cuda or ldx < plan.n:
        raise SuperdcError("X must be a contiguous CUDA float64 (m, >=n) tensor")
    if Y is None:
        Y = torch.empty((m, plan.n), dtype=torch.float64, device=X.device)
    o = opts if opts is not None else default_opts()
    _check(load_library().superdc_hss_apply(ctx.handle, plan.handle, int(trans), int(m), _ptr(X),
                                            int(ldx), _ptr(Y), int(Y.shape[1]), C.byref(o),
                                            _stream(stream)), "superdc_hss_apply")
    return Y


def hss_autotune(ctx, plan, gens, opts=None, stream=None):
    """superdc_hss_autotune: tune every level's launch shapes on one conquer of `gens`;
    returns the chosen shapes per level (as batch_shapes)."""
    lib = load_library()
    lib.superdc_hss_autotune.argtypes = [_P, _P, _P, _P, _P, _P, _P, C.POINTER(Opts), _P]
    lib.superdc_hss_autotune.restype = C.c_int
    lib.superdc_hss_batch_shapes.argtypes = [_P, C.c_int32, _P]
    lib.superdc_hss_batch_shapes.restype = C.c_int
    o = opts if opts is not None else default_opts()
    _check(lib.superdc_hss_autotune(ctx.handle, plan.handle, _ptr(gens["leaf_D"]),
                                    _ptr(gens["leaf_U"]), _ptr(gens["R"]), _ptr(gens["B"]),
                                    _ptr(gens["beta"]), C.byref(o), _stream(stream)),
           "superdc_hss_autotune")
    shapes = []
    for lvl in range(plan.depth):
        out = (C.c_int32 * 5)()
        _check(lib.superdc_hss_batch_shapes(plan.handle, lvl, out), "superdc_hss_batch_shapes")
        shapes.append(dict(sec_chunk=out[0], sec_split=out[1], vec_split=out[2],
                           bwd_split=out[3], fmm_split=out[4]))
    return shapes


def hss_set_timing(plan, enable=True):
    lib = load_library()
    lib.superdc_hss_set_timing.argtypes = [_P, C.c_int]
    lib.superdc_hss_set_timing.restype = C.c_int
    _check(lib.superdc_hss_set_timing(plan.handle, int(enable)), "superdc_hss_set_timing")


HSS_PHASES = ("leaf", "merge_assemble", "secular", "loewner_b", "apply", "copies")


def hss_phase_times(plan):
    """Per-phase milliseconds and timed-interval counts of the last conquer."""
    lib = load_library()
    lib.superdc_hss_phase_times.argtypes = [_P, _P, _P]
    lib.superdc_hss_phase_times.restype = C.c_int
    ms = (C.c_double * 6)()
    cnt = (C.c_int32 * 6)()
    _check(lib.superdc_hss_phase_times(plan.handle, ms, cnt), "superdc_hss_phase_times")
    return dict(zip(HSS_PHASES, list(ms))), dict(zip(HSS_PHASES, list(cnt)))


def hss_iterations(plan, stream=None):
    """Per-root evaluation counts of the last conquer: int32 tensor [depth, r, n]."""
    import torch
    lib = load_library()
    lib.superdc_hss_iterations.argtypes = [_P, _P, _P]
    lib.superdc_hss_iterations.restype = C.c_int
    out = torch.empty((plan.depth, plan.r, plan.n), dtype=torch.int32, device="cuda")
    _check(lib.superdc_hss_iterations(plan.handle, _ptr(out), _stream(stream)),
           "superdc_hss_iterations")
    return out
