#!/usr/bin/env python3
"""Benchmark of the conquering-stage hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload conquer|level|large|single|deflate|ex1]

A step is one pass of the whole rank-one path over one batch already resident in HBM:
validation and packing, the secular solve (midpoint pass plus middle-way iterations to
convergence), the Loewner vector and normalisation, and the Cauchy-like eigenvector
matrix applied to the batch's right-hand sides.  The batched form runs every phase as one
persistent launch over the whole batch; the plain form runs the same kernels once per
problem.  Both are timed; `value` is the batched form's whole-job throughput in roots/s.

Prints one JSON line.  The roofline object describes the dominant kernel of the step (the
kernel with the most time among those whose work has an algorithmic count): `achieved` is
its algorithmic FP64 rate -- 7 flops per pole-root pair evaluation of the secular sums
with the actual per-root evaluation counts, 5 and 6 per pair for the Loewner and b
passes, (2m + 3) per matrix entry plus 2nm for an apply to m vectors -- over its
duration measured with HIP events around each of its launches on the launch stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "secular roots/s + Cauchy-apply FP64 GFLOP/s, batched vs plain, at <=1e-12 rel err"
PEAK_FP64_VALU = 78.6    # TFLOP/s, MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
PEAK_FP64_MFMA = 78.6    # TFLOP/s, MI355X FP64 matrix
PEAK_HBM_GBPS = 8000.0   # GB/s, MI355X HBM3E
FLOPS_PER_PAIR = 7       # secular: 2 sub, 1 rcp, 1 mul, 1 add, 1 fma(2)
FLOPS_LOEWNER = 5        # per pair: 2 sub, 1 add, 2 mul
FLOPS_BNORM = 6          # per pair: 2 sub, 1 rcp, 1 mul, 1 fma(2)


FMM_CROSSOVER = 1024     # the library's default direct/FMM switch (roots per problem)
ITER_COUNT_MASK, ITER_UNMET, ITER_CAP = 0xFFFF, 1 << 16, 1 << 17  # iteration records

MU_DEFINITION = ("per level, the largest share over the r rank-one steps of roots that needed "
                 "more than 5 iterations after the midpoint pass, or whose iteration ended on "
                 "a step below rounding or a collapsed bracket (or the cap) before the "
                 "stopping test held")


def mu_levels(it, count_only=False):
    """The share mu (percent) of roots not converged within 5 iterations, per level, from
    iteration records of shape (depth, r, n)."""
    cnt = it & ITER_COUNT_MASK
    bad = cnt > 5 if count_only else (cnt > 5) | ((it & (ITER_UNMET | ITER_CAP)) != 0)
    return [float(100.0 * np.max(np.mean(bad[l], axis=1))) for l in range(it.shape[0])]


def unmet_levels(it):
    """Per level, the largest share (percent) over the steps of roots whose iteration ended
    before the stopping test held."""
    bad = (it & (ITER_UNMET | ITER_CAP)) != 0
    return [float(100.0 * np.max(np.mean(bad[l], axis=1))) for l in range(it.shape[0])]
MFMA_MIN_M = 4           # the library's automatic VALU/MFMA apply switch (columns)


def kernel_roofline(kt, flops, steps, workload=None):
    """Per-kernel table and the roofline object of the dominant kernel.

    kt: {kernel: (ms, launches)} from the library's per-kernel HIP-event timing over
    `steps` steps; flops: {kernel: algorithmic FP64 flops per step} for the kernels whose
    work has an algorithmic count.  The dominant kernel is the one with the largest time
    per step among those."""
    table = {}
    for name, (ms, nl) in sorted(kt.items(), key=lambda x: -x[1][0]):
        e = {"ms_per_step": ms / steps, "launches_per_step": nl / steps,
             "avg_launch_ms": ms / nl}
        if name in flops and ms > 0:
            e["algorithmic_tflops"] = flops[name] / (ms / steps * 1e-3) / 1e12
        table[name] = e
    cand = [k for k in table if k in flops and flops[k] > 0]
    if not cand:
        return table, None
    dom = max(cand, key=lambda k: table[k]["ms_per_step"])
    e = table[dom]
    achieved = e["algorithmic_tflops"]
    peak = PEAK_FP64_MFMA if dom == "k_apply_mfma" else PEAK_FP64_VALU
    roof = {"bound": "mfma" if dom == "k_apply_mfma" else "alu", "achieved": achieved,
            "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": kernel_traffic(dom, workload) if workload else None,
            "kernel": dom, "launches_per_step": e["launches_per_step"],
            "avg_launch_ms": e["avg_launch_ms"],
            "algorithmic_flops_per_launch": flops[dom] / e["launches_per_step"],
            "timing": "HIP events around each launch on its stream (library kernel timing)"}
    return table, roof


CALIB_BYTES = 512 << 20  # the calibration copy: this many bytes read and written
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2108_04209_amd", "csrc")


def kernel_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` in `workload` from the committed counter summary
    profiles/<kernel>_<workload>_traffic.md (FETCH_SIZE + WRITE_SIZE, each scaled by the
    same counter's reading for a copy of known size), or None if there is none or the
    kernel's sources changed since it was taken (their SHA-256 is recorded in it)."""
    import hashlib
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    try:
        srcs = fields["sources"].split(",")
        h = hashlib.sha256()
        for f in srcs:
            h.update(open(os.path.join(CSRC, f.strip()), "rb").read())
        if h.hexdigest() != fields["sources_sha256"]:
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def note(msg):
    """progress line on stderr (the JSON result is the only stdout line)"""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="conquer",
                    choices=["conquer", "level", "large", "single", "deflate", "ex1"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-level", action="store_true",
                    help="with --workload conquer, skip the batched-level and large-problem "
                         "side measurements")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fmm-crossover", type=int, default=0,
                    help="problems with at least this many roots use the FMM (0: the "
                         "library default, %d)" % FMM_CROSSOVER)
    ap.add_argument("--fmm-leaf", type=int, default=64,
                    help="poles per FMM leaf (multiple of 64, at most 1024; the library "
                         "default is 64)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 512 MiB device-to-device copy (the reference kernel "
                         "that scales the profiler's FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def workload(name):
    from paper_2108_04209_amd import gen
    if name == "level":
        batch, X = gen.cfg2()
        cfg = {"workload": "batched level: 4096 rank-one problems, n log-uniform in [64, 8192], "
                           "FP64, rho ~ U[0.1,2], 16 right-hand sides",
               "nprob": batch.nprob, "total_n": batch.total_n, "m": int(X.shape[1])}
    else:
        pr, X = gen.cfg0()
        batch = gen.concat([pr])
        cfg = {"workload": "single rank-one problem n=1024, 16 right-hand sides",
               "nprob": 1, "total_n": pr.n, "m": int(X.shape[1])}
    return batch, X, cfg


class Pipeline:
    """Preallocated device buffers and the four C-ABI calls of one step."""

    def __init__(self, batch, X, persistent, method=0, crossover=0, leaf=256):
        import torch
        from paper_2108_04209_amd import native
        self.torch = torch
        self.native = native
        self.ctx = native.Context()
        self.b = native.Batch(self.ctx, batch.off)
        dev = torch.device("cuda:0")
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
        self.d, self.z, self.rho = f(batch.d), f(batch.z), f(batch.rho)
        self.X = f(np.asarray(X).T)                      # (m, total): column-major batch
        tot, P = batch.total_n, batch.nprob
        self.out = dict(lam=torch.empty(tot, dtype=torch.float64, device=dev),
                        eta=torch.empty(tot, dtype=torch.float64, device=dev),
                        origin=torch.empty(tot, dtype=torch.int32, device=dev),
                        iters=torch.empty(tot, dtype=torch.int32, device=dev),
                        status=torch.empty(P, dtype=torch.int32, device=dev))
        self.zb = (torch.empty(tot, dtype=torch.float64, device=dev),
                   torch.empty(tot, dtype=torch.float64, device=dev))
        self.Y = torch.empty_like(self.X)
        self.opts = native.default_opts(persistent=persistent, method=method,
                                        fmm_crossover=crossover, fmm_leaf=leaf)

    def solve(self):
        self.native.secular_solve(self.ctx, self.b, self.d, self.z, self.rho, opts=self.opts,
                                  out=self.out)

    def vectors(self):
        o = self.out
        self.native.loewner(self.ctx, self.b, self.d, self.z, self.rho, o["eta"], o["origin"],
                            o["status"], opts=self.opts, out=self.zb)

    def apply(self):
        o = self.out
        self.native.cauchy_apply(self.ctx, self.b, self.d, self.zb[0], self.zb[1], o["eta"],
                                 o["origin"], o["status"], self.X, trans=1, opts=self.opts,
                                 Y=self.Y)

    def step(self):
        self.solve()
        self.vectors()
        self.apply()


def time_steps(pipe, steps, warmup):
    torch = pipe.torch
    for _ in range(warmup):
        pipe.step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        e = ev[s]
        e[0].record()
        pipe.solve()
        e[1].record()
        pipe.vectors()
        e[2].record()
        pipe.apply()
        e[3].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ph = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in ev])  # ms
    tot = np.array([e[0].elapsed_time(e[3]) for e in ev])
    return wall / steps * 1e3, tot, ph


def accuracy(pipe, batch, X, nsample=4):
    """Max |lambda - lambda_oracle| / ||A||_2 over a seeded sample of problems (largest
    included), and the apply error, against the CPU oracle."""
    import oracle
    o = {k: v.cpu().numpy() for k, v in pipe.out.items()}
    zh, bn = pipe.zb[0].cpu().numpy(), pipe.zb[1].cpu().numpy()
    Y = pipe.Y.cpu().numpy().T
    sizes = batch.sizes()
    rng = np.random.default_rng(1)
    pick = sorted({int(np.argmax(sizes))} | set(rng.choice(batch.nprob, min(nsample, batch.nprob), replace=False).tolist()))
    err, aerr = 0.0, 0.0
    for p in pick:
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        lam, eta, org, its, st = oracle.secular(pr.d, pr.z, pr.rho)
        err = max(err, np.abs(o["lam"][a:e] - lam).max() / np.abs(lam).max())
        z1 = oracle.loewner(pr.d, pr.z, pr.rho, eta, org)
        b1 = oracle.bnorm(pr.d, z1, eta, org)
        rows = np.arange(0, e - a, max(1, (e - a) // 64))
        Yo = oracle.cauchy_apply(pr.d, z1, b1, eta, org, X[a:e], trans=1, rows=rows)
        aerr = max(aerr, np.abs(Y[a:e][rows] - Yo).max() / np.abs(X[a:e]).max())
    return float(err), float(aerr), int(np.all(o["status"] == 0)), pick


def cpu_baseline(batch, X, seconds):
    """The oracle (plain FP64 C, OpenMP) on whole problems of the same workload, taken in a
    seeded order until `seconds` of wall time are spent; roots/s of the full path."""
    import oracle
    oracle.load()
    rng = np.random.default_rng(7)
    order = rng.permutation(batch.nprob)
    roots, t_used, probs = 0, 0.0, 0
    m = X.shape[1]
    for p in order:
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        t0 = time.perf_counter()
        lam, eta, org, its, st = oracle.secular(pr.d, pr.z, pr.rho)
        zh = oracle.loewner(pr.d, pr.z, pr.rho, eta, org)
        b = oracle.bnorm(pr.d, zh, eta, org)
        oracle.cauchy_apply(pr.d, zh, b, eta, org, X[a:e], trans=1)
        t_used += time.perf_counter() - t0
        roots += e - a
        probs += 1
        if t_used >= seconds:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": roots / t_used, "unit": "roots/s", "cores": cores, "kind": "oracle",
            "sample": f"{probs} whole problems ({roots} roots, seeded order) of the same "
                      f"workload, full path incl. apply to {m} vectors, {t_used:.1f} s"}


def bench_level(args, name):
    import torch
    batch, X, cfg = workload(name)
    tot = batch.total_n
    sizes = batch.sizes().astype(np.float64)
    m = X.shape[1]

    pipe = Pipeline(batch, X, persistent=1, crossover=args.fmm_crossover, leaf=args.fmm_leaf)
    wall_ms, tot_ms, ph = time_steps(pipe, args.steps, args.warmup)
    note(f"{name} batched {float(np.mean(tot_ms)):.2f} ms/step")
    iters = (pipe.out["iters"].cpu().numpy() & ITER_COUNT_MASK).astype(np.float64)
    status_ok = bool(np.all(pipe.out["status"].cpu().numpy() == 0))
    ms = float(np.mean(tot_ms))
    solve_ms, vec_ms, apply_ms = (float(x) for x in ph.mean(axis=0))

    # algorithmic work of one step
    n_of_root = np.repeat(sizes, batch.sizes())
    pairs = float(np.sum(n_of_root * (1.0 + iters)))
    sec_flops = FLOPS_PER_PAIR * pairs
    n2 = float(np.sum(sizes ** 2))
    vec_flops = (FLOPS_LOEWNER + FLOPS_BNORM) * n2
    apply_flops = (2 * m + 3) * n2 + 2 * tot * m

    # graph replay of the same step
    graph_ms = None
    try:
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            pipe.step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            pipe.step()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        graph_ms = e0.elapsed_time(e1) / args.steps
    except Exception as exc:  # report, do not hide
        graph_ms = f"capture failed: {exc!r}"

    err, aerr, st_ok, pick = accuracy(pipe, batch, X)

    plain_res = None
    if args.plain_steps > 0:
        plain = Pipeline(batch, X, persistent=0, crossover=args.fmm_crossover, leaf=args.fmm_leaf)
        p_wall, p_tot, p_ph = time_steps(plain, args.plain_steps, 1)
        p_ms = float(np.mean(p_tot))
        plain_res = {"ms_per_step": p_ms, "value": tot / (p_ms * 1e-3),
                     "phase_ms": dict(zip(["solve", "loewner_b", "apply"],
                                          (float(x) for x in p_ph.mean(axis=0)))),
                     "launches_per_phase": batch.nprob, "steps": args.plain_steps}

    # per-kernel timing pass
    pipe.native.kernel_timing(True)
    for _ in range(args.steps):
        pipe.step()
    torch.cuda.synchronize()
    kt = pipe.native.kernel_times()
    kw = pipe.native.kernel_work()
    pipe.native.kernel_timing(False)
    # direct kernels serve the problems below the FMM crossover only
    small = sizes[sizes < (args.fmm_crossover or FMM_CROSSOVER)]
    n2d = float(np.sum(small ** 2))
    kflops = {"k_loewner": FLOPS_LOEWNER * n2d, "k_bnorm": FLOPS_BNORM * n2d,
              ("k_apply_mfma" if m >= MFMA_MIN_M else "k_apply_valu"):
                  (2 * m + 3) * n2d + 2 * float(np.sum(small)) * m}
    for k in ("k_secular", "k_secular_fmm"):  # the solvers count their pair evaluations
        if k in kw:
            kflops[k] = FLOPS_PER_PAIR * kw[k] / args.steps
    kernels, roofline = kernel_roofline(kt, kflops, args.steps, name)
    res = {
        "metric": METRIC, "value": tot / (ms * 1e-3), "unit": "roots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators, no dataset)", "config": cfg,
        "secular_roots_per_s": tot / (solve_ms * 1e-3),
        "apply_gflops": apply_flops / (apply_ms * 1e-3) / 1e9,
        "phase_ms": {"solve": solve_ms, "loewner_b": vec_ms, "apply": apply_ms},
        "kernels": kernels,
        "mean_iters_after_midpoint": float(iters.mean()), "max_iters": int(iters.max()),
        "graph_ms_per_step": graph_ms, "wall_ms_per_step": wall_ms,
        "plain": plain_res,
        "speedup_batched_vs_plain": None if plain_res is None else plain_res["ms_per_step"] / ms,
        "accuracy": {"max_eig_err_rel_normA": err, "apply_err_rel": aerr,
                     "problems_checked": pick, "status_all_ok": status_ok},
        "roofline": roofline,
    }
    note(f"{name} graph/accuracy/plain done")
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(batch, X, args.cpu_seconds)
        note(f"{name} cpu baseline done")
    return res




def bench_large(args):
    """One rank-one problem, n = 65536, clustered poles (10% in clusters of 32 spaced
    1e-10, 1% of weights 1e-12), rho = 0.5, eigenvectors applied to 64 vectors: the
    triangular FMM (order 16, leaf 256) against direct sums, same kernels otherwise."""
    import oracle
    from paper_2108_04209_amd import gen
    pr, X = gen.cfg1()
    batch = gen.concat([pr])
    n, m = pr.n, X.shape[1]
    out = {}
    for name, method in (("fmm", 2), ("direct", 1)):
        pipe = Pipeline(batch, X, persistent=1, method=method, leaf=256)  # as specified
        wall_ms, tot_ms, ph = time_steps(pipe, args.steps, args.warmup)
        iters = (pipe.out["iters"].cpu().numpy() & ITER_COUNT_MASK).astype(np.float64)
        solve_ms, vec_ms, apply_ms = (float(x) for x in ph.mean(axis=0))
        ms = float(np.mean(tot_ms))
        note(f"large {name} {ms:.2f} ms/step")
        out[name] = {"ms_per_step": ms, "roots_per_s": n / (ms * 1e-3),
                     "phase_ms": {"solve": solve_ms, "loewner_b": vec_ms, "apply": apply_ms},
                     "mean_iters_after_midpoint": float(iters.mean()),
                     "max_iters": int(iters.max()),
                     "status": int(pipe.out["status"].cpu().numpy()[0]),
                     "_pipe": pipe}
    pf, pd = out["fmm"].pop("_pipe"), out["direct"].pop("_pipe")
    lam_f = pf.out["lam"].cpu().numpy()
    lam_d = pd.out["lam"].cpu().numpy()
    nA = float(np.abs(lam_d).max())
    # sampled oracle roots: the extreme ones, 30 random, 16 inside clusters
    rng = np.random.default_rng(8)
    tight = np.flatnonzero(np.diff(pr.d) < 1e-9)
    roots = np.unique(np.r_[0, n - 1, rng.choice(n, 30, replace=False),
                            rng.choice(tight, 16, replace=False)])
    lam_o, eta_o, org_o, its_o, st_o = oracle.secular(pr.d, pr.z, pr.rho, roots=roots)
    # sampled apply rows against the oracle fed the GPU's eta/origin (the oracle's own
    # zhat and b from them)
    eta_f = pf.out["eta"].cpu().numpy()
    org_f = pf.out["origin"].cpu().numpy()
    zh = oracle.loewner(pr.d, pr.z, pr.rho, eta_f, org_f)
    bn = oracle.bnorm(pr.d, zh, eta_f, org_f)
    rows = np.sort(rng.choice(n, 64, replace=False))
    Yo = oracle.cauchy_apply(pr.d, zh, bn, eta_f, org_f, X, trans=1, rows=rows)
    Yf = pf.Y.cpu().numpy().T
    fm = out["fmm"]
    best = min(("fmm", "direct"), key=lambda k: out[k]["ms_per_step"])
    return {
        "config": {"workload": "single rank-one problem n=65536, clustered poles, "
                               "64 right-hand sides, FMM order 16 leaf 256 vs direct",
                   "n": n, "m": int(m)},
        "value": out[best]["roots_per_s"], "faster": best, "fmm": out["fmm"],
        "direct": out["direct"],
        "apply_gflops_fmm_run": ((2 * m + 3) * float(n) ** 2 + 2 * n * m)
                                / (fm["phase_ms"]["apply"] * 1e-3) / 1e9,
        "accuracy": {"fmm_vs_direct_rel_normA": float(np.abs(lam_f - lam_d).max() / nA),
                     "fmm_vs_oracle_sampled_rel_normA": float(np.abs(lam_f[roots] - lam_o).max() / nA),
                     "origins_agree": bool(np.array_equal(org_f[roots], org_o)),
                     "apply_err_rel_sampled_rows": float(np.abs(Yf[rows] - Yo).max() / np.abs(X).max()),
                     "roots_checked": int(len(roots))},
    }


def bench_deflate(args):
    """Deflation (Remark 1) on a batched level: 4096 problems of log-uniform size in
    [64, 8192] drawn with repeated and nearly repeated poles and tiny or zero weights,
    tau = 1e-10.  One step: the deflation pass, the gather of the reduced problems, their
    solve, Loewner/b, Q^T X for 16 vectors (rotations, placement, Cauchy apply) and the
    scatter back.  The reduced batch (its sizes come from the pass) is built once."""
    import torch
    import oracle
    from paper_2108_04209_amd import gen, native
    tau = 1e-10
    sizes = gen.cfg2_sizes()
    batch, X = gen.deflation_batch(sizes, seed=5, m=16)
    dev = torch.device("cuda:0")
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    ctx = native.Context()
    b = native.Batch(ctx, batch.off)
    d, z, rho = f(batch.d), f(batch.z), f(batch.rho)
    Xt = f(np.asarray(X).T)
    df = native.deflate(ctx, b, d, z, rho, tau)
    kept = df["kept"].cpu().numpy()
    roff = np.concatenate([[0], np.cumsum(np.maximum(kept, 1))]).astype(np.int64)
    rb = native.Batch(ctx, roff)
    o = native.default_opts()
    rt = int(roff[-1])
    buf = {"dr": torch.empty((1, rt), dtype=torch.float64, device=dev),
           "zr": torch.empty((1, rt), dtype=torch.float64, device=dev),
           "V": torch.empty_like(Xt), "Vr": torch.empty((Xt.shape[0], rt), dtype=torch.float64, device=dev),
           "Wr": torch.empty((Xt.shape[0], rt), dtype=torch.float64, device=dev),
           "lam": torch.empty(batch.total_n, dtype=torch.float64, device=dev)}

    def step():
        native.deflate(ctx, b, d, z, rho, tau, out=df)
        native.batch_copy_rows(ctx, b, rb, df["d"], rows=df["kept"], fill=0.0, dst=buf["dr"])
        native.batch_copy_rows(ctx, b, rb, df["z"], rows=df["kept"], fill=1.0, dst=buf["zr"])
        dr, zr = buf["dr"].view(-1), buf["zr"].view(-1)
        s = native.secular_solve(ctx, rb, dr, zr, rho, opts=o)
        buf["lam"].copy_(df["d"])
        native.batch_copy_rows(ctx, rb, b, s["lam"], rows=df["kept"], dst=buf["lam"].view(1, -1))
        zh, bn = native.loewner(ctx, rb, dr, zr, rho, s["eta"], s["origin"], s["status"], opts=o)
        native.deflate_expand(ctx, b, df, Xt, trans=1, Y=buf["V"])
        native.batch_copy_rows(ctx, b, rb, buf["V"], rows=df["kept"], fill=0.0, dst=buf["Vr"])
        native.cauchy_apply(ctx, rb, dr, zh, bn, s["eta"], s["origin"], s["status"], buf["Vr"],
                            trans=1, opts=o, Y=buf["Wr"])
        native.batch_copy_rows(ctx, rb, b, buf["Wr"], rows=df["kept"], dst=buf["V"])
        return s

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        s = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    native.kernel_times()
    native.kernel_timing(True)
    try:
        for _ in range(args.steps):
            step()
        kt = native.kernel_times()
    finally:
        native.kernel_timing(False)
    note(f"deflate level {ms:.2f} ms/step")
    n = batch.total_n
    # the deflation pass: segment scans, joins, counts and placement (four launches)
    kd = kt.get("k_deflate", (0.0, 0))
    kd_ms = kd[0] / args.steps
    bytes_per_pole = 60  # d, z in; d, z, perm, two links, c, s out
    # accuracy: sampled problems against the oracle's deflation and reduced solve
    lam = buf["lam"].cpu().numpy()
    V = buf["V"].cpu().numpy().T
    dstat = df["status"].cpu().numpy()
    rng = np.random.default_rng(11)
    pick = sorted(set(rng.choice(batch.nprob, 4, replace=False).tolist()) | {int(np.argmax(sizes))})
    err, dec_ok, aerr = 0.0, True, 0.0
    for p in pick:
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        ref = oracle.deflated_eig(pr.d, pr.z, pr.rho, tau, vectors=(e - a) <= 1500)
        dec_ok &= int(kept[p]) == ref["deflate"]["kept"]
        err = max(err, float(np.abs(lam[a:e] - ref["lam"]).max() / np.abs(ref["lam"]).max()))
        if "Q" in ref:
            aerr = max(aerr, float(np.abs(V[a:e] - ref["Q"].T @ X[a:e]).max() / np.abs(X[a:e]).max()))
    return {
        "config": {"workload": "batched level with deflation: 4096 rank-one problems, n "
                               "log-uniform in [64, 8192], 5% repeated and 10% nearly repeated "
                               "poles, 5% tiny and 1% zero weights, tau = 1e-10, Q^T X for "
                               "16 vectors", "nprob": batch.nprob, "total_n": n, "tau": tau},
        "ms_per_step": ms, "roots_per_s": n / (ms * 1e-3),
        "deflated_fraction": float(1.0 - kept.sum() / n),
        "rule2_rotations": int((df["rot_right"].cpu().numpy() >= 0).sum()),
        "k_deflate": {"ms_per_pass": kd_ms, "launches_per_pass": kd[1] // max(1, args.steps),
                      "algorithmic_bytes_per_pole": bytes_per_pole,
                      "achieved_GBps": bytes_per_pole * n / (kd_ms * 1e-3) / 1e9 if kd_ms else None,
                      "peak_GBps": PEAK_HBM_GBPS},
        "kernels": {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
                    for k, v in sorted(kt.items(), key=lambda kv: -kv[1][0])},
        "accuracy": {"status": int(np.all(dstat == 0)) and int(np.all(s["status"].cpu().numpy() == 0)),
                     "decisions_agree_sampled": bool(dec_ok),
                     "lam_err_rel_normA_sampled": err, "QtX_err_rel_sampled": aerr,
                     "problems_checked": pick},
    }


def bench_ex1(args):
    """The paper's first example end to end: the symmetric tridiagonal matrix with 3 on the
    diagonal and -1 beside it, n = 65536, written as an HSS form of rank 2 (leaf 128).  One
    step: the dividing stage (balanced) and the conquering pass with deflation at the
    paper's tau = 1e-10; the eigenvalues are checked against the closed form
    3 - 2 cos(k pi / (n + 1)) and sampled eigenvectors against the matrix itself."""
    import torch
    from paper_2108_04209_amd import gen, native
    n, leaf = 65536, 128
    tree = gen.tridiag_hss(n, leaf)
    ctx = native.Context()
    plan = native.HSSPlan(ctx, tree.leaf, tree.depth, tree.r)
    dev = torch.device("cuda:0")
    gens = {k: torch.as_tensor(v, dtype=torch.float64, device=dev)
            for k, v in native.pack_hss(tree).items()}
    tau = 1e-10
    o = native.default_opts(persistent=1, fmm_crossover=args.fmm_crossover, fmm_leaf=args.fmm_leaf,
                            hss_tau=tau)
    dv = native.hss_divide(ctx, plan, gens)
    out = native.hss_conquer(ctx, plan, dv, opts=o)

    def step():
        native.hss_divide(ctx, plan, gens, out=dv)
        native.hss_conquer(ctx, plan, dv, opts=o, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    native.hss_set_timing(plan, True)
    native.hss_conquer(ctx, plan, dv, opts=o, out=out)
    phases, _ = native.hss_phase_times(plan)
    native.hss_set_timing(plan, False)
    native.kernel_times()
    native.kernel_timing(True)
    try:
        for _ in range(args.steps):
            native.hss_divide(ctx, plan, gens, out=dv)
        torch.cuda.synchronize()
        kt = native.kernel_times()
    finally:
        native.kernel_timing(False)
    div = kt.get("k_divide", (0.0, 0))
    lam = out["lam"].cpu().numpy()
    exact = np.sort(3.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    rng = np.random.default_rng(5)
    ks = np.sort(np.r_[0, n - 1, rng.choice(n, 30, replace=False)])
    E = np.zeros((len(ks), n))
    E[np.arange(len(ks)), ks] = 1.0
    Qs = native.hss_apply(ctx, plan, torch.as_tensor(E, device=dev), trans=0).cpu().numpy().T
    TQ = 3.0 * Qs
    TQ[:-1] -= Qs[1:]
    TQ[1:] -= Qs[:-1]
    resid = float((np.linalg.norm(TQ - Qs * lam[ks], axis=0) / 5.0).max())
    orth = float(np.abs(Qs.T @ Qs - np.eye(len(ks))).max())
    note(f"ex1 {ms:.2f} ms/step")
    # the paper's range of sizes (8192 .. 262144): time of divide + conquer and accuracy
    sweep = []
    for nn in (8192, 16384, 32768, 65536, 131072, 262144):
        tr = gen.tridiag_hss(nn, leaf)
        pl = native.HSSPlan(ctx, tr.leaf, tr.depth, tr.r)
        gg = {k: torch.as_tensor(v, dtype=torch.float64, device=dev)
              for k, v in native.pack_hss(tr).items()}
        dd = native.hss_divide(ctx, pl, gg)
        oo = native.hss_conquer(ctx, pl, dd, opts=o)  # warm-up: reduced batches, FMM plans
        torch.cuda.synchronize()
        reps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            native.hss_divide(ctx, pl, gg, out=dd)
            native.hss_conquer(ctx, pl, dd, opts=o, out=oo)
        e1.record()
        torch.cuda.synchronize()
        ex = np.sort(3.0 - 2.0 * np.cos(np.arange(1, nn + 1) * np.pi / (nn + 1)))
        sweep.append({"n": nn, "ms": e0.elapsed_time(e1) / reps,
                      "status": int(oo["status"].cpu().numpy()[0]),
                      "lam_err_rel_normA": float(np.abs(oo["lam"].cpu().numpy() - ex).max() / 5.0)})
        del pl, gg, dd, oo
    note("ex1 size sweep done")
    # the paper's accuracy measures on the whole eigenmatrix (its Ex. 1 table): residual
    # gamma = max_k ||A q_k - lambda_k q_k|| / (n ||A||), relative error
    # delta = ||lambda - lambda*|| / (n ||lambda*||) against the closed form, and loss of
    # orthogonality theta = max_k ||Q^T q_k - e_k|| / n; Q is formed column block by column
    # block through the structured eigenmatrix
    acc_table = []
    for nn in (8192, 16384):
        tr = gen.tridiag_hss(nn, leaf)
        pl = native.HSSPlan(ctx, tr.leaf, tr.depth, tr.r)
        gg = {k: torch.as_tensor(v, dtype=torch.float64, device=dev)
              for k, v in native.pack_hss(tr).items()}
        oo = native.hss_conquer(ctx, pl, native.hss_divide(ctx, pl, gg), opts=o)
        lam_t = oo["lam"]
        Q = torch.empty((nn, nn), dtype=torch.float64, device=dev)  # row c = column c of Q
        blk = 2048
        for c0 in range(0, nn, blk):
            E = torch.zeros((blk, nn), dtype=torch.float64, device=dev)
            E[torch.arange(blk, device=dev), torch.arange(c0, c0 + blk, device=dev)] = 1.0
            Q[c0:c0 + blk] = native.hss_apply(ctx, pl, E, trans=0)
        AQ = 3.0 * Q
        AQ[:, :-1] -= Q[:, 1:]
        AQ[:, 1:] -= Q[:, :-1]
        ex = torch.as_tensor(np.sort(3.0 - 2.0 * np.cos(np.arange(1, nn + 1) * np.pi / (nn + 1))),
                             device=dev)
        nA = float(ex.abs().max())
        gamma = float(torch.linalg.norm(AQ - Q * lam_t[:, None], dim=1).max()) / (nn * nA)
        del AQ
        G = Q @ Q.T
        G.diagonal().sub_(1.0)
        theta = float(torch.linalg.norm(G, dim=1).max()) / nn
        delta = float(torch.linalg.norm(lam_t - ex) / (nn * torch.linalg.norm(ex)))
        acc_table.append({"n": nn, "gamma": gamma, "delta": delta, "theta": theta})
        del Q, G, pl, gg, oo
    note("ex1 accuracy table done")
    return {"config": {"workload": "tridiagonal (3 on the diagonal, -1 beside it) as an HSS form "
                                   "of rank 2: n=65536, leaf 128, depth 9; balanced dividing "
                                   "stage + conquering pass with deflation, tau = 1e-10",
                       "n": n, "leaf": leaf,
                       "depth": tree.depth, "r": 2},
            "ms_per_step": ms, "conquer_phase_ms": phases, "divide_ms": div[0] / args.steps,
            "size_sweep": sweep, "accuracy_table": acc_table,
            "divide_launches": div[1] // max(1, args.steps),
            "accuracy": {"status": int(out["status"].cpu().numpy()[0]),
                         "lam_err_rel_normA": float(np.abs(lam - exact).max() / 5.0),
                         "max_resid_rel_normA_sampled": resid, "orth_err_sampled": orth,
                         "eigvecs_checked": len(ks)},
            "tau": tau}


# ---------------------------------------------------------------------------------------
# HSS conquering pass (n = 65536, leaf 128, depth 9, r = 8)
# ---------------------------------------------------------------------------------------
def conquer_flops(tree, iters):
    """Algorithmic FP64 work of one conquer from the per-root evaluation counts."""
    D, r, n = tree.depth, tree.r, tree.n
    sec = vec = app = 0.0
    for lvl in range(D):
        nl = tree.leaf << (D - lvl)
        sec += FLOPS_PER_PAIR * nl * float(np.sum(1.0 + iters[lvl]))
        vec += r * (FLOPS_LOEWNER + FLOPS_BNORM) * n * nl
        ncol = 2 * r if lvl > 0 else r
        for t in range(r):
            m = ncol - t - 1
            if m > 0:
                app += (2 * m + 3) * n * nl + 2 * n * m
    return sec, vec, app


def conquer_kernel_flops(tree, iters, crossover=FMM_CROSSOVER):
    """Algorithmic FP64 flops per kernel of one conquer for the direct kernels, mirroring the
    library's automatic choices: levels with nodes of at least `crossover` roots run
    through the FMM kernels (the solvers' pair evaluations are counted by the library)."""
    D, r, n = tree.depth, tree.r, tree.n
    k = dict(k_secular=0.0, k_loewner=0.0, k_bnorm=0.0, k_apply_mfma=0.0, k_apply_valu=0.0)
    for lvl in range(D):
        nl = tree.leaf << (D - lvl)
        if nl >= crossover:
            continue  # this level's solves, zhat, b and Q^T applies run through the FMM kernels
        k["k_loewner"] += r * FLOPS_LOEWNER * n * nl
        k["k_secular"] += FLOPS_PER_PAIR * nl * float(np.sum(1.0 + iters[lvl]))
        k["k_bnorm"] += r * FLOPS_BNORM * n * nl
        ncol = 2 * r if lvl > 0 else r
        for t in range(r):
            m = ncol - t - 1
            if m > 0:
                key = "k_apply_mfma" if m >= MFMA_MIN_M else "k_apply_valu"
                k[key] += (2 * m + 3) * n * nl + 2 * n * m
    return k


def conquer_cpu_baseline(seconds):
    """The HSS oracle (dense assembly of every node + LAPACK eigenvalues) on the subtree
    rooted at a level-l node of the same tree, the largest that fits the time budget; the
    roots the GPU path solves for that subtree (depth_s * r * n_s) per second."""
    import oracle.hss as ohss
    from paper_2108_04209_amd import gen
    best = None
    for ds in range(2, 7):
        sub = gen.hss_tree(n=128 << ds, leaf=128, r=8, cfg=3)
        t0 = time.perf_counter()
        ohss.level_eigenvalues(sub)
        dt = time.perf_counter() - t0
        best = (ds, sub.n, dt)
        if dt * 8.5 > seconds:   # the next depth costs ~8x (dense O(n^3))
            break
    ds, ns, dt = best
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": ds * 8 * ns / dt, "unit": "roots/s", "cores": cores, "kind": "oracle",
            "sample": f"HSS tree n={ns} (leaf 128, depth {ds}, r 8), same generator: dense "
                      f"assembly of every node and LAPACK eigenvalues, {dt:.1f} s; counted as "
                      f"the {ds * 8 * ns} roots the GPU path solves for that tree"}


def bench_conquer(args):
    import torch
    import oracle.hss as ohss
    from paper_2108_04209_amd import gen, native
    tree = gen.hss_tree()
    ctx = native.Context()
    plan = native.HSSPlan(ctx, tree.leaf, tree.depth, tree.r)
    dev = torch.device("cuda:0")
    gens = {k: torch.as_tensor(v, dtype=torch.float64, device=dev)
            for k, v in native.pack_hss(tree).items()}
    opts1 = native.default_opts(persistent=1, fmm_crossover=args.fmm_crossover,
                                fmm_leaf=args.fmm_leaf)
    out = native.hss_conquer(ctx, plan, gens, opts=opts1)
    native.hss_set_timing(plan, True)

    def timed(opts, steps, warm):
        for _ in range(warm):
            native.hss_conquer(ctx, plan, gens, opts=opts, out=out)
        torch.cuda.synchronize()
        tot, phases = [], {k: 0.0 for k in native.HSS_PHASES}
        counts = None
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            native.hss_conquer(ctx, plan, gens, opts=opts, out=out)
            e1.record()
            torch.cuda.synchronize()
            tot.append(e0.elapsed_time(e1))
            ph, counts = native.hss_phase_times(plan)
            for k in phases:
                phases[k] += ph[k] / steps
        return float(np.mean(tot)), phases, counts

    ms, phases, counts = timed(opts1, args.steps, args.warmup)
    note(f"conquer batched {ms:.2f} ms/step")
    status = int(out["status"].cpu().numpy()[0])
    it_raw = native.hss_iterations(plan).cpu().numpy()
    iters = (it_raw & ITER_COUNT_MASK).astype(np.float64)
    lam = out["lam"].cpu().numpy()
    sec_f, vec_f, app_f = conquer_flops(tree, iters)
    roots = tree.depth * tree.r * tree.n

    # ablation of the local shifting (Sec. 4.2.2): the same conquer with the iterate kept as
    # lambda itself; per level, the largest share over the r rank-one steps of roots that
    # needed more than 5 iterations, and the eigenvalues against the shifted run
    abl = None
    if not args.no_level:
        o_un = native.default_opts(persistent=1, fmm_crossover=args.fmm_crossover,
                                   fmm_leaf=args.fmm_leaf, unshifted=1)
        un = native.hss_conquer(ctx, plan, gens, opts=o_un)
        torch.cuda.synchronize()
        it_un = native.hss_iterations(plan).cpu().numpy()
        lam_un = un["lam"].cpu().numpy()
        abl = {"levels_n": [int(tree.leaf << (tree.depth - l)) for l in range(tree.depth)],
               "mu_definition": MU_DEFINITION,
               "mu_percent_shifted": mu_levels(it_raw), "mu_percent_unshifted": mu_levels(it_un),
               "mu_percent_count_only_shifted": mu_levels(it_raw, count_only=True),
               "mu_percent_count_only_unshifted": mu_levels(it_un, count_only=True),
               "unmet_percent_shifted": unmet_levels(it_raw),
               "unmet_percent_unshifted": unmet_levels(it_un),
               "status_unshifted": int(un["status"].cpu().numpy()[0]),
               "nonfinite_unshifted": int(np.count_nonzero(~np.isfinite(lam_un)))}
        fin = np.isfinite(lam_un)
        abl["max_lam_diff_rel_normA_finite"] = (
            float(np.abs(lam_un[fin] - lam[fin]).max() / np.abs(lam).max()) if fin.any() else None)
        # the hybrid interpolation of [li93] (middle way and fixed weight) in place of the
        # middle way alone, with local shifting
        o_hy = native.default_opts(persistent=1, fmm_crossover=args.fmm_crossover,
                                   fmm_leaf=args.fmm_leaf, interp=1)
        native.hss_conquer(ctx, plan, gens, opts=o_hy)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        hy = native.hss_conquer(ctx, plan, gens, opts=o_hy)
        e1.record()
        torch.cuda.synchronize()
        it_hy = native.hss_iterations(plan).cpu().numpy()
        abl["hybrid_li93"] = {"mu_percent": mu_levels(it_hy),
                              "mean_iters": float((it_hy & ITER_COUNT_MASK).mean()),
                              "mean_iters_middle_way": float(iters.mean()),
                              "ms_per_step": e0.elapsed_time(e1),
                              "status": int(hy["status"].cpu().numpy()[0]),
                              "max_lam_diff_rel_normA": float(np.abs(hy["lam"].cpu().numpy() - lam).max()
                                                              / np.abs(lam).max())}
        native.hss_conquer(ctx, plan, gens, opts=opts1, out=out)  # restore the shifted state
        torch.cuda.synchronize()
    # graph replay of the same step (timing events off while capturing)
    graph_ms = None
    native.hss_set_timing(plan, False)
    try:
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            native.hss_conquer(ctx, plan, gens, opts=opts1, out=out)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            native.hss_conquer(ctx, plan, gens, opts=opts1, out=out)
        g.replay()
        torch.cuda.synchronize()
        glam = out["lam"].cpu().numpy()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        graph_ms = {"ms_per_step": e0.elapsed_time(e1) / args.steps,
                    "replay_equals_eager": bool(np.array_equal(glam, lam))}
    except Exception as exc:  # report, do not hide
        graph_ms = f"capture failed: {exc!r}"
    # per-kernel timing pass (phase events off)
    native.kernel_timing(True)
    for _ in range(args.steps):
        native.hss_conquer(ctx, plan, gens, opts=opts1, out=out)
    torch.cuda.synchronize()
    kt = native.kernel_times()
    kw = native.kernel_work()
    native.kernel_timing(False)
    kflops = conquer_kernel_flops(tree, iters, args.fmm_crossover or FMM_CROSSOVER)
    for k in ("k_secular", "k_secular_fmm"):  # the solvers count their pair evaluations
        if k in kw:
            kflops[k] = FLOPS_PER_PAIR * kw[k] / args.steps
    kernels, roofline = kernel_roofline(kt, kflops, args.steps, "conquer")
    native.hss_set_timing(plan, True)

    # accuracy: trace identity and sampled eigenpair residuals with the oracle's product
    nA = float(np.abs(lam).max())
    tr_err = abs(lam.sum() - ohss.trace(tree)) / (tree.n * nA)
    rng = np.random.default_rng(5)
    ks = np.sort(np.r_[0, tree.n - 1, rng.choice(tree.n, 30, replace=False)])
    E = np.zeros((len(ks), tree.n))
    E[np.arange(len(ks)), ks] = 1.0
    Qs = native.hss_apply(ctx, plan, torch.as_tensor(E, device=dev), trans=0).cpu().numpy().T
    resid = float((np.linalg.norm(ohss.matvec(tree, Qs) - Qs * lam[ks], axis=0) / nA).max())
    orth = float(np.abs(Qs.T @ Qs - np.eye(len(ks))).max())

    plain_res = None
    if args.plain_steps > 0:
        p_ms, p_ph, _ = timed(native.default_opts(persistent=0, fmm_crossover=args.fmm_crossover,
                                                  fmm_leaf=args.fmm_leaf),
                              args.plain_steps, 1)
        plain_res = {"ms_per_step": p_ms, "value": roots / (p_ms * 1e-3),
                     "phase_ms": p_ph, "steps": args.plain_steps,
                     "launches": "one per node per phase"}

    cfg = {"workload": "HSS conquering pass: n=65536, leaf 128, depth 9, rank 8 "
                       "(8 sequential rank-one updates per node), FP64, all nodes of a level "
                       "batched per call",
           "n": tree.n, "leaf": tree.leaf, "depth": tree.depth, "r": tree.r,
           "rank_one_roots_per_step": roots}
    res = {
        "metric": METRIC, "value": roots / (ms * 1e-3), "unit": "roots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators, no dataset)", "config": cfg,
        "secular_roots_per_s": roots / (phases["secular"] * 1e-3),
        # the dense (2m + 3) n_l^2 work of every apply over the apply phase's time: levels whose
        # nodes reach the FMM crossover do far less work than counted here
        "apply_gflops_direct_equivalent": app_f / (phases["apply"] * 1e-3) / 1e9,
        "phase_ms": phases, "phase_intervals": counts, "kernels": kernels,
        "mean_iters_after_midpoint": float(iters.mean()), "max_iters": int(iters.max()),
        "graph": graph_ms,
        "ablation_unshifted": abl,
        "plain": plain_res,
        "speedup_batched_vs_plain": None if plain_res is None else plain_res["ms_per_step"] / ms,
        "accuracy": {"status": status, "trace_err_rel": tr_err,
                     "max_resid_rel_normA_sampled": resid, "orth_err_sampled": orth,
                     "eigvecs_checked": len(ks)},
        "roofline": roofline,
    }
    note("conquer graph/accuracy/plain done")
    if not args.no_cpu:
        res["cpu_baseline"] = conquer_cpu_baseline(args.cpu_seconds)
        note("conquer cpu baseline done")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "the path has no multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        x = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        note(f"calibration copy of {CALIB_BYTES} bytes done")
        del x, y
    if args.workload == "conquer":
        res = bench_conquer(args)
        if not args.no_level:
            lv = bench_level(argparse.Namespace(**{**vars(args), "no_cpu": True}), "level")
            res["level"] = {k: lv[k] for k in ("config", "value", "ms_per_step",
                                               "secular_roots_per_s", "apply_gflops",
                                               "phase_ms", "kernels", "graph_ms_per_step", "plain",
                                               "speedup_batched_vs_plain", "accuracy",
                                               "roofline")}
            res["large"] = bench_large(argparse.Namespace(**{**vars(args), "steps": min(args.steps, 5)}))
            res["deflate"] = bench_deflate(argparse.Namespace(**{**vars(args), "steps": min(args.steps, 5)}))
            res["ex1"] = bench_ex1(argparse.Namespace(**{**vars(args), "steps": min(args.steps, 5)}))
    elif args.workload == "deflate":
        dfl = bench_deflate(args)
        res = {"metric": METRIC, "value": dfl["roots_per_s"], "unit": "roots/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": dfl["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic (seeded generators, no dataset)", **dfl}
    elif args.workload == "ex1":
        ex = bench_ex1(args)
        res = {"metric": METRIC, "value": 2 * (ex["config"]["depth"]) * ex["config"]["n"] / (ex["ms_per_step"] * 1e-3),
               "unit": "roots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": ex["ms_per_step"], "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f64", "data": "synthetic (closed-form matrix)", **ex}
    elif args.workload == "large":
        lg = bench_large(args)
        ms = lg[lg["faster"]]["ms_per_step"]
        res = {"metric": METRIC, "value": lg["value"], "unit": "roots/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic (seeded generators, no dataset)", **lg}
    else:
        res = bench_level(args, args.workload)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
