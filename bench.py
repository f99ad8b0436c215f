#!/usr/bin/env python3
"""Benchmark of the conquering-stage hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload conquer|level|large|single|deflate|ex1|grad]

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
ITER_COUNT_MASK, ITER_UNMET, ITER_CAP, ITER_SKIPPED = 0xFFFF, 1 << 16, 1 << 17, 1 << 18

MU_DEFINITION = ("per level, the largest share over the r rank-one steps of roots that needed "
                 "more than 5 iterations after the midpoint pass, or whose iteration ended on "
                 "a step below rounding or a collapsed bracket (or the cap) before the "
                 "stopping test held")


def _per_level(bad, lam_ok):
    """Per level, the largest share (percent) over the steps of the flagged roots among the
    roots of problems that were solved (lam_ok: not skipped for invalid input); None for a
    level with no solved problem."""
    out = []
    for l in range(bad.shape[0]):
        v = [float(100.0 * np.mean(bad[l, t][lam_ok[l, t]])) for t in range(bad.shape[1])
             if lam_ok[l, t].any()]
        out.append(max(v) if v else None)
    return out


def mu_levels(it, count_only=False):
    """The share mu (percent) of roots not converged within 5 iterations, per level, from
    iteration records of shape (depth, r, n), over the roots of the problems solved."""
    lam_ok = (it & ITER_SKIPPED) == 0
    cnt = it & ITER_COUNT_MASK
    bad = cnt > 5 if count_only else (cnt > 5) | ((it & (ITER_UNMET | ITER_CAP)) != 0)
    return _per_level(bad, lam_ok)


def unmet_levels(it):
    """Per level, the largest share (percent) over the steps of roots whose iteration ended
    before the stopping test held, over the roots of the problems solved."""
    return _per_level((it & (ITER_UNMET | ITER_CAP)) != 0, (it & ITER_SKIPPED) == 0)
MFMA_MIN_M = 4           # the library's automatic VALU/MFMA apply switch (columns)


MFMA_KERNELS = ("k_apply_mfma", "k_fmmv_eval_mfma")  # FP64 matrix-core kernels
APPLY_KERNELS = ("k_apply_mfma", "k_apply_valu", "k_fmmv_eval_mfma", "k_fmmv_eval")
SOLVER_KERNELS = ("k_secular", "k_secular_fmm")


def kernel_peak(name):
    return PEAK_FP64_MFMA if name in MFMA_KERNELS else PEAK_FP64_VALU


def counted_flops(kw, steps):
    """Algorithmic flops per step from the library's device counters: the solvers count
    pole-root pair evaluations (7 flops each), the apply and FMM evaluation kernels count
    their algorithmic flops directly."""
    out = {}
    for k, v in kw.items():
        if k in SOLVER_KERNELS:
            out[k] = FLOPS_PER_PAIR * v / steps
        elif k in APPLY_KERNELS:
            out[k] = v / steps
    return out


def collect_counters(native):
    """The library's device counters since the last collection: work per kernel (for
    counted_flops) and, per solver, the share of wavefront lanes that held a live root over
    all of its passes."""
    kc = native.kernel_counters()
    kw = {k: v[0] for k, v in kc.items()}
    lanes = {k: v[1] / v[2] for k, v in kc.items() if k in SOLVER_KERNELS and v[2] > 0}
    return kw, lanes


def kernel_pass(native, run, steps, counters=True):
    """Per-kernel measurement in two passes of `steps` steps each: HIP events alone (the
    kernel times; no counter atomics in the kernels), then the device counters alone (the
    work; skipped with counters=False, so that every launch of a profiled run is one of the
    timed kind).  Returns ({kernel: (ms, launches)}, work, live-lane fractions)."""
    import torch
    native.kernel_times()  # drop anything recorded before
    native.kernel_timing(True, mode="events")
    kw, lanes = {}, {}
    try:
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        kt = native.kernel_times()
        if counters:
            native.kernel_timing(True, mode="counters")
            for _ in range(steps):
                run()
            torch.cuda.synchronize()
            kw, lanes = collect_counters(native)
    finally:
        native.kernel_timing(False)
    return kt, kw, lanes


def kernel_roofline(kt, flops, steps, workload=None):
    """Per-kernel table and the roofline object of the dominant kernel.

    kt: {kernel: (ms, launches)} from the library's per-kernel HIP-event timing over
    `steps` steps; flops: {kernel: algorithmic FP64 flops per step} for the kernels whose
    work has an algorithmic count.  Every such kernel gets its achieved rate and its
    fraction of its own peak (the FP64 matrix peak for the MFMA kernels, the FP64 vector
    peak otherwise).  The dominant kernel is the one with the largest time per step among
    them."""
    table = {}
    for name, (ms, nl) in sorted(kt.items(), key=lambda x: -x[1][0]):
        e = {"ms_per_step": ms / steps, "launches_per_step": nl / steps,
             "avg_launch_ms": ms / nl}
        if name in flops and flops[name] > 0 and ms > 0:
            a = flops[name] / (ms / steps * 1e-3) / 1e12
            e["algorithmic_tflops"] = a
            e["peak_tflops"] = kernel_peak(name)
            e["frac"] = a / kernel_peak(name)
            e["bound"] = "mfma" if name in MFMA_KERNELS else "alu"
        table[name] = e
    cand = [k for k in table if "frac" in table[k]]
    if not cand:
        return table, None
    dom = max(cand, key=lambda k: table[k]["ms_per_step"])
    e = table[dom]
    roof = {"bound": e["bound"], "achieved": e["algorithmic_tflops"], "peak": e["peak_tflops"],
            "unit": "TFLOP/s", "frac": e["frac"],
            "traffic": kernel_traffic(dom, workload) if workload else None,
            "kernel": dom, "launches_per_step": e["launches_per_step"],
            "avg_launch_ms": e["avg_launch_ms"],
            "algorithmic_flops_per_launch": flops[dom] / e["launches_per_step"],
            "timing": "HIP events around each launch on its stream (library kernel timing)"}
    return table, roof


def apply_summary(table):
    """The apply half of the metric: every Cauchy-apply kernel's algorithmic rate and its
    fraction of its peak, and the whole apply's rate (their flops over their time)."""
    ks = {k: table[k] for k in APPLY_KERNELS if k in table and "frac" in table[k]}
    if not ks:
        return None
    fl = sum(v["algorithmic_tflops"] * v["ms_per_step"] for v in ks.values())
    ms = sum(v["ms_per_step"] for v in ks.values())
    return {"kernels": {k: {"algorithmic_tflops": v["algorithmic_tflops"], "frac": v["frac"],
                            "peak_tflops": v["peak_tflops"], "ms_per_step": v["ms_per_step"]}
                        for k, v in ks.items()},
            "algorithmic_tflops": fl / ms, "ms_per_step": ms,
            "count": "device counters: (2m + 3) flops per Cauchy entry (pole or equivalent "
                     "source against root, m columns including a fused b) plus the output "
                     "scaling"}


def counted_fp64(workload, kt_table):
    """The rocprof-counted FP64 rate of the solvers, from the committed instruction-mix
    summary profiles/<workload>_instruction_mix.md (per-step FP64 flops from the
    SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 counters, 64 lanes per wave instruction, an FMA
    as 2), over this run's measured kernel time; None if the summary is missing or the
    kernels' sources changed since it was taken."""
    fields = _profile_fields(os.path.join(PROFILES, f"{workload}_instruction_mix.md"))
    if not fields:
        return None
    out = {}
    for k in SOLVER_KERNELS:
        key = f"{k}_fp64_flops_per_step"
        if key in fields and k in kt_table:
            f = float(fields[key])
            out[k] = {"counted_tflops": f / (kt_table[k]["ms_per_step"] * 1e-3) / 1e12,
                      "frac_vector_peak": f / (kt_table[k]["ms_per_step"] * 1e-3) / 1e12 / PEAK_FP64_VALU,
                      "algorithmic_tflops": kt_table[k].get("algorithmic_tflops")}
    return out or None


CALIB_BYTES = 512 << 20  # the calibration copy: this many bytes read and written
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2108_04209_amd", "csrc")


def _profile_fields(path):
    """The "- key: value" lines of a committed summary, or None if it is missing or the
    sources it names changed since it was taken (their SHA-256 is recorded in it)."""
    import hashlib
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    try:
        h = hashlib.sha256()
        for f in fields["sources"].split(","):
            h.update(open(os.path.join(CSRC, f.strip()), "rb").read())
        if h.hexdigest() != fields["sources_sha256"]:
            return None
    except (KeyError, OSError):
        return None
    return fields


def kernel_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` in `workload` from the committed counter summary
    profiles/<kernel>_<workload>_traffic.md (FETCH_SIZE + WRITE_SIZE, each scaled by the
    same counter's reading for a copy of known size), or None if there is none or the
    kernel's sources changed since it was taken."""
    fields = _profile_fields(os.path.join(PROFILES, f"{kernel}_{workload}_traffic.md"))
    try:
        return float(fields["hbm_bytes_per_launch"]) if fields else None
    except (KeyError, ValueError):
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
                    choices=["conquer", "level", "large", "single", "deflate", "ex1", "grad"])
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
    ap.add_argument("--tune-cache", default=None,
                    help="file that keeps the autotuner's choices between runs (the library's "
                         "SUPERDC_TUNE_CACHE); a run that finds its shapes there does not tune")
    ap.add_argument("--profile", action="store_true",
                    help="the run a kernel-trace profile wraps (conquer): tuned launch shapes "
                         "only (no heuristic-shape timing) and no device-counter pass, so the "
                         "profiler's per-kernel averages cover the launches bench.py times")
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
    # the heuristic launch shapes first, then the autotuner's on the same data
    h_wall, h_tot, h_ph = time_steps(pipe, args.steps, args.warmup)
    heur = {"ms_per_step": float(np.mean(h_tot)), "shapes": pipe.native.batch_shapes(pipe.b)}
    tuned_shapes = pipe.native.autotune(pipe.ctx, pipe.b, pipe.d, pipe.z, pipe.rho, opts=pipe.opts)
    wall_ms, tot_ms, ph = time_steps(pipe, args.steps, args.warmup)
    note(f"{name} batched {float(np.mean(tot_ms)):.2f} ms/step (heuristic shapes "
         f"{heur['ms_per_step']:.2f})")
    iters = (pipe.out["iters"].cpu().numpy() & ITER_COUNT_MASK).astype(np.float64)
    status_ok = bool(np.all(pipe.out["status"].cpu().numpy() == 0))
    ms = float(np.mean(tot_ms))
    solve_ms, vec_ms, apply_ms = (float(x) for x in ph.mean(axis=0))

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

    # per-kernel timing and work
    kt, kw, lanes = kernel_pass(pipe.native, pipe.step, args.steps)
    # Loewner and b by direct sums serve the problems below the FMM crossover only; the
    # solvers and the apply kernels count their work on the device
    small = sizes[sizes < (args.fmm_crossover or FMM_CROSSOVER)]
    n2d = float(np.sum(small ** 2))
    kflops = {"k_loewner": FLOPS_LOEWNER * n2d, "k_bnorm": FLOPS_BNORM * n2d}
    kflops.update(counted_flops(kw, args.steps))
    kernels, roofline = kernel_roofline(kt, kflops, args.steps, name)
    res = {
        "metric": METRIC, "value": tot / (ms * 1e-3), "unit": "roots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators, no dataset)", "config": cfg,
        "secular_roots_per_s": tot / (solve_ms * 1e-3),
        "apply": apply_summary(kernels),
        "active_lane_fraction": lanes,
        "phase_ms": {"solve": solve_ms, "loewner_b": vec_ms, "apply": apply_ms},
        "autotune": {"tuned_shapes": tuned_shapes, "tuned_ms_per_step": ms,
                     "heuristic": heur},
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
    # per-kernel timing of the FMM run, with the device-counted work
    kt, kw, lanes = kernel_pass(pf.native, pf.step, args.steps)
    kernels, roofline = kernel_roofline(kt, counted_flops(kw, args.steps), args.steps)
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
    best = min(("fmm", "direct"), key=lambda k: out[k]["ms_per_step"])
    return {
        "config": {"workload": "single rank-one problem n=65536, clustered poles, "
                               "64 right-hand sides, FMM order 16 leaf 256 vs direct",
                   "n": n, "m": int(m)},
        "value": out[best]["roots_per_s"], "faster": best, "fmm": out["fmm"],
        "direct": out["direct"], "fmm_kernels": kernels, "fmm_roofline": roofline,
        "fmm_active_lane_fraction": lanes,
        "fmm_apply": apply_summary(kernels),
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
    native.kernel_timing(True, mode="events")
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
    native.kernel_timing(True, mode="events")
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


FLOPS_BWD_PAIR = 29  # adjoint with projections: 12 per pair in the roots pass, 17 in the poles pass


def bench_grad(args):
    """The differentiation workload: 1024 problems, n uniform in [256, 4096].  One step is
    the forward pass (solve, Loewner/b, projections p = Qhat^T u) and the backward pass of
    the loss sum_k wl_k lambda_k + sum_k wp_k p_k^2 through the hand-written adjoint
    (superdc_secular_backward: dlambda/d(d, z, rho) and the projection terms), all through
    the C ABI on preallocated buffers."""
    import torch
    import oracle
    from paper_2108_04209_amd import gen, native
    full = gen.cfg4()
    dev = torch.device("cuda:0")
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    ctx = native.Context()
    b = native.Batch(ctx, full.off)
    d, z, rho = f(full.d), f(full.z), f(full.rho)
    u, wl, wp = f(full.extra["u"]), f(full.extra["wl"]), f(full.extra["wp"])
    tot, P = full.total_n, full.nprob
    o = native.default_opts()
    sol = dict(lam=torch.empty(tot, dtype=torch.float64, device=dev),
               eta=torch.empty(tot, dtype=torch.float64, device=dev),
               origin=torch.empty(tot, dtype=torch.int32, device=dev),
               iters=torch.empty(tot, dtype=torch.int32, device=dev),
               status=torch.empty(P, dtype=torch.int32, device=dev))
    zb = (torch.empty(tot, dtype=torch.float64, device=dev),
          torch.empty(tot, dtype=torch.float64, device=dev))
    pr_ = torch.empty((1, tot), dtype=torch.float64, device=dev)
    gp = torch.empty(tot, dtype=torch.float64, device=dev)
    g = (torch.empty(tot, dtype=torch.float64, device=dev),
         torch.empty(tot, dtype=torch.float64, device=dev),
         torch.empty(P, dtype=torch.float64, device=dev))
    u2 = u.view(1, -1)

    def forward():
        native.secular_solve(ctx, b, d, z, rho, opts=o, out=sol)
        native.loewner(ctx, b, d, z, rho, sol["eta"], sol["origin"], sol["status"], opts=o, out=zb)
        native.cauchy_apply(ctx, b, d, zb[0], zb[1], sol["eta"], sol["origin"], sol["status"],
                            u2, trans=1, opts=o, Y=pr_)

    def backward():
        torch.mul(pr_.view(-1), wp, out=gp).mul_(2.0)  # dL/dp = 2 wp p
        native.secular_backward(ctx, b, d, z, rho, sol["eta"], sol["origin"], sol["status"],
                                g_lam=wl, g_proj=gp, u=u, opts=o, out=g)

    for _ in range(args.warmup):
        forward()
        backward()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for e in ev:
        e[0].record()
        forward()
        e[1].record()
        backward()
        e[2].record()
    torch.cuda.synchronize()
    fw = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    bw = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    note(f"grad forward {fw:.2f} ms, backward {bw:.2f} ms")
    def fwd_bwd():
        forward()
        backward()

    kt, kw, lanes = kernel_pass(native, fwd_bwd, args.steps)
    sizes = full.sizes().astype(np.float64)
    n2 = float(np.sum(sizes ** 2))
    small = sizes[sizes < FMM_CROSSOVER]
    kflops = {"k_bwd": FLOPS_BWD_PAIR * n2, "k_loewner": FLOPS_LOEWNER * float(np.sum(small ** 2)),
              "k_bnorm": FLOPS_BNORM * float(np.sum(small ** 2))}
    kflops.update(counted_flops(kw, args.steps))
    kernels, roofline = kernel_roofline(kt, kflops, args.steps)
    # gradients of a seeded sample of problems against the oracle's adjoint, fed the
    # oracle's own forward
    gd, gz, gr = (x.cpu().numpy() for x in g)
    err = 0.0
    for p in np.random.default_rng(3).choice(P, 3, replace=False):
        a, e = int(full.off[p]), int(full.off[p + 1])
        pr = full.problem(p)
        lam, eta, org, its, st = oracle.secular(pr.d, pr.z, pr.rho)
        zh = oracle.loewner(pr.d, pr.z, pr.rho, eta, org)
        bb = oracle.bnorm(pr.d, zh, eta, org)
        pp = oracle.cauchy_apply(pr.d, zh, bb, eta, org, full.extra["u"][a:e], trans=1)[:, 0]
        od, oz, orr = oracle.backward(pr.d, pr.z, pr.rho, eta, org, g_lam=full.extra["wl"][a:e],
                                      g_proj=2 * full.extra["wp"][a:e] * pp, u=full.extra["u"][a:e])
        sc = max(np.abs(od).max(), np.abs(oz).max())
        err = max(err, float(np.abs(gd[a:e] - od).max() / sc), float(np.abs(gz[a:e] - oz).max() / sc),
                  float(abs(gr[p] - orr) / max(abs(orr), sc)))
    ms = fw + bw
    return {"config": {"workload": "differentiation batch: 1024 rank-one problems, n uniform in "
                                   "[256, 4096], FP64, loss sum wl lambda + sum wp (q^T u)^2, "
                                   "forward + hand-written adjoint",
                       "nprob": P, "total_n": tot},
            "ms_per_step": ms, "roots_per_s": tot / (ms * 1e-3),
            "forward_ms": fw, "backward_ms": bw, "kernels": kernels, "roofline": roofline,
            "grad_err_rel_vs_oracle_sampled": err,
            "status_all_ok": bool(np.all(sol["status"].cpu().numpy() == 0))}


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


CPU_SAMPLE_FRAC = 0.02  # share of each stand-in problem's roots (and poles) the oracle runs


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def conquer_cpu_sample(frac=CPU_SAMPLE_FRAC):
    """The oracle (plain FP64 C, OpenMP over roots) on the rank-one problems of the HSS
    conquer (n = 65536, leaf 128, depth 9, r = 8): per level l, 2^l problems of n / 2^l
    roots, each solved r times with an apply of Qhat^T to m = 2r - t - 1 columns at step t
    (r - t - 1 at the root).  One seeded stand-in problem per level (the single-problem
    generator at that size) is run on a seeded `frac` of its roots (at least 256, so all
    the roots of the smallest levels): the solve on those
    roots, Loewner's zhat on as many poles, b and the apply on as many rows.  Loewner, b
    and the apply cost a fixed number of operations per pole-root pair, so they run with
    interval midpoints as stand-in roots.  Every time is scaled linearly to the whole
    level (roots are independent given the poles) and summed: seconds per conquer."""
    import oracle
    from paper_2108_04209_amd import gen
    oracle.load()
    n, depth, r = 65536, 9, 8
    rng = np.random.default_rng(17)
    levels, total = [], 0.0
    for lvl in range(depth):
        nl, count = n >> lvl, 1 << lvl
        pr = gen.uniform_problem(nl, gen.rng_for(6, lvl), rho=1.0, gap=1e-6)
        k = min(nl, max(int(round(frac * nl)), 256))  # at least 256 roots (all of small ones)
        idx = np.sort(rng.choice(nl, k, replace=False))
        scale = nl / k
        t0 = time.perf_counter()
        oracle.secular(pr.d, pr.z, pr.rho, roots=idx)
        t_solve = time.perf_counter() - t0
        org = np.arange(nl, dtype=np.int32)
        eta = np.empty(nl)
        eta[:-1] = 0.5 * np.diff(pr.d)
        eta[-1] = 0.5 * pr.rho * float(pr.z @ pr.z)
        t0 = time.perf_counter()
        oracle.loewner(pr.d, pr.z, pr.rho, eta, org, poles=idx)
        oracle.bnorm(pr.d, pr.z, eta, org, roots=idx)
        t_vec = time.perf_counter() - t0
        ncol = 2 * r if lvl > 0 else r
        t_app = 0.0
        for t in range(r):
            m = ncol - t - 1
            if m <= 0:
                continue
            X = rng.standard_normal((nl, m))
            t0 = time.perf_counter()
            oracle.cauchy_apply(pr.d, pr.z, pr.z, eta, org, X, trans=1, rows=idx)
            t_app += time.perf_counter() - t0
        lvl_s = count * scale * (r * (t_solve + t_vec) + t_app)
        levels.append({"n": nl, "problems": count, "sampled_roots": k,
                       "sample_s": t_solve + t_vec + t_app, "extrapolated_s": lvl_s})
        total += lvl_s
    return {"conquer_s": total, "levels": levels}


def conquer_cpu_baseline():
    """conquer_cpu_sample on all host threads and on one (a child process with
    OMP_NUM_THREADS=1), as rank-one roots per second of the whole conquer."""
    import subprocess
    roots = 9 * 8 * 65536
    allc = conquer_cpu_sample()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = None
    try:
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample-conquer"],
                             env=env, capture_output=True, text=True, timeout=600, check=True)
        one = json.loads(out.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError) as exc:
        one = {"error": repr(exc)}
    res = {"value": roots / allc["conquer_s"], "unit": "roots/s", "cores": cores,
           "kind": "oracle",
           "sample": f"the C oracle on one seeded stand-in rank-one problem per conquer level "
                     f"(n = 65536 ... 256), {CPU_SAMPLE_FRAC:.0%} of its roots (at least 256): solve, Loewner "
                     f"zhat and b on as many poles and roots, Q^T applied to the level's "
                     f"m = 2r - t - 1 columns on as many rows; extrapolated linearly to the "
                     f"2^l problems x 8 steps of every level (EXTRAPOLATED)",
           "extrapolated": True, "conquer_s": allc["conquer_s"], "levels": allc["levels"],
           "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count()}
    if "conquer_s" in one:
        res["one_core"] = {"value": roots / one["conquer_s"], "unit": "roots/s", "cores": 1,
                           "conquer_s": one["conquer_s"]}
    else:
        res["one_core"] = one
    return res


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

    def timed(opts, steps, warm):
        # the timed steps run without the phase events (a few hundred event records a step,
        # about a millisecond); the phase breakdown comes from as many passes after them
        native.hss_set_timing(plan, False)
        for _ in range(warm):
            native.hss_conquer(ctx, plan, gens, opts=opts, out=out)
        torch.cuda.synchronize()
        tot = []
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            native.hss_conquer(ctx, plan, gens, opts=opts, out=out)
            e1.record()
            torch.cuda.synchronize()
            tot.append(e0.elapsed_time(e1))
        native.hss_set_timing(plan, True)
        phases, counts = {k: 0.0 for k in native.HSS_PHASES}, None
        for _ in range(steps):
            native.hss_conquer(ctx, plan, gens, opts=opts, out=out)
            torch.cuda.synchronize()
            ph, counts = native.hss_phase_times(plan)
            for k in phases:
                phases[k] += ph[k] / steps
        native.hss_set_timing(plan, False)
        return float(np.mean(tot)), phases, counts

    # the heuristic launch shapes first, then every level's batch tuned on its own problems
    h_ms = None if args.profile else timed(opts1, args.steps, args.warmup)[0]
    tuned_shapes = native.hss_autotune(ctx, plan, gens, opts=opts1)
    ms, phases, counts = timed(opts1, args.steps, args.warmup)
    note(f"conquer batched {ms:.2f} ms/step (heuristic shapes {h_ms})")
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
               "skipped_percent_unshifted": [float(100.0 * np.mean((it_un[l] & ITER_SKIPPED) != 0))
                                             for l in range(it_un.shape[0])],
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
                              "unmet_percent": unmet_levels(it_hy),
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
    # per-kernel timing and work (phase events off)
    kt, kw, lanes = kernel_pass(native, lambda: native.hss_conquer(ctx, plan, gens, opts=opts1,
                                                                   out=out), args.steps,
                                counters=not args.profile)
    kflops = conquer_kernel_flops(tree, iters, args.fmm_crossover or FMM_CROSSOVER)
    kflops.update(counted_flops(kw, args.steps))  # solvers and apply kernels: device counts
    kernels, roofline = kernel_roofline(kt, kflops, args.steps, "conquer")

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
        "apply": apply_summary(kernels),
        "counted_fp64": counted_fp64("hss_conquer_n65536", kernels),
        "active_lane_fraction": lanes,
        "autotune": {"tuned_ms_per_step": ms, "heuristic_ms_per_step": h_ms,
                     "tuned_shapes_per_level": tuned_shapes},
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
        res["cpu_baseline"] = conquer_cpu_baseline()
        note("conquer cpu baseline done")
    return res


def main():
    if "--cpu-sample-conquer" in sys.argv:  # child of conquer_cpu_baseline: CPU only
        print(json.dumps(conquer_cpu_sample()), flush=True)
        return
    args = parse()
    if args.tune_cache:
        os.environ["SUPERDC_TUNE_CACHE"] = args.tune_cache
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
                                               "secular_roots_per_s", "apply", "autotune",
                                               "phase_ms", "kernels", "graph_ms_per_step", "plain",
                                               "active_lane_fraction",
                                               "speedup_batched_vs_plain", "accuracy",
                                               "roofline")}
            res["large"] = bench_large(argparse.Namespace(**{**vars(args), "steps": min(args.steps, 5)}))
            res["deflate"] = bench_deflate(argparse.Namespace(**{**vars(args), "steps": min(args.steps, 5)}))
            res["ex1"] = bench_ex1(argparse.Namespace(**{**vars(args), "steps": min(args.steps, 5)}))
            res["grad"] = bench_grad(argparse.Namespace(**{**vars(args), "steps": min(args.steps, 5)}))
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
    elif args.workload == "grad":
        gr = bench_grad(args)
        res = {"metric": METRIC, "value": gr["roots_per_s"], "unit": "roots/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": gr["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic (seeded generators, no dataset)", **gr}
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
