"""Graph capture of the batched path.

A batched step -- every problem of a level solved, ẑ and b formed, and the eigenvector
matrix applied, one persistent launch per phase -- allocates nothing and never waits for
the host after a warm-up call of its shape, so it can be captured into a hipGraph (through
torch.cuda.graph, on the capture stream the binding passes).  Every replay must give the
eager result bit for bit: the persistent work queues reset themselves at the end of each
launch, so a replay starts from zero without any memset.  The replays are interleaved with
eager calls on the same context and buffers, and with host synchronisations, and each
replay is checked on its own after its outputs were overwritten.
"""
import numpy as np
import pytest

from paper_2108_04209_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _capture(step):
    """Warm up on a side stream, then capture one step."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    return g


def _snapshot(bufs):
    return {k: v.clone() for k, v in bufs.items()}


def _scramble(bufs):
    for v in bufs.values():
        if v.dtype == torch.float64:
            v.fill_(float("nan"))
        else:
            v.fill_(-7)


def _check_replays(g, step, bufs, eager, reps=3):
    for rep in range(reps):
        _scramble(bufs)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in eager.items():
            assert torch.equal(bufs[k], v), (rep, k)
        # eager work on the same context and buffers between the replays
        step()
        torch.cuda.synchronize()
        for k, v in eager.items():
            assert torch.equal(bufs[k], v), ("eager", rep, k)


def test_level_graph_replay():
    """A mixed level (sizes log-uniform in [64, 4096], a quarter of them above the FMM
    crossover): solve -> Loewner/b -> Qhat^T X and Qhat X captured as one graph."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    rng = np.random.default_rng(31)
    sizes = np.round(np.exp(rng.uniform(np.log(64), np.log(4096), 96))).astype(int)
    sizes[:3] = [4096, 1024, 2000]
    batch, X = gen.small_batch(sizes.tolist(), seed=31, m=16)
    print(f"graph level: {batch.nprob} problems, total {batch.total_n}", flush=True)
    ctx = native.Context()
    b = native.Batch(ctx, batch.off)
    d, z, rho = gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho)
    Xt = gp.to_dev(np.asarray(X).T)
    tot, P = batch.total_n, batch.nprob
    dev = gp.dev()
    bufs = dict(lam=torch.empty(tot, dtype=torch.float64, device=dev),
                eta=torch.empty(tot, dtype=torch.float64, device=dev),
                origin=torch.empty(tot, dtype=torch.int32, device=dev),
                iters=torch.empty(tot, dtype=torch.int32, device=dev),
                status=torch.empty(P, dtype=torch.int32, device=dev),
                zhat=torch.empty(tot, dtype=torch.float64, device=dev),
                b=torch.empty(tot, dtype=torch.float64, device=dev),
                Y1=torch.empty_like(Xt), Y0=torch.empty_like(Xt))
    o = native.default_opts(persistent=1)
    sol = {k: bufs[k] for k in ("lam", "eta", "origin", "iters", "status")}

    def step():
        native.secular_solve(ctx, b, d, z, rho, opts=o, out=sol)
        native.loewner(ctx, b, d, z, rho, bufs["eta"], bufs["origin"], bufs["status"], opts=o,
                       out=(bufs["zhat"], bufs["b"]))
        native.cauchy_apply(ctx, b, d, bufs["zhat"], bufs["b"], bufs["eta"], bufs["origin"],
                            bufs["status"], Xt, trans=1, opts=o, Y=bufs["Y1"])
        native.cauchy_apply(ctx, b, d, bufs["zhat"], bufs["b"], bufs["eta"], bufs["origin"],
                            bufs["status"], bufs["Y1"], trans=0, opts=o, Y=bufs["Y0"])

    step()
    torch.cuda.synchronize()
    eager = _snapshot(bufs)
    assert int(eager["status"].abs().sum()) == 0
    # the round trip Qhat (Qhat^T X) = X: the eager result is a valid one
    assert float((eager["Y0"] - Xt).abs().max()) <= 1e-12 * float(Xt.abs().max()) * 10
    g = _capture(step)
    _check_replays(g, step, bufs, eager)


def test_conquer_graph_replay():
    """A whole HSS conquering pass (n = 4096, leaf 128, r = 8, depth 5; the top two levels
    through the FMM) captured as one graph, with every level's eigenvalues."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    tree = gen.hss_tree(n=4096, leaf=128, r=8, cfg=3)
    print("graph conquer: n=4096 leaf 128 r 8", flush=True)
    ctx = native.Context()
    plan = native.HSSPlan(ctx, tree.leaf, tree.depth, tree.r)
    gens = {k: gp.to_dev(v) for k, v in native.pack_hss(tree).items()}
    dev = gp.dev()
    bufs = dict(lam=torch.empty(tree.n, dtype=torch.float64, device=dev),
                lam_levels=torch.empty((tree.depth + 1, tree.n), dtype=torch.float64, device=dev),
                status=torch.empty(1, dtype=torch.int32, device=dev))
    o = native.default_opts(persistent=1)

    def step():
        native.hss_conquer(ctx, plan, gens, opts=o, out=bufs)

    step()
    torch.cuda.synchronize()
    eager = _snapshot(bufs)
    assert int(eager["status"][0]) == 0
    g = _capture(step)
    _check_replays(g, step, bufs, eager)
    # the structured eigenmatrix left by a replay is the eager one
    E = torch.eye(tree.n, dtype=torch.float64, device=dev)[:64].contiguous()
    _scramble(bufs)
    g.replay()
    Qg = native.hss_apply(ctx, plan, E, trans=0)
    torch.cuda.synchronize()
    step()
    Qe = native.hss_apply(ctx, plan, E, trans=0)
    torch.cuda.synchronize()
    assert torch.equal(Qg, Qe)
