"""The allocation-free solve (superdc_secular_solve_noalloc) against the regular entry
point with direct sums, through the C ABI.

Both run the same kernels with the same launch shapes, so every output must agree bit for
bit; the per-call buffers of the allocation-free variant live in one fixed device array
that keeps the last call's contents, so two calls in a row -- the second on a smaller
batch -- must each agree with the regular call on the same input.  Argument errors that
the host can see (a batch above the array's capacity, the FMM method) are refused before
any work is enqueued.
"""
import numpy as np
import pytest

from paper_2108_04209_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve_pair(ctx, batch, persistent):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    b = native.Batch(ctx, batch.off)
    d, z, rho = gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho)
    o = native.default_opts(method=1, persistent=persistent)
    reg = native.secular_solve(ctx, b, d, z, rho, opts=o)
    na = native.secular_solve_noalloc(ctx, b, d, z, rho, opts=o)
    torch.cuda.synchronize()
    return b, reg, na


@pytest.mark.parametrize("persistent", [1, 0])
def test_noalloc_matches_regular_twice(persistent):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    ctx = native.Context()
    first = gen.small_batch([1024, 70, 3000, 64, 1, 513], seed=71)
    second = gen.small_batch([300, 9, 128], seed=72)   # smaller: stale contents above it
    for name, batch in (("first", first), ("second", second)):
        print(f"noalloc {name}: {batch.nprob} problems, total {batch.total_n}, "
              f"persistent {persistent}", flush=True)
        _, reg, na = _solve_pair(ctx, batch, persistent)
        for k in ("lam", "eta", "origin", "iters", "status"):
            assert torch.equal(reg[k], na[k]), (name, k)
        assert int(na["status"].abs().sum()) == 0
    # against the oracle as well, on one problem of each call
    import oracle
    for batch in (first, second):
        _, _, na = _solve_pair(ctx, batch, persistent)
        lam = na["lam"].cpu().numpy()
        p = int(np.argmax(batch.sizes()))
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        ol = oracle.secular(pr.d, pr.z, pr.rho)[0]
        assert np.abs(lam[a:e] - ol).max() <= 1e-12 * np.abs(ol).max()


def test_noalloc_refuses_what_it_cannot_hold():
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    ctx = native.Context()
    lib = native.load_library()
    dummy = gp.to_dev(np.zeros(8))
    idummy = torch.zeros(8, dtype=torch.int32, device=gp.dev())
    p = lambda t: native._ptr(t)
    # a batch larger than the fixed array: refused on the host, nothing enqueued
    big = native.Batch(ctx, np.array([0, 3_000_000, 4_000_001], dtype=np.int64))
    o = native.default_opts(method=1)
    rc = lib.superdc_secular_solve_noalloc(ctx.handle, big.handle, p(dummy), p(dummy), p(dummy),
                                           p(dummy), p(dummy), p(idummy), None, p(idummy),
                                           native.C.byref(o), native._stream(None))
    assert rc == -1
    small = native.Batch(ctx, np.array([0, 8], dtype=np.int64))
    o2 = native.default_opts(method=2)
    rc = lib.superdc_secular_solve_noalloc(ctx.handle, small.handle, p(dummy), p(dummy), p(dummy),
                                           p(dummy), p(dummy), p(idummy), None, p(idummy),
                                           native.C.byref(o2), native._stream(None))
    assert rc == -1
    torch.cuda.synchronize()


def test_noalloc_graph_replay():
    """Captured into a graph after one eager call, every replay equals the eager result."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    ctx = native.Context()
    batch = gen.small_batch([2048, 500, 64, 1500], seed=73)
    b = native.Batch(ctx, batch.off)
    d, z, rho = gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho)
    o = native.default_opts(method=1)
    tot, P = batch.total_n, batch.nprob
    out = dict(lam=torch.empty(tot, dtype=torch.float64, device=gp.dev()),
               eta=torch.empty(tot, dtype=torch.float64, device=gp.dev()),
               origin=torch.empty(tot, dtype=torch.int32, device=gp.dev()),
               iters=torch.empty(tot, dtype=torch.int32, device=gp.dev()),
               status=torch.empty(P, dtype=torch.int32, device=gp.dev()))
    native.secular_solve_noalloc(ctx, b, d, z, rho, opts=o, out=out)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in out.items()}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        native.secular_solve_noalloc(ctx, b, d, z, rho, opts=o, out=out)
    for rep in range(3):
        for v in out.values():
            v.fill_(-3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in eager.items():
            assert torch.equal(out[k], v), (rep, k)
