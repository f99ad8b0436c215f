"""The autotuner picks shapes in range, the tuned batch still matches the oracle, and the
cache file reproduces the choice in a new batch of the same sizes."""
import numpy as np
import pytest

from paper_2108_04209_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_autotune_and_cache(orc, tmp_path, monkeypatch):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    monkeypatch.setenv("SUPERDC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    sizes = [4096, 3000, 777, 64, 2048, 1500] * 8
    batch = gen.small_batch(sizes, seed=71, kind="uniform")
    ctx = gp.context()
    b = native.Batch(ctx, batch.off)
    d, z, rho = gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho)
    sh = native.autotune(ctx, b, d, z, rho)
    assert sh["sec_chunk"] in (64, 128, 256, 512)
    assert sh["sec_split"] in (1, 2, 4, 8, 16)
    assert sh["vec_split"] in (1, 2, 4, 8, 16) and sh["bwd_split"] in (1, 2, 4, 8, 16)
    assert sh["fmm_split"] in (1, 2, 4, 8)  # problems of 1024 roots and more use the FMM
    res = native.secular_solve(ctx, b, d, z, rho)
    torch.cuda.synchronize()
    lam = res["lam"].cpu().numpy()
    assert (res["status"].cpu().numpy() == 0).all()
    for p in range(batch.nprob):
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        ol, oe, oo, oi, os_ = orc.secular(pr.d, pr.z, pr.rho)
        assert np.abs(lam[a:e] - ol).max() <= 1e-12 * np.abs(ol).max()
    # a second batch of the same sizes reads the cached shapes
    b2 = native.Batch(ctx, batch.off)
    assert native.autotune(ctx, b2, d, z, rho) == sh
    lines = (tmp_path / "tune.txt").read_text().split("\n")
    assert len([x for x in lines if x.strip()]) == 1


def test_kernel_timing():
    """Per-kernel timing brackets each launch: one solve gives one validation and one
    solver launch with positive durations; with timing off nothing is collected."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    batch = gen.small_batch([300, 1200], seed=72)
    ctx = gp.context()
    b = native.Batch(ctx, batch.off)
    d, z, rho = gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho)
    native.kernel_times()  # drop anything collected before
    native.kernel_timing(True)
    try:
        res = native.secular_solve(ctx, b, d, z, rho, opts=native.default_opts(method=1))
        kt = native.kernel_times()
        kw = native.kernel_work()
    finally:
        native.kernel_timing(False)
    assert kt["k_validate"][1] == 1 and kt["k_secular"][1] == 1
    assert kt["k_secular"][0] > 0.0
    # the solver's pair count: every pass (the midpoint pass and each iteration) of every
    # root sums over all n_p poles
    its = res["iters"].cpu().numpy().astype(np.int64) & native.ITER_COUNT_MASK
    want = sum(int(batch.off[p + 1] - batch.off[p]) * int(np.sum(1 + its[batch.off[p]:batch.off[p + 1]]))
               for p in range(batch.nprob))
    assert kw["k_secular"] == want
    native.secular_solve(ctx, b, d, z, rho)
    torch.cuda.synchronize()
    assert native.kernel_times() == {}


def test_device_counters():
    """The counters alone (no events): the direct Cauchy apply counts (2m + 3) flops per
    matrix entry plus 2m per output row, exactly; the solver's live-lane count covers every
    pass of every root and never exceeds the lanes its wavefronts had; the events alone
    record times and no work."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    batch, X = gen.small_batch([300, 1200, 64, 77], seed=74, m=5)
    ctx = gp.context()
    b = native.Batch(ctx, batch.off)
    d, z, rho = gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho)
    o = native.default_opts(method=1, apply_kernel=2)
    s = native.secular_solve(ctx, b, d, z, rho, opts=o)
    zh, bn = native.loewner(ctx, b, d, z, rho, s["eta"], s["origin"], s["status"], opts=o)
    Xt = gp.to_dev(np.asarray(X).T)
    torch.cuda.synchronize()
    native.kernel_times()
    native.kernel_timing(True, mode="counters")
    try:
        res = native.secular_solve(ctx, b, d, z, rho, opts=o)
        native.cauchy_apply(ctx, b, d, zh, bn, s["eta"], s["origin"], s["status"], Xt, trans=1,
                            opts=o)
        kc = native.kernel_counters()
        kt = native.kernel_times()
    finally:
        native.kernel_timing(False)
    assert kt == {}  # no events were recorded
    n = np.diff(batch.off).astype(np.int64)
    m = X.shape[1]
    assert kc["k_apply_mfma"][0] == float(np.sum(n * n * (2 * m + 3) + 2 * n * m))
    its = res["iters"].cpu().numpy().astype(np.int64) & native.ITER_COUNT_MASK
    work, live, slots = kc["k_secular"]
    assert live >= np.sum(1 + its) and 0 < live <= slots
    native.kernel_timing(True, mode="events")
    try:
        native.secular_solve(ctx, b, d, z, rho, opts=o)
        kt = native.kernel_times()
        kw = native.kernel_work()
    finally:
        native.kernel_timing(False)
    assert kt["k_secular"][1] == 1 and kw == {}
