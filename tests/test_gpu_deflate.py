"""GPU parity of deflation (Remark 1) against the CPU oracle, through the C ABI.

Bars:
  decisions     kept counts, placements (perm) and rotation links identical: both sides
                evaluate the rule-2 test and the rotation with the same FP64 expressions in
                the same order, without fused multiply-adds
  values        deflated eigenvalues, reduced poles and weights, rotation c and s: bit for
                bit (the same expressions; FP64 square root and division are correctly
                rounded on both sides)
  eigenvalues   full pipeline (deflate, reduced solve) within 1e-12 ||A||_2 of the oracle's
  Q X, Q^T X    within 1e-12 of the oracle's dense Q applied to X, relative to ||X||
"""
import numpy as np
import pytest

from paper_2108_04209_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [1, 2, 3, 63, 64, 65, 200, 777, 1500, 4100]


def ulps(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    scale = np.maximum(np.spacing(np.abs(a)), np.spacing(np.abs(b)))
    return np.where(a == b, 0.0, np.abs(a - b) / scale)


@pytest.mark.parametrize("tau", [1e-10, 1e-7, 0.0])
def test_deflate_matches_oracle(orc, tau):
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    batch = gen.deflation_batch(SIZES, seed=1)
    ctx = gp.context()
    b = native.Batch(ctx, batch.off)
    df = native.deflate(ctx, b, gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho), tau)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in df.items()}
    assert (g["status"] == 0).all()
    for p in range(batch.nprob):
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        ref = orc.deflate(pr.d, pr.z, pr.rho, tau)
        assert g["kept"][p] == ref["kept"], p
        for k, r in (("perm", "perm"), ("rot_right", "rright"), ("rot_left", "rleft")):
            assert np.array_equal(g[k][a:e], ref[r]), (p, k)
        for k, r in (("d", "d"), ("z", "z"), ("rot_c", "c"), ("rot_s", "s")):
            assert ulps(g[k][a:e], ref[r]).max() == 0, (p, k)
        if tau == 0.0:
            assert ref["kept"] == e - a


def test_deflate_edge_cases(orc):
    """every pole deflated by rule 1, all poles equal (one chain), invalid inputs"""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    probs = [gen.RankOne(np.linspace(0, 1, 100), np.zeros(100), 1.0),
             gen.RankOne(np.full(130, 0.25), np.ones(130) / np.sqrt(130), 2.0),
             gen.RankOne(np.array([0.0, 1.0, 0.5]), np.ones(3), 1.0),
             gen.RankOne(np.array([0.0, 1.0]), np.array([1.0, np.nan]), 1.0),
             gen.RankOne(np.array([0.0, 1.0]), np.ones(2), -1.0)]
    batch = gen.concat(probs)
    ctx = gp.context()
    b = native.Batch(ctx, batch.off)
    df = native.deflate(ctx, b, gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho), 1e-12)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in df.items()}
    assert list(g["status"][:2]) == [0, 0]
    assert g["kept"][0] == 0 and g["kept"][1] == 1
    # one chain through all 130 equal poles: every link, the survivor the last pole
    a = int(batch.off[1])
    assert np.array_equal(g["rot_right"][a:a + 129], np.arange(1, 130))
    assert g["z"][a] == pytest.approx(np.linalg.norm(probs[1].z), rel=1e-14)
    ref = orc.deflate(probs[1].d, probs[1].z, probs[1].rho, 1e-12)
    assert ulps(g["z"][a:a + 130], ref["z"]).max() == 0
    st = g["status"]
    assert st[2] & 1  # decreasing d
    assert st[3] & 4  # non-finite z
    assert st[4] & 8  # rho <= 0


@pytest.mark.parametrize("tau", [1e-10, 1e-6])
def test_deflated_pipeline(orc, tau):
    from tests import gpu_pipeline as gp
    batch, X = gen.deflation_batch([5, 64, 300, 1000], seed=2, m=6)
    res = gp.deflated_run(batch, tau, X=X)
    assert (res["dstatus"] == 0).all() and (res["rstatus"] == 0).all()
    for p in range(batch.nprob):
        a, e = int(batch.off[p]), int(batch.off[p + 1])
        pr = batch.problem(p)
        ref = orc.deflated_eig(pr.d, pr.z, pr.rho, tau, vectors=True)
        nA = np.abs(ref["lam"]).max()
        assert np.abs(res["lam"][a:e] - ref["lam"]).max() <= 1e-12 * nA, p
        Q = ref["Q"]
        Xp = X[a:e]
        nx = np.abs(Xp).max()
        assert np.abs(res["Y0"][a:e] - Q @ Xp).max() <= 1e-12 * nx * np.sqrt(e - a), p
        assert np.abs(res["Y1"][a:e] - Q.T @ Xp).max() <= 1e-12 * nx * np.sqrt(e - a), p


def test_deflated_pipeline_large(orc):
    """n = 20000 with many clusters: eigenvalues on sampled positions, orthogonality by
    the round trip Q^T (Q X) = X on the GPU"""
    from tests import gpu_pipeline as gp
    batch, X = gen.deflation_batch([20000], seed=3, m=4)
    res = gp.deflated_run(batch, 1e-10, X=X)
    assert (res["dstatus"] == 0).all() and (res["rstatus"] == 0).all()
    pr = batch.problem(0)
    df = orc.deflate(pr.d, pr.z, pr.rho, 1e-10)
    assert res["kept"][0] == df["kept"]
    k = df["kept"]
    # deflated eigenvalues are the deflation's own values; reduced roots against the oracle's
    # solver on sampled roots
    assert ulps(res["lam"][k:], df["d"][k:]).max() == 0
    rng = np.random.default_rng(0)
    roots = np.sort(rng.choice(k, size=min(k, 200), replace=False))
    lam_or = orc.secular(df["d"][:k], df["z"][:k], pr.rho, roots=roots)[0]
    nA = max(abs(df["d"][0]), abs(df["d"][k - 1]) + pr.rho * float(np.sum(df["z"][:k] ** 2)))
    assert np.abs(res["lam"][roots] - lam_or).max() <= 1e-12 * nA
    # Q^T (Q X) = X through the GPU path
    Y = res["Y0"]
    back = gp.deflated_run(batch, 1e-10, X=Y)["Y1"]
    assert np.abs(back - X).max() <= 1e-11 * np.abs(X).max()


def test_deflate_across_scan_segments(orc):
    """Problems longer than one segment of the parallel scan: a chain of 5000 equal poles
    that runs through every segment end (each join must rescan the next segment from the
    incoming pole), and long clustered problems, against the oracle's sequential scan,
    decisions and values bit for bit."""
    from paper_2108_04209_amd import native
    from tests import gpu_pipeline as gp
    g = gen.rng_for(905, 0)
    probs = [gen.RankOne(np.full(5000, 0.5), np.abs(g.standard_normal(5000)) + 0.1, 1.0)]
    for n in (9000, 4097, 6144):
        probs.append(gen.deflation_problem(n, g, rho=float(g.uniform(0.2, 2.0))))
    batch = gen.concat(probs)
    ctx = gp.context()
    b = native.Batch(ctx, batch.off)
    for tau in (1e-10, 1e-6):
        df = native.deflate(ctx, b, gp.to_dev(batch.d), gp.to_dev(batch.z), gp.to_dev(batch.rho), tau)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in df.items()}
        assert (res["status"] == 0).all()
        for p, pr in enumerate(probs):
            a, e = int(batch.off[p]), int(batch.off[p + 1])
            ref = orc.deflate(pr.d, pr.z, pr.rho, tau)
            assert res["kept"][p] == ref["kept"], (p, tau)
            for k, r in (("perm", "perm"), ("rot_right", "rright"), ("rot_left", "rleft")):
                assert np.array_equal(res[k][a:e], ref[r]), (p, k, tau)
            for k, r in (("d", "d"), ("z", "z"), ("rot_c", "c"), ("rot_s", "s")):
                assert ulps(res[k][a:e], ref[r]).max() == 0, (p, k, tau)
    assert res["kept"][0] == 1  # the whole chain ends in one survivor
