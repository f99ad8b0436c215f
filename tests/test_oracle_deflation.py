"""Pins of the oracle's deflation (Remark 1) against facts fixed by the mathematics.

The paper prints no deflation example, so the pins are:
  - a worked 3 x 3 case solved by hand (two equal poles, all of z equal to one);
  - tau = 0 deflates nothing;
  - exact zeros of z and exactly repeated poles deflate with no perturbation at all, so
    the spectrum must match LAPACK's to rounding;
  - for any tau the deflated matrix Qhat-side reconstruction differs from A by a
    perturbation whose norm the two rules bound, so Weyl's inequality bounds every
    eigenvalue error; the full eigenvector matrix is orthogonal and diagonalises the
    deflated matrix;
  - structural invariants: kept poles strictly increasing, perm a permutation, rotation
    links consistent, every rule-2 off-diagonal entry below tau.
"""
import numpy as np
import pytest

from paper_2108_04209_amd import gen

EPS = np.finfo(np.float64).eps


def dense(d, z, rho):
    return np.diag(d) + rho * np.outer(z, z)


def test_worked_3x3(orc):
    # A = diag(0, 0, 1) + 1 1^T: the equal poles rotate with c = s = 1/sqrt(2); pole 0
    # deflates with eigenvalue 0 (eigenvector (1, -1, 0)/sqrt(2)), the reduced problem is
    # diag(0, 1) + (sqrt 2, 1)(sqrt 2, 1)^T with eigenvalues 2 -+ sqrt(2).
    d, z = np.array([0.0, 0.0, 1.0]), np.array([1.0, 1.0, 1.0])
    r = orc.deflated_eig(d, z, 1.0, 1e-10)
    df = r["deflate"]
    assert df["kept"] == 2
    assert list(df["perm"]) == [1, 2, 0]
    assert list(df["rright"]) == [1, -1, -1] and list(df["rleft"]) == [-1, 0, -1]
    assert df["c"][0] == pytest.approx(np.sqrt(0.5), rel=2 * EPS)
    assert df["s"][0] == pytest.approx(np.sqrt(0.5), rel=2 * EPS)
    assert np.allclose(df["d"], [0.0, 1.0, 0.0], atol=0.0)
    assert df["z"][0] == pytest.approx(np.sqrt(2.0), rel=2 * EPS) and df["z"][1] == 1.0
    want = [2.0 - np.sqrt(2.0), 2.0 + np.sqrt(2.0), 0.0]
    assert np.abs(r["lam"] - want).max() <= 8 * EPS
    v = r["Q"][:, 2]
    assert np.abs(np.abs(v) - [np.sqrt(0.5), np.sqrt(0.5), 0.0]).max() <= 4 * EPS
    assert v[0] * v[1] < 0


def test_tau_zero_is_identity(orc):
    g = gen.rng_for(900, 0)
    pr = gen.uniform_problem(200, g, rho=0.7)
    df = orc.deflate(pr.d, pr.z, pr.rho, 0.0)
    assert df["kept"] == 200
    assert (df["perm"] == np.arange(200)).all()
    assert (df["rright"] == -1).all() and (df["rleft"] == -1).all()
    assert (df["d"] == pr.d).all() and (df["z"] == pr.z).all()


@pytest.mark.parametrize("seed", range(3))
def test_exact_cases_match_lapack(orc, seed):
    # zeros of z and repeated poles: the rules act with nothing dropped
    g = gen.rng_for(901, seed)
    n = 60
    d = np.sort(g.uniform(-1, 1, n))
    rep = g.random(n) < 0.2
    for i in range(1, n):
        if rep[i]:
            d[i] = d[i - 1]
    z = g.standard_normal(n)
    z[g.random(n) < 0.1] = 0.0
    rho = 1.3
    r = orc.deflated_eig(d, z, rho, 1e-300)
    assert r["status"] == 0
    df = r["deflate"]
    assert df["kept"] < n
    A = dense(d, z, rho)
    nrm = np.abs(np.linalg.eigvalsh(A)).max()
    assert np.abs(np.sort(r["lam"]) - np.linalg.eigvalsh(A)).max() <= 64 * EPS * nrm
    Q = r["Q"]
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 64 * EPS
    assert np.abs(Q.T @ A @ Q - np.diag(r["lam"])).max() <= 64 * EPS * nrm
    # a deflated zero of z returns its own pole exactly
    for j in range(df["kept"], n):
        i = df["perm"][j]
        if z[i] == 0.0:
            assert df["d"][j] == d[i]


@pytest.mark.parametrize("tau", [1e-12, 1e-9, 1e-6])
@pytest.mark.parametrize("seed", range(3))
def test_weyl_bound_and_orthogonality(orc, tau, seed):
    g = gen.rng_for(902, seed)
    pr = gen.deflation_problem(150, g, rho=g.uniform(0.1, 2.0))
    d, z, rho = pr.d, pr.z, pr.rho
    r = orc.deflated_eig(d, z, rho, tau)
    assert r["status"] == 0
    df = r["deflate"]
    n, k = d.size, df["kept"]
    v = np.sqrt(rho) * z
    nv = np.linalg.norm(v)
    # the perturbation each rule drops: rule 1 removes v_k's coupling, rule 2 an
    # off-diagonal entry cs (d_a - d_b) of size below tau
    rule2 = df["rright"] >= 0
    rule1 = np.zeros(n, dtype=bool)
    rule1[df["perm"][k:]] = True
    rule1 &= ~rule2
    bound = np.sum(2.0 * np.abs(v[rule1]) * nv + v[rule1] ** 2) + tau * np.count_nonzero(rule2)
    A = dense(d, z, rho)
    ev = np.linalg.eigvalsh(A)
    nrm = np.abs(ev).max()
    assert np.abs(np.sort(r["lam"]) - ev).max() <= bound + 1e-13 * nrm
    Q = r["Q"]
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-13
    # Q diagonalises A up to the dropped perturbation
    assert np.abs(Q.T @ A @ Q - np.diag(r["lam"])).max() <= bound + 1e-13 * nrm


@pytest.mark.parametrize("tau", [1e-10, 1e-7])
def test_structure(orc, tau):
    g = gen.rng_for(903, 0)
    pr = gen.deflation_problem(3000, g, rho=0.9)
    df = orc.deflate(pr.d, pr.z, pr.rho, tau)
    n, k = pr.n, df["kept"]
    assert 0 < k < n
    assert (np.diff(df["d"][:k]) > 0).all()
    assert (df["z"][k:] == 0.0).all() and (df["z"][:k] != 0.0).all()
    assert np.array_equal(np.sort(df["perm"]), np.arange(n))
    assert (np.diff(df["perm"][k:]) > 0).all() and (np.diff(df["perm"][:k]) > 0).all()
    for a in np.nonzero(df["rright"] >= 0)[0]:
        b = df["rright"][a]
        assert b > a and df["rleft"][b] == a
        c, s = df["c"][a], df["s"][a]
        assert abs(c * c + s * s - 1.0) <= 4 * EPS
    # rule 1 exactly where |sqrt(rho) z| < tau
    v = np.sqrt(pr.rho) * pr.z
    defl = np.zeros(n, dtype=bool)
    defl[df["perm"][k:]] = True
    assert (defl[np.abs(v) < tau]).all()
    # chains: runs of repeated poles rotate one into the next
    assert np.count_nonzero((df["rright"] >= 0) & (df["rleft"] >= 0)) > 0


def test_expand_roundtrip(orc):
    g = gen.rng_for(904, 0)
    pr = gen.deflation_problem(80, g, rho=1.1)
    df = orc.deflate(pr.d, pr.z, pr.rho, 1e-9)
    X = g.standard_normal((80, 3))
    Y = orc.deflate_expand(df, X, 0)
    assert np.abs(orc.deflate_expand(df, Y, 1) - X).max() <= 1e-14
    assert np.linalg.norm(Y) == pytest.approx(np.linalg.norm(X), rel=1e-14)
