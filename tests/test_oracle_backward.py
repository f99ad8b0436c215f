"""Pins of the oracle's adjoint (d lambda, d p against d, z, rho) by closed forms,
central finite differences and torch.linalg.eigh autograd on the dense matrix.

Closed forms (A = diag(d) + rho z z^T, eigenpairs (lambda_k, q_k), p_k = q_k^T u):
  L = sum lambda_k         = tr A        -> dL/dd = 1, dL/dz = 2 rho z, dL/drho = ||z||^2
  L = sum lambda_k^2       = ||A||_F^2   -> dL/dd = 2(d + rho z^2),
                                            dL/dz = 4 rho d*z + 4 rho^2 ||z||^2 z,
                                            dL/drho = 2 sum d z^2 + 2 rho ||z||^4
  L = sum lambda_k p_k^2   = u^T A u     -> dL/dd = u^2, dL/dz = 2 rho (z.u) u, dL/drho = (z.u)^2
  L = sum p_k^2            = ||u||^2     -> all zero
The third exercises both the eigenvalue and the eigenvector parts of the adjoint.
"""
import numpy as np
import pytest
import torch

from paper_2108_04209_amd import gen
from tests import refcheck


def forward(orc, d, z, rho):
    lam, eta, org, its, st = orc.secular(d, z, rho)
    assert st == 0
    zh = orc.loewner(d, z, rho, eta, org)
    b = orc.bnorm(d, zh, eta, org)
    return lam, eta, org, zh, b


def proj(orc, d, zh, b, eta, org, u):
    return orc.cauchy_apply(d, zh, b, eta, org, u.reshape(-1, 1), trans=1)[:, 0]


def problem(n, seed, rho=None):
    g = gen.rng_for(950, seed)
    pr = gen.uniform_problem(n, g, rho=rho if rho is not None else g.uniform(0.1, 2.0), gap=1e-3)
    u = g.standard_normal(n)
    return pr, u, g


@pytest.mark.parametrize("n", [1, 2, 17, 100])
def test_closed_forms(orc, n):
    pr, u, _ = problem(n, n)
    d, z, rho = pr.d, pr.z, pr.rho
    lam, eta, org, zh, b = forward(orc, d, z, rho)
    p = proj(orc, d, zh, b, eta, org, u)
    zz = z @ z
    tol = 1e-11

    gd, gz, gr = orc.backward(d, z, rho, eta, org, g_lam=np.ones(n))
    np.testing.assert_allclose(gd, np.ones(n), atol=tol)
    np.testing.assert_allclose(gz, 2 * rho * z, atol=tol)
    assert gr == pytest.approx(zz, rel=tol)

    gd, gz, gr = orc.backward(d, z, rho, eta, org, g_lam=2 * lam)
    np.testing.assert_allclose(gd, 2 * (d + rho * z * z), atol=tol)
    np.testing.assert_allclose(gz, 4 * rho * d * z + 4 * rho ** 2 * zz * z, atol=tol)
    assert gr == pytest.approx(2 * np.sum(d * z * z) + 2 * rho * zz ** 2, rel=tol)

    zu = z @ u
    gd, gz, gr = orc.backward(d, z, rho, eta, org, g_lam=p * p, g_proj=2 * lam * p, u=u)
    np.testing.assert_allclose(gd, u * u, atol=1e-9)
    np.testing.assert_allclose(gz, 2 * rho * zu * u, atol=1e-9)
    assert gr == pytest.approx(zu ** 2, rel=1e-9, abs=1e-9)

    gd, gz, gr = orc.backward(d, z, rho, eta, org, g_proj=2 * p, u=u)
    np.testing.assert_allclose(gd, 0, atol=1e-9)
    np.testing.assert_allclose(gz, 0, atol=1e-9)
    assert abs(gr) <= 1e-9


def loss(orc, d, z, rho, u, wl, wp):
    lam, eta, org, zh, b = forward(orc, d, z, rho)
    p = proj(orc, d, zh, b, eta, org, u)
    return float(wl @ lam + wp @ (p * p))


@pytest.mark.parametrize("n,seed", [(12, 0), (40, 1), (96, 2)])
def test_central_fd(orc, n, seed):
    pr, u, g = problem(n, 100 + seed)
    d, z, rho = pr.d, pr.z, pr.rho
    wl = g.standard_normal(n)
    wp = g.standard_normal(n)
    lam, eta, org, zh, b = forward(orc, d, z, rho)
    p = proj(orc, d, zh, b, eta, org, u)
    gd, gz, gr = orc.backward(d, z, rho, eta, org, g_lam=wl, g_proj=2 * wp * p, u=u)
    # direction that keeps d sorted: |h v_d| <= 1% of the adjacent gaps
    gaps = np.diff(d)
    room = np.minimum(np.r_[gaps, np.inf], np.r_[np.inf, gaps])
    for trial in range(3):
        vd = g.standard_normal(n)
        vz = g.standard_normal(n)
        vr = g.standard_normal()
        h = 1e-6
        scale = min(1.0, 0.01 * room.min() / (h * np.abs(vd).max()))
        vd *= scale
        Lp = loss(orc, d + h * vd, z + h * vz, rho + h * vr, u, wl, wp)
        Lm = loss(orc, d - h * vd, z - h * vz, rho - h * vr, u, wl, wp)
        fd = (Lp - Lm) / (2 * h)
        an = gd @ vd + gz @ vz + gr * vr
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * (np.abs(gd) @ np.abs(vd) + np.abs(gz) @ np.abs(vz)))


@pytest.mark.parametrize("n,seed", [(8, 0), (64, 1)])
def test_torch_eigh(orc, n, seed):
    pr, u, g = problem(n, 200 + seed)
    wl = g.standard_normal(n)
    wp = g.standard_normal(n)
    d = torch.tensor(pr.d, dtype=torch.float64, requires_grad=True)
    z = torch.tensor(pr.z, dtype=torch.float64, requires_grad=True)
    rho = torch.tensor(pr.rho, dtype=torch.float64, requires_grad=True)
    A = torch.diag(d) + rho * torch.outer(z, z)
    A = 0.5 * (A + A.T)
    w, V = torch.linalg.eigh(A)
    p = V.T @ torch.tensor(u)
    L = torch.tensor(wl) @ w + torch.tensor(wp) @ (p * p)
    L.backward()
    lam, eta, org, zh, b = forward(orc, pr.d, pr.z, pr.rho)
    pp = proj(orc, pr.d, zh, b, eta, org, u)
    gd, gz, gr = orc.backward(pr.d, pr.z, pr.rho, eta, org, g_lam=wl, g_proj=2 * wp * pp, u=u)
    ref = np.r_[d.grad.numpy(), z.grad.numpy(), rho.grad.numpy()]
    got = np.r_[gd, gz, gr]
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()
