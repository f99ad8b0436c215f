"""Seeded synthetic inputs for diagonal-plus-rank-one eigenproblems and HSS conquer passes.

The rank-one problem is diag(d) + rho * z z^T with d strictly increasing (Sec. 2.2,
eq. rank1upd, with v = sqrt(rho) z).  The HSS inputs are the generators of Sec. 2.1
(eq. hss) for a perfect binary tree.

This module only draws random numbers and lays them out.  It is shared by the CPU
oracle and the HIP path and contains none of the method's arithmetic: no secular
sums, no Loewner products, no eigenvector formulas.

Every draw comes from numpy's PCG64 seeded by SeedSequence([210804209, cfg, index]),
so the same (cfg, index) always gives the same arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 210804209


def rng_for(cfg: int, index: int = 0) -> np.random.Generator:
    """Independent stream for workload `cfg`, item `index`."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([MASTER_SEED, cfg, index])))


# ----------------------------------------------------------------------------------------
# single rank-one problems
# ----------------------------------------------------------------------------------------

@dataclass
class RankOne:
    d: np.ndarray          # float64[n], strictly increasing poles
    z: np.ndarray          # float64[n], update vector
    rho: float             # > 0

    @property
    def n(self) -> int:
        return int(self.d.shape[0])


def gapped_uniform(g: np.random.Generator, n: int, lo: float, hi: float, gap: float) -> np.ndarray:
    """Sorted uniform points on [lo, hi) with every neighbour gap >= `gap`.

    Sorted uniforms u are lifted as u*(1-(n-1)*gap') + i*gap' on the unit interval,
    then mapped to [lo, hi); gap' is `gap` expressed on the unit interval.
    """
    u = np.sort(g.random(n))
    unit_gap = gap / (hi - lo)
    if (n - 1) * unit_gap >= 1.0:
        raise ValueError("gap too large for n points in the interval")
    t = u * (1.0 - (n - 1) * unit_gap) + np.arange(n) * unit_gap
    return lo + (hi - lo) * t


def uniform_problem(n: int, g: np.random.Generator, rho: float = 1.0, gap: float = 1e-6,
                    lo: float = 0.0, hi: float = 1.0) -> RankOne:
    """The basic workload: gapped sorted uniform poles, z ~ N(0,1) normalised, given rho."""
    d = gapped_uniform(g, n, lo, hi, gap)
    z = g.standard_normal(n)
    z /= np.linalg.norm(z)
    return RankOne(d=d, z=z, rho=float(rho))


def cfg0(n: int = 1024, m: int = 16):
    """One problem, n=1024: poles sorted U[0,1) with min gap 1e-6, ||z||=1, rho=1, m RHS."""
    g = rng_for(0, 0)
    prob = uniform_problem(n, g, rho=1.0, gap=1e-6)
    X = g.standard_normal((n, m))
    return prob, np.asfortranarray(X)


def clustered_problem(n: int, g: np.random.Generator, rho: float = 0.5, cluster: int = 32,
                      cluster_frac: float = 0.10, cluster_step: float = 1e-10,
                      tiny_frac: float = 0.01, tiny_value: float = 1e-12,
                      min_sep: float = 5e-11) -> RankOne:
    """Poles on U[-1,1) with a share of them packed into tight clusters, z ~ N(0,1)/sqrt(n)
    with a share of entries replaced by a tiny constant (not renormalised)."""
    ncl = int(cluster_frac * n) // cluster
    centers = g.uniform(-1.0, 1.0, ncl)
    clus = (centers[:, None] + cluster_step * np.arange(cluster)[None, :]).ravel()
    nfree = n - clus.size
    free = g.uniform(-1.0, 1.0, nfree)
    # redraw free points that land within min_sep of any other point
    for _ in range(100):
        allp = np.concatenate([clus, free])
        order = np.argsort(allp, kind="stable")
        s = allp[order]
        close = np.zeros(s.size, dtype=bool)
        dif = np.diff(s) < min_sep
        close[:-1] |= dif
        close[1:] |= dif
        is_free = order >= clus.size
        bad = order[close & is_free] - clus.size
        # a free point next to a cluster point or another free point must move;
        # cluster points are never moved (their spacing is the design)
        if bad.size == 0:
            break
        free[bad] = g.uniform(-1.0, 1.0, bad.size)
    else:  # pragma: no cover - vanishingly unlikely
        raise RuntimeError("could not separate points")
    d = np.sort(np.concatenate([clus, free]))
    if np.any(np.diff(d) <= 0):
        raise RuntimeError("generator produced repeated poles")
    z = g.standard_normal(n) / np.sqrt(n)
    ntiny = int(round(tiny_frac * n))
    idx = g.choice(n, size=ntiny, replace=False)
    z[idx] = tiny_value
    return RankOne(d=d, z=z, rho=float(rho))


def cfg1(n: int = 65536, m: int = 64):
    """One large clustered problem: 10% of poles in clusters of 32 spaced 1e-10,
    1% of z entries set to 1e-12, rho=0.5, m RHS."""
    g = rng_for(1, 0)
    prob = clustered_problem(n, g, rho=0.5)
    X = g.standard_normal((n, m))
    return prob, np.asfortranarray(X)


# ----------------------------------------------------------------------------------------
# batches (CSR layout: problem p owns rows off[p]:off[p+1])
# ----------------------------------------------------------------------------------------

@dataclass
class Batch:
    off: np.ndarray        # int64[P+1]
    d: np.ndarray          # float64[sum n]
    z: np.ndarray          # float64[sum n]
    rho: np.ndarray        # float64[P]
    extra: dict = field(default_factory=dict)

    @property
    def nprob(self) -> int:
        return int(self.rho.shape[0])

    @property
    def total_n(self) -> int:
        return int(self.off[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.off)

    def problem(self, p: int) -> RankOne:
        a, b = int(self.off[p]), int(self.off[p + 1])
        return RankOne(d=self.d[a:b], z=self.z[a:b], rho=float(self.rho[p]))


def concat(problems) -> Batch:
    sizes = np.array([pr.n for pr in problems], dtype=np.int64)
    off = np.zeros(len(problems) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    d = np.concatenate([pr.d for pr in problems]) if problems else np.zeros(0)
    z = np.concatenate([pr.z for pr in problems]) if problems else np.zeros(0)
    rho = np.array([pr.rho for pr in problems], dtype=np.float64)
    return Batch(off=off, d=d, z=z, rho=rho)


def cfg2_sizes(nprob: int = 4096, nmin: int = 64, nmax: int = 8192) -> np.ndarray:
    g = rng_for(2, 1 << 30)
    return np.rint(np.exp(g.uniform(np.log(nmin), np.log(nmax), nprob))).astype(np.int64)


def cfg2(nprob: int = 4096, m: int = 16, nmin: int = 64, nmax: int = 8192):
    """Batched level: sizes log-uniform in [nmin, nmax], each problem drawn like cfg0 with
    its own seed, rho ~ U[0.1, 2], m RHS stacked column-major over the whole batch."""
    sizes = cfg2_sizes(nprob, nmin, nmax)
    probs = []
    for p, n in enumerate(sizes):
        g = rng_for(2, p)
        rho = g.uniform(0.1, 2.0)
        probs.append(uniform_problem(int(n), g, rho=rho, gap=1e-6))
    b = concat(probs)
    gx = rng_for(2, 1 << 31)
    X = np.asfortranarray(gx.standard_normal((b.total_n, m)))
    return b, X


def cfg4(nprob: int = 1024, nmin: int = 256, nmax: int = 4096):
    """Differentiation batch: sizes uniform in [nmin, nmax], cfg0-style draws, rho ~ U[0.1,2];
    loss weights wl ~ N(0,1) per eigenvalue and projection vectors u ~ N(0,1)."""
    gs = rng_for(4, 1 << 30)
    sizes = gs.integers(nmin, nmax + 1, nprob)
    probs = []
    for p, n in enumerate(sizes):
        g = rng_for(4, p)
        rho = g.uniform(0.1, 2.0)
        probs.append(uniform_problem(int(n), g, rho=rho, gap=1e-6))
    b = concat(probs)
    gw = rng_for(4, 1 << 31)
    b.extra["wl"] = gw.standard_normal(b.total_n)
    b.extra["u"] = gw.standard_normal(b.total_n)
    b.extra["wp"] = gw.standard_normal(b.total_n)
    return b


def small_batch(sizes, seed: int = 0, kind: str = "uniform", m: int = 0):
    """Test batches of given sizes.  kind: 'uniform' (cfg0 draws, rho~U[0.1,2]),
    'clustered' (cfg1 draws at this size), 'tinyrho' (rho = 1e-20)."""
    probs = []
    for p, n in enumerate(sizes):
        g = rng_for(100 + seed, p)
        if kind == "uniform":
            probs.append(uniform_problem(int(n), g, rho=g.uniform(0.1, 2.0), gap=1e-6))
        elif kind == "clustered":
            probs.append(clustered_problem(int(n), g, rho=0.5, cluster=min(32, max(2, n // 8)),
                                           cluster_frac=0.10 if n >= 64 else 0.0))
        elif kind == "tinyrho":
            probs.append(uniform_problem(int(n), g, rho=1e-20, gap=1e-6))
        else:
            raise ValueError(kind)
    b = concat(probs)
    if m:
        gx = rng_for(100 + seed, 1 << 31)
        return b, np.asfortranarray(gx.standard_normal((b.total_n, m)))
    return b


def deflation_problem(n: int, g: np.random.Generator, rho: float = 1.0, dup_frac: float = 0.05,
                      near_frac: float = 0.10, tiny_frac: float = 0.05,
                      zero_frac: float = 0.01) -> RankOne:
    """Poles that call for deflation: sorted U[0,1) points at least 1e-6 apart, where a share
    of the poles repeats its left neighbour exactly (duplicates, also in runs) and a share
    sits a tiny distance 10^U[-15,-9] above it; z ~ N(0,1) normalised, with a share of
    entries replaced by tiny values +-10^U[-14,-9] and a share by exact zeros.  d is
    non-decreasing, not strictly increasing."""
    base = gapped_uniform(g, n, 0.0, 1.0, 1e-6) if n > 1 else g.random(n)
    kind = g.random(n)
    kind[0] = 1.0
    step = np.where(kind < dup_frac, 0.0, 10.0 ** g.uniform(-15, -9, n))
    follow = kind < dup_frac + near_frac          # placed relative to its left neighbour
    head = np.maximum.accumulate(np.where(follow, 0, np.arange(n)))
    # offsets inside each run of followers: cumulative steps since the run's head
    cs = np.cumsum(np.where(follow, step, 0.0))
    d = base[head] + (cs - cs[head])
    z = g.standard_normal(n)
    z /= np.linalg.norm(z)
    zk = g.random(n)
    tiny = zk < tiny_frac
    z[tiny] = np.sign(z[tiny]) * 10.0 ** g.uniform(-14, -9, int(tiny.sum()))
    z[(zk >= tiny_frac) & (zk < tiny_frac + zero_frac)] = 0.0
    return RankOne(d=d, z=z, rho=float(rho))


def deflation_batch(sizes, seed: int = 0, m: int = 0):
    """Batches of deflation_problem draws with rho ~ U[0.1, 2]."""
    probs = []
    for p, n in enumerate(sizes):
        g = rng_for(300 + seed, p)
        probs.append(deflation_problem(int(n), g, rho=g.uniform(0.1, 2.0)))
    b = concat(probs)
    if m:
        gx = rng_for(300 + seed, 1 << 31)
        return b, np.asfortranarray(gx.standard_normal((b.total_n, m)))
    return b


# ----------------------------------------------------------------------------------------
# HSS generators for a conquer pass (perfect binary tree, Sec. 2.1 eq. hss)
# ----------------------------------------------------------------------------------------

@dataclass
class HSSTree:
    """Generators of a symmetric HSS matrix on a perfect binary tree.

    Levels are numbered as in the paper: the root is level 0 and the leaves are level
    `depth`.  Nodes of level l are indexed 0..2^l-1 from left to right.

    leaf_D : float64[nleaf, leaf, leaf]   symmetric leaf blocks (taken as already divided)
    leaf_U : float64[nleaf, leaf, r]      orthonormal leaf bases
    R[l]   : float64[2^l, r, r]           transfer matrices of the level-l nodes (l >= 1);
                                          for each sibling pair the stacked [R_c1; R_c2]
                                          has orthonormal columns
    B[l]   : float64[2^l, r, r]           coupling generator of the children pair of each
                                          level-l node (l < depth)
    beta[l]: float64[2^l]                 positive balancing scalar of that pair (||B||_2)
    """
    n: int
    leaf: int
    depth: int
    r: int
    leaf_D: np.ndarray
    leaf_U: np.ndarray
    R: dict
    B: dict
    beta: dict


def _orthonormal(g: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    q, rr = np.linalg.qr(g.standard_normal((rows, cols)))
    return q * np.sign(np.diag(rr))[None, :]


def hss_tree(n: int = 65536, leaf: int = 128, r: int = 8, cfg: int = 3) -> HSSTree:
    """HSS conquer workload: leaf blocks N(0,1)/sqrt(leaf) symmetrised from the upper
    triangle, orthonormal U and stacked R, B ~ N(0,1)."""
    nleaf = n // leaf
    depth = int(round(np.log2(nleaf)))
    if leaf * (1 << depth) != n:
        raise ValueError("n must be leaf * 2^depth")
    g = rng_for(cfg, 0)
    G = g.standard_normal((nleaf, leaf, leaf)) / np.sqrt(leaf)
    up = np.triu(G)
    leaf_D = up + np.transpose(np.triu(G, 1), (0, 2, 1))
    leaf_U = np.stack([_orthonormal(g, leaf, r) for _ in range(nleaf)])
    R, B, beta = {}, {}, {}
    for lvl in range(1, depth + 1):
        cnt = 1 << lvl
        Rl = np.empty((cnt, r, r))
        for pair in range(cnt // 2):
            q = _orthonormal(g, 2 * r, r)
            Rl[2 * pair], Rl[2 * pair + 1] = q[:r], q[r:]
        R[lvl] = Rl
    for lvl in range(0, depth):
        cnt = 1 << lvl
        Bl = g.standard_normal((cnt, r, r))
        B[lvl] = Bl
        beta[lvl] = np.array([np.linalg.norm(Bl[i], 2) for i in range(cnt)])
    return HSSTree(n=n, leaf=leaf, depth=depth, r=r, leaf_D=leaf_D, leaf_U=leaf_U,
                   R=R, B=B, beta=beta)


def hss_original(n: int = 65536, leaf: int = 128, r: int = 8, cfg: int = 5) -> HSSTree:
    """Generators of an HSS matrix before the dividing stage (eq. hss): leaf blocks
    N(0,1)/sqrt(leaf) symmetrised, orthonormal U and stacked R, couplings B ~ N(0,1)
    (the coupling of node p's children is U_c1 B_p U_c2^T).  beta holds ||B||_2 of the
    undivided couplings, for reference only."""
    t = hss_tree(n, leaf, r, cfg)
    return t


def tridiag_hss(n: int, leaf: int, diag=3.0, off=-1.0) -> HSSTree:
    """The symmetric tridiagonal matrix with the given diagonal and off-diagonal (scalars or
    arrays of n and n-1 entries) as an HSS form of rank 2 (the paper's first example):
    node bases [e_first, e_last] of the node's rows, R_c1 = [[1, 0], [0, 0]],
    R_c2 = [[0, 0], [0, 1]], and the coupling of siblings c1, c2 is off[k] e_last(c1)
    e_first(c2)^T, i.e. B = [[0, 0], [off[k], 0]] with k the last row of c1."""
    nleaf = n // leaf
    depth = int(round(np.log2(nleaf)))
    if leaf * (1 << depth) != n or leaf < 2:
        raise ValueError("n must be leaf * 2^depth with leaf >= 2")
    dg = np.broadcast_to(np.asarray(diag, dtype=np.float64), (n,)).copy()
    od = np.broadcast_to(np.asarray(off, dtype=np.float64), (n - 1,)).copy()
    leaf_D = np.zeros((nleaf, leaf, leaf))
    for q in range(nleaf):
        a = q * leaf
        leaf_D[q][np.arange(leaf), np.arange(leaf)] = dg[a:a + leaf]
        leaf_D[q][np.arange(leaf - 1), np.arange(1, leaf)] = od[a:a + leaf - 1]
        leaf_D[q][np.arange(1, leaf), np.arange(leaf - 1)] = od[a:a + leaf - 1]
    leaf_U = np.zeros((nleaf, leaf, 2))
    leaf_U[:, 0, 0] = 1.0
    leaf_U[:, leaf - 1, 1] = 1.0
    R, B, beta = {}, {}, {}
    for lvl in range(1, depth + 1):
        Rl = np.zeros((1 << lvl, 2, 2))
        Rl[0::2, 0, 0] = 1.0
        Rl[1::2, 1, 1] = 1.0
        R[lvl] = Rl
    for lvl in range(depth):
        cnt = 1 << lvl
        size = leaf << (depth - lvl)
        Bl = np.zeros((cnt, 2, 2))
        for q in range(cnt):
            Bl[q, 1, 0] = od[q * size + size // 2 - 1]
        B[lvl] = Bl
        beta[lvl] = np.abs(Bl[:, 1, 0])
    return HSSTree(n=n, leaf=leaf, depth=depth, r=2, leaf_D=leaf_D, leaf_U=leaf_U,
                   R=R, B=B, beta=beta)
