"""Graph generators: stochastic block models (Sec. 5 of the paper), their perturbations
(edge redrawing and node reassignment, Sec. 5.1), a Chung-Lu graph with planted
communities, and small textbook graphs whose spectra are known in closed form.

Every generator returns a :class:`Graph` holding the symmetric weight matrix W in CSR
form (int64 row pointers, int32 column indices sorted within each row, float64
weights, no self-loops).  Nothing here touches the Laplacian or any step of the
clustering method.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    rowptr: np.ndarray  # int64, n + 1
    colidx: np.ndarray  # int32, nnz
    w: np.ndarray  # float64, nnz
    labels: np.ndarray | None = None  # planted community of every node (int32)
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def edge_keys(self) -> np.ndarray:
        """Sorted int64 keys ``u * n + v`` of the undirected edges with ``u < v``."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.rowptr))
        cols = self.colidx.astype(np.int64)
        m = rows < cols
        return rows[m] * self.n + cols[m]


# --------------------------------------------------------------------------------------
# helpers


def edges_to_graph(n: int, keys: np.ndarray, labels=None, weights=None, meta=None) -> Graph:
    """CSR of the symmetric graph whose undirected edges are ``keys = u * n + v`` (u < v).

    ``weights`` (optional, one per key) default to 1.
    """
    keys = np.asarray(keys, dtype=np.int64)
    u = keys // n
    v = keys - u * n
    if weights is None:
        wk = np.ones(keys.shape[0], dtype=np.float64)
    else:
        wk = np.asarray(weights, dtype=np.float64)
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    ww = np.concatenate([wk, wk])
    order = np.argsort(rows * n + cols, kind="stable")
    rows = rows[order]
    cols = cols[order]
    ww = ww[order]
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return Graph(n=n, rowptr=rowptr, colidx=cols.astype(np.int32), w=ww,
                 labels=None if labels is None else np.asarray(labels, dtype=np.int32),
                 meta=dict(meta or {}))


def _canon_unique(i: np.ndarray, j: np.ndarray, n: int) -> np.ndarray:
    """Keys of the distinct unordered pairs among (i, j), self-pairs dropped."""
    keep = i != j
    i = i[keep]
    j = j[keep]
    lo = np.minimum(i, j).astype(np.int64)
    hi = np.maximum(i, j).astype(np.int64)
    return np.unique(lo * n + hi)


def block_sizes_equal(n: int, k: int) -> np.ndarray:
    """k blocks whose sizes differ by at most one."""
    base = np.full(k, n // k, dtype=np.int64)
    base[: n - base.sum()] += 1
    return base


def block_sizes_zipf(n: int, k: int, s: float) -> np.ndarray:
    """k block sizes proportional to ``r ** -s`` (r = 1..k), rounded by largest remainder."""
    p = np.arange(1, k + 1, dtype=np.float64) ** (-s)
    p /= p.sum()
    raw = p * n
    sizes = np.floor(raw).astype(np.int64)
    short = n - sizes.sum()
    order = np.argsort(-(raw - sizes), kind="stable")
    sizes[order[:short]] += 1
    if np.any(sizes < 2):
        raise ValueError("zipf sizes leave a block with fewer than two nodes")
    return sizes


def _sbm_q1(sizes: np.ndarray, mean_degree: float, ratio: float) -> float:
    """Intra-block edge probability q1 (with q2 = ratio * q1) giving the requested mean degree."""
    n = float(sizes.sum())
    sz = sizes.astype(np.float64)
    denom = np.sum(sz * ((sz - 1.0) + ratio * (n - sz)))
    q1 = mean_degree * n / denom
    if q1 > 1.0:
        raise ValueError("mean degree too large for these block sizes")
    return q1


def _sample_pairs_exact(rng, count: int, draw) -> np.ndarray:
    """``count`` distinct pair keys, drawn by repeatedly calling ``draw(size)``."""
    if count <= 0:
        return np.zeros(0, dtype=np.int64)
    got = np.zeros(0, dtype=np.int64)
    need = count
    while True:
        extra = int(need * 1.05) + 16
        got = np.union1d(got, draw(extra))
        if got.size >= count:
            break
        need = count - got.size
    if got.size > count:
        got = np.sort(rng.choice(got, size=count, replace=False))
    return got


# --------------------------------------------------------------------------------------
# stochastic block model (Sec. 5): q1 inside a block, q2 = ratio * q1 across blocks


def sbm(n: int, k: int, mean_degree: float, ratio: float, seed: int,
        sizes: np.ndarray | None = None) -> Graph:
    """Planted-partition SBM, unweighted and symmetric.

    Blocks are contiguous node ranges of the given ``sizes`` (equal by default).  For
    every block pair the number of edges is Binomial(#pairs, q) and that many distinct
    pairs are drawn uniformly, so the law is exactly the SBM's.
    """
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = block_sizes_equal(n, k)
    sizes = np.asarray(sizes, dtype=np.int64)
    assert sizes.sum() == n and sizes.size == k
    q1 = _sbm_q1(sizes, mean_degree, ratio)
    q2 = ratio * q1
    off = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    parts = []
    for a in range(k):
        na = int(sizes[a])
        oa = int(off[a])
        # within block a
        npairs = na * (na - 1) // 2
        cnt = int(rng.binomial(npairs, q1))

        def draw_in(sz, oa=oa, na=na):
            i = oa + rng.integers(0, na, size=sz)
            j = oa + rng.integers(0, na, size=sz)
            return _canon_unique(i, j, n)

        parts.append(_sample_pairs_exact(rng, cnt, draw_in))
        for b in range(a + 1, k):
            nb = int(sizes[b])
            ob = int(off[b])
            cnt = int(rng.binomial(na * nb, q2))

            def draw_x(sz, oa=oa, na=na, ob=ob, nb=nb):
                i = oa + rng.integers(0, na, size=sz)
                j = ob + rng.integers(0, nb, size=sz)
                return _canon_unique(i, j, n)

            parts.append(_sample_pairs_exact(rng, cnt, draw_x))
    keys = np.sort(np.concatenate(parts)) if parts else np.zeros(0, np.int64)
    labels = np.repeat(np.arange(k, dtype=np.int32), sizes)
    return edges_to_graph(n, keys, labels=labels,
                          meta=dict(kind="sbm", k=k, q1=q1, q2=q2, mean_degree=mean_degree,
                                    ratio=ratio, seed=seed))


class DynamicSBM:
    """A sequence of SBM snapshots under the two perturbations of Sec. 5.1.

    * edge redrawing: delete a fraction of the existing edges uniformly at random and add
      as many new ones drawn from the model (pair (i, j) accepted with probability
      q(i, j) / q1);
    * node reassignment: pick a fraction of the nodes, delete every edge touching them,
      move each to a different block chosen uniformly, and reconnect it by drawing a
      Poisson number of new neighbours with the model's probabilities.

    ``q1`` and ``q2`` stay those of the initial graph.
    """

    def __init__(self, g0: Graph, seed: int):
        self.n = g0.n
        self.k = int(g0.meta["k"])
        self.q1 = float(g0.meta["q1"])
        self.q2 = float(g0.meta["q2"])
        self.ratio = self.q2 / self.q1
        self.labels = g0.labels.copy()
        self.keys = g0.edge_keys()
        self.rng = np.random.default_rng(seed)
        self.t = 1

    def graph(self) -> Graph:
        return edges_to_graph(self.n, self.keys, labels=self.labels,
                              meta=dict(kind="dyn-sbm", k=self.k, q1=self.q1, q2=self.q2, t=self.t))

    def _draw_model_pairs(self, count: int) -> np.ndarray:
        rng = self.rng
        n = self.n
        out = np.zeros(0, dtype=np.int64)
        while out.size < count:
            sz = int((count - out.size) / max(self.ratio, 0.05)) + 64
            i = rng.integers(0, n, size=sz)
            j = rng.integers(0, n, size=sz)
            same = self.labels[i] == self.labels[j]
            acc = same | (rng.random(sz) < self.ratio)
            cand = _canon_unique(i[acc], j[acc], n)
            cand = cand[~np.isin(cand, self.keys, assume_unique=True)]
            cand = np.setdiff1d(cand, out, assume_unique=True)
            out = np.union1d(out, cand)
        if out.size > count:
            out = np.sort(rng.choice(out, size=count, replace=False))
        return out

    def step(self, rewire_frac: float, move_frac: float) -> Graph:
        rng = self.rng
        n = self.n
        # edge redrawing
        ne = self.keys.size
        nrew = int(round(rewire_frac * ne))
        if nrew > 0:
            drop = rng.choice(ne, size=nrew, replace=False)
            keep = np.ones(ne, dtype=bool)
            keep[drop] = False
            self.keys = self.keys[keep]
            self.keys = np.union1d(self.keys, self._draw_model_pairs(nrew))
        # node reassignment
        nmove = int(round(move_frac * n))
        if nmove > 0:
            moved = rng.choice(n, size=nmove, replace=False)
            mark = np.zeros(n, dtype=bool)
            mark[moved] = True
            u = self.keys // n
            v = self.keys - u * n
            self.keys = self.keys[~(mark[u] | mark[v])]
            shift = rng.integers(1, self.k, size=nmove)
            self.labels[moved] = (self.labels[moved] + shift) % self.k
            sizes = np.bincount(self.labels, minlength=self.k).astype(np.int64)
            order = np.argsort(self.labels, kind="stable")
            off = np.zeros(self.k + 1, dtype=np.int64)
            np.cumsum(sizes, out=off[1:])
            b = self.labels[moved].astype(np.int64)
            nb = sizes[b]
            mu_in = self.q1 * (nb - 1)
            mu_out = self.q2 * (n - nb)
            deg = rng.poisson(mu_in + mu_out)
            src = np.repeat(moved.astype(np.int64), deg)
            bb = np.repeat(b, deg)
            p_in = np.repeat(mu_in / np.maximum(mu_in + mu_out, 1e-300), deg)
            inside = rng.random(src.size) < p_in
            dst = np.empty(src.size, dtype=np.int64)
            # a partner inside the new block
            r_in = rng.integers(0, 1 << 62, size=src.size)
            dst_in = order[off[bb] + (r_in % sizes[bb])]
            # a partner outside: uniform over the nodes of the other blocks
            r_out = rng.integers(0, 1 << 62, size=src.size)
            outside_n = n - sizes[bb]
            pos = r_out % np.maximum(outside_n, 1)
            pos = np.where(pos >= off[bb], pos + sizes[bb], pos)
            dst_out = order[pos]
            dst[inside] = dst_in[inside]
            dst[~inside] = dst_out[~inside]
            new = _canon_unique(src, dst, n)
            self.keys = np.union1d(self.keys, new)
        self.t += 1
        return self.graph()


# --------------------------------------------------------------------------------------
# Chung-Lu graph with planted communities


def _sample_weighted(cdf: np.ndarray, count: int, rng) -> np.ndarray:
    """``count`` i.i.d. indices with P(i) = cdf[i] - cdf[i-1] (cdf normalised to end at 1),
    in random order.  The uniforms are searched in sorted order (NumPy's binary search then
    starts from the previous hit) and the results shuffled."""
    u = np.sort(rng.random(count))
    idx = np.minimum(np.searchsorted(cdf, u, side="right"), cdf.size - 1)
    return rng.permutation(idx)


def chung_lu(n: int, k: int, mean_degree: float, exponent: float, ratio: float,
             seed: int) -> Graph:
    """Power-law expected degrees with planted communities.

    Expected-degree weights ``theta_i ∝ (i + i0) ** (-1 / (exponent - 1))`` scaled to the
    requested mean and capped at ``sqrt(sum theta)``; nodes are placed in k equal
    communities at random.  Candidate pairs follow P(a, b) ∝ theta_a theta_b w(a, b) with
    w = 1 inside a community and ``ratio`` across: the within-community share of the
    candidates is drawn first, then within-community endpoints from each community's
    weights and cross-community endpoints from all weights (same-community draws redrawn).
    Duplicates and self-pairs are dropped and the edge count is trimmed to
    ``n * mean_degree / 2``.
    """
    rng = np.random.default_rng(seed)
    i0 = 10.0
    theta = (np.arange(n, dtype=np.float64) + i0) ** (-1.0 / (exponent - 1.0))
    theta *= mean_degree / theta.mean()
    cap = np.sqrt(theta.sum())
    theta = np.minimum(theta, cap)
    theta *= mean_degree / theta.mean()
    comm = rng.permutation(np.repeat(np.arange(k, dtype=np.int32), (n + k - 1) // k)[:n])
    target = int(n * mean_degree / 2)
    cdf = np.cumsum(theta)
    cdf /= cdf[-1]
    members = [np.flatnonzero(comm == c) for c in range(k)]
    ccdf = []
    for mem in members:
        w = np.cumsum(theta[mem])
        ccdf.append(w / w[-1] if w.size else w)
    S = np.array([theta[mem].sum() for mem in members])
    m_in = float(np.sum(S * S))
    m_out = ratio * (float(S.sum()) ** 2 - m_in)
    p_in = m_in / (m_in + m_out)
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < target:
        draw = int((target - keys.size) * 1.05) + 1024
        n_in = int(rng.binomial(draw, p_in))
        chunks = []
        per_c = rng.multinomial(n_in, S * S / m_in)
        for c, cnt in enumerate(per_c):
            if cnt == 0 or members[c].size < 2:
                continue
            a = members[c][_sample_weighted(ccdf[c], int(cnt), rng)]
            b = members[c][_sample_weighted(ccdf[c], int(cnt), rng)]
            chunks.append(_canon_unique(a, b, n))
        need = draw - n_in
        while need > 0:
            a = _sample_weighted(cdf, need, rng)
            b = _sample_weighted(cdf, need, rng)
            cross = comm[a] != comm[b]
            chunks.append(_canon_unique(a[cross], b[cross], n))
            need -= int(cross.sum())
        keys = np.union1d(keys, np.concatenate(chunks))
    if keys.size > target:
        keys = np.sort(rng.choice(keys, size=target, replace=False))
    return edges_to_graph(n, keys, labels=comm,
                          meta=dict(kind="chung-lu", k=k, exponent=exponent, ratio=ratio,
                                    mean_degree=mean_degree, seed=seed))


def rewire_model_free(g: Graph, frac: float, seed: int, ratio: float) -> Graph:
    """Edge redrawing for graphs without block probabilities (the Chung-Lu sequence):
    delete ``frac`` of the edges and add as many pairs drawn by degree-proportional
    endpoint sampling, cross-community pairs kept with probability ``ratio``."""
    rng = np.random.default_rng(seed)
    n = g.n
    keys = g.edge_keys()
    nrew = int(round(frac * keys.size))
    if nrew == 0:
        return g
    drop = rng.choice(keys.size, size=nrew, replace=False)
    keep = np.ones(keys.size, dtype=bool)
    keep[drop] = False
    keys = keys[keep]
    deg = np.diff(g.rowptr).astype(np.float64) + 1e-3
    cdf = np.cumsum(deg)
    cdf /= cdf[-1]
    comm = g.labels
    new = np.zeros(0, dtype=np.int64)
    while new.size < nrew:
        sz = 4 * (nrew - new.size) + 1024
        a = _sample_weighted(cdf, sz, rng)
        b = _sample_weighted(cdf, sz, rng)
        ok = (comm[a] == comm[b]) | (rng.random(sz) < ratio)
        cand = _canon_unique(a[ok], b[ok], n)
        # keys is sorted: membership by binary search instead of a re-sort
        pos = np.minimum(np.searchsorted(keys, cand), keys.size - 1)
        cand = cand[keys[pos] != cand]
        new = np.union1d(new, cand)
    if new.size > nrew:
        new = rng.choice(new, size=nrew, replace=False)
    keys = np.union1d(keys, new)
    return edges_to_graph(n, keys, labels=comm, meta=dict(g.meta))


# --------------------------------------------------------------------------------------
# textbook graphs


def cycle_graph(n: int) -> Graph:
    """The n-cycle; its normalized Laplacian has eigenvalues 1 - cos(2 pi j / n)."""
    u = np.arange(n, dtype=np.int64)
    v = (u + 1) % n
    keys = np.unique(np.minimum(u, v) * n + np.maximum(u, v))
    return edges_to_graph(n, keys, meta=dict(kind="cycle"))


def disjoint_cliques(k: int, size: int) -> Graph:
    """k disjoint complete graphs of ``size`` nodes each."""
    n = k * size
    parts = []
    for a in range(k):
        i, j = np.triu_indices(size, 1)
        parts.append((a * size + i).astype(np.int64) * n + (a * size + j))
    labels = np.repeat(np.arange(k, dtype=np.int32), size)
    return edges_to_graph(n, np.sort(np.concatenate(parts)), labels=labels,
                          meta=dict(kind="cliques", k=k))
