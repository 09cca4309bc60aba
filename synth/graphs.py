"""Seeded synthetic graph generators.

These build the inputs that both the oracle and the HIP path consume.  They
hold none of the clustering method's arithmetic: only random graph models and
CSR assembly.  Every generator returns a `Graph` whose CSR stores both
directions of each undirected edge (nnz = 2m), sorted by row then column, with
no self-loops.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class Graph:
    n: int
    indptr: np.ndarray            # int64 [n+1]
    indices: np.ndarray           # int32 [nnz]
    data: Optional[np.ndarray]    # float64 [nnz] or None (unit weights)
    labels: Optional[np.ndarray] = None   # planted cluster of each vertex

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])


def csr_from_edges(n, u, v, w=None) -> Graph:
    """Symmetric CSR from an undirected edge list (u[i], v[i]) with u != v.
    Duplicate pairs are merged (first weight kept)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if w is not None:
        w = np.asarray(w, dtype=np.float64)[keep]
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    key = lo * n + hi
    key, first = np.unique(key, return_index=True)
    lo, hi = key // n, key % n
    if w is not None:
        w = w[first]
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    order = np.argsort(rows * n + cols, kind="stable")
    rows, cols = rows[order], cols[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=indptr[1:])
    data = None if w is None else np.concatenate([w, w])[order]
    return Graph(n, indptr, cols.astype(np.int32), data)


def _pairs_within(rng, lo, size, p, dense_limit=1 << 24):
    """Bernoulli(p) edges among vertices [lo, lo+size): exact per-pair coin
    flips when the block is small, otherwise a Binomial edge count followed by
    uniform pair draws (duplicates merged later)."""
    npairs = size * (size - 1) // 2
    if npairs == 0 or p <= 0:
        return np.empty(0, np.int64), np.empty(0, np.int64)
    if npairs <= dense_limit:
        iu, ju = np.triu_indices(size, k=1)
        m = rng.random(iu.size) < p
        return iu[m] + lo, ju[m] + lo
    cnt = rng.binomial(npairs, p)
    a = rng.integers(0, size, cnt)
    b = rng.integers(0, size, cnt)
    return a + lo, b + lo


def _pairs_between(rng, lo_a, size_a, lo_b, size_b, p, dense_limit=1 << 24):
    npairs = size_a * size_b
    if npairs == 0 or p <= 0:
        return np.empty(0, np.int64), np.empty(0, np.int64)
    if npairs <= dense_limit:
        m = rng.random((size_a, size_b)) < p
        a, b = np.nonzero(m)
        return a + lo_a, b + lo_b
    cnt = rng.binomial(npairs, p)
    return rng.integers(0, size_a, cnt) + lo_a, rng.integers(0, size_b, cnt) + lo_b


def sbm(n, k, p_in, p_out, seed, permute=False) -> Graph:
    """Stochastic block model as in the paper's synthetic experiments (Sec. 4.1):
    k clusters of (nearly) equal size, each pair inside a cluster joined with
    probability p_in and across clusters with p_out, unit weights.  Cluster
    sizes differ by at most one (the remainder goes to the first clusters).
    With permute=True the vertex ids are shuffled (seeded)."""
    rng = np.random.default_rng(seed)
    sizes = np.full(k, n // k, dtype=np.int64)
    sizes[: n % k] += 1
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    us, vs = [], []
    for a in range(k):
        u, v = _pairs_within(rng, int(starts[a]), int(sizes[a]), p_in)
        us.append(u); vs.append(v)
        for b in range(a + 1, k):
            u, v = _pairs_between(rng, int(starts[a]), int(sizes[a]),
                                  int(starts[b]), int(sizes[b]), p_out)
            us.append(u); vs.append(v)
    u = np.concatenate(us); v = np.concatenate(vs)
    labels = np.repeat(np.arange(k, dtype=np.int32), sizes)
    if permute:
        perm = rng.permutation(n)
        u, v = perm[u], perm[v]
        lab = np.empty(n, dtype=np.int32)
        lab[perm] = labels
        labels = lab
    g = csr_from_edges(n, u, v)
    g.labels = labels
    return g


def sbm_by_degree(n, k, deg_in, deg_out, seed, permute=False) -> Graph:
    """SBM parameterised by expected in-cluster and out-of-cluster degree."""
    size = n / k
    p_in = deg_in / max(size - 1, 1)
    p_out = deg_out / max(n - size, 1)
    return sbm(n, k, min(p_in, 1.0), min(p_out, 1.0), seed, permute)


def disjoint_cliques(k, s) -> Graph:
    """k disjoint complete graphs K_s (vertices of clique c are c*s..c*s+s-1)."""
    us, vs = [], []
    iu, ju = np.triu_indices(s, k=1)
    for c in range(k):
        us.append(iu + c * s); vs.append(ju + c * s)
    g = csr_from_edges(k * s, np.concatenate(us), np.concatenate(vs))
    g.labels = np.repeat(np.arange(k, dtype=np.int32), s)
    return g


def cycle(n) -> Graph:
    """The cycle C_n (n >= 3)."""
    i = np.arange(n)
    return csr_from_edges(n, i, (i + 1) % n)


def complete_bipartite(a, b) -> Graph:
    """K_{a,b}: vertices 0..a-1 on one side, a..a+b-1 on the other."""
    u, v = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return csr_from_edges(a + b, u.ravel(), v.ravel())


def random_weighted(n, m, seed, hubs=0, hub_degree=0, isolated=0, weighted=True) -> Graph:
    """A ragged test graph: m uniform random edges, plus `hubs` vertices each
    joined to `hub_degree` random others, and the last `isolated` vertices left
    without edges.  Weights are uniform in (0.5, 2) when weighted."""
    rng = np.random.default_rng(seed)
    live = n - isolated
    u = rng.integers(0, live, m)
    v = rng.integers(0, live, m)
    if hubs:
        hu = np.repeat(rng.choice(live, hubs, replace=False), hub_degree)
        hv = rng.integers(0, live, hu.size)
        u = np.concatenate([u, hu]); v = np.concatenate([v, hv])
    w = rng.uniform(0.5, 2.0, u.size) if weighted else None
    return csr_from_edges(n, u, v, w)


def gaussian_mixture(n_per, k, dim, seed, mean_scale=2.0):
    """Points of a mixture of k isotropic Gaussians: means ~ N(0, mean_scale^2 I),
    unit covariance, n_per points per component (component c occupies rows
    c*n_per..).  Returns (X float32 [k*n_per, dim], labels)."""
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((k, dim)) * mean_scale
    X = np.repeat(means, n_per, axis=0) + rng.standard_normal((k * n_per, dim))
    return X.astype(np.float32), np.repeat(np.arange(k, dtype=np.int32), n_per)


def knn_graph(X, knn=10, block=4096) -> Graph:
    """Symmetrised k-nearest-neighbour graph of the rows of X (the paper's
    pre-processing of its real-world data, Sec. 4.2, with k = 10).  Exact
    neighbours by squared Euclidean distance, self excluded, ties to the lower
    index; union symmetrisation; weight exp(-d^2 / sigma^2) with sigma^2 the
    median of the directed neighbour distances."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    sq = (X * X).sum(axis=1)
    nbr = np.empty((n, knn), dtype=np.int64)
    dist = np.empty((n, knn))
    for s in range(0, n, block):
        e = min(n, s + block)
        D = sq[s:e, None] + sq[None, :] - 2.0 * (X[s:e] @ X.T)
        D[np.arange(e - s), np.arange(s, e)] = np.inf
        part = np.argpartition(D, knn, axis=1)[:, : knn + 1]
        pd = np.take_along_axis(D, part, axis=1)
        order = np.lexsort((part, pd), axis=1)[:, :knn]
        nbr[s:e] = np.take_along_axis(part, order, axis=1)
        dist[s:e] = np.maximum(np.take_along_axis(pd, order, axis=1), 0.0)
    sigma2 = float(np.median(dist))
    u = np.repeat(np.arange(n), knn)
    v = nbr.ravel()
    w = np.exp(-dist.ravel() / sigma2)
    return csr_from_edges(n, u, v, w)


def knn_mixture(n_per, k, dim, seed, knn=10) -> Graph:
    X, lab = gaussian_mixture(n_per, k, dim, seed)
    g = knn_graph(X, knn)
    g.labels = lab
    return g


# ---------------------------------------------------------------------------
# Device-side generation for workloads too large for host numpy (torch is used
# only as a device array library here; the graph models are the ones above).
# ---------------------------------------------------------------------------
def knn_mixture_device(n_per, k, dim, seed, knn=10, device="cuda", block=2048):
    """The symmetrised k-NN graph of `knn_graph` over the points of
    `gaussian_mixture`, built on the device: the same points, exact
    neighbours by FP32 squared distance (self excluded, a stable sort so ties
    go to the lower index), sigma^2 the median of the directed neighbour
    distances (mean of the two middle values), weight exp(-d^2 / sigma^2),
    union symmetrisation keeping the first weight of a pair.  Returns device
    (indptr int64, indices int32, weights float32) and the host labels."""
    import torch
    X_h, lab = gaussian_mixture(n_per, k, dim, seed)
    X = torch.from_numpy(X_h).to(device)
    n = X.shape[0]
    sq = (X * X).sum(1)
    nbr = torch.empty((n, knn), dtype=torch.int64, device=device)
    dist = torch.empty((n, knn), dtype=torch.float32, device=device)
    XT = X.t().contiguous()
    for s in range(0, n, block):
        e = min(n, s + block)
        D = sq[s:e, None] + sq[None, :] - 2.0 * (X[s:e] @ XT)
        D[torch.arange(e - s, device=device), torch.arange(s, e, device=device)] = float("inf")
        val, idx = torch.sort(D, dim=1, stable=True)
        nbr[s:e] = idx[:, :knn]
        dist[s:e] = val[:, :knn].clamp_min(0.0)
        del D, val, idx
    flat = torch.sort(dist.flatten()).values
    m = flat.numel() // 2
    sigma2 = float(flat[m]) if flat.numel() % 2 else 0.5 * (float(flat[m - 1]) + float(flat[m]))
    u = torch.arange(n, device=device).repeat_interleave(knn)
    v = nbr.flatten()
    w = torch.exp(-dist.flatten().double() / sigma2)
    lo, hi = torch.minimum(u, v), torch.maximum(u, v)
    key = lo * n + hi
    key_s, order = torch.sort(key, stable=True)
    first = torch.ones_like(key_s, dtype=torch.bool)
    first[1:] = key_s[1:] != key_s[:-1]
    key_u, w_u = key_s[first], w[order][first]
    lo, hi = key_u // n, key_u % n
    rows = torch.cat([lo, hi])
    cols = torch.cat([hi, lo])
    ww = torch.cat([w_u, w_u])
    order = torch.argsort(rows * n + cols)
    rows, cols, ww = rows[order], cols[order], ww[order]
    indptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    indptr[1:] = torch.cumsum(torch.bincount(rows, minlength=n), 0)
    return indptr, cols.to(torch.int32), ww.to(torch.float32), lab

def sbm_device(n, k, deg_in, deg_out, seed, device="cuda"):
    """SBM with k near-equal clusters and expected in/out-cluster degree
    deg_in/deg_out, built on the device.  Edge counts per block (within) and
    across blocks are Binomial draws from a host generator; endpoints are
    uniform draws from a seeded device generator; self-pairs are dropped and
    duplicate pairs merged.  Returns (indptr int64, indices int32, labels
    int32) device tensors."""
    import torch
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    sizes = np.full(k, n // k, dtype=np.int64)
    sizes[: n % k] += 1
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    size = n / k
    p_in = min(deg_in / max(size - 1, 1), 1.0)
    p_out = min(deg_out / max(n - size, 1), 1.0)
    us, vs = [], []
    for b in range(k):
        s = int(sizes[b])
        m = int(rng.binomial(s * (s - 1) // 2, p_in)) if s > 1 else 0
        if m:
            us.append(torch.randint(0, s, (m,), generator=gen, device=device) + int(starts[b]))
            vs.append(torch.randint(0, s, (m,), generator=gen, device=device) + int(starts[b]))
    cross_pairs = (n * n - int((sizes ** 2).sum())) // 2
    m = int(rng.binomial(cross_pairs, p_out)) if cross_pairs > 0 else 0
    lab = torch.repeat_interleave(torch.arange(k, device=device, dtype=torch.int64),
                                  torch.from_numpy(sizes).to(device))
    got = 0
    while got < m:
        want = int((m - got) * 1.3) + 16
        u = torch.randint(0, n, (want,), generator=gen, device=device)
        v = torch.randint(0, n, (want,), generator=gen, device=device)
        keep = lab[u] != lab[v]
        u, v = u[keep][: m - got], v[keep][: m - got]
        us.append(u)
        vs.append(v)
        got += u.numel()
    if us:
        u = torch.cat(us)
        v = torch.cat(vs)
    else:
        u = v = torch.empty(0, dtype=torch.int64, device=device)
    keep = u != v
    u, v = u[keep], v[keep]
    lo, hi = torch.minimum(u, v), torch.maximum(u, v)
    key = torch.unique(lo * n + hi)
    lo, hi = key // n, key % n
    rows = torch.cat([lo, hi])
    cols = torch.cat([hi, lo])
    order = torch.argsort(rows * n + cols)
    rows, cols = rows[order], cols[order]
    indptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    indptr[1:] = torch.cumsum(torch.bincount(rows, minlength=n), 0)
    return indptr, cols.to(torch.int32), lab.to(torch.int32)


def batched_sbm_params(count=512, seed=0):
    """Per-graph parameters of the batched workload: n uniform in
    [1000, 200000], k uniform in [2, 20], expected degree uniform in [8, 64]
    split 9:1 into in- and out-cluster degree, l = ceil(log2 k) + 1,
    t = ceil(3 ln n), graph seed derived from (seed, index)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(1000, 200001))
        k = int(rng.integers(2, 21))
        d = float(rng.uniform(8.0, 64.0))
        out.append(dict(n=n, k=k, deg_in=0.9 * d, deg_out=0.1 * d, l=int(np.ceil(np.log2(k))) + 1,
                        t=int(np.ceil(3.0 * np.log(n))), seed=int(seed) * 1_000_003 + i))
    return out


def _csr_device(n, u, v):
    """Symmetric CSR (dropping self-pairs, merging duplicates) from device
    endpoint arrays."""
    import torch
    keep = u != v
    u, v = u[keep], v[keep]
    lo, hi = torch.minimum(u, v), torch.maximum(u, v)
    key = torch.unique(lo * n + hi)
    lo, hi = key // n, key % n
    rows = torch.cat([lo, hi])
    cols = torch.cat([hi, lo])
    order = torch.argsort(rows * n + cols)
    rows, cols = rows[order], cols[order]
    indptr = torch.zeros(n + 1, dtype=torch.int64, device=u.device)
    indptr[1:] = torch.cumsum(torch.bincount(rows, minlength=n), 0)
    return indptr, cols.to(torch.int32)


def dcsbm_device(n, k, mean_deg, seed, alpha=2.5, in_frac=0.9, device="cuda"):
    """Degree-corrected SBM (Karrer and Newman style): k near-equal contiguous
    clusters; degree propensities theta ~ Pareto with density exponent alpha
    and mean mean_deg (x_min = mean_deg (alpha-2)/(alpha-1)); a fraction
    in_frac of each vertex's expected degree inside its cluster.  Edges are
    Chung-Lu draws: endpoints chosen with probability proportional to theta
    (inside a cluster for the in-cluster edges, across clusters for the
    rest); self-pairs dropped, duplicates merged.  Returns (indptr, indices,
    labels) device tensors."""
    import torch
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    xmin = mean_deg * (alpha - 2.0) / (alpha - 1.0)
    u01 = torch.rand(n, generator=gen, device=device, dtype=torch.float64)
    theta = xmin * (1.0 - u01) ** (-1.0 / (alpha - 1.0))
    sizes = np.full(k, n // k, dtype=np.int64)
    sizes[: n % k] += 1
    starts = np.concatenate([[0], np.cumsum(sizes)])
    lab = torch.repeat_interleave(torch.arange(k, device=device, dtype=torch.int64),
                                  torch.from_numpy(sizes).to(device))
    cum = torch.cumsum(theta, 0)
    cum0 = torch.cat([torch.zeros(1, dtype=torch.float64, device=device), cum])
    Theta = (cum0[torch.from_numpy(starts[1:]).to(device)] - cum0[torch.from_numpy(starts[:-1]).to(device)]).cpu().numpy()
    total = float(cum0[-1])
    # in-cluster edges: per cluster a Poisson count, endpoints theta-weighted
    m_in = rng.poisson(in_frac * Theta / 2.0)
    blk = torch.repeat_interleave(torch.arange(k, device=device), torch.from_numpy(m_in).to(device))
    lo_c = cum0[torch.from_numpy(starts[:-1]).to(device)][blk]
    span = (cum0[torch.from_numpy(starts[1:]).to(device)] - cum0[torch.from_numpy(starts[:-1]).to(device)])[blk]
    def draw_in():
        r = lo_c + torch.rand(blk.numel(), generator=gen, device=device, dtype=torch.float64) * span
        return torch.clamp(torch.searchsorted(cum, r, right=True), max=n - 1)
    u_in, v_in = draw_in(), draw_in()
    # cross-cluster edges: theta-weighted endpoints, same-cluster pairs redrawn
    m_out = int(rng.poisson((1.0 - in_frac) * total / 2.0))
    us, vs, got = [], [], 0
    while got < m_out:
        want = int((m_out - got) * 1.3) + 16
        a = torch.clamp(torch.searchsorted(cum, torch.rand(want, generator=gen, device=device,
                                                             dtype=torch.float64) * total, right=True), max=n - 1)
        b = torch.clamp(torch.searchsorted(cum, torch.rand(want, generator=gen, device=device,
                                                             dtype=torch.float64) * total, right=True), max=n - 1)
        keep = lab[a] != lab[b]
        a, b = a[keep][: m_out - got], b[keep][: m_out - got]
        us.append(a)
        vs.append(b)
        got += a.numel()
    u = torch.cat([u_in] + us)
    v = torch.cat([v_in] + vs)
    indptr, indices = _csr_device(n, u, v)
    return indptr, indices, lab.to(torch.int32)


def learned_params(count, seed0):
    """Per-graph parameters of the learned-form workload: n uniform in
    [100000, 2000000], k uniform in [2, 50], mean degree log-uniform in
    [8, 64], degree-propensity exponent alpha uniform in [2.2, 8] (heavy-tailed
    to nearly uniform degrees), in-cluster fraction uniform in [0.85, 0.95],
    l = ceil(log2 k) + 1, t = ceil(3 ln n), graph seed seed0 + index."""
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(count):
        n = int(rng.integers(100_000, 2_000_001))
        k = int(rng.integers(2, 51))
        deg = float(np.exp(rng.uniform(np.log(8.0), np.log(64.0))))
        alpha = float(rng.uniform(2.2, 8.0))
        in_frac = float(rng.uniform(0.85, 0.95))
        out.append(dict(n=n, k=k, l=int(np.ceil(np.log2(k))) + 1, t=int(np.ceil(3.0 * np.log(n))),
                        deg=deg, alpha=alpha, in_frac=in_frac, seed=seed0 + i))
    return out


def learned_graph(spec, device="cuda"):
    """The DC-SBM of one learned-form spec: (indptr, indices, labels)."""
    return dcsbm_device(spec["n"], spec["k"], spec["deg"], spec["seed"], alpha=spec["alpha"],
                        in_frac=spec["in_frac"], device=device)


def graph_agreement(a, b):
    """How two device CSR graphs (indptr, indices, weights) of the same n
    agree: the fraction of each one's entries the other holds, and the
    largest relative weight difference over the shared entries."""
    import torch
    out = []
    keys = []
    for ip, ix, _ in (a, b):
        n = ip.numel() - 1
        rows = torch.repeat_interleave(torch.arange(n, device=ip.device), ip[1:] - ip[:-1])
        keys.append(rows * n + ix.long())
    ka, kb = keys
    wa, wb = a[2].double(), b[2].double()
    oa, ob = torch.argsort(ka), torch.argsort(kb)
    ka, kb, wa, wb = ka[oa], kb[ob], wa[oa], wb[ob]
    pos = torch.searchsorted(kb, ka).clamp(max=kb.numel() - 1)
    hit = kb[pos] == ka
    common = int(hit.sum())
    rel = ((wa[hit] - wb[pos[hit]]).abs() / wb[pos[hit]].abs().clamp_min(1e-300)).max() if common else torch.zeros(())
    return {"entries": [int(ka.numel()), int(kb.numel())], "common": common,
            "common_frac": [common / max(1, ka.numel()), common / max(1, kb.numel())],
            "weight_max_rel_diff": float(rel)}
