"""Plain FP64 CPU oracle for FastSpectralCluster.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module: it is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  It shares no code with the HIP path.

Every function follows the paper ("Fast and Simple Spectral Clustering in
Theory and Practice", Macgregor, NeurIPS 2023) step by step in float64, with
numpy/scipy primitives (a sparse matrix product, a dense eigendecomposition in
the checks) as the only library steps.  Readings where the paper is silent are
marked "Reading:" and are listed in the design notes.

Sections of the paper referenced below:
  * Sec. 2 (Preliminaries): degree, Laplacian, normalised Laplacian N, the
    halved signless Laplacian M = I - N/2 with eigenvalues in [0, 1].
  * Sec. 2.2: the k-means cost; Lloyd's algorithm with k-means++ seeding.
  * Sec. 2.3, Algorithm 1 (PowerMethod): x_i = M x_{i-1}, no normalisation.
  * Sec. 3.2, Algorithm 2 (FastSpectralCluster): l Gaussian vectors, each run
    through PowerMethod for t steps, k-means on D^{-1/2} Y.
  * Sec. 4: PM with k vectors, the comparison method of Boutsidis et al.
  * Sec. 4.2: ARI and NMI as the accuracy scores.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------
# Counter-based random numbers.
# Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random
# numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter, a 2x32-bit key,
# ten rounds of two 32x32->64 multiplies with a Weyl-sequence key schedule.
# The paper only fixes the distribution N(0, I) of the start vectors
# (Sec. 3.1 and Algorithm 2); the generator is this build's reading.
# ----------------------------------------------------------------------------
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = np.uint64(0x9E3779B9)
_PHILOX_W1 = np.uint64(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on arrays of 32-bit words (held in uint64 containers).

    Returns the four output words as uint64 arrays with values < 2**32.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK32 for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _PHILOX_W0) & _MASK32
            k1 = (k1 + _PHILOX_W1) & _MASK32
        p0 = _PHILOX_M0 * c0          # < 2**64, exact in uint64
        p1 = _PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform53(hi, lo):
    """Map a pair of 32-bit words to a double in (0, 1): the top 53 bits of
    the 64-bit word hi:lo, offset by half a step so that 0 is never hit."""
    hi = np.asarray(hi, dtype=np.uint64)
    lo = np.asarray(lo, dtype=np.uint64)
    w = (hi << np.uint64(32)) | lo
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def _key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def gaussian_block(n, l, seed):
    """Start block X0 in R^{n x l} with i.i.d. N(0, 1) entries (Algorithm 2,
    the l Gaussian vectors; Sec. 3.1 for the distribution).

    Entry (i, j) uses Philox counter (i_lo, i_hi, j, 0) under key = seed; the
    four output words give two uniforms u1, u2 and the Box-Muller (1958)
    transform z = sqrt(-2 ln u1) cos(2 pi u2) in float64.
    """
    k0, k1 = _key(seed)
    i = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(l, dtype=np.uint64)[None, :]
    i, j = np.broadcast_arrays(i, j)
    r0, r1, r2, r3 = philox4x32_10(i & _MASK32, i >> np.uint64(32), j, 0, k0, k1)
    u1 = uniform53(r0, r1)
    u2 = uniform53(r2, r3)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def uniform_draw(seed, counter, stream):
    """One uniform in (0, 1) from Philox counter (counter_lo, counter_hi, 0,
    stream) under key = seed (used by the k-means++ sampling)."""
    k0, k1 = _key(seed)
    c = int(counter)
    r0, r1, _, _ = philox4x32_10(c & 0xFFFFFFFF, c >> 32, 0, stream, k0, k1)
    return float(uniform53(r0, r1))


# ----------------------------------------------------------------------------
# Graph quantities (Sec. 2, Preliminaries)
# ----------------------------------------------------------------------------
def validate_graph(n, indptr, indices, data=None):
    """Checks the graph is a weighted undirected graph as Sec. 2 assumes:
    symmetric A, no self-loops (the degree sums over u != v), weights finite
    and non-negative.  Raises ValueError otherwise."""
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    if indptr.shape != (n + 1,) or indptr[0] != 0 or np.any(np.diff(indptr) < 0):
        raise ValueError("bad row pointer")
    if indices.size and (indices.min() < 0 or indices.max() >= n):
        raise ValueError("column index out of range")
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(indptr))
    if np.any(rows == indices):
        raise ValueError("self-loop")
    w = np.ones(indices.size) if data is None else np.asarray(data, dtype=np.float64)
    if not np.all(np.isfinite(w)) or np.any(w < 0):
        raise ValueError("weights must be finite and non-negative")
    A = sp.csr_matrix((w, indices, indptr), shape=(n, n))
    if abs(A - A.T).sum() != 0.0:
        raise ValueError("adjacency is not symmetric")


def adjacency(n, indptr, indices, data=None):
    """A as a float64 sparse matrix (unit weights when data is None)."""
    w = np.ones(len(indices)) if data is None else np.asarray(data, dtype=np.float64)
    return sp.csr_matrix((w, np.asarray(indices), np.asarray(indptr)), shape=(n, n))


def degrees(n, indptr, indices, data=None):
    """deg(v) = sum_{u != v} w(u, v) (Sec. 2), summed in float64 over the
    entries of row v in the order the row stores them."""
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    w = np.ones(len(indices)) if data is None else np.asarray(data, dtype=np.float64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(indptr))
    w = np.where(indices != rows, w, 0.0)
    d = np.zeros(n)
    np.add.at(d, rows, w)      # unbuffered, in entry order
    return d


def inv_sqrt_degree(d):
    """D^{-1/2} as a vector.  Reading: an isolated vertex (d = 0) has no
    defined D^{-1/2}; it is taken as 0, so its embedding row is 0."""
    out = np.zeros_like(d)
    pos = d > 0
    out[pos] = 1.0 / np.sqrt(d[pos])
    return out


def signless_laplacian(n, indptr, indices, data=None):
    """M = I - N/2 = (I + D^{-1/2} A D^{-1/2}) / 2 (Sec. 2, with the paper's
    halving so that the eigenvalues gamma_i = 1 - lambda_i/2 lie in [0, 1]),
    as a sparse matrix.  An isolated vertex gets the row e_v / 2."""
    A = adjacency(n, indptr, indices, data)
    s = inv_sqrt_degree(degrees(n, indptr, indices, data))
    S = sp.diags(s)
    return (0.5 * (sp.identity(n, format="csr") + S @ A @ S)).tocsr()


# ----------------------------------------------------------------------------
# Algorithm 1 (PowerMethod) and the embedding of Algorithm 2
# ----------------------------------------------------------------------------
def power_method(M, x0, t):
    """Algorithm 1: x_i = M x_{i-1} for i = 1..t; returns x_t.  Applied to
    every column of x0 independently (no normalisation, no
    orthogonalisation)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    for _ in range(t):
        x = M @ x
    return x


def power_method_traced(M, x0, t, rows=None):
    """Algorithm 1 with the per-step column statistics recorded:
    sqnorm[i, j] = ||x_i^{(j)}||^2 for i = 0..t and
    rayleigh[i, j] = x_i^T M x_i / x_i^T x_i = x_i^T x_{i+1} / ||x_i||^2 for
    i = 0..t-1 (a Rayleigh quotient of M, so it lies in [0, 1] by Sec. 2).
    `rows` (a boolean mask) restricts the statistics to those rows."""
    x = np.array(x0, dtype=np.float64, copy=True)
    m = np.ones(x.shape[0], dtype=bool) if rows is None else np.asarray(rows, dtype=bool)
    sq = [np.einsum("ij,ij->j", x[m], x[m])]
    ray = []
    for _ in range(t):
        xn = M @ x
        num = np.einsum("ij,ij->j", x[m], xn[m])
        den = sq[-1]
        ray.append(np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0))
        x = xn
        sq.append(np.einsum("ij,ij->j", x[m], x[m]))
    return x, np.array(sq), np.array(ray).reshape(t, x.shape[1])


def embed(n, indptr, indices, data, l, t, seed=None, x0=None, traced=False):
    """The embedding that Algorithm 2 hands to k-means: D^{-1/2} Y, where the
    columns of Y are PowerMethod(M, x_i, t) for l Gaussian x_i.

    x0 (n x l) overrides the seeded start block.  With traced=True it also
    returns the per-step squared norms and Rayleigh quotients of the y_i.
    Reading: the statistics are taken over the non-isolated vertices only
    (an isolated vertex has no D^{-1/2}, see inv_sqrt_degree).
    """
    if x0 is None:
        x0 = gaussian_block(n, l, seed)
    x0 = np.asarray(x0, dtype=np.float64).reshape(n, l)
    M = signless_laplacian(n, indptr, indices, data)
    d = degrees(n, indptr, indices, data)
    s = inv_sqrt_degree(d)
    if traced:
        Y, sq, ray = power_method_traced(M, x0, t, rows=d > 0)
        return s[:, None] * Y, sq, ray
    Y = power_method(M, x0, t)
    return s[:, None] * Y


# ----------------------------------------------------------------------------
# k-means (Sec. 2.2): k-means++ seeding, then Lloyd's algorithm
# ----------------------------------------------------------------------------
def kmeans_cost(B, labels, k):
    """COST_B(A_1..A_k) = sum_i sum_{u in A_i} ||B(u,:) - mu_i||^2 with mu_i the
    mean of the rows in A_i (Sec. 2.2)."""
    B = np.asarray(B, dtype=np.float64)
    total = 0.0
    for i in range(k):
        rows = B[labels == i]
        if len(rows):
            total += float(((rows - rows.mean(axis=0)) ** 2).sum())
    return total


def kmeanspp_trials(k):
    """Candidates per round of the greedy seeding: 2 + floor(ln k)."""
    return 2 + int(np.floor(np.log(k)))


def kmeanspp(P, k, seed, eligible=None, trials=None):
    """k-means++ seeding (Arthur and Vassilvitskii, as cited in Sec. 2.2), in
    its greedy form: each round draws several candidates by D^2 sampling and
    keeps the one that lowers the potential sum_v min(D2(v), ||P_v - c||^2)
    most.

    Reading of the sampling, with the Philox uniforms of this module:
      * centre 0: with u from stream 1, the row v whose inclusive running
        count of eligible rows first exceeds u * n_eligible;
      * centre r >= 1: D2(v) = min over chosen centres of ||P_v - c||^2 on
        eligible rows (0 on the others); candidate j (0 <= j < L, L = trials,
        by default 2 + floor(ln k)) takes u from stream 3, counter r * L + j,
        and is the smallest v whose inclusive float64 running sum of D2
        exceeds u * sum(D2); the candidate with the smallest potential over
        the eligible rows wins, ties to the lower j;
      * if sum(D2) == 0: every candidate is the smallest eligible row not
        chosen yet, else the smallest row not chosen yet.
    trials = 1 is plain D^2 sampling.  Returns the chosen row indices.
    """
    P = np.asarray(P, dtype=np.float64)
    n = P.shape[0]
    elig = np.ones(n, dtype=bool) if eligible is None else np.asarray(eligible, dtype=bool)
    L = kmeanspp_trials(k) if trials is None else int(trials)
    chosen = []

    def pick(weights, u):
        run = np.cumsum(weights)        # inclusive running sum, index order
        total = float(run[-1]) if n else 0.0
        if total > 0.0:
            v = int(np.searchsorted(run, u * total, side="right"))
            if v >= n:  # rounding left the target at the very end
                v = int(np.nonzero(weights > 0)[0][-1])
            return v
        for v in range(n):
            if elig[v] and v not in chosen:
                return v
        for v in range(n):
            if v not in chosen:
                return v
        raise ValueError("k exceeds n")

    chosen.append(pick(elig.astype(np.float64), uniform_draw(seed, 0, 1)))
    d2 = np.full(n, np.inf)
    for r in range(1, k):
        d2 = np.minimum(d2, ((P - P[chosen[-1]]) ** 2).sum(axis=1))
        w = np.where(elig, d2, 0.0)
        best, best_pot = None, None
        for j in range(L):
            v = pick(w, uniform_draw(seed, r * L + j, 3))
            pot = float(np.where(elig, np.minimum(d2, ((P - P[v]) ** 2).sum(axis=1)), 0.0).sum())
            if best is None or pot < best_pot:
                best, best_pot = v, pot
        chosen.append(best)
    return chosen


def assign(P, centres):
    """Nearest centre by the direct float64 squared distance; ties go to the
    lowest centre index."""
    P = np.asarray(P, dtype=np.float64)
    C = np.asarray(centres, dtype=np.float64)
    out = np.empty(P.shape[0], dtype=np.int64)
    step = 1 << 15
    for s in range(0, P.shape[0], step):
        blk = P[s:s + step]
        dist = ((blk[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
        out[s:s + step] = np.argmin(dist, axis=1)  # first minimum wins
    return out


def lloyd(P, centres, iters, eligible=None):
    """Lloyd's algorithm (Sec. 2.2): `iters` rounds of (assign every row to its
    nearest centre, move every centre to the mean of its eligible rows).
    Reading: a centre with no rows keeps its position; a final assignment
    makes the labels agree with the returned centres."""
    P = np.asarray(P, dtype=np.float64)
    C = np.array(centres, dtype=np.float64, copy=True)
    n = P.shape[0]
    elig = np.ones(n, dtype=bool) if eligible is None else np.asarray(eligible, dtype=bool)
    for _ in range(iters):
        lab = assign(P, C)
        for j in range(C.shape[0]):
            rows = P[(lab == j) & elig]
            if len(rows):
                C[j] = rows.sum(axis=0) / len(rows)
    return assign(P, C), C


def kmeans(P, k, iters, seed, eligible=None):
    """k-means++ seeding followed by `iters` Lloyd rounds."""
    P = np.asarray(P, dtype=np.float64)
    idx = kmeanspp(P, k, seed, eligible)
    return lloyd(P, P[idx], iters, eligible)


def fast_spectral_cluster(n, indptr, indices, data, k, l, t, seed, kmeans_iters,
                          x0=None):
    """Algorithm 2 end to end: embedding D^{-1/2} Y, then k-means on it.
    Isolated vertices (reading: d = 0) take no part in the k-means fit and are
    labelled by their nearest final centre.  Returns (labels, centres, E)."""
    E = embed(n, indptr, indices, data, l, t, seed=seed, x0=x0)
    d = degrees(n, indptr, indices, data)
    labels, C = kmeans(E, k, kmeans_iters, seed, eligible=d > 0)
    return labels, C, E


# ----------------------------------------------------------------------------
# The eigenvector baselines of Sec. 4 ("k Eigenvectors", "log(k) Eigenvectors")
# ----------------------------------------------------------------------------
def eigs_embed(n, indptr, indices, data, m):
    """The m leading eigenvectors F of M (the m smallest of the normalised
    Laplacian, Sec. 2) from a dense symmetric eigendecomposition, embedded as
    D^{-1/2} F like Algorithm 2's D^{-1/2} Y (isolated rows 0).  Returns
    (E, gamma) with gamma the m largest eigenvalues, descending."""
    M = signless_laplacian(n, indptr, indices, data).toarray()
    gam, F = np.linalg.eigh(M)
    F = F[:, ::-1][:, :m]
    d = degrees(n, indptr, indices, data)
    return inv_sqrt_degree(d)[:, None] * F, gam[::-1][:m].copy()


def eigs_cluster(n, indptr, indices, data, k, m, seed, kmeans_iters):
    """k-means (as in fast_spectral_cluster) on eigs_embed."""
    E, _ = eigs_embed(n, indptr, indices, data, m)
    d = degrees(n, indptr, indices, data)
    labels, C = kmeans(E, k, kmeans_iters, seed, eligible=d > 0)
    return labels, C, E


# ----------------------------------------------------------------------------
# k nearest neighbours: the pre-processing of the real-world data (Sec. 4.2)
# ----------------------------------------------------------------------------
def knn_rows(X, rows, knn):
    """The knn nearest other points of each listed row of X by squared
    Euclidean distance, brute force in float64 from the coordinate
    differences; ties to the lower index.  Returns (indices, squared
    distances), each len(rows) x knn, nearest first."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    nbr = np.empty((len(rows), knn), dtype=np.int64)
    dist = np.empty((len(rows), knn))
    for i, q in enumerate(rows):
        d = ((X - X[q]) ** 2).sum(axis=1)
        d[q] = np.inf
        order = np.lexsort((np.arange(n), d))[:knn]
        nbr[i] = order
        dist[i] = d[order]
    return nbr, dist


def knn(X, knn):
    """knn_rows over every row."""
    return knn_rows(X, np.arange(np.asarray(X).shape[0]), knn)


def knn_graph(X, k):
    """The symmetrised kNN graph (Sec. 4.2 joins each point to its k
    nearest).  Readings: the union of the directed edges; weight
    exp(-d / sigma^2) with sigma^2 the median of the directed squared
    distances and d taken from the list of the pair's lower-indexed endpoint
    when it holds the pair (all weights 1 if sigma^2 = 0).  Returns CSR
    (indptr, indices, weights) with both directions, rows sorted by column."""
    nbr, dist = knn(X, k)
    n = nbr.shape[0]
    sigma2 = float(np.median(dist))
    pairs = {}
    for u in range(n):
        for j in range(k):
            v = int(nbr[u, j])
            key = (min(u, v), max(u, v))
            if key not in pairs:
                pairs[key] = np.exp(-dist[u, j] / sigma2) if sigma2 > 0 else 1.0
    rows, cols, ws = [], [], []
    for (a, b), w in pairs.items():
        rows += [a, b]
        cols += [b, a]
        ws += [w, w]
    A = sp.csr_matrix((ws, (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int64), A.data


# ----------------------------------------------------------------------------
# PM with k vectors: the comparison method of Sec. 4, whose embedding is k
# mutually orthogonal vectors obtained by the power method (the algorithm of
# Boutsidis et al.; Sec. 1.1 notes its extra singular value decomposition)
# ----------------------------------------------------------------------------
PMK_CUT = 1e-12


def orthonormal_basis(Y):
    """An orthonormal basis of the columns of Y (rows x k): the left singular
    vectors (LAPACK's SVD in float64), in descending order of singular value,
    a column whose singular value is at most PMK_CUT of the largest set to 0
    (float64 cannot tell that direction from none).  Fewer rows than k leave
    the trailing columns 0.  Returns (U, sigma), both padded to k columns."""
    rows, k = Y.shape
    U = np.zeros((rows, k))
    sigma = np.zeros(k)
    if rows == 0:
        return U, sigma
    u, sv, _ = np.linalg.svd(Y, full_matrices=False)
    r = len(sv)
    sigma[:r] = sv
    keep = (sv > 0) & (sv > PMK_CUT * sv[0])
    U[:, :r] = np.where(keep[None, :], u, 0.0)
    return U, sigma


def pm_k_iterate(n, indptr, indices, data, k, t, seed=None, x0=None):
    """Orthogonal (subspace) iteration on k vectors, over the non-isolated
    rows: Q_0 = basis(X0), then for i = 1..t, Y_i = M Q_{i-1} and
    Q_i = basis(Y_i), with basis() the orthonormalisation above after every
    step.  In exact arithmetic span(Q_t) = span(M^t X0), so this is the power
    method on k vectors kept orthogonal; the per-step orthonormalisation keeps
    every direction that float64 resolves at any t (without it the columns of
    M^t X0 all turn towards the leading eigenvector).

    Returns (U, sigma): U = Q_t (n x k, isolated rows 0), sigma the singular
    values of Y_t (of X0 when t = 0), descending.  Reading: each column's sign
    makes its largest-magnitude entry positive (the first such entry on a
    tie); an isolated vertex has no D^{-1/2} and takes no part."""
    if x0 is None:
        x0 = gaussian_block(n, k, seed)
    x0 = np.asarray(x0, dtype=np.float64).reshape(n, k)
    d = degrees(n, indptr, indices, data)
    rows = np.flatnonzero(d > 0)
    M = signless_laplacian(n, indptr, indices, data)[rows][:, rows]
    Q, sigma = orthonormal_basis(x0[rows])
    for _ in range(t):
        Q, sigma = orthonormal_basis(M @ Q)
    for j in range(k):
        if Q.shape[0] and Q[int(np.argmax(np.abs(Q[:, j]))), j] < 0:
            Q[:, j] = -Q[:, j]
    U = np.zeros((n, k))
    U[rows] = Q
    return U, sigma


def pm_k_embed(n, indptr, indices, data, k, t, seed=None, x0=None):
    """The embedding of PM with k vectors: D^{-1/2} U with U = pm_k_iterate's
    orthonormal basis, the rows k-means sees (as Algorithm 2 embeds
    D^{-1/2} Y)."""
    U, _ = pm_k_iterate(n, indptr, indices, data, k, t, seed=seed, x0=x0)
    return inv_sqrt_degree(degrees(n, indptr, indices, data))[:, None] * U


def pm_k_cluster(n, indptr, indices, data, k, t, seed, kmeans_iters, x0=None):
    """PM with k vectors end to end: pm_k_embed, then k-means exactly as in
    fast_spectral_cluster (isolated vertices out of the fit).  Returns
    (labels, centres, E)."""
    E = pm_k_embed(n, indptr, indices, data, k, t, seed=seed, x0=x0)
    d = degrees(n, indptr, indices, data)
    labels, C = kmeans(E, k, kmeans_iters, seed, eligible=d > 0)
    return labels, C, E


# ----------------------------------------------------------------------------
# Accuracy scores of Sec. 4.2: normalised mutual information and the
# adjusted Rand index (Hubert and Arabie)
# ----------------------------------------------------------------------------
def nmi(a, b):
    """Normalised mutual information (the second accuracy score of Sec. 4.2)
    from the contingency table, natural logarithms:
    I(A; B) / ((H(A) + H(B)) / 2).  Readings: the paper cites the score
    without fixing its normalisation; this is the arithmetic mean of the two
    entropies.  When both entropies are 0 (each labeling one cluster) the
    score is 1; I is clipped at 0 against rounding."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    n = a.size
    if n == 0:
        return 1.0
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    table = np.zeros((ai.max() + 1, bi.max() + 1))
    np.add.at(table, (ai, bi), 1.0)
    pa = table.sum(axis=1) / n
    pb = table.sum(axis=0) / n
    ha = -float(np.sum(pa * np.log(pa)))
    hb = -float(np.sum(pb * np.log(pb)))
    nz = table > 0
    pij = table[nz] / n
    mi = float(np.sum(pij * np.log(pij / np.outer(pa, pb)[nz])))
    mi = max(mi, 0.0)
    if ha + hb == 0.0:
        return 1.0
    return mi / (0.5 * (ha + hb))


def _comb2(x):
    x = np.asarray(x, dtype=np.float64)
    return x * (x - 1.0) / 2.0


def ari(a, b):
    """ARI from the contingency table:
    (sum_ij C(n_ij, 2) - E) / (mean(sum_i C(a_i,2), sum_j C(b_j,2)) - E), with
    E = sum_i C(a_i,2) sum_j C(b_j,2) / C(n, 2).  Reading: when the
    denominator vanishes (both labelings trivial) the score is 1."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    n = a.size
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    table = np.zeros((ai.max() + 1 if n else 1, bi.max() + 1 if n else 1))
    np.add.at(table, (ai, bi), 1.0)
    sum_ij = _comb2(table).sum()
    sa = _comb2(table.sum(axis=1)).sum()
    sb = _comb2(table.sum(axis=0)).sum()
    total = _comb2(n)
    expected = sa * sb / total if total > 0 else 0.0
    denom = 0.5 * (sa + sb) - expected
    if denom == 0.0:
        return 1.0
    return float((sum_ij - expected) / denom)
