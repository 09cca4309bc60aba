"""Pins for the FP64 oracle: every check below compares the oracle with
something other than itself -- published known-answer vectors, closed forms
from the spectra of special graphs, library routines (scipy's normalised
Laplacian, numpy's eigensolver and FFT, scikit-learn's Lloyd and ARI),
brute force, and statistical facts the paper states."""
import itertools
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
from scipy import stats

import synth
from oracle import fsc_oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def test_philox_known_answers():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        c0, c1, c2, c3, k0, k1 = (int(x, 16) for x in r[:6])
        want = [int(x, 16) for x in r[6:]]
        got = [int(x) for x in o.philox4x32_10(c0, c1, c2, c3, k0, k1)]
        assert got == want


def test_uniform53_endpoints():
    # closed form: the map is ((w >> 11) + 1/2) * 2^-53 on the 64-bit word w
    assert o.uniform53(0, 0) == 0.5 * 2.0 ** -53
    assert o.uniform53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 0.5 * 2.0 ** -53
    assert o.uniform53(0x80000000, 0) == 0.5 + 0.5 * 2.0 ** -53


def test_gaussian_block_distribution():
    # Sec. 3.1 / Algorithm 2: start vectors are N(0, I).  KS test against the
    # normal CDF, and the chi-square facts of Lemma A.1 (E||x||^2 = n,
    # ||x||^2 <= 6n).
    n, l = 200_000, 4
    X = o.gaussian_block(n, l, seed=1234)
    assert X.shape == (n, l)
    for j in range(l):
        assert stats.kstest(X[:, j], "norm").pvalue > 1e-4
        sq = float((X[:, j] ** 2).sum())
        assert abs(sq - n) < 6 * np.sqrt(2 * n)        # chi^2_n: sd sqrt(2n)
        assert sq <= 6 * n
    # columns are independent: correlations at the 1/sqrt(n) scale
    c = np.corrcoef(X.T)
    assert np.abs(c - np.eye(l)).max() < 5 / np.sqrt(n)
    # seeds give different streams, the same seed the same one
    assert np.array_equal(X[:100], o.gaussian_block(100, l, seed=1234))
    assert not np.allclose(X[:100], o.gaussian_block(100, l, seed=1235))


# --------------------------------------------------------------------------
# Degrees and the signless Laplacian (Sec. 2)
# --------------------------------------------------------------------------
def _hand_graph():
    # path 0-1-2 with weights 2, 3 and a pendant 3-1 with weight 0.5
    return synth.csr_from_edges(4, [0, 1, 3], [1, 2, 1], [2.0, 3.0, 0.5])


def test_degrees_by_hand():
    g = _hand_graph()
    d = o.degrees(g.n, g.indptr, g.indices, g.data)
    assert d.tolist() == [2.0, 5.5, 3.0, 0.5]


def test_degree_sum_is_twice_edge_weight():
    g = synth.random_weighted(300, 1500, seed=3)
    d = o.degrees(g.n, g.indptr, g.indices, g.data)
    # every undirected edge appears twice in the CSR
    assert np.isclose(d.sum(), g.data.sum(), rtol=1e-14)


def _lib_signless(g):
    """M from scipy's own normalised Laplacian: M = I - N/2 (Sec. 2)."""
    A = sp.csr_matrix((np.ones(g.nnz) if g.data is None else g.data, g.indices, g.indptr),
                      shape=(g.n, g.n))
    N = csgraph.laplacian(A.toarray(), normed=True)
    return np.eye(g.n) - 0.5 * N


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_signless_laplacian_matches_scipy(seed):
    g = synth.random_weighted(120, 900, seed=seed)
    assert np.all(o.degrees(g.n, g.indptr, g.indices, g.data) > 0)
    M = o.signless_laplacian(g.n, g.indptr, g.indices, g.data).toarray()
    assert np.abs(M - _lib_signless(g)).max() < 1e-15


@pytest.mark.parametrize("seed", [0, 1])
def test_power_method_equals_eigen_expansion(seed):
    # x_t = sum_i a_i gamma_i^t f_i (Sec. 3.1), with the spectrum from a
    # library eigensolver of scipy's normalised Laplacian; gamma in [0, 1].
    g = synth.random_weighted(150, 1200, seed=seed)
    l, t = 3, 17
    Mlib = _lib_signless(g)
    gam, F = np.linalg.eigh(Mlib)
    assert gam.min() > -1e-12 and gam.max() < 1 + 1e-12
    assert abs(gam.max() - 1.0) < 1e-12               # gamma_1 = 1
    X0 = o.gaussian_block(g.n, l, seed=seed + 10)
    want = F @ (gam[:, None] ** t * (F.T @ X0))
    M = o.signless_laplacian(g.n, g.indptr, g.indices, g.data)
    got = o.power_method(M, X0, t)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # the embedding is D^{-1/2} of that
    d = np.asarray(sp.csr_matrix((g.data, g.indices, g.indptr)).sum(axis=1)).ravel()
    E = o.embed(g.n, g.indptr, g.indices, g.data, l, t, x0=X0)
    assert np.abs(E - want / np.sqrt(d)[:, None]).max() < 1e-12 * np.abs(want).max()


def test_cliques_closed_form():
    # k disjoint K_s: the top eigenspace (gamma = 1, multiplicity k) holds the
    # per-clique constants; every other eigenvalue is (s-2)/(2(s-1)).  So
    # Y_t = PX + g^t (X - PX) with PX the per-clique column mean, and the
    # embedding is constant per clique up to g^t.
    k, s, l, t = 4, 9, 3, 11
    g = synth.disjoint_cliques(k, s)
    X0 = o.gaussian_block(g.n, l, seed=5)
    PX = np.repeat(X0.reshape(k, s, l).mean(axis=1), s, axis=0)
    gam = (s - 2) / (2 * (s - 1))
    want = (PX + gam ** t * (X0 - PX)) / np.sqrt(s - 1)
    E = o.embed(g.n, g.indptr, g.indices, None, l, t, x0=X0)
    assert np.abs(E - want).max() < 1e-14
    E40 = o.embed(g.n, g.indptr, g.indices, None, l, 40, x0=X0)
    spread = np.abs(E40.reshape(k, s, l) - E40.reshape(k, s, l).mean(axis=1, keepdims=True)).max()
    assert spread < 1e-12


def test_cycle_fourier_closed_form():
    # C_n: M is a circulant with eigenvalues cos^2(pi j / n) on the Fourier modes
    n, t = 64, 9
    g = synth.cycle(n)
    x = o.gaussian_block(n, 1, seed=2)[:, 0]
    lam = np.cos(np.pi * np.arange(n) / n) ** 2
    want = np.real(np.fft.ifft(np.fft.fft(x) * lam ** t))
    M = o.signless_laplacian(n, g.indptr, g.indices, None)
    assert np.abs(o.power_method(M, x[:, None], t)[:, 0] - want).max() < 1e-13


def test_complete_bipartite_extreme_eigenvectors():
    # K_{a,b}: D^{1/2} (+1 on one side, -1 on the other) has gamma = 0, and
    # D^{1/2} 1 has gamma = 1.
    a, b = 5, 8
    g = synth.complete_bipartite(a, b)
    M = o.signless_laplacian(g.n, g.indptr, g.indices, None)
    sd = np.sqrt(np.r_[np.full(a, b), np.full(b, a)].astype(float))
    f0 = sd * np.r_[np.ones(a), -np.ones(b)]
    f1 = sd
    assert np.abs(M @ f0).max() < 1e-14
    assert np.abs(M @ f1 - f1).max() < 1e-14


def test_large_t_embedding_is_constant_on_connected_graph():
    # D^{-1/2} f_1 is constant (Sec. 2): after many steps on a connected,
    # non-bipartite graph every column of E is (nearly) constant.
    g = synth.sbm(200, 1, 0.2, 0.0, seed=1)
    assert csgraph.connected_components(sp.csr_matrix((np.ones(g.nnz), g.indices, g.indptr)))[0] == 1
    E = o.embed(g.n, g.indptr, g.indices, None, 2, 400, seed=9)
    assert (E.std(axis=0) / np.abs(E.mean(axis=0))).max() < 1e-8


def test_trace_rayleigh_quotients():
    # Rayleigh quotients of M lie in [0, 1] and equal x^T M x / x^T x computed
    # with the library M; squared norms never grow (||M|| <= 1).
    g = synth.random_weighted(100, 700, seed=4)
    X0 = o.gaussian_block(g.n, 2, seed=1)
    E, sq, ray = o.embed(g.n, g.indptr, g.indices, g.data, 2, 6, x0=X0, traced=True)
    Mlib = _lib_signless(g)
    x = X0.copy()
    for i in range(6):
        want = np.einsum("ij,ij->j", x, Mlib @ x) / np.einsum("ij,ij->j", x, x)
        assert np.abs(ray[i] - want).max() < 1e-13
        assert np.abs(sq[i] - np.einsum("ij,ij->j", x, x)).max() < 1e-10 * sq[i].max()
        x = Mlib @ x
    assert np.all((ray >= 0) & (ray <= 1))
    assert np.all(np.diff(sq, axis=0) <= 1e-12 * sq[:-1])


def test_isolated_vertices_embed_to_zero():
    g = synth.random_weighted(50, 200, seed=1, isolated=5)
    E = o.embed(g.n, g.indptr, g.indices, g.data, 3, 5, seed=1)
    assert np.all(E[-5:] == 0.0)
    assert np.all(np.abs(E[:-5]).sum(axis=1) > 0)


def test_validate_graph_rejects_bad_graphs():
    g = _hand_graph()
    o.validate_graph(g.n, g.indptr, g.indices, g.data)
    with pytest.raises(ValueError):
        o.validate_graph(2, [0, 1, 1], [0], None)                   # self-loop
    with pytest.raises(ValueError):
        o.validate_graph(2, [0, 1, 1], [1], None)                   # asymmetric
    with pytest.raises(ValueError):
        o.validate_graph(2, [0, 1, 2], [1, 0], [-1.0, -1.0])        # negative
    with pytest.raises(ValueError):
        o.validate_graph(2, [0, 1, 2], [1, 2], None)                # out of range


# --------------------------------------------------------------------------
# k-means (Sec. 2.2)
# --------------------------------------------------------------------------
def test_kmeans_cost_matrix_identity():
    # COST_B = ||B - X X^T B||_F^2 with X the scaled partition indicator
    # (the identity the appendix uses to bound the k-means cost).
    rng = np.random.default_rng(0)
    B = rng.standard_normal((40, 3))
    lab = rng.integers(0, 4, 40)
    X = np.zeros((40, 4))
    for i in range(4):
        m = lab == i
        X[m, i] = 1 / np.sqrt(m.sum())
    assert np.isclose(o.kmeans_cost(B, lab, 4), np.linalg.norm(B - X @ X.T @ B) ** 2, rtol=1e-12)


def test_kmeans_not_below_brute_force_optimum():
    rng = np.random.default_rng(1)
    for trial in range(5):
        P = rng.standard_normal((8, 2))
        k = 3
        best = min(o.kmeans_cost(P, np.array(lab), k)
                   for lab in itertools.product(range(k), repeat=8) if len(set(lab)) == k)
        lab, C = o.kmeans(P, k, 20, seed=trial)
        assert o.kmeans_cost(P, lab, k) >= best - 1e-12
    # well separated: Lloyd reaches the optimum
    P = np.r_[rng.normal(0, .05, (3, 2)), rng.normal(5, .05, (3, 2)), rng.normal([0, 5], .05, (2, 2))]
    best = min(o.kmeans_cost(P, np.array(lab), 3)
               for lab in itertools.product(range(3), repeat=8) if len(set(lab)) == 3)
    lab, C = o.kmeans(P, 3, 20, seed=0)
    assert np.isclose(o.kmeans_cost(P, lab, 3), best, rtol=1e-12)


def test_lloyd_matches_sklearn():
    from sklearn.cluster import KMeans
    X, _ = synth.gaussian_mixture(300, 5, 4, seed=2, mean_scale=3.0)
    X = X.astype(np.float64)
    init = X[[0, 300, 600, 900, 1200]] + 0.3
    lab, C = o.lloyd(X, init, 50)
    km = KMeans(5, init=init, n_init=1, max_iter=50, tol=0.0, algorithm="lloyd").fit(X)
    assert np.array_equal(lab, km.labels_)
    assert np.abs(C - km.cluster_centers_).max() < 1e-10


def test_lloyd_fixed_point_and_empty_cluster():
    X, _ = synth.gaussian_mixture(100, 3, 2, seed=3, mean_scale=4.0)
    X = X.astype(np.float64)
    # a fourth centre far away never gets a row: it must keep its position
    init = np.r_[X[[0, 100, 200]], [[1e3, 1e3]]]
    lab, C = o.lloyd(X, init, 30)
    assert np.array_equal(C[3], [1e3, 1e3])
    for j in range(3):
        assert np.allclose(C[j], X[lab == j].mean(axis=0), atol=1e-12)
    d = ((X[:, None] - C[None]) ** 2).sum(-1)
    assert np.all(d[np.arange(len(X)), lab] <= d.min(axis=1))


def test_kmeanspp_samples_proportional_to_d2():
    # k-means++: the second centre is drawn with probability D^2 / sum D^2
    # (the first is uniform).  Empirical frequencies over many seeds.
    P = np.array([[0.0], [1.0], [3.0], [6.0], [10.0]])
    trials = 6000
    first = np.zeros(5)
    second = np.zeros((5, 5))
    for s in range(trials):
        c = o.kmeanspp(P, 2, seed=s, trials=1)
        first[c[0]] += 1
        second[c[0], c[1]] += 1
    assert stats.chisquare(first).pvalue > 1e-4
    for a in range(5):
        d2 = (P[:, 0] - P[a, 0]) ** 2
        exp = d2 / d2.sum() * second[a].sum()
        m = exp > 0
        assert second[a, ~m].sum() == 0                # the centre itself never again
        assert stats.chisquare(second[a, m], exp[m]).pvalue > 1e-4


def test_greedy_kmeanspp_keeps_the_best_candidate():
    """Each round's winner is the candidate (drawn by D^2 sampling, checked
    by rerunning the plain sampling with the same uniforms) whose potential,
    recomputed here by brute force over the rows, is smallest."""
    rng = np.random.default_rng(5)
    P = rng.standard_normal((40, 3))
    elig = np.ones(40, dtype=bool)
    elig[[3, 17]] = False
    k = 5
    L = o.kmeanspp_trials(k)
    assert L == 2 + int(np.floor(np.log(k)))
    for seed in range(10):
        c = o.kmeanspp(P, k, seed, eligible=elig)
        for r in range(1, k):
            d2 = np.array([min(((P[v] - P[x]) ** 2).sum() for x in c[:r]) for v in range(40)])
            w = np.where(elig, d2, 0.0)
            cands = []
            for j in range(L):
                u = o.uniform_draw(seed, r * L + j, 3)
                run = np.cumsum(w)
                cands.append(int(np.searchsorted(run, u * run[-1], side="right")))
            pots = [sum(min(w[v], ((P[v] - P[x]) ** 2).sum()) for v in range(40) if elig[v]) for x in cands]
            assert c[r] == cands[int(np.argmin(pots))]
            assert elig[c[r]]


def test_greedy_kmeanspp_separates_well_spread_blobs():
    """Five tight blobs far apart: the greedy seeding puts one centre in
    each blob for every seed (plain D^2 sampling may put two in one)."""
    rng = np.random.default_rng(1)
    means = np.array([[0, 0], [10, 0], [0, 10], [10, 10], [5, 25]], dtype=float)
    sizes = [400, 30, 30, 200, 10]
    P = np.concatenate([m + 0.1 * rng.standard_normal((s_, 2)) for m, s_ in zip(means, sizes)])
    blob = np.repeat(np.arange(5), sizes)
    for seed in range(30):
        c = o.kmeanspp(P, 5, seed)
        assert sorted(blob[c]) == [0, 1, 2, 3, 4]


def test_kmeanspp_respects_eligibility_and_degenerate_case():
    P = np.zeros((6, 2))                               # all points equal: sum D^2 = 0
    elig = np.array([0, 1, 0, 1, 1, 0], dtype=bool)
    c = o.kmeanspp(P, 4, seed=3, eligible=elig)
    assert sorted(c[:1]) and elig[c[0]]
    # after the first draw the rule takes the smallest unchosen eligible rows,
    # then the smallest unchosen rows
    rest = [v for v in [1, 3, 4] if v != c[0]]
    assert c[1:3] == rest and c[3] == 0
    P = np.random.default_rng(0).standard_normal((50, 2))
    elig = np.arange(50) % 3 == 0
    for s in range(20):
        assert all(elig[v] for v in o.kmeanspp(P, 5, seed=s, eligible=elig))


# --------------------------------------------------------------------------
# ARI (Sec. 4.2)
# --------------------------------------------------------------------------
def test_ari_matches_sklearn():
    from sklearn.metrics import adjusted_rand_score
    rng = np.random.default_rng(0)
    for _ in range(20):
        n = int(rng.integers(2, 500))
        a = rng.integers(0, rng.integers(1, 8), n)
        b = np.where(rng.random(n) < 0.7, a, rng.integers(0, 6, n))
        assert abs(o.ari(a, b) - adjusted_rand_score(a, b)) < 1e-12
    a = rng.integers(0, 5, 100)
    assert o.ari(a, a) == 1.0
    perm = np.array([3, 1, 4, 0, 2])
    assert abs(o.ari(a, perm[a]) - 1.0) < 1e-15
    assert o.ari(np.zeros(10), np.zeros(10)) == 1.0


# --------------------------------------------------------------------------
# Whole pipeline (Algorithm 2)
# --------------------------------------------------------------------------
def test_pipeline_recovers_cliques_and_small_sbm():
    g = synth.disjoint_cliques(5, 12)
    lab, C, E = o.fast_spectral_cluster(g.n, g.indptr, g.indices, None, 5, 3, 30, 7, 20)
    assert o.ari(lab, g.labels) == 1.0
    # the small SBM the paper's synthetic experiments describe: every method
    # recovers the planted clusters (Sec. 4.1)
    g = synth.sbm(1000, 5, 0.5, 0.01, seed=0)
    lab, C, E = o.fast_spectral_cluster(g.n, g.indptr, g.indices, None, 5, 3, 20, 0, 20)
    assert o.ari(lab, g.labels) > 0.99


def test_nmi_matches_scikit_learn_and_closed_forms():
    from sklearn.metrics import normalized_mutual_info_score as sk_nmi
    rng = np.random.default_rng(4)
    for n, ka, kb in [(50, 3, 4), (1000, 10, 10), (333, 2, 7)]:
        a = rng.integers(0, ka, n)
        b = np.where(rng.random(n) < 0.6, a % kb, rng.integers(0, kb, n))
        assert abs(o.nmi(a, b) - sk_nmi(a, b, average_method="arithmetic")) < 1e-12
    a = rng.integers(0, 5, 200)
    assert abs(o.nmi(a, (a + 3) % 5) - 1.0) < 1e-12          # a relabelling
    i = np.arange(9 * 40)
    assert abs(o.nmi(i % 3, (i // 3) % 3)) < 1e-12              # independent: I = 0
    assert o.nmi(np.zeros(7), np.zeros(7)) == 1.0                # both one cluster
    assert o.nmi(np.zeros(8), np.arange(8) % 2) == 0.0           # one trivial labeling


# ---- PM with k vectors (the comparison method of Sec. 4) ----
def _dense_M(g):
    """M = (I + D^{-1/2} A D^{-1/2}) / 2 built densely from the edge list, an
    isolated vertex's D^{-1/2} taken as 0 (its row of M is e_v / 2)."""
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.indptr))
    A[rows, g.indices] = 1.0 if g.data is None else g.data
    d = A.sum(axis=1)
    s = np.where(d > 0, 1.0 / np.sqrt(np.where(d > 0, d, 1.0)), 0.0)
    return 0.5 * (np.eye(g.n) + s[:, None] * A * s[None, :]), d


def test_pm_k_on_disjoint_cliques_spans_the_cluster_indicators():
    g = synth.disjoint_cliques(4, 6)
    E = o.pm_k_embed(g.n, g.indptr, g.indices, g.data, 4, 80, seed=3)
    d = np.full(g.n, 5.0)
    U = np.sqrt(d)[:, None] * E
    B = np.zeros((g.n, 4))
    B[np.arange(g.n), g.labels] = 1.0 / np.sqrt(6.0)      # orthonormal cluster indicators
    cos = np.linalg.svd(B.T @ U, compute_uv=False)
    assert cos.min() > 1 - 1e-12
    lab, _, _ = o.pm_k_cluster(g.n, g.indptr, g.indices, g.data, 4, 80, 3, 10)
    assert o.ari(lab, g.labels) == 1.0


def test_pm_k_columns_are_orthonormal_and_span_the_power_iterate():
    g = synth.random_weighted(60, 150, seed=5, isolated=3)
    k, t, seed = 5, 7, 11
    E = o.pm_k_embed(g.n, g.indptr, g.indices, g.data, k, t, seed=seed)
    U_all, sigma = o.pm_k_iterate(g.n, g.indptr, g.indices, g.data, k, t, seed=seed)
    M, d = _dense_M(g)
    live = d > 0
    assert np.all(E[~live] == 0.0)
    U = np.sqrt(d[live])[:, None] * E[live]
    assert np.abs(U - U_all[live]).max() < 1e-14
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12
    # M^t X0 from the dense eigendecomposition, not from repeated products
    gam, F = np.linalg.eigh(M)
    X0 = o.gaussian_block(g.n, k, seed)
    Y = (F * gam ** t) @ F.T @ X0
    Yl = Y[live]
    assert np.linalg.norm(Yl - U @ (U.T @ Yl)) < 1e-10 * np.linalg.norm(Yl)
    # sigma: the singular values of M applied to an orthonormal basis of
    # M^(t-1) X0 (a Householder QR of the dense expansion)
    B = np.linalg.qr(((F * gam ** (t - 1)) @ F.T @ X0)[live])[0]
    sv = np.linalg.svd(M[np.ix_(live, live)] @ B, compute_uv=False)
    assert np.allclose(sigma, sv, rtol=1e-10)
    assert np.all(np.diff(sigma) <= 0)
    # the sign rule: each column's largest-magnitude entry is positive
    assert all(U[np.argmax(np.abs(U[:, j])), j] > 0 for j in range(k))


def test_pm_k_converges_to_the_top_eigenvectors():
    # three planted clusters: gamma_2, gamma_3 ~ 0.95, the rest of the
    # spectrum below 0.6; at t = 300 gamma_3^t ~ 1e-7, yet all three
    # orthogonal vectors survive and span the leading eigenvectors
    g = synth.sbm(300, 3, 0.5, 0.02, seed=2)
    t = 300
    E = o.pm_k_embed(g.n, g.indptr, g.indices, g.data, 3, t, seed=1)
    _, sigma = o.pm_k_iterate(g.n, g.indptr, g.indices, g.data, 3, t, seed=1)
    M, d = _dense_M(g)
    gam, F = np.linalg.eigh(M)
    assert (gam[-4] / gam[-3]) ** t < 1e-30 and gam[-3] ** t < 1e-6
    U = np.sqrt(d)[:, None] * E
    assert np.abs(U.T @ U - np.eye(3)).max() < 1e-12
    cos = np.linalg.svd(F[:, -3:].T @ U, compute_uv=False)
    assert cos.min() > 1 - 1e-12
    # once converged, M Q = Q diag(gamma): the singular values are the
    # leading eigenvalues
    assert np.allclose(sigma, gam[::-1][:3], rtol=1e-12, atol=0)


def test_pm_k_keeps_every_direction_where_the_plain_iterate_underflows():
    # distinct leading eigenvalues, t large enough that gamma_4^t underflows
    # to 0 in float64: M^t X0 itself has lost columns 2..4, the orthogonal
    # iteration has not
    g = synth.random_weighted(40, 160, seed=3)
    M, d = _dense_M(g)
    assert np.all(d > 0)
    gam, F = np.linalg.eigh(M)
    k, t = 4, 3000
    assert gam[-4] - gam[-5] > 1e-3 and gam[-4] ** t == 0.0
    E = o.pm_k_embed(g.n, g.indptr, g.indices, g.data, k, t, seed=2)
    _, sigma = o.pm_k_iterate(g.n, g.indptr, g.indices, g.data, k, t, seed=2)
    U = np.sqrt(d)[:, None] * E
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12
    cos = np.linalg.svd(F[:, -k:].T @ U, compute_uv=False)
    assert cos.min() > 1 - 1e-12
    assert np.allclose(sigma, gam[::-1][:k], rtol=1e-12, atol=0)
    # where the gaps between the leading eigenvalues are wide, every column is
    # the eigenvector itself (up to the sign rule)
    gaps = np.abs(np.diff(gam[::-1][: k + 1]))
    for j in range(k):
        if min(gaps[max(j - 1, 0)], gaps[j]) > 1e-2:
            f = F[:, -1 - j]
            assert abs(abs(f @ U[:, j]) - 1.0) < 1e-10


def test_pm_k_rank_deficient_block_leaves_zero_columns():
    # a triangle and four isolated vertices: Y has rank at most 3
    g = synth.csr_from_edges(7, np.array([0, 1, 2]), np.array([1, 2, 0]))
    E = o.pm_k_embed(g.n, g.indptr, g.indices, g.data, 5, 3, seed=4)
    assert np.all(E[3:] == 0.0)
    assert np.all(E[:, 3:] == 0.0)
    U = np.sqrt(2.0) * E[:3, :3]
    assert np.abs(U.T @ U - np.eye(3)).max() < 1e-12


# ---- k nearest neighbours (the pre-processing of Sec. 4.2) ----
def test_knn_on_a_line_is_the_closed_form():
    # x_i = i on the first axis: the neighbours of i are i-1, i+1, i-2, i+2, ...
    # (each equal pair to the lower index first), clipped at the ends
    n = 40
    X = np.zeros((n, 4))
    X[:, 0] = np.arange(n)
    nbr, dist = o.knn(X, 6)
    for i in range(n):
        want = sorted((j for j in range(n) if j != i), key=lambda j: ((j - i) ** 2, j))[:6]
        assert list(nbr[i]) == want
        assert np.array_equal(dist[i], [(j - i) ** 2 for j in want])
    assert list(nbr[10]) == [9, 11, 8, 12, 7, 13]


def test_knn_matches_a_kd_tree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(6)
    X = rng.standard_normal((500, 12))
    nbr, dist = o.knn(X, 10)
    dd, ii = cKDTree(X).query(X, k=11)
    assert np.array_equal(nbr, ii[:, 1:])
    assert np.allclose(dist, dd[:, 1:] ** 2, rtol=1e-12)


def test_knn_ties_and_duplicates_go_to_the_lower_index():
    X = np.zeros((6, 4))
    X[3:] = 1.0                      # two groups of three identical points
    nbr, dist = o.knn(X, 4)
    assert list(nbr[0]) == [1, 2, 3, 4] and list(dist[0]) == [0, 0, 4, 4]
    assert list(nbr[4]) == [3, 5, 0, 1]


def test_knn_graph_on_a_line_is_the_closed_form():
    # x_i = i, 2 neighbours: the path plus the pairs {0, 2} and {n-3, n-1};
    # directed distances are 1 except the two ends' second neighbours (4), so
    # sigma^2 = 1
    n = 30
    X = np.zeros((n, 4))
    X[:, 0] = np.arange(n)
    indptr, indices, w = o.knn_graph(X, 2)
    A = sp.csr_matrix((w, indices, indptr), shape=(n, n)).toarray()
    want = np.zeros((n, n))
    for i in range(n - 1):
        want[i, i + 1] = want[i + 1, i] = np.exp(-1.0)
    want[0, 2] = want[2, 0] = want[n - 3, n - 1] = want[n - 1, n - 3] = np.exp(-4.0)
    assert np.array_equal(A, want)
    assert all(np.all(np.diff(indices[indptr[r]:indptr[r + 1]]) > 0) for r in range(n))


def test_knn_graph_is_the_union_of_the_directed_lists():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((200, 8))
    nbr, dist = o.knn(X, 5)
    indptr, indices, w = o.knn_graph(X, 5)
    A = sp.csr_matrix((w, indices, indptr), shape=(200, 200))
    assert (A != A.T).nnz == 0
    D = np.zeros((200, 200), dtype=bool)
    D[np.repeat(np.arange(200), 5), nbr.ravel()] = True
    assert np.array_equal(A.toarray() > 0, D | D.T)
    s2 = np.median(dist)
    assert np.allclose(A[0, nbr[0, 0]], np.exp(-dist[0, 0] / s2), rtol=1e-15)


# ---- eigenvector baselines (Sec. 4) ----
def test_eigs_on_disjoint_cliques_spans_the_cluster_indicators():
    g = synth.disjoint_cliques(3, 7)
    E, gam = o.eigs_embed(g.n, g.indptr, g.indices, g.data, 3)
    assert np.allclose(gam, 1.0, atol=1e-12)                 # eigenvalue 1 once per component
    U = np.sqrt(6.0) * E
    B = np.zeros((g.n, 3))
    B[np.arange(g.n), g.labels] = 1.0 / np.sqrt(7.0)
    assert np.linalg.svd(B.T @ U, compute_uv=False).min() > 1 - 1e-12


def test_eigs_satisfy_the_eigen_equation_and_match_a_sparse_solver():
    from scipy.sparse.linalg import eigsh
    g = synth.sbm(400, 4, 0.2, 0.01, seed=3)
    E, gam = o.eigs_embed(g.n, g.indptr, g.indices, g.data, 4)
    M, d = _dense_M(g)
    F = np.sqrt(d)[:, None] * E
    assert np.abs(M @ F - F * gam).max() < 1e-12
    assert np.abs(F.T @ F - np.eye(4)).max() < 1e-12
    w, V = eigsh(M, k=4, which="LA", tol=1e-14)
    assert np.allclose(np.sort(w)[::-1], gam, atol=1e-10)
    assert np.linalg.svd(V.T @ F, compute_uv=False).min() > 1 - 1e-10
