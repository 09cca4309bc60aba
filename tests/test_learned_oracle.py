"""Pins for the learned-form oracle: dense eigen closed forms of the filter,
the exact Chebyshev expansion of gamma^8, the scatter statistics against the
k-means cost of Sec. 2.2 and against pairwise distances, the loss's lower
bound (smallest generalised eigenvalue), and gradients against central
finite differences and torch's autograd."""
import numpy as np
import pytest
import scipy.sparse.csgraph as csgraph
import scipy.sparse as sp
from numpy.polynomial import Chebyshev as Ch
from numpy.polynomial import chebyshev as C

import synth
from oracle import fsc_learned as fl
from oracle import fsc_oracle as o


def _graph():
    g = synth.random_weighted(120, 800, seed=3)
    M = o.signless_laplacian(g.n, g.indptr, g.indices, g.data)
    A = sp.csr_matrix((g.data, g.indices, g.indptr), shape=(g.n, g.n)).toarray()
    Mlib = np.eye(g.n) - 0.5 * csgraph.laplacian(A, normed=True)
    return g, M, Mlib


def test_chebyshev_basis_matches_spectral_form():
    g, M, Mlib = _graph()
    gam, F = np.linalg.eigh(Mlib)
    X0 = o.gaussian_block(g.n, 3, seed=1)
    B = fl.cheb_basis(M, X0)
    for j in range(fl.NCOEF):
        e = np.zeros(j + 1); e[-1] = 1.0
        Tj = C.chebval(2 * gam - 1, e)          # library Chebyshev T_j at 2 gamma - 1
        want = F @ (Tj[:, None] * (F.T @ X0))
        assert np.abs(B[j] - want).max() < 1e-11 * max(1.0, np.abs(want).max())


def test_gamma8_expansion_reproduces_power_method():
    # gamma^8 = ((x + 1) / 2)^8 with x = 2 gamma - 1; its Chebyshev series in x
    # (numpy's poly2cheb) are the filter coefficients of M^8
    g, M, _ = _graph()
    poly = np.polynomial.polynomial.polypow([0.5, 0.5], 8)
    c = C.poly2cheb(poly)
    assert abs(c.sum() - 1.0) < 1e-14               # p(1) = 1
    X0 = o.gaussian_block(g.n, 2, seed=2)
    got = fl.filter_apply(M, X0, c)
    want = o.power_method(M, X0, 8)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    c_full = fl.full_coefficients(c[1:])
    assert np.allclose(c_full, c, atol=1e-15)


def test_filter_keeps_trivial_eigenvector():
    g, M, _ = _graph()
    d = o.degrees(g.n, g.indptr, g.indices, g.data)
    f1 = np.sqrt(d)[:, None]
    c = fl.full_coefficients(np.random.default_rng(0).standard_normal(8))
    assert np.abs(fl.filter_apply(M, f1, c) - f1).max() < 1e-11


def _stats_graph():
    # 3 planted clusters plus 4 isolated vertices (excluded from the scatter)
    g = synth.sbm(300, 3, 0.1, 0.01, seed=2)
    n = g.n + 4
    indptr = np.concatenate([g.indptr, np.full(4, g.indptr[-1])])
    return n, indptr, g.indices


def test_scatter_stats_are_the_kmeans_cost():
    n, ip, ix = _stats_graph()
    F, W, T, labels = fl.graph_stats(n, ip, ix, None, 3, 2, 15, seed=4)
    assert W.shape == T.shape == (9, 9) and np.allclose(W, W.T) and np.allclose(T, T.T)
    X0 = o.gaussian_block(n, 2, 4)
    M = o.signless_laplacian(n, ip, ix, None)
    d = o.degrees(n, ip, ix, None)
    m = d > 0
    s = o.inv_sqrt_degree(d)
    rng = np.random.default_rng(1)
    for _ in range(3):
        c = fl.full_coefficients(rng.standard_normal(8) * 0.3)
        E = (s[:, None] * fl.filter_apply(M, X0, c))[m]
        assert abs(c @ W @ c - o.kmeans_cost(E, labels[m], 3)) <= 1e-10 * (c @ T @ c)
        # total scatter: the cost of one cluster holding every row
        assert abs(c @ T @ c - o.kmeans_cost(E, np.zeros(m.sum(), dtype=int), 1)) <= 1e-10 * (c @ T @ c)
    # the labels are the plain method's (Algorithm 2)
    lab_p, _, _ = o.fast_spectral_cluster(n, ip, ix, None, 3, 2, 15, 4, 30)
    assert np.array_equal(labels[m], np.asarray(lab_p)[m])
    assert F.shape == (9,)
    # Rayleigh features are quotients of M: inside [0, 1]
    assert np.all((F[5:] >= 0) & (F[5:] <= 1))


def test_scatter_by_pairwise_distances():
    """Within scatter of a cluster C = sum over pairs u < v in C of
    ||e_u - e_v||^2 / |C| (no means involved), on a tiny brute-force case;
    T - W (the between-cluster scatter) is positive semidefinite."""
    rng = np.random.default_rng(3)
    n, l = 23, 3
    Bz = [rng.standard_normal((n, l)) for _ in range(9)]
    labels = rng.integers(0, 4, n)
    mask = np.ones(n, dtype=bool)
    mask[[2, 9]] = False
    W, T = fl.scatter_stats(Bz, labels, mask)
    c = rng.standard_normal(9)
    E = sum(cj * b for cj, b in zip(c, Bz))
    idx = np.nonzero(mask)[0]
    want_w = want_t = 0.0
    for a_ in range(len(idx)):
        for b_ in range(a_ + 1, len(idx)):
            u, v = idx[a_], idx[b_]
            dist = ((E[u] - E[v]) ** 2).sum()
            want_t += dist / len(idx)
            if labels[u] == labels[v]:
                want_w += dist / np.sum(labels[idx] == labels[u])
    assert abs(c @ W @ c - want_w) < 1e-10 * want_t
    assert abs(c @ T @ c - want_t) < 1e-10 * want_t
    assert np.linalg.eigvalsh(W).min() > -1e-10 * np.abs(T).max()
    assert np.linalg.eigvalsh(T - W).min() > -1e-10 * np.abs(T).max()


def test_loss_at_gamma_t_is_the_plain_embeddings_cost():
    """With t = 8 the coefficients of gamma^8 give E(c) = the plain embedding
    (Algorithm 1 output in z-space), so the loss is that embedding's k-means
    cost under its own labels over its total scatter."""
    n, ip, ix = _stats_graph()
    F, W, T, labels = fl.graph_stats(n, ip, ix, None, 3, 2, 8, seed=6)
    c8 = C.poly2cheb(np.polynomial.polynomial.polypow([0.5, 0.5], 8))
    m = o.degrees(n, ip, ix, None) > 0
    E = o.embed(n, ip, ix, None, 2, 8, seed=6)[m]
    want = o.kmeans_cost(E, labels[m], 3) / o.kmeans_cost(E, np.zeros(m.sum(), dtype=int), 1)
    assert abs(fl.ratio(c8, W, T) - want) < 1e-10


def _T8_closed(u):
    """T_8 by its closed forms: cos(8 arccos u) inside [-1, 1], cosh(8
    arccosh |u|) outside (T_8 is even)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    inside = np.abs(u) <= 1
    out[inside] = np.cos(8 * np.arccos(u[inside]))
    out[~inside] = np.cosh(8 * np.arccosh(np.abs(u[~inside])))
    return out


@pytest.mark.parametrize("alpha,beta", [(np.log(0.52), np.log(0.28)), (0.3, -4.0), (-2.5, -1.0), (-0.7, -0.2)])
def test_head_is_the_chebyshev_polynomial_of_the_interval(alpha, beta):
    a, b = fl.interval(alpha, beta)
    assert a < b < 1
    c = fl.full_coefficients(fl.coefficients([[alpha, beta]])[0])
    assert abs(c.sum() - 1.0) < 1e-12                        # p(1) = 1
    g = np.concatenate([np.linspace(0, 1, 101), np.random.default_rng(0).random(50)])
    p = C.chebval(2 * g - 1, c)                              # numpy's Chebyshev series at 2g - 1
    u = lambda x: (2 * x - a - b) / (b - a)
    want = _T8_closed(u(g)) / _T8_closed(u(np.array([1.0])))[0]
    assert np.abs(p - want).max() < 1e-10 * max(1.0, np.abs(want).max())
    # numpy's own change of domain gives the same coefficients
    q = Ch([0] * 8 + [1], domain=[a, b]).convert(domain=[0, 1], kind=Ch).coef
    assert np.abs(q / q.sum() - c).max() < 1e-10 * max(1.0, np.abs(c).max())
    # minimax: on [a, b] |p| reaches its maximum 1 / T_8(u(1)) at the 9
    # extrema of T_8
    ext = (a + b) / 2 + (b - a) / 2 * np.cos(np.pi * np.arange(9) / 8)
    pe = C.chebval(2 * ext - 1, c)
    bound = 1.0 / _T8_closed(u(np.array([1.0])))[0]
    inner = np.linspace(a, b, 1001)
    # rounding: coefficient errors of order eps each, times |T_j(x)| <=
    # T_j(max(1, |x|)) (large where the interval reaches below 0)
    tol = 1e-14 * C.chebval(np.maximum(1.0, np.abs(2 * inner - 1)), np.ones(9)).max()
    assert np.allclose(np.abs(pe), bound, rtol=1e-8, atol=tol)
    assert np.abs(C.chebval(2 * inner - 1, c)).max() <= bound * (1 + 1e-8) + tol


def test_head_derivatives_match_finite_differences():
    for alpha, beta in [(np.log(0.52), np.log(0.28)), (-1.3, -2.2), (0.2, -0.5)]:
        q, qa, qb = fl.head(alpha, beta)
        eps = 1e-6
        fa = (fl.head(alpha + eps, beta)[0] - fl.head(alpha - eps, beta)[0]) / (2 * eps)
        fb = (fl.head(alpha, beta + eps)[0] - fl.head(alpha, beta - eps)[0]) / (2 * eps)
        scale = np.abs(q).max()
        assert np.abs(qa - fa).max() <= 1e-6 * scale
        assert np.abs(qb - fb).max() <= 1e-6 * scale


def test_initial_parameters_give_the_initial_interval():
    p = fl.init_params(0)
    out, _ = fl.mlp_forward(p, np.zeros((1, fl.NFEAT)))
    a, b = fl.interval(out[0, 0], out[0, 1])
    assert abs(a - fl.INIT_A) < 1e-12 and abs(b - fl.INIT_B) < 1e-12
    assert fl.param_count() == 9 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 2 + 2


def _batch(B=5, seed=0):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((B, fl.NFEAT))
    W, T = [], []
    for _ in range(B):
        A = rng.standard_normal((9, 14))
        Bm = rng.standard_normal((9, 5))
        W.append(A @ A.T)
        T.append(A @ A.T + Bm @ Bm.T)      # T = W + a positive semidefinite between part
    return F, np.array(W), np.array(T)


def _lambda_min(W, T):
    """Smallest generalised eigenvalue of (W, T): the least possible ratio."""
    Lc = np.linalg.cholesky(T)
    Li = np.linalg.inv(Lc)
    return float(np.linalg.eigvalsh(Li @ W @ Li.T).min())


def test_gradient_matches_finite_differences():
    p = fl.init_params(1)
    p[-258:-2] *= 20.0       # output weights large enough for the features to matter
    F, W, T = _batch()
    L, g = fl.loss_and_grad(p, F, W, T)
    rng = np.random.default_rng(2)
    idx = rng.choice(p.size, 60, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p); e[i] = eps
        fd = (fl.loss(p + e, F, W, T) - fl.loss(p - e, F, W, T)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd))


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p = fl.init_params(3)
    p[-258:-2] *= 20.0
    F, W, T = _batch(4, seed=5)
    L, g = fl.loss_and_grad(p, F, W, T)
    P = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    pos, x = 0, torch.tensor(F)
    for li, (i, o_) in enumerate(fl.LAYERS):
        Wl = P[pos:pos + i * o_].view(o_, i); pos += i * o_
        b = P[pos:pos + o_]; pos += o_
        x = x @ Wl.T + b
        if li < len(fl.LAYERS) - 1:
            x = torch.relu(x)
    # the head in torch: T_8 of the interval at the Chebyshev-Gauss nodes,
    # projected on T_0..T_8 (autograd through every step)
    b_ = 1 - torch.exp(x[:, 1:2])
    a_ = b_ - torch.exp(x[:, 0:1])
    nodes = torch.cos(torch.pi * (torch.arange(9, dtype=torch.float64) + 0.5) / 9)
    u = (nodes[None] + 1 - a_ - b_) / (b_ - a_)
    t0, t1 = torch.ones_like(u), u
    for _ in range(7):
        t0, t1 = t1, 2 * u * t1 - t0
    Tn = torch.cos(torch.outer(torch.arange(9, dtype=torch.float64), torch.arccos(nodes)))
    q = (2.0 / 9) * t1 @ Tn.T
    q = torch.cat([q[:, :1] / 2, q[:, 1:]], 1)
    Wt, Tt = torch.tensor(W), torch.tensor(T)
    num = torch.bmm(torch.bmm(q[:, None, :], Wt), q[:, :, None]).flatten()
    den = torch.bmm(torch.bmm(q[:, None, :], Tt), q[:, :, None]).flatten()
    Lt = (num / den).mean()
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-12
    assert np.abs(P.grad.numpy() - g).max() < 1e-10


def test_adam_reduces_loss_to_no_less_than_the_bound():
    F, W, T = _batch(8, seed=7)
    p = fl.init_params(4)
    m = np.zeros_like(p); v = np.zeros_like(p)
    L0 = fl.loss(p, F, W, T)
    for step in range(1, 201):
        _, g = fl.loss_and_grad(p, F, W, T)
        p, m, v = fl.adam_step(p, g, m, v, step, 1e-3)
    L1 = fl.loss(p, F, W, T)
    bound = np.mean([_lambda_min(W[b], T[b]) for b in range(8)])
    assert L1 < L0 - 0.3 * (L0 - bound)
    # the ratio never goes below the smallest generalised eigenvalue, and the
    # eigenvector (scaled so p(1) = 1) attains it
    for b in range(8):
        lam = _lambda_min(W[b], T[b])
        Lb, _ = fl.loss_terms(fl.mlp_forward(p, F[b:b + 1])[0], W[b][None], T[b][None])
        assert Lb[0] >= lam - 1e-12
        ev, V = np.linalg.eig(np.linalg.solve(T[b], W[b]))
        x = np.real(V[:, np.argmin(np.real(ev))])
        assert abs(fl.ratio(x, W[b], T[b]) - lam) < 1e-9


def test_adam_matches_torch_optimizer():
    """adam_step against torch.optim.Adam (CPU, float64) on the same gradient
    sequence: Kingma and Ba's bias-corrected update."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    p = rng.standard_normal(50)
    m = np.zeros_like(p); v = np.zeros_like(p)
    P = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([P], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 31):
        g = rng.standard_normal(50) * (1 + step % 3)
        p, m, v = fl.adam_step(p, g, m, v, step, 3e-3)
        opt.zero_grad()
        P.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    assert np.abs(P.detach().numpy() - p).max() < 1e-12


def test_features_closed_form_on_a_cycle():
    """On a cycle every degree is 2: mean 2, coefficient of variation 0,
    max/mean 1; the shifted and scaled raw statistics follow."""
    n, k = 40, 3
    d = np.full(n, 2.0)
    ray = [0.5, 0.6, 0.7, 0.8]
    f = fl.features(n, k, d, ray)
    raw = np.array([np.log(n), np.log(k), np.log(2.0), 0.0, 0.0, *ray])
    want = (raw - fl.FEAT_SHIFT) / fl.FEAT_SCALE
    assert np.allclose(f, want, rtol=0, atol=1e-15)
    # isolated vertices do not enter the degree statistics
    d2 = np.concatenate([d, np.zeros(5)])
    assert np.allclose(fl.features(n + 5, k, d2, ray)[2:], want[2:], rtol=0, atol=1e-15)
