"""Pins for the learned-form oracle: dense eigen closed forms of the filter,
the exact Chebyshev expansion of gamma^8, the loss identity, and gradients
against central finite differences and torch's autograd."""
import numpy as np
import pytest
import scipy.sparse.csgraph as csgraph
import scipy.sparse as sp
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


def test_loss_identity_against_explicit_blocks():
    g = synth.sbm(300, 3, 0.1, 0.01, seed=2)
    F, G, h, yy = fl.graph_stats(g.n, g.indptr, g.indices, None, 3, 2, 15, seed=4)
    assert G.shape == (9, 9) and np.allclose(G, G.T)
    assert np.all(np.linalg.eigvalsh(G) > -1e-9 * np.abs(G).max())
    c_rest = np.random.default_rng(1).standard_normal(8) * 0.1
    L, _ = fl.loss_terms(c_rest[None], G[None], h[None], np.array([yy]))
    X0 = o.gaussian_block(g.n, 2, 4)
    M = o.signless_laplacian(g.n, g.indptr, g.indices, None)
    S = fl.filter_apply(M, X0, fl.full_coefficients(c_rest))
    Y = o.power_method(M, X0, 15)
    assert abs(L[0] - ((S - Y) ** 2).sum() / (Y ** 2).sum()) < 1e-10
    assert F.shape == (9,)
    # Rayleigh features are quotients of M: inside [0, 1]
    assert np.all((F[5:] >= 0) & (F[5:] <= 1))


def _batch(B=5, seed=0):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((B, fl.NFEAT))
    G, h, yy = [], [], []
    for _ in range(B):
        A = rng.standard_normal((9, 12))
        G.append(A @ A.T)
        h.append(rng.standard_normal(9))
        yy.append(float(rng.uniform(1, 3)))
    return F, np.array(G), np.array(h), np.array(yy)


def test_gradient_matches_finite_differences():
    p = fl.init_params(1)
    p[-1000:] *= 100.0       # a last layer large enough to give the loss curvature
    F, G, h, yy = _batch()
    L, g = fl.loss_and_grad(p, F, G, h, yy)
    rng = np.random.default_rng(2)
    idx = rng.choice(p.size, 60, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p); e[i] = eps
        fd = (fl.loss(p + e, F, G, h, yy) - fl.loss(p - e, F, G, h, yy)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd))


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p = fl.init_params(3)
    F, G, h, yy = _batch(4, seed=5)
    L, g = fl.loss_and_grad(p, F, G, h, yy)
    P = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    pos, x = 0, torch.tensor(F)
    for li, (i, o_) in enumerate(fl.LAYERS):
        W = P[pos:pos + i * o_].view(o_, i); pos += i * o_
        b = P[pos:pos + o_]; pos += o_
        x = x @ W.T + b
        if li < len(fl.LAYERS) - 1:
            x = torch.relu(x)
    c = torch.cat([1 - x.sum(1, keepdim=True), x], 1)
    Gt, ht, yt = torch.tensor(G), torch.tensor(h), torch.tensor(yy)
    Lt = ((torch.einsum("bi,bij,bj->b", c, Gt, c) - 2 * (ht * c).sum(1) + yt) / yt).mean()
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-12
    assert np.abs(P.grad.numpy() - g).max() < 1e-10


def test_adam_reduces_loss():
    F, G, h, yy = _batch(8, seed=7)
    p = fl.init_params(4)
    m = np.zeros_like(p); v = np.zeros_like(p)
    L0 = fl.loss(p, F, G, h, yy)
    for step in range(1, 201):
        _, g = fl.loss_and_grad(p, F, G, h, yy)
        p, m, v = fl.adam_step(p, g, m, v, step, 1e-3)
    assert fl.loss(p, F, G, h, yy) < 0.5 * L0
    # the optimum per graph is the least-squares solution: the loss never
    # goes below it
    for b in range(8):
        A = np.eye(9)[:, 1:] - np.outer(np.eye(9)[0], np.ones(8))   # c = e0 + A c_rest
        e0 = np.eye(9)[0]
        Gr = A.T @ G[b] @ A
        rhs = A.T @ (h[b] - G[b] @ e0)
        cr = np.linalg.solve(Gr, rhs)
        Lmin, _ = fl.loss_terms(cr[None], G[b][None], h[b][None], yy[b:b + 1])
        Lb, _ = fl.loss_terms(fl.mlp_forward(p, F[b:b + 1])[0], G[b][None], h[b][None], yy[b:b + 1])
        assert Lb[0] >= Lmin[0] - 1e-9


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
