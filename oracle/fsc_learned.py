"""FP64 oracle of the learned polynomial-filter form.

TEST INFRASTRUCTURE ONLY (tests, smoke and the CPU baseline use it; the
product path never does).

The paper computes M^t X0 (Algorithm 1) to project a Gaussian block onto the
top eigenvectors of M (Sec. 3.1: x_t = sum_i a_i gamma_i^t f_i).  The learned
form replaces gamma^t by a degree-8 polynomial p(gamma) = sum_j c_j T*_j(gamma)
in the shifted Chebyshev basis of [0, 1] (T*_j(g) = T_j(2g - 1)), with p(1) = 1
so the trivial eigenvector (gamma_1 = 1) keeps its weight.

Readings (the paper has no learned part):
* The filter.  What the top eigenvectors need is that the bulk of the
  spectrum, where the noise directions lie, is damped while the eigenvalues
  near 1 are kept.  The degree-8 polynomial with the smallest maximum on an
  interval [a, b] among those with p(1) = 1 is the Chebyshev polynomial of
  that interval, p(g) = T_8(u(g)) / T_8(u(1)), u(g) = (2g - a - b) / (b - a).
  The MLP (9 features, 3 hidden layers of 128 with ReLU) outputs two numbers
  (alpha, beta) that fix the interval, b = 1 - e^beta and a = b - e^alpha (so
  a < b < 1 always), and a fixed head turns them into c_0..c_8.  Coefficients
  output directly by a network are hopeless here: damping the bulk by four
  orders of magnitude needs them to about 1e-4, and training in that space
  does not converge.
* The loss.  The filter is trained on the plain method's clustering: the
  plain method (t power steps, then k-means, Algorithm 2) labels a graph's
  vertices, and the loss is the normalised k-means cost (Sec. 2.2) of the
  filtered embedding E(c) = D^{-1/2} p(M) X0 under those labels, within-
  cluster over total scatter.  Both are quadratic forms in c (c^T W c /
  c^T T c), so training needs only per-graph 9 x 9 scatter statistics of the
  basis blocks; the ratio does not depend on the scale of c.
Parity of this part is pinned internally (the k-means cost, the closed form
of the head, numpy's Chebyshev conversion, finite differences, autograd, the
generalised eigenvalue bound), not by the paper.
"""
from __future__ import annotations

import numpy as np

from . import fsc_oracle as o

DEG = 8            # polynomial degree
NCOEF = DEG + 1    # c_0..c_8
NFEAT = 9          # features per graph
HID = 128          # hidden width
NOUT = 2           # (alpha, beta): the damped interval
LAYERS = [(NFEAT, HID), (HID, HID), (HID, HID), (HID, NOUT)]
# initial interval [0.2, 0.72]: about 0.5 +- 1/sqrt(20), the bulk of M for a
# random graph of mean degree 20
INIT_A, INIT_B = 0.2, 0.72


# ---------------------------------------------------------------------------
# Chebyshev basis and the filter
# ---------------------------------------------------------------------------
def cheb_basis(M, X0, deg=DEG):
    """B_j = T*_j(M) X0 for j = 0..deg by the three-term recurrence
    T*_0 = I, T*_1 = 2M - I, T*_{j+1} = 2 (2M - I) T*_j - T*_{j-1}."""
    X0 = np.asarray(X0, dtype=np.float64)
    B = [X0.copy()]
    if deg >= 1:
        B.append(2.0 * (M @ X0) - X0)
    for _ in range(2, deg + 1):
        Bj = B[-1]
        B.append(2.0 * (2.0 * (M @ Bj) - Bj) - B[-2])
    return B


def full_coefficients(c_rest):
    """(c_0, c_1..c_8) with c_0 = 1 - sum(c_1..c_8), so that p(1) = 1."""
    c_rest = np.asarray(c_rest, dtype=np.float64)
    return np.concatenate([[1.0 - c_rest.sum()], c_rest])


def filter_apply(M, X0, c):
    """S = p(M) X0 = sum_j c_j T*_j(M) X0 (c has 9 entries)."""
    B = cheb_basis(M, X0, len(c) - 1)
    return sum(cj * Bj for cj, Bj in zip(c, B))


def filter_embed(n, indptr, indices, data, l, c, seed=None, x0=None):
    """The filtered embedding D^{-1/2} p(M) X0 (the learned form's analogue of
    the embedding handed to k-means in Algorithm 2)."""
    if x0 is None:
        x0 = o.gaussian_block(n, l, seed)
    M = o.signless_laplacian(n, indptr, indices, data)
    s = o.inv_sqrt_degree(o.degrees(n, indptr, indices, data))
    return s[:, None] * filter_apply(M, np.asarray(x0, dtype=np.float64).reshape(n, l), c)


# ---------------------------------------------------------------------------
# Training statistics of one graph
# ---------------------------------------------------------------------------
# fixed centring/scaling of the raw statistics, so the inputs are O(1)
FEAT_SHIFT = np.array([12.0, 2.0, 3.0, 1.0, 5.0, 0.0, 0.0, 0.0, 0.0])
FEAT_SCALE = np.array([2.0, 1.0, 1.0, 1.0, 2.0, 1.0, 1.0, 1.0, 1.0])


def features(n, k, d, rayleigh4):
    """log n, log k, log mean degree, log(1 + degree coefficient of
    variation), log(max/mean degree) -- over non-isolated vertices -- and the
    column-mean Rayleigh quotients x^T M x / x^T x of the basis vectors
    B_0..B_3, then (raw - FEAT_SHIFT) / FEAT_SCALE."""
    d = np.asarray(d, dtype=np.float64)
    dd = d[d > 0]
    mean = dd.mean()
    cv = dd.std() / mean
    raw = np.array([np.log(n), np.log(k), np.log(mean), np.log1p(cv), np.log(dd.max() / mean),
                    *np.asarray(rayleigh4, dtype=np.float64)])
    return (raw - FEAT_SHIFT) / FEAT_SCALE


def scatter_stats(Bz, labels, mask):
    """W, T (9 x 9) with c^T W c the within-cluster scatter and c^T T c the
    total scatter of the rows v in `mask` of E(c) = sum_j c_j Bz[j] (the sum
    of squared distances to the cluster's mean, respectively to the mean of
    all those rows), by centring the blocks and taking inner products."""
    mask = np.asarray(mask, dtype=bool)
    X = np.stack([np.asarray(b, dtype=np.float64)[mask] for b in Bz])   # nb x m x l
    L = np.asarray(labels)[mask]
    Xt = X - X.mean(axis=1, keepdims=True)
    Xw = X.copy()
    for c in np.unique(L):
        sel = L == c
        Xw[:, sel] -= X[:, sel].mean(axis=1, keepdims=True)
    W = np.einsum("imq,jmq->ij", Xw, Xw)
    T = np.einsum("imq,jmq->ij", Xt, Xt)
    return W, T


def graph_stats(n, indptr, indices, data, k, l, t, seed, kmeans_iters=30):
    """Everything the trainer needs from one graph: features, the scatter
    statistics W, T of the z-space basis blocks D^{-1/2} T*_j(M) X0 over the
    non-isolated vertices, under the labels of the plain method (t steps,
    k-means with kmeans_iters Lloyd rounds, Algorithm 2), and those labels."""
    X0 = o.gaussian_block(n, l, seed)
    M = o.signless_laplacian(n, indptr, indices, data)
    d = o.degrees(n, indptr, indices, data)
    m = d > 0
    s = o.inv_sqrt_degree(d)
    B = cheb_basis(M, X0)
    E = s[:, None] * o.power_method(M, X0, t)
    labels, _ = o.kmeans(E, k, kmeans_iters, seed, eligible=m)
    W, T = scatter_stats([s[:, None] * b for b in B], labels, m)
    ray = []
    for j in range(4):
        Bj = B[j][m]
        MB = (M @ B[j])[m]
        ray.append(float(np.mean(np.einsum("ij,ij->j", Bj, MB) / np.einsum("ij,ij->j", Bj, Bj))))
    return features(n, k, d, ray), W, T, labels


# ---------------------------------------------------------------------------
# The MLP: 3 hidden layers of 128 with ReLU, 8 outputs
# ---------------------------------------------------------------------------
def param_count():
    return sum(i * o_ + o_ for i, o_ in LAYERS)


def unpack(params):
    """Flat layout: for each layer, W (out x in, row-major) then b (out)."""
    params = np.asarray(params, dtype=np.float64)
    out, pos = [], 0
    for i, o_ in LAYERS:
        W = params[pos:pos + i * o_].reshape(o_, i)
        pos += i * o_
        b = params[pos:pos + o_]
        pos += o_
        out.append((W, b))
    return out


def init_params(seed):
    """He-uniform weights, zero biases (from numpy's generator); the output
    layer's weights scaled by 0.01 and its biases set to the initial
    interval, so every graph starts near the filter of [INIT_A, INIT_B]."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (i, o_) in enumerate(LAYERS):
        lim = np.sqrt(6.0 / i)
        Wl = rng.uniform(-lim, lim, size=(o_, i))
        bl = np.zeros(o_)
        if li == len(LAYERS) - 1:
            Wl *= 0.01
            bl = np.array([np.log(INIT_B - INIT_A), np.log(1.0 - INIT_B)])
        parts += [Wl.ravel(), bl]
    return np.concatenate(parts)


def mlp_forward(params, F):
    """F: (batch, 9) -> (outputs (batch, 2) = (alpha, beta), activations)."""
    x = np.asarray(F, dtype=np.float64)
    acts = [x]
    layers = unpack(params)
    for li, (W, b) in enumerate(layers):
        z = x @ W.T + b
        x = np.maximum(z, 0.0) if li < len(layers) - 1 else z
        acts.append(x)
    return x, acts


# ---------------------------------------------------------------------------
# The head: (alpha, beta) -> the Chebyshev polynomial of the interval [a, b]
# ---------------------------------------------------------------------------
def interval(alpha, beta):
    """b = 1 - e^beta, a = b - e^alpha."""
    b = 1.0 - np.exp(beta)
    return b - np.exp(alpha), b


def _cheb_T(m, u):
    """T_m(u) for any real u, by the three-term recurrence."""
    t0, t1 = np.ones_like(u), u
    if m == 0:
        return t0
    for _ in range(m - 1):
        t0, t1 = t1, 2.0 * u * t1 - t0
    return t1


def _cheb_dT(m, u):
    """T_m'(u) = m U_{m-1}(u), U by its three-term recurrence."""
    u0, u1 = np.ones_like(u), 2.0 * u
    if m == 1:
        return np.ones_like(u)
    for _ in range(m - 2):
        u0, u1 = u1, 2.0 * u * u1 - u0
    return m * u1


# Chebyshev-Gauss nodes of [-1, 1]: the discrete orthogonality of T_0..T_8 on
# 9 nodes gives the exact coefficients of any polynomial of degree <= 8
_NODES = np.cos(np.pi * (np.arange(NCOEF) + 0.5) / NCOEF)
_TNODES = np.cos(np.outer(np.arange(NCOEF), np.arccos(_NODES)))   # T_j(x_k)


def _project(values):
    """Chebyshev coefficients (in x = 2 gamma - 1) of the degree-8
    polynomial taking `values` at the nodes."""
    q = (2.0 / NCOEF) * (_TNODES @ values)
    q[0] *= 0.5
    return q


def head(alpha, beta):
    """Unnormalised coefficients q (9) of T_8(u(gamma)) in the T*_j basis,
    u = (2 gamma - a - b) / (b - a), and dq/dalpha, dq/dbeta."""
    a, b = interval(alpha, beta)
    g1 = _NODES + 1.0                      # 2 gamma at the nodes
    u = (g1 - a - b) / (b - a)
    dT = _cheb_dT(DEG, u)
    du_da = (g1 - 2.0 * b) / (b - a) ** 2
    du_db = (2.0 * a - g1) / (b - a) ** 2
    da_dalpha = -np.exp(alpha)
    db_dbeta = -np.exp(beta)               # a = b - e^alpha moves with b
    q = _project(_cheb_T(DEG, u))
    dq_dalpha = _project(dT * du_da) * da_dalpha
    dq_dbeta = _project(dT * (du_da + du_db)) * db_dbeta
    return q, dq_dalpha, dq_dbeta


def coefficients(out):
    """c_1..c_8 (batch, 8) of the filters for MLP outputs (batch, 2):
    q / p_q(1) with p_q(1) = sum_j q_j (T*_j(1) = 1)."""
    out = np.atleast_2d(out)
    cs = []
    for al, be in out:
        q, _, _ = head(al, be)
        cs.append(q[1:] / q.sum())
    return np.array(cs)


def ratio(c, W, T):
    """c^T W c / c^T T c for full coefficients c (9)."""
    c = np.asarray(c, dtype=np.float64)
    return float(c @ W @ c) / float(c @ T @ c)


def loss_terms(out, W, T):
    """Per-graph normalised k-means cost of the filter of MLP outputs
    out (batch, 2) and its gradient in out.  The ratio does not depend on the
    scale of the coefficients, so it is taken on q directly.  With zero total
    scatter (every row equal) the ratio is undefined; such a graph counts 0
    with a zero gradient."""
    out = np.atleast_2d(out)
    L, dout = [], []
    for b in range(out.shape[0]):
        q, qa, qb = head(out[b, 0], out[b, 1])
        num = q @ W[b] @ q
        den = q @ T[b] @ q
        if not den > 0:
            L.append(0.0)
            dout.append(np.zeros(NOUT))
            continue
        Lb = num / den
        L.append(Lb)
        gq = 2.0 * (W[b] @ q - Lb * (T[b] @ q)) / den
        dout.append([gq @ qa, gq @ qb])
    return np.array(L), np.array(dout)


def loss(params, F, W, T):
    """Mean normalised cost over the batch."""
    out, _ = mlp_forward(params, F)
    L, _ = loss_terms(out, W, T)
    return float(L.mean())


def loss_and_grad(params, F, W, T):
    """Mean loss and its gradient in the flat parameters (hand-written
    backward pass)."""
    out, acts = mlp_forward(params, F)
    L, dout = loss_terms(out, W, T)
    B = out.shape[0]
    delta = dout / B
    layers = unpack(params)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W_, b = layers[li]
        a_in = acts[li]
        grads.append((delta.T @ a_in, delta.sum(axis=0)))
        if li > 0:
            delta = (delta @ W_) * (acts[li] > 0)
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return float(L.mean()), flat


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected; returns new
    (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
