"""Exact k nearest neighbours (the pre-processing of Sec. 4.2) through the
C ABI, against the FP64 brute-force oracle.

Distances are FP32 (the dot products on the matrix cores), so near-ties may
order differently from the oracle's.  The checks: every returned squared
distance equals the exact one of the returned index within
1e-5 (|x_q|^2 + |x_c|^2); every returned neighbour lies within the exact
knn-th distance plus twice that bound; no self, no repeats; and the index
list equals the oracle's wherever the oracle's gaps exceed the bound.  With
small integer coordinates every value is exact in FP32 and the lists must
match the oracle's exactly, ties included.
"""
import time

import numpy as np
import pytest
import torch

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _check(fsc, X, knn, rows=None, exact=False):
    n = X.shape[0]
    say(f"knn n={n} dim={X.shape[1]} k={knn}")
    nbr, dist = fsc.knn(torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda(), knn)
    nbr, dist = nbr.cpu().numpy(), dist.cpu().numpy()
    rows = np.arange(n) if rows is None else np.asarray(rows)
    on, od = o.knn_rows(X, rows, min(knn + 1, n - 1))
    X64 = X.astype(np.float64)
    sq = (X64 * X64).sum(axis=1)
    for i, q in enumerate(rows):
        g = nbr[q].astype(np.int64)
        if exact:
            assert np.array_equal(g, on[i, :knn]), (q, g, on[i])
            assert np.array_equal(dist[q], od[i, :knn])
            continue
        assert len(set(g.tolist())) == knn and q not in g and g.min() >= 0 and g.max() < n
        ex = ((X64[g] - X64[q]) ** 2).sum(axis=1)
        tol = 1e-5 * (sq[q] + sq[g])
        assert np.all(np.abs(dist[q] - ex) <= tol), q
        assert np.all(ex <= od[i, knn - 1] + 2 * tol.max()), q
        gaps = np.diff(od[i])
        if np.all(gaps > 2 * 1e-5 * (sq[q] + sq.max())):
            assert np.array_equal(g, on[i, :knn]), q


def test_knn_gaussian_mixture(gpu_lib):
    X, _ = synth.gaussian_mixture(300, 5, 784, seed=1)     # 1500 rows: ragged tiles
    _check(gpu_lib, X, 10)


def test_knn_ragged_dim_and_largest_k(gpu_lib):
    X = np.random.default_rng(2).standard_normal((1001, 100)).astype(np.float32)
    _check(gpu_lib, X, 16)


@pytest.mark.parametrize("dim", [800, 804, 1024])
def test_knn_both_block_shapes(gpu_lib, dim):
    # up to 800 dimensions the 8-wave block, above it the 4-wave one
    X = np.random.default_rng(dim).standard_normal((700, dim)).astype(np.float32)
    _check(gpu_lib, X, 10)


def test_knn_smallest_case(gpu_lib):
    X = np.array([[0, 0, 0, 0], [1, 2, 3, 4]], dtype=np.float32)
    _check(gpu_lib, X, 1, exact=True)


def test_knn_exact_ties_with_integer_coordinates(gpu_lib):
    rng = np.random.default_rng(3)
    base = rng.integers(0, 3, (5, 8))
    X = base[rng.integers(0, 5, 203)].astype(np.float32)   # many identical points
    _check(gpu_lib, X, 16, exact=True)
    X = rng.integers(-2, 3, (777, 12)).astype(np.float32)
    _check(gpu_lib, X, 10, exact=True)


def test_knn_rejects_bad_shapes(gpu_lib):
    X = torch.zeros((10, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.FscError, match="dim"):
        gpu_lib.knn(X, 3)
    X = torch.zeros((10, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.FscError, match="knn"):
        gpu_lib.knn(X, 17)


def test_knn_full_size_sampled_rows(gpu_lib):
    # 70,000 points of 10 Gaussians in 784 dimensions (the kNN workload's points)
    X, _ = synth.gaussian_mixture(7000, 10, 784, seed=0)
    Xt = torch.from_numpy(X).cuda()
    gpu_lib.knn(Xt, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gpu_lib.knn(Xt, 10)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    flops = 2.0 * X.shape[0] ** 2 * X.shape[1]
    say(f"  knn 70000 x 784, k=10: {ms:.1f} ms, {flops / ms / 1e9:.1f} TFLOP/s (FP32)")
    rows = np.concatenate([[0, 1, 69999], np.random.default_rng(4).integers(0, 70000, 29)])
    _check(gpu_lib, X, 10, rows=rows)
    # the whole graph builder at this size: timing and the CSR's invariants
    gpu_lib.knn_graph(Xt, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ip, ix, w = gpu_lib.knn_graph(Xt, 10)
    torch.cuda.synchronize()
    say(f"  knn graph 70000 x 784, k=10: {(time.perf_counter() - t0) * 1e3:.1f} ms, nnz {int(ip[-1])}")
    deg = torch.diff(ip)
    assert int(deg.min()) >= 10 and 700000 <= int(ip[-1]) <= 1400000
    assert float(w.min()) > 0.0 and float(w.max()) <= 1.0


def _graph(fsc, X, k):
    ip, ix, w = fsc.knn_graph(torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda(), k)
    return ip.cpu().numpy(), ix.cpu().numpy().astype(np.int64), w.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("case", ["line", "integer"])
def test_knn_graph_exact_structure(gpu_lib, case):
    rng = np.random.default_rng(5)
    if case == "line":
        X = np.zeros((301, 4), dtype=np.float32)
        X[:, 0] = np.arange(301)
        k = 2
    else:
        X = rng.integers(-2, 3, (1203, 12)).astype(np.float32)
        k = 10
    say(f"knn graph {case} n={X.shape[0]} k={k}")
    ip, ix, w = _graph(gpu_lib, X, k)
    oip, oix, ow = o.knn_graph(X, k)
    assert np.array_equal(ip, oip) and np.array_equal(ix, oix)
    assert np.all(np.abs(w - ow) <= 1e-6 * ow)


def test_knn_graph_gaussian_mixture(gpu_lib):
    X, _ = synth.gaussian_mixture(200, 5, 784, seed=2)
    n, k = X.shape[0], 10
    ip, ix, w = _graph(gpu_lib, X, k)
    oip, oix, ow = o.knn_graph(X, k)
    say(f"knn graph mixture n={n}: nnz {ip[-1]} vs oracle {oip[-1]}")
    import scipy.sparse as sp
    A = sp.csr_matrix((w, ix, ip), shape=(n, n))
    B = sp.csr_matrix((ow, oix, oip), shape=(n, n))
    assert (A != A.T).nnz == 0
    assert np.all(np.diff(ip) >= k)
    assert all(np.all(np.diff(ix[ip[r]:ip[r + 1]]) > 0) for r in range(n))
    common = A.multiply(B > 0)
    assert common.nnz >= 0.999 * B.nnz
    rel = np.abs(common - B.multiply(A > 0)).max() / ow.min()
    assert rel <= 1e-5
