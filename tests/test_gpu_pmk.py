"""PM with k vectors (the comparison method of Sec. 4) through the C ABI,
against the FP64 oracle.

The embedding is compared where it is unique: the singular values of Y, the
subspace its columns span (principal angles), orthonormality of
U = D^{1/2} E over the non-isolated rows, and each column alone where its
singular value is well separated from its neighbours (sign-aligned, since a
near-tie in the sign rule's largest entry may resolve either way in FP32).
Tolerances follow from FP32 rows: relative error 1e-5 in the rows, amplified
by sigma_max / sigma_j in column j.  Labels: ARI >= 0.99 against the oracle.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import host_weights, say, to_device

pytestmark = pytest.mark.gpu


def _u(E, d):
    live = d > 0
    return np.sqrt(d[live])[:, None] * E[live]


def _span_cos(Uo, U):
    """Cosines of the principal angles between span(Uo) (orthonormal) and
    span(U); U is re-orthonormalised first, so that its own small departure
    from orthonormality (checked separately) does not enter."""
    return np.linalg.svd(Uo.T @ np.linalg.qr(U)[0], compute_uv=False)


def _check_against_oracle(fsc, g, data, k, t, seed, ari_bar=0.99):
    ip, ix, dd = data
    say(f"pmk n={g.n} k={k} t={t} seed={seed}")
    lab, E, sv = (x.cpu().numpy() for x in fsc.cluster_pmk(ip, ix, dd, k, t, seed))
    hw = host_weights(dd)
    Eo = o.pm_k_embed(g.n, g.indptr, g.indices, hw, k, t, seed=seed)
    d = o.degrees(g.n, g.indptr, g.indices, hw)
    assert np.all(E[d == 0] == 0.0)
    Y = np.sqrt(d)[:, None] * o.embed(g.n, g.indptr, g.indices, hw, k, t, seed=seed)
    svo = np.linalg.svd(Y[d > 0], compute_uv=False)
    cond = svo[0] / svo
    assert np.all(np.abs(sv - svo) <= 1e-5 * svo * cond ** 2), (sv, svo)
    keep = svo > 1e-6 * svo[0]
    U, Uo = _u(E, d)[:, keep], _u(Eo, d)[:, keep]
    assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-4
    cos = _span_cos(Uo, U)
    assert cos.min() > 1 - 1e-6, cos
    for j in np.flatnonzero(keep):
        gap = min([abs(svo[j] - svo[i]) for i in range(k) if i != j] + [np.inf]) / svo[j]
        if gap > 0.1:
            a, b = _u(E, d)[:, j], _u(Eo, d)[:, j]
            a = a * np.sign(a @ b)
            assert np.linalg.norm(a - b) <= 1e-5 * cond[j] ** 2 / gap, (j, np.linalg.norm(a - b))
    lab_o, _, _ = o.pm_k_cluster(g.n, g.indptr, g.indices, hw, k, t, seed, 30)
    a = o.ari(lab, lab_o)
    say("  ARI vs oracle", a)
    assert a >= ari_bar
    return lab


@pytest.mark.parametrize("k,t", [(3, 12), (5, 15), (8, 20)])
def test_pmk_matches_oracle_on_sbm(gpu_lib, k, t):
    g = synth.sbm(2000, k, 0.1, 0.005, seed=k)
    lab = _check_against_oracle(gpu_lib, g, to_device(g), k, t, seed=7)
    assert o.ari(lab, g.labels) >= 0.99


def test_pmk_on_ragged_weighted_graph_with_isolated_vertices(gpu_lib):
    # hubs, light rows and isolated vertices; weights in FP32
    g = synth.random_weighted(30000, 90000, seed=8, hubs=4, hub_degree=3000, isolated=17)
    ip, ix, dd = to_device(g, weights="f32")
    say("pmk ragged weighted n=30000")
    lab, E, sv = gpu_lib.cluster_pmk(ip, ix, dd, 6, 5, 3)
    E = E.cpu().numpy()
    hw = host_weights(dd)
    d = o.degrees(g.n, g.indptr, g.indices, hw)
    assert np.all(E[d == 0] == 0.0)
    Eo = o.pm_k_embed(g.n, g.indptr, g.indices, hw, 6, 5, seed=3)
    svo = np.linalg.svd(np.sqrt(d)[:, None][d > 0] * o.embed(g.n, g.indptr, g.indices, hw, 6, 5, seed=3)[d > 0],
                        compute_uv=False)
    cond = svo[0] / svo
    assert np.all(np.abs(sv.cpu().numpy() - svo) <= 1e-5 * svo * cond ** 2)
    U, Uo = _u(E, d), _u(Eo, d)
    assert np.abs(U.T @ U - np.eye(6)).max() < 1e-4
    assert _span_cos(Uo, U).min() > 1 - 1e-6
    lab = lab.cpu().numpy()
    assert lab.min() >= 0 and lab.max() < 6


def test_pmk_rank_deficient_block(gpu_lib):
    # a triangle and four isolated vertices: Y has rank 3, columns 3 and 4 are 0
    g = synth.csr_from_edges(7, np.array([0, 1, 2]), np.array([1, 2, 0]))
    ip, ix, dd = to_device(g)
    lab, E, sv = gpu_lib.cluster_pmk(ip, ix, dd, 5, 3, 4)
    E = E.cpu().numpy()
    Eo = o.pm_k_embed(g.n, g.indptr, g.indices, None, 5, 3, seed=4)
    assert np.all(E[3:] == 0.0) and np.all(E[:, 3:] == 0.0)
    U, Uo = np.sqrt(2.0) * E[:3, :3], np.sqrt(2.0) * Eo[:3, :3]
    assert np.abs(U.T @ U - np.eye(3)).max() < 1e-5
    assert _span_cos(Uo, U).min() > 1 - 1e-6


def test_pmk_rejects_k_above_eight(gpu_lib):
    g = synth.sbm(100, 2, 0.3, 0.01, seed=1)
    ip, ix, dd = to_device(g)
    with pytest.raises(gpu_lib.FscError, match="k must be"):
        gpu_lib.cluster_pmk(ip, ix, dd, 9, 3, 1)


def test_pmk_full_size_sbm(gpu_lib):
    # 1M vertices, 8 planted clusters, mean degree 40, vertex ids permuted: the
    # shape of the benchmark's graph with k = 8
    g = synth.sbm_by_degree(1_000_000, 8, 36, 4, seed=0, permute=True)
    ip, ix, _ = to_device(g)
    dd = torch.ones(g.nnz, dtype=torch.float32, device="cuda")
    say("pmk full size n=1e6 k=8 t=30")
    lab, E, sv = gpu_lib.cluster_pmk(ip, ix, dd, 8, 30, 5)
    d = np.diff(g.indptr).astype(np.float64)
    U = _u(E.cpu().numpy(), d)
    assert np.abs(U.T @ U - np.eye(8)).max() < 1e-4
    a = o.ari(lab.cpu().numpy(), g.labels)
    say("  ARI vs planted", a, "sigma", sv.cpu().numpy())
    assert a >= 0.99
