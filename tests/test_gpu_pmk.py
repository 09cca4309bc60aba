"""PM with k vectors (the comparison method of Sec. 4: k orthogonal vectors
from the power method) through the C ABI, against the FP64 oracle's
orthogonal iteration.

Both sides orthonormalise after every step, so the columns are the left
singular vectors of the last step's block.  The embedding is compared where
it is unique: the last step's singular values, the subspace the columns span
(the sine of the largest principal angle), orthonormality of U = D^{1/2} E
over the non-isolated rows, and each column alone where its singular value is
separated from its neighbours (error bounded by the FP32 row error over the
gap).  Where a column's largest entry is also separated from its runner-up,
the sign rule must agree exactly.  Labels: ARI >= 0.99 against the oracle.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import host_weights, say, to_device

pytestmark = pytest.mark.gpu

# FP32 rows: each step rounds the block at ~6e-8 relative; the errors of
# earlier steps decay with the spectral gap, so the subspace and the
# singular values stay within a few 1e-6 of the FP64 iteration.
SPAN_TOL = 2e-5
SIGMA_TOL = 1e-5


def _u(E, d):
    live = d > 0
    return np.sqrt(d[live])[:, None] * E[live]


def _sin_angle(A, B):
    """sin of the largest principal angle between span(A) and span(B), each
    re-orthonormalised first (their own small departure from orthonormality
    is checked separately)."""
    qa = np.linalg.qr(A)[0]
    qb = np.linalg.qr(B)[0]
    return float(np.linalg.norm(qb - qa @ (qa.T @ qb), 2))


def _check_columns(U, Uo, svo):
    """Columns with a separated singular value match one by one; where the
    largest entry is also separated from the runner-up, without sign
    alignment (the sign rule)."""
    k = U.shape[1]
    for j in range(k):
        if svo[j] <= 0:
            continue
        gap = min([abs(svo[j] - svo[i]) for i in range(k) if i != j] + [np.inf]) / svo[j]
        if gap <= 0.05:
            continue
        a, b = U[:, j], Uo[:, j]
        tol = 2e-5 / gap
        top = np.sort(np.abs(b))[::-1]
        if len(top) > 1 and top[0] - top[1] > 10 * tol:
            assert np.linalg.norm(a - b) <= tol, (j, np.linalg.norm(a - b), "sign rule")
        else:
            assert np.linalg.norm(a * np.sign(a @ b) - b) <= tol, (j, np.linalg.norm(a - b))


def _check_against_oracle(fsc, g, data, k, t, seed, ari_bar=0.99):
    ip, ix, dd = data
    say(f"pmk n={g.n} k={k} t={t} seed={seed}")
    lab, E, sv = (x.cpu().numpy() for x in fsc.cluster_pmk(ip, ix, dd, k, t, seed))
    hw = host_weights(dd)
    Uo_all, svo = o.pm_k_iterate(g.n, g.indptr, g.indices, hw, k, t, seed=seed)
    d = o.degrees(g.n, g.indptr, g.indices, hw)
    assert np.all(E[d == 0] == 0.0)
    assert np.all(np.abs(sv - svo) <= SIGMA_TOL * svo[0]), (sv, svo)
    keep = svo > 1e-6 * svo[0]
    U, Uo = _u(E, d), Uo_all[d > 0]
    assert np.all(U[:, ~keep] == 0.0)
    U, Uo = U[:, keep], Uo[:, keep]
    assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-5
    s = _sin_angle(Uo, U)
    say("  sin(angle) vs oracle", s)
    assert s <= SPAN_TOL
    _check_columns(U, Uo, svo[keep])
    lab_o, _, _ = o.pm_k_cluster(g.n, g.indptr, g.indices, hw, k, t, seed, 30)
    a = o.ari(lab, lab_o)
    say("  ARI vs oracle", a)
    assert a >= ari_bar
    return lab, U, sv


@pytest.mark.parametrize("k,t", [(3, 12), (5, 15), (8, 20)])
def test_pmk_matches_oracle_on_sbm(gpu_lib, k, t):
    g = synth.sbm(2000, k, 0.1, 0.005, seed=k)
    lab, _, _ = _check_against_oracle(gpu_lib, g, to_device(g), k, t, seed=7)
    assert o.ari(lab, g.labels) >= 0.99


def test_pmk_at_t300_keeps_every_column(gpu_lib):
    # three planted clusters: gamma_2, gamma_3 ~ 0.95 and gamma_3^300 ~ 1e-7,
    # below what FP32 resolves in M^t X0; the orthogonal vectors all survive
    # and span the leading eigenvectors, whose eigenvalues are the singular
    # values of the last step
    g = synth.sbm(300, 3, 0.5, 0.02, seed=2)
    lab, U, sv = _check_against_oracle(gpu_lib, g, to_device(g), 3, 300, seed=1)
    assert U.shape[1] == 3
    M = o.signless_laplacian(g.n, g.indptr, g.indices, None).toarray()
    gam, F = np.linalg.eigh(M)
    assert gam[-3] ** 300 < 1e-6
    assert _sin_angle(F[:, -3:], U) <= SPAN_TOL
    assert np.abs(sv - gam[::-1][:3]).max() <= SIGMA_TOL
    assert o.ari(lab, g.labels) == 1.0


def test_pmk_at_t0_is_the_orthonormal_start_block(gpu_lib):
    g = synth.sbm(500, 4, 0.1, 0.01, seed=3)
    _check_against_oracle(gpu_lib, g, to_device(g), 4, 0, seed=9, ari_bar=0.0)


def test_pmk_on_ragged_weighted_graph_with_isolated_vertices(gpu_lib):
    # hubs, light rows and isolated vertices; weights in FP32
    g = synth.random_weighted(30000, 90000, seed=8, hubs=4, hub_degree=3000, isolated=17)
    data = to_device(g, weights="f32")
    lab, U, _ = _check_against_oracle(gpu_lib, g, data, 6, 5, 3, ari_bar=0.0)
    assert U.shape[1] == 6


def test_pmk_rank_deficient_block(gpu_lib):
    # a triangle and four isolated vertices: Y has rank 3, columns 3 and 4 are 0
    g = synth.csr_from_edges(7, np.array([0, 1, 2]), np.array([1, 2, 0]))
    ip, ix, dd = to_device(g)
    lab, E, sv = gpu_lib.cluster_pmk(ip, ix, dd, 5, 3, 4)
    E = E.cpu().numpy()
    Uo, _ = o.pm_k_iterate(g.n, g.indptr, g.indices, None, 5, 3, seed=4)
    assert np.all(E[3:] == 0.0) and np.all(E[:, 3:] == 0.0)
    U = np.sqrt(2.0) * E[:3, :3]
    assert np.abs(U.T @ U - np.eye(3)).max() < 1e-5
    assert _sin_angle(Uo[:3, :3], U) <= SPAN_TOL


def test_pmk_rejects_k_above_eight(gpu_lib):
    g = synth.sbm(100, 2, 0.3, 0.01, seed=1)
    ip, ix, dd = to_device(g)
    with pytest.raises(gpu_lib.FscError, match="k must be"):
        gpu_lib.cluster_pmk(ip, ix, dd, 9, 3, 1)


def test_pmk_rejects_bf16_vectors(gpu_lib):
    g = synth.sbm(100, 2, 0.3, 0.01, seed=1)
    ip, ix, dd = to_device(g)
    with pytest.raises(gpu_lib.FscError, match="FP32 or FP64"):
        gpu_lib.cluster_pmk(ip, ix, dd, 2, 3, 1, vec_dtype="bf16")


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
    sv = sv.cpu().numpy()
    say("  ARI vs planted", a, "sigma", sv)
    # the leading eigenvalue of M is 1 (Sec. 2); after 30 steps the block is
    # close to the leading eigenspace (the other 7 planted clusters'
    # eigenvalues sit near 0.946), so sigma_1 is just below 1
    assert 1.0 - 1e-4 < sv[0] <= 1.0 + 1e-6 and sv[-1] > 0.8
    assert a >= 0.99
