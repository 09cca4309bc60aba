"""The eigenvector baselines of Sec. 4 (orthogonal iteration to the m leading
eigenvectors of M) through the C ABI, against the FP64 oracle's dense
eigendecomposition.

Compared where unique: the eigenvalue estimates, the span of the embedding
(the sine of the largest principal angle, after re-orthonormalising the FP32
rows), orthonormality of U = D^{1/2} E, and the labels (ARI >= 0.99 against
the oracle's k-means on its own eigenvectors).  The test graphs have a clear
gap below the m-th eigenvalue, so cycles * steps orthogonalised steps
converge far below FP32 rounding; on the path graph the m-th eigenvalue is
small (gamma_m^30 < 1e-6), which a restart from the unorthogonalised block
M^30 X0 could not resolve.
"""
import numpy as np
import pytest

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import say, to_device

pytestmark = pytest.mark.gpu


def _sin_angle(A, B):
    qa = np.linalg.qr(A)[0]
    qb = np.linalg.qr(B)[0]
    return float(np.linalg.norm(qb - qa @ (qa.T @ qb), 2))


@pytest.mark.parametrize("k", [4, 8])
def test_k_eigenvectors_match_oracle_on_sbm(gpu_lib, k):
    g = synth.sbm(2000, k, 0.1, 0.005, seed=10 + k)
    ip, ix, dd = to_device(g)
    say(f"eigs n=2000 k=m={k}")
    lab, E, gam = (x.cpu().numpy() for x in gpu_lib.cluster_eigs(ip, ix, dd, k, k, 6, 20, 5))
    Eo, gamo = o.eigs_embed(g.n, g.indptr, g.indices, None, k)
    d = o.degrees(g.n, g.indptr, g.indices, None)
    assert np.abs(gam - gamo).max() < 1e-5, (gam, gamo)
    U = np.sqrt(d)[:, None] * E
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-5
    assert _sin_angle(np.sqrt(d)[:, None] * Eo, U) < 2e-5
    lab_o, _, _ = o.eigs_cluster(g.n, g.indptr, g.indices, None, k, k, 5, 30)
    assert o.ari(lab, lab_o) >= 0.99
    assert o.ari(lab, g.labels) >= 0.99


@pytest.mark.parametrize("m", [5, 8])
def test_small_leading_eigenvalues_keep_every_column(gpu_lib, m):
    # the path on 10 vertices: eigenvalues cos^2(pi j / 18), all distinct;
    # gamma_5 = 0.587 and gamma_8 = 0.117, so gamma_m^30 < 1e-6, yet every
    # column survives and is the eigenvector itself (up to sign)
    n = 10
    g = synth.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    ip, ix, dd = to_device(g)
    lab, E, gam = (x.cpu().numpy() for x in gpu_lib.cluster_eigs(ip, ix, dd, 2, m, 4, 30, 3))
    Eo, gamo = o.eigs_embed(g.n, g.indptr, g.indices, None, m)
    assert np.allclose(gamo, np.cos(np.pi * np.arange(m) / 18) ** 2, atol=1e-12)
    assert gamo[m - 1] ** 30 < 1e-6
    assert np.abs(gam - gamo).max() < 1e-5, (gam, gamo)
    d = o.degrees(g.n, g.indptr, g.indices, None)
    U, Uo = np.sqrt(d)[:, None] * E, np.sqrt(d)[:, None] * Eo
    assert np.abs(U.T @ U - np.eye(m)).max() < 1e-5
    for j in range(m):
        assert abs(abs(U[:, j] @ Uo[:, j]) - 1.0) < 1e-5, j


def test_eigenvectors_of_cliques_with_isolated_vertices(gpu_lib):
    # 5 cliques of 9 and 4 isolated vertices: the leading eigenspace is
    # spanned by the degree-weighted clique indicators (eigenvalue 1)
    c = synth.disjoint_cliques(5, 9)
    rows = np.repeat(np.arange(c.n), np.diff(c.indptr))
    g = synth.csr_from_edges(49, rows[rows < c.indices], c.indices[rows < c.indices])
    ip, ix, dd = to_device(g)
    lab, E, gam = (x.cpu().numpy() for x in gpu_lib.cluster_eigs(ip, ix, dd, 5, 5, 3, 10, 2))
    assert np.all(E[45:] == 0.0)
    assert np.abs(gam - 1.0).max() < 1e-5
    B = np.zeros((45, 5))
    B[np.arange(45), c.labels] = 1.0
    assert _sin_angle(B, np.sqrt(8.0) * E[:45]) < 1e-5
    assert o.ari(lab[:45], c.labels) == 1.0


def test_eigs_rejects_m_above_eight(gpu_lib):
    g = synth.sbm(100, 2, 0.3, 0.01, seed=1)
    ip, ix, dd = to_device(g)
    with pytest.raises(gpu_lib.FscError, match="m must be"):
        gpu_lib.cluster_eigs(ip, ix, dd, 2, 9, 2, 5, 1)
