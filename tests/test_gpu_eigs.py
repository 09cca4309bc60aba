"""The eigenvector baselines of Sec. 4 (subspace iteration) through the C
ABI, against the FP64 oracle's dense eigendecomposition.

Compared where unique: the eigenvalue estimates, the span of the embedding
(principal angles, after re-orthonormalising the FP32 rows), orthonormality
of U = D^{1/2} E, and the labels (ARI >= 0.99 against the oracle's k-means on
its own eigenvectors).  The test graphs have a clear gap below the m-th
eigenvalue, so cycles * steps power steps converge far below FP32 rounding.
"""
import numpy as np
import pytest

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import say, to_device

pytestmark = pytest.mark.gpu


def _span_cos(A, B):
    return np.linalg.svd(np.linalg.qr(A)[0].T @ np.linalg.qr(B)[0], compute_uv=False)


@pytest.mark.parametrize("k", [4, 8])
def test_k_eigenvectors_match_oracle_on_sbm(gpu_lib, k):
    g = synth.sbm(2000, k, 0.1, 0.005, seed=10 + k)
    ip, ix, dd = to_device(g)
    say(f"eigs n=2000 k=m={k}")
    lab, E, gam = (x.cpu().numpy() for x in gpu_lib.cluster_eigs(ip, ix, dd, k, k, 6, 20, 5))
    Eo, gamo = o.eigs_embed(g.n, g.indptr, g.indices, None, k)
    d = o.degrees(g.n, g.indptr, g.indices, None)
    assert np.abs(gam - gamo).max() < 1e-4, (gam, gamo)
    U = np.sqrt(d)[:, None] * E
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-4
    assert _span_cos(U, np.sqrt(d)[:, None] * Eo).min() > 1 - 1e-5
    lab_o, _, _ = o.eigs_cluster(g.n, g.indptr, g.indices, None, k, k, 5, 30)
    assert o.ari(lab, lab_o) >= 0.99
    assert o.ari(lab, g.labels) >= 0.99


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
    assert _span_cos(np.sqrt(8.0) * E[:45], B).min() > 1 - 1e-6
    assert o.ari(lab[:45], c.labels) == 1.0


def test_eigs_rejects_m_above_eight(gpu_lib):
    g = synth.sbm(100, 2, 0.3, 0.01, seed=1)
    ip, ix, dd = to_device(g)
    with pytest.raises(gpu_lib.FscError, match="m must be"):
        gpu_lib.cluster_eigs(ip, ix, dd, 2, 9, 2, 5, 1)
