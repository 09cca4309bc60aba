"""Boundary options of fsc_embed / fsc_cluster through the C ABI:

* validate = 2, the on-device symmetry check (Sec. 2: G is undirected):
  symmetric graphs pass and give the same embedding as without the check;
  a missing mirror entry, a weight that differs by one unit in the last
  place, and duplicates that do not add up to the mirror are rejected with
  FSC_E_GRAPH; duplicates that do add up, and explicit zeros without a
  mirror, pass.  Each verdict equals the oracle's validate_graph on the same
  arrays.
* return_y: fsc_embed writes Y = M^t X0 (Algorithm 1's iterates) instead of
  D^{-1/2} Y, against the oracle's PowerMethod; isolated rows are 2^-t X0.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import check_elems, col_rel_err, host_weights, say

pytestmark = pytest.mark.gpu


def _dev(indptr, indices, data, wdt):
    ip = torch.from_numpy(np.asarray(indptr, dtype=np.int64)).cuda()
    ix = torch.from_numpy(np.asarray(indices, dtype=np.int32)).cuda()
    if data is None:
        return ip, ix, None
    d = torch.from_numpy(np.asarray(data, dtype=np.float64))
    d = {"f64": d, "f32": d.float(), "bf16": d.to(torch.bfloat16)}[wdt]
    return ip, ix, d.cuda()


def _verdicts(fsc, n, indptr, indices, data, wdt):
    """(device accepts, oracle accepts) for validate = 2."""
    ip, ix, d = _dev(indptr, indices, data, wdt)
    vec = "f64" if wdt == "f64" else "bf16" if wdt == "bf16" else "f32"
    try:
        fsc.embed(ip, ix, d, 2, 2, seed=0, vec_dtype=vec, validate=2)
        dev_ok = True
    except fsc.FscError as e:
        assert e.code == -2, e
        assert "symmetric" in str(e)
        dev_ok = False
    try:
        o.validate_graph(n, indptr, indices, host_weights(d))
        ora_ok = True
    except ValueError:
        ora_ok = False
    return dev_ok, ora_ok


def _drop(indptr, indices, data, j):
    """The CSR without its entry j."""
    rows = np.repeat(np.arange(len(indptr) - 1), np.diff(indptr))
    keep = np.ones(len(indices), dtype=bool)
    keep[j] = False
    ip = np.zeros_like(indptr)
    np.add.at(ip, rows[keep] + 1, 1)
    return np.cumsum(ip), indices[keep], None if data is None else data[keep]


@pytest.mark.parametrize("wdt", ["none", "f64", "f32", "bf16"])
def test_symmetric_graphs_pass_and_change_nothing(gpu_lib, wdt):
    g = synth.random_weighted(4000, 20000, seed=3, hubs=3, hub_degree=900, isolated=7)
    data = None if wdt == "none" else g.data
    ip, ix, d = _dev(g.indptr, g.indices, data, wdt)
    vec = "f64" if wdt == "f64" else "f32"
    a = gpu_lib.embed(ip, ix, d, 3, 6, seed=1, vec_dtype=vec, validate=2)
    b = gpu_lib.embed(ip, ix, d, 3, 6, seed=1, vec_dtype=vec)
    assert torch.equal(a, b)
    lab = gpu_lib.cluster(ip, ix, d, 4, 3, 6, 1, vec_dtype=vec, validate=2)
    assert torch.equal(lab, gpu_lib.cluster(ip, ix, d, 4, 3, 6, 1, vec_dtype=vec))


@pytest.mark.parametrize("wdt", ["none", "f32", "bf16", "f64"])
def test_a_missing_mirror_entry_is_rejected(gpu_lib, wdt):
    g = synth.random_weighted(500, 2000, seed=4)
    data = None if wdt == "none" else g.data
    rng = np.random.default_rng(0)
    for j in rng.choice(g.nnz, 5, replace=False):
        ip, ix, dd = _drop(g.indptr, g.indices, data, j)
        dev_ok, ora_ok = _verdicts(gpu_lib, g.n, ip, ix, dd, wdt)
        assert not dev_ok and not ora_ok
        # the cheap checks do not see it
        ipd, ixd, ddd = _dev(ip, ix, dd, wdt)
        vec = "f64" if wdt == "f64" else "bf16" if wdt == "bf16" else "f32"
        gpu_lib.embed(ipd, ixd, ddd, 2, 2, seed=0, vec_dtype=vec, validate=1)


def test_a_weight_one_ulp_off_is_rejected(gpu_lib):
    g = synth.random_weighted(500, 2000, seed=5)
    w = g.data.astype(np.float32)
    w[17] = np.nextafter(w[17], np.float32(np.inf))
    dev_ok, ora_ok = _verdicts(gpu_lib, g.n, g.indptr, g.indices, w.astype(np.float64), "f32")
    assert not dev_ok and not ora_ok


def _pair_graph(entries, n=4):
    """CSR from (row, col, weight) entries, in the given order within rows."""
    entries = sorted(entries, key=lambda e: e[0])
    indptr = np.zeros(n + 1, dtype=np.int64)
    for r, _, _ in entries:
        indptr[r + 1] += 1
    return np.cumsum(indptr), np.array([e[1] for e in entries]), np.array([e[2] for e in entries], dtype=np.float64)


@pytest.mark.parametrize("entries,symmetric", [
    # duplicates of (0, 1) add up to its mirror
    ([(0, 1, 1.0), (0, 1, 2.0), (1, 0, 3.0), (2, 3, 0.5), (3, 2, 0.5)], True),
    # ... or do not
    ([(0, 1, 1.0), (0, 1, 2.0), (1, 0, 2.5), (2, 3, 0.5), (3, 2, 0.5)], False),
    # an explicit zero with no mirror is a zero of A
    ([(0, 1, 1.0), (1, 0, 1.0), (2, 3, 0.0)], True),
    # a directed edge
    ([(0, 1, 1.0), (1, 0, 1.0), (2, 3, 0.25)], False),
    # mirrored duplicates in another order within the row
    ([(0, 1, 2.0), (0, 2, 1.0), (0, 1, 1.0), (1, 0, 1.0), (1, 0, 2.0), (2, 0, 1.0)], True),
])
@pytest.mark.parametrize("wdt", ["f64", "f32"])
def test_duplicates_and_zeros_follow_the_matrix(gpu_lib, entries, symmetric, wdt):
    ip, ix, w = _pair_graph(entries)
    dev_ok, ora_ok = _verdicts(gpu_lib, 4, ip, ix, w, wdt)
    assert dev_ok == ora_ok == symmetric


def test_random_perturbations_agree_with_the_oracle(gpu_lib):
    g = synth.random_weighted(300, 1200, seed=6)
    rng = np.random.default_rng(1)
    seen = set()
    for trial in range(12):
        w = g.data.copy()
        ix = g.indices.copy()
        kind = trial % 3
        j = int(rng.integers(g.nnz))
        if kind == 0:
            w[j] *= 1.5                     # one weight changed
        elif kind == 1:
            r = np.searchsorted(g.indptr, j, side="right") - 1
            c = int(rng.integers(g.n))
            if c != r:
                ix[j] = c                   # one column moved
        dev_ok, ora_ok = _verdicts(gpu_lib, g.n, g.indptr, ix, w, "f64")
        assert dev_ok == ora_ok, (trial, kind)
        seen.add(dev_ok)
    assert seen == {True, False}


def test_validate_level_out_of_range(gpu_lib):
    g = synth.sbm(100, 2, 0.2, 0.01, seed=0)
    ip, ix, d = _dev(g.indptr, g.indices, None, "none")
    with pytest.raises(gpu_lib.FscError) as e:
        gpu_lib.embed(ip, ix, d, 2, 3, seed=0, validate=3)
    assert e.value.code == -1


def test_symmetry_check_at_full_size(gpu_lib):
    g = synth.sbm_by_degree(1_000_000, 10, 36, 4, seed=0, permute=True)
    ip, ix, _ = _dev(g.indptr, g.indices, None, "none")
    d = torch.ones(g.nnz, dtype=torch.float32, device="cuda")
    say(f"symmetry check n={g.n} nnz={g.nnz}")
    gpu_lib.embed(ip, ix, d, 4, 1, seed=0, validate=2)
    # one weight of 40M off by one unit in the last place
    d[123_456] = torch.nextafter(d[123_456], torch.tensor(2.0, device="cuda"))
    with pytest.raises(gpu_lib.FscError, match="symmetric"):
        gpu_lib.embed(ip, ix, d, 4, 1, seed=0, validate=2)


@pytest.mark.parametrize("vec", ["f64", "f32", "bf16"])
def test_return_y_is_the_power_iterate(gpu_lib, vec):
    g = synth.random_weighted(3000, 12000, seed=9, hubs=2, hub_degree=800, isolated=11)
    wdt = {"f64": "f64", "f32": "f32", "bf16": "bf16"}[vec]
    ip, ix, d = _dev(g.indptr, g.indices, g.data, wdt)
    hw = host_weights(d)
    t, l = 9, 3
    Y = gpu_lib.embed(ip, ix, d, l, t, seed=4, vec_dtype=vec, return_y=True).double().cpu().numpy()
    x0 = o.gaussian_block(g.n, l, 4)
    want = o.power_method(o.signless_laplacian(g.n, g.indptr, g.indices, hw), x0, t)
    err = col_rel_err(Y, want)
    say(f"return_y {vec}: rel err {err:.2e}")
    assert err <= {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}[vec]
    check_elems(Y, want, vec, "Y")
    deg = o.degrees(g.n, g.indptr, g.indices, hw)
    iso = deg == 0
    assert iso.sum() >= 11   # the 11 planted ones, and any the draw left alone
    tol = {"f64": 1e-15, "f32": 1e-7, "bf16": 8e-3}[vec]
    assert np.allclose(Y[iso], x0[iso] * 2.0 ** -t, rtol=tol, atol=0)
    # E = D^{-1/2} Y is what fsc_embed writes without the option
    E = gpu_lib.embed(ip, ix, d, l, t, seed=4, vec_dtype=vec).double().cpu().numpy()
    live = ~iso
    assert col_rel_err(E[live] * np.sqrt(deg[live])[:, None], Y[live]) <= {"f64": 1e-14, "f32": 1e-6, "bf16": 8e-3}[vec]


def test_return_y_with_a_given_start_block(gpu_lib):
    g = synth.random_weighted(1000, 4000, seed=2, isolated=5)
    ip, ix, d = _dev(g.indptr, g.indices, g.data, "f64")
    x0 = np.random.default_rng(3).standard_normal((g.n, 4))
    xt = torch.from_numpy(x0).cuda()
    Y = gpu_lib.embed(ip, ix, d, 4, 5, seed=0, vec_dtype="f64", x0=xt, return_y=True).cpu().numpy()
    want = o.power_method(o.signless_laplacian(g.n, g.indptr, g.indices, g.data), x0, 5)
    assert col_rel_err(Y, want) <= 1e-12


# ---------------------------------------------------------------------------
# Degenerate graphs of Sec. 2's setting, through the C ABI against the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [300, 100_000])
def test_graph_without_edges(gpu_lib, n):
    """No edges: every vertex isolated (d = 0), so every embedding row is 0
    and no row takes part in the k-means fit; the seeding falls back to the
    smallest unchosen rows, every centre is 0 and every label is 0 (the
    lowest centre on a tie), as in the oracle.  100,000 vertices take the
    column-slab form with nothing in it."""
    ip = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    ix = torch.zeros(0, dtype=torch.int32, device="cuda")
    E = gpu_lib.embed(ip, ix, None, 3, 5, seed=1).cpu().numpy()
    assert E.shape == (n, 3) and not E.any()
    lab, E2 = gpu_lib.cluster(ip, ix, None, 4, 3, 5, 1, kmeans_iters=10, return_embedding=True)
    lab_o, _, E_o = o.fast_spectral_cluster(n, np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int64), None,
                                            4, 3, 5, 1, 10)
    assert not E_o.any() and not E2.cpu().numpy().any()
    assert np.array_equal(lab.cpu().numpy(), np.asarray(lab_o, dtype=np.int32))
    assert not lab.cpu().numpy().any()


def test_single_vertex(gpu_lib):
    ip = torch.zeros(2, dtype=torch.int64, device="cuda")
    ix = torch.zeros(0, dtype=torch.int32, device="cuda")
    lab, E = gpu_lib.cluster(ip, ix, None, 1, 1, 3, 0, kmeans_iters=5, return_embedding=True)
    assert lab.cpu().numpy().tolist() == [0] and E.cpu().numpy().tolist() == [[0.0]]


@pytest.mark.parametrize("vec", ["f64", "f32"])
def test_one_edge(gpu_lib, vec):
    """Two vertices joined by one edge: M = [[1/2, 1/2], [1/2, 1/2]] projects
    onto the constant vector after one step, so both embedding rows are
    equal; k = 2 then puts both vertices in cluster 0 (the second centre is
    the first's copy and ties go to the lower index), as in the oracle."""
    indptr = np.array([0, 1, 2], dtype=np.int64)
    indices = np.array([1, 0], dtype=np.int64)
    ip, ix, _ = _dev(indptr, indices, None, "f64")
    E = gpu_lib.embed(ip, ix, None, 2, 3, seed=5, vec_dtype=vec).double().cpu().numpy()
    want = o.embed(2, indptr, indices, None, 2, 3, seed=5)
    assert col_rel_err(E, want) <= (1e-12 if vec == "f64" else 1e-6)
    assert np.allclose(E[0], E[1], rtol=1e-6, atol=0)
    lab = gpu_lib.cluster(ip, ix, None, 2, 2, 3, 5, kmeans_iters=5, vec_dtype=vec).cpu().numpy()
    lab_o, _, _ = o.fast_spectral_cluster(2, indptr, indices, None, 2, 2, 3, 5, 5)
    assert np.array_equal(lab, np.asarray(lab_o, dtype=np.int32))


def test_t0_cluster_is_kmeans_of_the_start_block(gpu_lib):
    """t = 0: no power step; the labels are k-means of D^{-1/2} X0."""
    g = synth.random_weighted(2000, 8000, seed=8, isolated=3)
    ip, ix, d = _dev(g.indptr, g.indices, g.data, "f64")
    lab = gpu_lib.cluster(ip, ix, d, 4, 3, 0, 2, kmeans_iters=15, vec_dtype="f64").cpu().numpy()
    lab_o, _, _ = o.fast_spectral_cluster(g.n, g.indptr, g.indices, g.data, 4, 3, 0, 2, 15)
    assert o.ari(lab, lab_o) >= 0.99
