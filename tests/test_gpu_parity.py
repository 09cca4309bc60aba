"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: FP64 vectors 1e-12 relative per column; FP32 1e-5; BF16 storage
2e-2 (against the oracle run on the same bf16-rounded weights).  Labels: ARI
>= 0.99 against the oracle, plus validity (every label is a nearest centre).
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import check_elems, col_rel_err, host_weights, say, to_device

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


def oracle_embed(g, data_host, l, t, seed, traced=False):
    return o.embed(g.n, g.indptr, g.indices, data_host, l, t, seed=seed, traced=traced)


def test_native_library_is_loaded(gpu_lib):
    maps = open("/proc/self/maps").read()
    assert os.path.join("paper_2310_10939_amd", "libfsc.so") in maps


# --------------------------------------------------------------------------
# Embedding
# --------------------------------------------------------------------------
def test_start_block_t0_matches_oracle_philox(gpu_lib):
    g = synth.sbm(500, 4, 0.1, 0.01, seed=3)
    ip, ix, _ = to_device(g)
    say("t=0 start block, n=500")
    E = gpu_lib.embed(ip, ix, None, 4, 0, seed=77, vec_dtype="f64").cpu().numpy()
    want = oracle_embed(g, None, 4, 0, 77)
    assert np.abs(E - want).max() <= 1e-14 * np.abs(want).max()


def test_small_sbm_fp64(gpu_lib):
    g = synth.sbm(1000, 5, 0.5, 0.01, seed=0)
    ip, ix, _ = to_device(g)
    say("C1 sbm fp64 l=3 t=20")
    E = gpu_lib.embed(ip, ix, None, 3, 20, seed=0, vec_dtype="f64").cpu().numpy()
    want = oracle_embed(g, None, 3, 20, 0)
    err = col_rel_err(E, want)
    say("fp64 rel err", err)
    assert err <= TOL["f64"]
    check_elems(E, want, "f64")


@pytest.mark.parametrize("l", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("vec", ["f64", "f32"])
def test_ragged_weighted_graph(gpu_lib, l, vec):
    # hubs make long rows (chunked, combined in order), isolated vertices make
    # empty rows; a small tile size gives many tiles and a ragged tail
    g = synth.random_weighted(3000, 12000, seed=l, hubs=4, hub_degree=1500, isolated=13)
    ip, ix, d = to_device(g, "keep" if vec == "f64" else "f32")
    say(f"ragged n=3000 nnz={g.nnz} l={l} vec={vec}")
    for tile in (64, 0):
        E = gpu_lib.embed(ip, ix, d, l, 9, seed=5, vec_dtype=vec, tile_nnz=tile).cpu().numpy()
        want = oracle_embed(g, host_weights(d), l, 9, 5)
        err = col_rel_err(E, want)
        say("  tile", tile, "rel err", err)
        assert err <= TOL[vec]
        check_elems(E, want, vec)
        assert np.all(E[-13:] == 0)


def test_bf16_storage_on_knn_graph(gpu_lib):
    g = synth.knn_mixture(300, 5, 32, seed=1)
    ip, ix, d = to_device(g, "bf16")
    say(f"knn bf16 n={g.n} nnz={g.nnz}")
    E = gpu_lib.embed(ip, ix, d, 4, 40, seed=2, vec_dtype="bf16").float().cpu().numpy()
    want = oracle_embed(g, host_weights(d), 4, 40, 2)
    err = col_rel_err(E, want)
    say("bf16 rel err", err)
    assert err <= TOL["bf16"]
    check_elems(E, want, "bf16")
    # f32 vectors with bf16 weights
    E32 = gpu_lib.embed(ip, ix, d, 4, 40, seed=2, vec_dtype="f32").cpu().numpy()
    assert col_rel_err(E32, want) <= TOL["f32"]


def test_cliques_constant_per_component(gpu_lib):
    g = synth.disjoint_cliques(6, 40)
    ip, ix, _ = to_device(g)
    E = gpu_lib.embed(ip, ix, None, 3, 30, seed=1, vec_dtype="f32").cpu().numpy().reshape(6, 40, 3)
    spread = np.abs(E - E.mean(axis=1, keepdims=True)).max()
    # gamma' = 38/78 per step: after 30 steps the non-constant part is ~1e-9
    assert spread <= 1e-6 * np.abs(E).max()


def test_traces_and_renorm(gpu_lib):
    g = synth.random_weighted(2000, 9000, seed=11, hubs=2, hub_degree=900, isolated=5)
    ip, ix, d = to_device(g, "keep")
    _, sq_o, ray_o = oracle_embed(g, host_weights(d), 3, 12, 4, traced=True)
    for vec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        dd = d if vec == "f64" else d.float()
        E, sq, ray = gpu_lib.embed(ip, ix, dd, 3, 12, seed=4, vec_dtype=vec, traces=True, tile_nnz=128)
        sq, ray = sq.cpu().numpy(), ray.cpu().numpy()
        assert np.abs(sq - sq_o).max() <= tol * 10 * np.abs(sq_o).max()
        assert np.abs(ray - ray_o).max() <= tol * 10
        assert np.all((ray >= -tol) & (ray <= 1 + tol))
        # re-normalised iterations return the un-normalised result
        En, sqn, rayn = gpu_lib.embed(ip, ix, dd, 3, 12, seed=4, vec_dtype=vec, traces=True, renorm=True,
                                      tile_nnz=128)
        assert col_rel_err(En.cpu().numpy(), E.cpu().numpy()) <= 10 * tol
        assert np.abs(sqn.cpu().numpy() - sq_o).max() <= tol * 10 * np.abs(sq_o).max()


def test_deterministic(gpu_lib):
    g = synth.random_weighted(5000, 40000, seed=2, hubs=3, hub_degree=3000)
    ip, ix, d = to_device(g, "f32")
    a = gpu_lib.embed(ip, ix, d, 4, 10, seed=9, traces=True, tile_nnz=256)
    b = gpu_lib.embed(ip, ix, d, 4, 10, seed=9, traces=True, tile_nnz=256)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_caller_start_block(gpu_lib):
    g = synth.sbm(800, 4, 0.05, 0.005, seed=8)
    ip, ix, _ = to_device(g)
    x0 = np.random.default_rng(0).standard_normal((g.n, 2))
    E = gpu_lib.embed(ip, ix, None, 2, 7, seed=0, vec_dtype="f64",
                      x0=torch.from_numpy(x0).cuda()).cpu().numpy()
    want = o.embed(g.n, g.indptr, g.indices, None, 2, 7, x0=x0)
    assert col_rel_err(E, want) <= 1e-12


# --------------------------------------------------------------------------
# k-means and ARI
# --------------------------------------------------------------------------
def _valid_assignment(P, labels, C, tol):
    d = ((P[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    own = d[np.arange(len(P)), labels]
    return np.all(own <= d.min(axis=1) + tol * (1 + d.min(axis=1)))


@pytest.mark.parametrize("k,l", [(5, 4), (17, 4), (40, 8), (3, 2), (10, 6)])
def test_kmeans_parity(gpu_lib, k, l):
    X, truth = synth.gaussian_mixture(400, k, l, seed=k, mean_scale=6.0)
    X = X.astype(np.float32)
    say(f"kmeans k={k} l={l} n={len(X)}")
    lab_o, C_o = o.kmeans(X.astype(np.float64), k, 20, seed=3)
    lab, C = gpu_lib.kmeans(torch.from_numpy(X).cuda(), k, 20, seed=3)
    lab, C = lab.cpu().numpy(), C.cpu().numpy()
    assert lab.min() >= 0 and lab.max() < k
    a = o.ari(lab, lab_o)
    say("  ARI vs oracle", a)
    assert a >= 0.99
    assert _valid_assignment(X.astype(np.float64), lab, C.astype(np.float64), 1e-4)


@pytest.mark.parametrize("n,l,k", [(5, 2, 1), (64, 1, 64), (700, 3, 2), (5000, 3, 7), (40000, 8, 33), (20000, 4, 64)])
def test_kmeanspp_seeds_match_oracle_exactly(gpu_lib, n, l, k):
    """Greedy k-means++ on points of an integer grid: every squared distance
    and every running sum is exact on both sides, so the GPU must choose the
    oracle's rows, candidate for candidate (0 Lloyd steps leave the seeds as
    the centres).  Some rows are ineligible."""
    rng = np.random.default_rng(n + k)
    X = rng.integers(-100, 101, size=(n, l)).astype(np.float32)
    elig = (np.arange(n) % 5 != 2)
    idx = o.kmeanspp(X.astype(np.float64), k, 11, eligible=elig)
    _, C = gpu_lib.kmeans(torch.from_numpy(X).cuda(), k, 0, seed=11,
                          eligible=torch.from_numpy(elig.astype(np.uint8)).cuda())
    say(f"kmeans++ n={n} l={l} k={k}")
    assert np.array_equal(C.cpu().numpy(), X[idx])


def test_kmeanspp_with_fewer_distinct_points_than_k(gpu_lib):
    """Three distinct points repeated, k = 6: after three centres every D^2
    is 0 and the seeding takes unchosen rows; the centres are the oracle's
    and every label is valid."""
    X = np.repeat(np.array([[0, 0], [5, 1], [-3, 7]], dtype=np.float32), [40, 25, 35], axis=0)
    idx = o.kmeanspp(X.astype(np.float64), 6, 2)
    lab, C = gpu_lib.kmeans(torch.from_numpy(X).cuda(), 6, 5, seed=2)
    lab = lab.cpu().numpy()
    assert lab.min() >= 0 and lab.max() < 6
    _, C0 = gpu_lib.kmeans(torch.from_numpy(X).cuda(), 6, 0, seed=2)
    assert np.array_equal(C0.cpu().numpy(), X[idx])
    assert _valid_assignment(X.astype(np.float64), lab, C.cpu().numpy().astype(np.float64), 1e-6)


def test_lloyd_stops_at_its_fixed_point(gpu_lib):
    """Overlapping clusters take several Lloyd steps to settle.  The results
    for 0, 1, 2, ... steps change until a step changes no label, and from
    then on every step count gives the same labels and centres bit for bit
    (the library skips the steps after such a step, which would repeat it)."""
    X, _ = synth.gaussian_mixture(2000, 12, 6, seed=5, mean_scale=2.0)
    Xt = torch.from_numpy(X.astype(np.float32)).cuda()
    runs = []
    for it in range(0, 41):
        lab, C = gpu_lib.kmeans(Xt, 12, it, seed=4)
        runs.append((lab.cpu().numpy(), C.cpu().numpy()))
    same = [np.array_equal(runs[i][0], runs[i - 1][0]) and np.array_equal(runs[i][1], runs[i - 1][1])
            for i in range(1, len(runs))]
    first = next((i + 1 for i, v in enumerate(same) if v), None)
    say(f"lloyd settles after {first} steps")
    assert first is not None and first >= 3
    for it in list(range(first, len(runs))) + [200]:
        lab, C = runs[it] if it < len(runs) else (x.cpu().numpy() for x in gpu_lib.kmeans(Xt, 12, it, seed=4))
        assert np.array_equal(lab, runs[first][0]) and np.array_equal(C, runs[first][1]), it
    lab_o, _ = o.kmeans(X.astype(np.float64), 12, first, seed=4)
    assert o.ari(runs[first][0], lab_o) >= 0.99


def test_kmeans_eligibility_and_fp64_points(gpu_lib):
    X, _ = synth.gaussian_mixture(300, 4, 3, seed=1, mean_scale=5.0)
    X = X.astype(np.float64)
    elig = (np.arange(len(X)) % 5 != 0).astype(np.uint8)
    lab_o, C_o = o.kmeans(X, 4, 15, seed=2, eligible=elig.astype(bool))
    lab, C = gpu_lib.kmeans(torch.from_numpy(X).cuda(), 4, 15, seed=2,
                            eligible=torch.from_numpy(elig).cuda())
    assert o.ari(lab.cpu().numpy(), lab_o) >= 0.99


def test_ari_kernel(gpu_lib):
    rng = np.random.default_rng(0)
    for n in [1, 7, 1000, 100000]:
        a = rng.integers(0, 6, n).astype(np.int32)
        b = np.where(rng.random(n) < 0.6, a, rng.integers(0, 9, n)).astype(np.int32)
        got = float(gpu_lib.ari(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), 6, 9))
        assert abs(got - o.ari(a, b)) < 1e-12
    # tables counted in LDS per block (up to 8192 cells) and in global memory
    # (larger); agreeing labelings put most pairs in a few cells
    for n, ka, kb in [(1_000_000, 10, 10), (50_000, 64, 64), (20_000, 100, 100), (30_000, 8192, 2)]:
        a = rng.integers(0, ka, n).astype(np.int32)
        b = np.where(rng.random(n) < 0.97, a % kb, rng.integers(0, kb, n)).astype(np.int32)
        got = float(gpu_lib.ari(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), ka, kb))
        assert abs(got - o.ari(a, b)) < 1e-12, (n, ka, kb)


def test_nmi_kernel(gpu_lib):
    rng = np.random.default_rng(1)
    for n, ka, kb in [(1, 6, 9), (7, 6, 9), (1000, 6, 9), (100000, 10, 10), (300000, 2048, 2048)]:
        a = rng.integers(0, ka, n).astype(np.int32)
        b = np.where(rng.random(n) < 0.6, a % kb, rng.integers(0, kb, n)).astype(np.int32)
        got = float(gpu_lib.nmi(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), ka, kb))
        assert abs(got - o.nmi(a, b)) < 1e-12, (n, ka, kb)


def test_nmi_degenerate_cases(gpu_lib):
    z = torch.zeros(50, dtype=torch.int32, device="cuda")
    assert float(gpu_lib.nmi(z, z, 1, 1)) == 1.0                       # both one cluster
    assert float(gpu_lib.nmi(z[:0], z[:0], 3, 3)) == 1.0               # no items
    alt = torch.arange(50, dtype=torch.int32, device="cuda") % 2
    assert float(gpu_lib.nmi(z, alt, 1, 2)) == 0.0                     # one trivial labeling
    # out-of-range labels drop their pair
    rng = np.random.default_rng(2)
    a = rng.integers(0, 5, 4000).astype(np.int32)
    b = np.where(rng.random(4000) < 0.7, a, rng.integers(0, 5, 4000)).astype(np.int32)
    a[::13] = -1
    b[5::17] = 5
    keep = (a >= 0) & (b < 5)
    got = float(gpu_lib.nmi(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), 5, 5))
    assert abs(got - o.nmi(a[keep], b[keep])) < 1e-12


# --------------------------------------------------------------------------
# Whole pipeline
# --------------------------------------------------------------------------
def test_cluster_small_sbm(gpu_lib):
    # 10 trials of the small SBM (FP64, l = 3, t = 20, 20 Lloyd steps)
    for trial in range(10):
        g = synth.sbm(1000, 5, 0.5, 0.01, seed=trial)
        ip, ix, _ = to_device(g)
        lab = gpu_lib.cluster(ip, ix, None, 5, 3, 20, seed=trial, kmeans_iters=20, vec_dtype="f64").cpu().numpy()
        lab_o, _, _ = o.fast_spectral_cluster(g.n, g.indptr, g.indices, None, 5, 3, 20, trial, 20)
        assert o.ari(lab, lab_o) >= 0.99
        assert o.ari(lab, g.labels) >= 0.99


def test_cluster_outputs_and_isolated(gpu_lib):
    g = synth.sbm(3000, 6, 0.02, 0.0005, seed=4)
    # add isolated vertices at the end
    n = g.n + 7
    indptr = np.concatenate([g.indptr, np.full(7, g.indptr[-1])])
    g2 = synth.Graph(n, indptr, g.indices, None, np.concatenate([g.labels, np.zeros(7, np.int32)]))
    ip, ix, _ = to_device(g2)
    lab, E, C = gpu_lib.cluster(ip, ix, None, 6, 4, 25, seed=1, kmeans_iters=25, return_embedding=True,
                                return_centres=True)
    lab, E, C = lab.cpu().numpy(), E.cpu().numpy(), C.cpu().numpy()
    lab_o, C_o, E_o = o.fast_spectral_cluster(n, indptr, g.indices, None, 6, 4, 25, 1, 25)
    assert col_rel_err(E, E_o) <= 1e-5
    assert np.all(E[-7:] == 0)
    assert o.ari(lab[:-7], lab_o[:-7]) >= 0.99
    assert _valid_assignment(E.astype(np.float64), lab, C.astype(np.float64), 1e-3)


def test_errors_are_reported(gpu_lib):
    g = synth.sbm(100, 2, 0.2, 0.01, seed=0)
    ip, ix, _ = to_device(g)
    with pytest.raises(gpu_lib.FscError) as e:
        gpu_lib.embed(ip, ix, None, 9, 3, seed=0)
    assert e.value.code == -1
    with pytest.raises(gpu_lib.FscError):
        gpu_lib.cluster(ip, ix, None, 101, 2, 3, seed=0)
    # validation: a self-loop and an out-of-range column
    bad = ix.clone()
    bad[0] = 0
    with pytest.raises(gpu_lib.FscError) as e:
        gpu_lib.embed(ip, bad, None, 2, 3, seed=0, validate=True)
    assert e.value.code == -2
    bad[0] = 100
    with pytest.raises(gpu_lib.FscError) as e:
        gpu_lib.embed(ip, bad, None, 2, 3, seed=0, validate=True)
    assert e.value.code == -2
    neg = -torch.ones(ix.numel(), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.FscError) as e:
        gpu_lib.embed(ip, ix, neg, 2, 3, seed=0, validate=True)
    assert e.value.code == -2
    # a valid graph passes validation
    gpu_lib.embed(ip, ix, None, 2, 3, seed=0, validate=True)
