"""Column-slab form of the sparse product: parity with the FP64 oracle and
with the plain tile kernel.

All three forms are checked: phases (every block walks the slabs), per-XCD
(8 slabs, partial sums added by a second kernel) and waves (every wave takes
its 64 rows through the slabs, sums in registers; bit-identical to phases).  Small graphs are cut into
many slabs by a small slab size (4 KiB of the block), with long rows (hubs, summed by chunks of the original CSR),
isolated vertices and a ragged last tile of rows.  The full-size test runs
the 1M-vertex SBM (vertex ids permuted, as the benchmark's default workload)
in the launch configuration the benchmark times (default tuning: 1 MiB
slabs) and compares the whole embedding and the labels with the oracle.  Tolerances as in the other parity tests: FP32 1e-5, BF16 2e-2
(relative, per column), ARI >= 0.99.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import check_elems, col_rel_err, host_weights, say, to_device

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}


@pytest.fixture
def slab(gpu_lib):
    def set_kb(kb, mode=0):
        return gpu_lib.tuning(slab_kb=kb, slab_mode=mode)
    yield set_kb
    gpu_lib.tuning(slab_kb=1024, slab_mode=3)


def test_slab_size_is_reported(gpu_lib, slab):
    assert slab(4)["slab_kb"] == 4
    assert slab(-1)["slab_kb"] == -1
    assert slab(1024)["slab_kb"] == 1024
    assert slab(0, 1)["slab_mode"] == 1
    assert slab(0, 2)["slab_mode"] == 2
    assert slab(0, 3)["slab_mode"] == 3
    assert slab(0, 4)["slab_mode"] == 4
    with pytest.raises(RuntimeError):
        slab(0, 5)


@pytest.mark.parametrize("mode", [1, 2, 4])
@pytest.mark.parametrize("l", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("vec,wt", [("f32", "f32"), ("f32", "none"), ("bf16", "bf16")])
def test_slab_matches_oracle_and_tiles(gpu_lib, slab, l, vec, wt, mode):
    # 5000 rows: 20 tiles of 256 rows, the last one ragged; hubs of 1200
    # nonzeros are long rows; 17 isolated vertices at the end
    g = synth.random_weighted(5000, 30000, seed=20 + l, hubs=5, hub_degree=1200, isolated=17)
    ip, ix, d = to_device(g, wt)
    want = o.embed(g.n, g.indptr, g.indices, host_weights(d), l, 7, seed=3)
    say(f"slab n=5000 nnz={g.nnz} l={l} vec={vec} weights={wt} mode={mode}")
    slab(-1)
    plain = gpu_lib.embed(ip, ix, d, l, 7, seed=3, vec_dtype=vec).float().cpu().numpy()
    slab(4, mode)
    E = gpu_lib.embed(ip, ix, d, l, 7, seed=3, vec_dtype=vec).float().cpu().numpy()
    err, err_plain = col_rel_err(E, want), col_rel_err(plain, want)
    say("  rel err slab", err, "tiles", err_plain)
    assert err <= TOL[vec]
    check_elems(E, want, vec)
    assert np.all(E[-17:] == 0)
    if vec == "f32":
        assert col_rel_err(E, plain) <= 1e-5


@pytest.mark.parametrize("mode", [1, 2, 4])
def test_slab_traces_and_renorm(gpu_lib, slab, mode):
    g = synth.random_weighted(4000, 20000, seed=11, hubs=3, hub_degree=900, isolated=5)
    ip, ix, d = to_device(g, "f32")
    _, sq_o, ray_o = o.embed(g.n, g.indptr, g.indices, host_weights(d), 3, 12, seed=4, traced=True)
    slab(4, mode)
    E, sq, ray = gpu_lib.embed(ip, ix, d, 3, 12, seed=4, traces=True)
    sq, ray = sq.cpu().numpy(), ray.cpu().numpy()
    assert np.abs(sq - sq_o).max() <= 1e-4 * np.abs(sq_o).max()
    assert np.abs(ray - ray_o).max() <= 1e-4
    En, sqn, _ = gpu_lib.embed(ip, ix, d, 3, 12, seed=4, traces=True, renorm=True)
    assert col_rel_err(En.cpu().numpy(), E.cpu().numpy()) <= 1e-4
    assert np.abs(sqn.cpu().numpy() - sq_o).max() <= 1e-4 * np.abs(sq_o).max()


@pytest.mark.parametrize("mode", [1, 2, 4])
def test_slab_unit_weight_tiles(gpu_lib, slab, mode):
    """Tiles whose weights are all exactly 1 skip the weight loads: stored
    unit weights give the same bits as no weights, and a graph where one
    edge pair weighs 2.5 (so only the tiles of its two rows load weights)
    matches the oracle."""
    g = synth.random_weighted(5000, 30000, seed=7, hubs=2, hub_degree=800, isolated=3)
    ip, ix, _ = to_device(g, "none")
    slab(4, mode)
    ones = torch.ones(g.nnz, dtype=torch.float32, device="cuda")
    a = gpu_lib.embed(ip, ix, ones, 4, 6, seed=1)
    b = gpu_lib.embed(ip, ix, None, 4, 6, seed=1)
    assert torch.equal(a, b)
    w = np.ones(g.nnz)
    r = 2500
    j = int(g.indptr[r])
    c = int(g.indices[j])
    k = int(g.indptr[c]) + int(np.nonzero(g.indices[g.indptr[c]:g.indptr[c + 1]] == r)[0][0])
    w[j] = w[k] = 2.5
    d = torch.from_numpy(w.astype(np.float32)).cuda()
    E = gpu_lib.embed(ip, ix, d, 4, 6, seed=1).cpu().numpy()
    want = o.embed(g.n, g.indptr, g.indices, w, 4, 6, seed=1)
    assert col_rel_err(E, want) <= TOL["f32"]


@pytest.mark.parametrize("mode", [1, 2, 4])
def test_slab_deterministic(gpu_lib, slab, mode):
    g = synth.random_weighted(6000, 50000, seed=2, hubs=3, hub_degree=3000)
    ip, ix, d = to_device(g, "f32")
    slab(8, mode)
    a = gpu_lib.embed(ip, ix, d, 4, 10, seed=9, traces=True)
    b = gpu_lib.embed(ip, ix, d, 4, 10, seed=9, traces=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("mode", [1, 2, 4])
def test_slab_cluster_small(gpu_lib, slab, mode):
    g = synth.sbm_by_degree(20000, 6, 24, 3, seed=5, permute=True)
    ip, ix, _ = to_device(g)
    slab(16, mode)
    lab = gpu_lib.cluster(ip, ix, None, 6, 4, 25, 1, kmeans_iters=20)
    lab_o, _, _ = o.fast_spectral_cluster(g.n, g.indptr, g.indices, None, 6, 4, 25, 1, 20)
    ari = float(gpu_lib.ari(lab, torch.from_numpy(np.asarray(lab_o, dtype=np.int32)).cuda(), 6, 6))
    say("slab cluster ARI vs oracle", ari)
    assert ari >= 0.99


@pytest.mark.parametrize("kb", [4, 64])
@pytest.mark.parametrize("l", [1, 3, 4, 8])
@pytest.mark.parametrize("wt", ["f32", "none", "bf16"])
def test_wave_form_equals_phase_form(gpu_lib, slab, kb, l, wt):
    """The wave form sums every row in the phase form's order, so the two
    give the same bits (the FP64 statistics are summed over the rows in
    another order and are compared to 1e-10)."""
    g = synth.random_weighted(9000, 60000, seed=40 + l, hubs=4, hub_degree=1500, isolated=9)
    ip, ix, d = to_device(g, wt)
    vec = "bf16" if wt == "bf16" else "f32"
    slab(kb, 1)
    a, sqa, raa = gpu_lib.embed(ip, ix, d, l, 9, seed=5, vec_dtype=vec, traces=True)
    slab(kb, 4)
    b, sqb, rab = gpu_lib.embed(ip, ix, d, l, 9, seed=5, vec_dtype=vec, traces=True)
    say(f"wave vs phases kb={kb} l={l} weights={wt}")
    assert torch.equal(a, b)
    assert torch.allclose(sqa, sqb, rtol=1e-10, atol=0)
    assert torch.allclose(raa, rab, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("kb", [4, 64])
def test_group_build_degrees_in_csr_order(gpu_lib, slab, kb):
    """The phase form's layout builder reads each row with eight lanes and
    counts the ones while every weight of a row so far is exactly 1, then
    sums the remaining weights in CSR order.  Rows here switch between the
    two at various positions, with weights whose FP64 sum depends on the
    order (1e8 and 1e-8 among ones); the wave form, whose builder sums each
    row in one thread, must give the same bits."""
    g = synth.random_weighted(9000, 60000, seed=61, hubs=4, hub_degree=1500, isolated=9)
    w = np.ones(g.nnz, dtype=np.float32)
    j = np.arange(g.nnz)
    w[j % 13 == 11] = 1e8
    w[j % 29 == 17] = 1e-8
    w[j % 31 == 0] = 0.1
    ip, ix, _ = to_device(g, "none")
    d = torch.from_numpy(w).cuda()
    slab(kb, 1)
    a, sqa, _ = gpu_lib.embed(ip, ix, d, 4, 9, seed=5, traces=True)
    slab(kb, 4)
    b, sqb, _ = gpu_lib.embed(ip, ix, d, 4, 9, seed=5, traces=True)
    say(f"group-form degrees kb={kb}")
    assert torch.equal(a, b)
    assert torch.allclose(sqa, sqb, rtol=1e-10, atol=0)
    E = a.cpu().numpy()
    want = o.embed(g.n, g.indptr, g.indices, w.astype(np.float64), 4, 9, seed=5)
    assert col_rel_err(E, want) <= TOL["f32"]


def test_full_size_sbm_matches_oracle(gpu_lib):
    """The 1M-vertex SBM (k = 10, in-degree 36, out-degree 4, fp32 unit
    weights, l = 4, t = 30, 30 Lloyd steps) in the benchmark's launch
    configuration: the whole FP32 embedding against the FP64 oracle, and
    the labels against the oracle's k-means on the oracle embedding."""
    g = synth.sbm_by_degree(1_000_000, 10, 36, 4, seed=0, permute=True)
    ip, ix, _ = to_device(g)
    data = torch.ones(g.nnz, dtype=torch.float32, device="cuda")
    say(f"full-size SBM n={g.n} nnz={g.nnz}")
    E = gpu_lib.embed(ip, ix, data, 4, 30, seed=0).cpu().numpy()
    want = o.embed(g.n, g.indptr, g.indices, None, 4, 30, seed=0)
    err = col_rel_err(E, want)
    say("  rel err", err)
    assert err <= TOL["f32"]
    check_elems(E, want, "f32", "1M SBM")
    lab = gpu_lib.cluster(ip, ix, data, 10, 4, 30, 0, kmeans_iters=30)
    d = o.degrees(g.n, g.indptr, g.indices, None)
    lab_o, _ = o.kmeans(want, 10, 30, 0, eligible=d > 0)
    ari = float(gpu_lib.ari(lab, torch.from_numpy(np.asarray(lab_o, dtype=np.int32)).cuda(), 10, 10))
    say("  ARI vs oracle", ari)
    assert ari >= 0.99
