"""The batched form against the single-graph path and the oracle: a batch of
small graphs of every block width (with hubs, isolated vertices, t = 0), and
a batch of graphs larger than one column slab (which the single-graph path
runs in the slab form), all in the shared XCD-affine level launches."""
import numpy as np
import pytest
import torch

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import check_elems, col_rel_err, host_weights, say, to_device

pytestmark = pytest.mark.gpu


def _batch():
    specs = [
        # (graph, k, l, t)
        (synth.sbm(1500, 5, 0.05, 0.002, seed=1), 5, 3, 12),
        (synth.random_weighted(3000, 12000, seed=2, hubs=3, hub_degree=1500, isolated=9), 4, 4, 9),
        (synth.sbm(400, 2, 0.1, 0.01, seed=3), 2, 1, 7),
        (synth.sbm(2500, 8, 0.03, 0.001, seed=4), 8, 5, 14),
        (synth.random_weighted(800, 3000, seed=5, weighted=False), 3, 2, 0),
        (synth.sbm(6000, 12, 0.02, 0.0003, seed=6), 12, 7, 10),
        (synth.disjoint_cliques(6, 30), 6, 4, 11),
        (synth.random_weighted(1200, 5000, seed=7, hubs=1, hub_degree=1100), 5, 8, 6),
    ]
    return specs


def test_batched_matches_single_graph_path(gpu_lib):
    specs = _batch()
    dev = []
    for g, k, l, t in specs:
        ip, ix, d = to_device(g, "f32")
        dev.append((ip, ix, d))
    ks = [s[1] for s in specs]
    ls = [s[2] for s in specs]
    ts = [s[3] for s in specs]
    seed = 11
    say("batched: graphs", len(specs))
    lab, emb, off, eoff = gpu_lib.cluster_batched(dev, ks, ls, ts, seed, kmeans_iters=20, return_embedding=True)
    lab2, emb2, _, _ = gpu_lib.cluster_batched(dev, ks, ls, ts, seed, kmeans_iters=20, return_embedding=True)
    lab3, emb3, _, _ = gpu_lib.cluster_batched(dev, ks, ls, ts, seed, kmeans_iters=20, return_embedding=True,
                                               use_graph=False)
    assert torch.equal(lab, lab2) and torch.equal(emb, emb2)       # graph replay
    assert torch.equal(lab, lab3) and torch.equal(emb, emb3)       # direct launches
    lab = lab.cpu().numpy()
    emb = emb.cpu().numpy()
    for gi, ((g, k, l, t), (ip, ix, d)) in enumerate(zip(specs, dev)):
        E = emb[eoff[gi]:eoff[gi + 1]].reshape(g.n, l)
        L = lab[off[gi]:off[gi + 1]]
        # single-graph path with the same seed
        Ls, Es = gpu_lib.cluster(ip, ix, d, k, l, t, seed + gi, kmeans_iters=20, return_embedding=True)
        Ls, Es = Ls.cpu().numpy(), Es.cpu().numpy()
        err_single = col_rel_err(E, Es)
        want = o.embed(g.n, g.indptr, g.indices, host_weights(d), l, t, seed=seed + gi)
        err_oracle = col_rel_err(E, want)
        a = o.ari(L, Ls)
        say(f"  graph {gi}: n={g.n} k={k} l={l} t={t} err vs single {err_single:.1e} vs oracle {err_oracle:.1e} ARI {a:.4f}")
        assert err_oracle <= 1e-5
        assert err_single <= 1e-5
        check_elems(E, want, "f32", "vs oracle")
        check_elems(E, Es, "f32", "vs single")
        assert a >= 0.99
        assert L.min() >= 0 and L.max() < k


def test_batched_errors(gpu_lib):
    g = synth.sbm(300, 3, 0.1, 0.01, seed=0)
    ip, ix, _ = to_device(g)
    with pytest.raises(gpu_lib.FscError):
        gpu_lib.cluster_batched([(ip, ix, None)], [3], [9], [5], 0)
    with pytest.raises(gpu_lib.FscError):
        gpu_lib.cluster_batched([(ip, ix, None)], [301], [2], [5], 0)


def test_batched_graphs_larger_than_a_slab(gpu_lib):
    # n x l blocks of 1.1 to 3.2 MB, above the 1 MB column slab: the single
    # path takes the slab form, the batch the XCD-affine tile launches
    specs = [(synth.sbm_by_degree(70000, 4, 18, 2, seed=31, permute=True), 4, 3, 34),
             (synth.sbm_by_degree(120000, 9, 27, 3, seed=32, permute=True), 9, 5, 36),
             (synth.sbm_by_degree(200000, 12, 45, 5, seed=33, permute=True), 12, 5, 37)]
    dev = [to_device(g, "f32") for g, _, _, _ in specs]
    ks, ls, ts = [s[1] for s in specs], [s[2] for s in specs], [s[3] for s in specs]
    seed = 5
    lab, emb, off, eoff = gpu_lib.cluster_batched(dev, ks, ls, ts, seed, kmeans_iters=30, return_embedding=True)
    lab, emb = lab.cpu().numpy(), emb.cpu().numpy()
    for gi, ((g, k, l, t), (ip, ix, d)) in enumerate(zip(specs, dev)):
        E = emb[eoff[gi]:eoff[gi + 1]].reshape(g.n, l)
        L = lab[off[gi]:off[gi + 1]]
        want = o.embed(g.n, g.indptr, g.indices, host_weights(d), l, t, seed=seed + gi)
        err = col_rel_err(E, want)
        Ls, Es = gpu_lib.cluster(ip, ix, d, k, l, t, seed + gi, kmeans_iters=30, return_embedding=True)
        a = o.ari(L, Ls.cpu().numpy())
        say(f"  graph {gi}: n={g.n} k={k} l={l} t={t} err vs oracle {err:.1e} ARI vs single {a:.4f} "
            f"vs planted {o.ari(L, g.labels):.4f}")
        assert err <= 1e-5
        check_elems(E, want, "f32", "vs oracle")
        check_elems(E, Es.cpu().numpy(), "f32", "vs single")
        assert a >= 0.99
