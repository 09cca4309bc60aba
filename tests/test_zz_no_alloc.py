"""fsc_cluster_noalloc (the entry point that allocates no device memory)
against fsc_cluster through the C ABI: labels, embedding and centres equal
bit for bit on two calls in a row, the second with a smaller graph (the
scratch array keeps the first call's contents), and a graph whose workspace
exceeds the scratch array is rejected with FSC_E_NOMEM."""
import numpy as np
import pytest
import torch

import synth
from oracle import fsc_oracle as o
from tests.gpu_util import say, to_device

pytestmark = pytest.mark.gpu


def _both(fsc, g, k, l, t, seed, vec="f32", weights="f32"):
    ip, ix, d = to_device(g, weights)
    a = fsc.cluster(ip, ix, d, k, l, t, seed, kmeans_iters=20, vec_dtype=vec, return_embedding=True,
                    return_centres=True)
    b = fsc.cluster_noalloc(ip, ix, d, k, l, t, seed, kmeans_iters=20, vec_dtype=vec, return_embedding=True,
                            return_centres=True)
    torch.cuda.synchronize()
    return a, b


def _same(a, b):
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_noalloc_equals_cluster_on_two_calls_the_second_smaller(gpu_lib):
    # a graph on the column-slab path (block larger than 1 MiB), then a
    # smaller one on the tile path
    big = synth.sbm_by_degree(120_000, 6, 18, 2, seed=4, permute=True)
    small = synth.sbm(3000, 4, 0.05, 0.002, seed=5)
    say(f"noalloc call 1: n={big.n} nnz={big.nnz}")
    a, b = _both(gpu_lib, big, 6, 4, 20, 3)
    _same(a, b)
    assert o.ari(b[0].cpu().numpy(), big.labels) >= 0.99
    say(f"noalloc call 2: n={small.n} nnz={small.nnz}")
    a, b = _both(gpu_lib, small, 4, 3, 12, 8)
    _same(a, b)
    assert o.ari(b[0].cpu().numpy(), small.labels) >= 0.99


def test_noalloc_other_precisions_and_shapes(gpu_lib):
    g = synth.random_weighted(5000, 30000, seed=21, hubs=3, hub_degree=1200, isolated=11)
    for vec, wt, l in [("f64", "keep", 3), ("bf16", "bf16", 4), ("f32", "none", 8)]:
        say(f"noalloc vec={vec} weights={wt} l={l}")
        a, b = _both(gpu_lib, g, 5, l, 9, 2, vec=vec, weights=wt)
        _same(a, b)


def test_noalloc_rejects_a_graph_beyond_the_scratch(gpu_lib):
    g = synth.sbm_by_degree(400_000, 4, 36, 4, seed=1)
    ip, ix, d = to_device(g, "f32")
    with pytest.raises(gpu_lib.FscError, match="scratch array") as e:
        gpu_lib.cluster_noalloc(ip, ix, d, 4, 4, 5, 0)
    assert e.value.code == -4
