#!/usr/bin/env python
"""Benchmark of FastSpectralCluster (Algorithm 2) on one MI355X.

Default workload: the large SBM -- n = 1,000,000 vertices, k = 10 equal
clusters, expected in-degree 36 and out-degree 4 (Bernoulli edges), vertex
ids randomly permuted, CSR with int32 columns and fp32 unit weights; l = 4
Gaussian vectors, t = 30 power
steps with per-step FP64 column norms and Rayleigh quotients; k-means++ then
30 Lloyd steps.  One step = one full fsc_cluster call on inputs already in
HBM.  value = nnz * l * t / step time (edge x vector x iteration per second).

The JSON line also carries the roofline of the dominant kernel (the sparse
product of one power step, timed with HIP events inside the library on the
call's stream; as stored and pattern-only), the FP64 CPU oracle's whole run
on the same graph (all host threads and one), and the GPU result against it
(FP64 relative error of the embedding, ARI of the labels).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges×vectors×iters/s (SpMM GB/s vs HBM peak) + clustering time at ARI parity"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "spmm_sbm1m_counters.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2310_10939_amd", "csrc", f)
                  for f in ("fsc_embed.hip", "fsc_slab.hpp", "fsc_slab.hip", "fsc_tiles.hpp", "fsc_device.hpp")]

WORKLOADS = {
    # name: (n, k, deg_in, deg_out, l, t, lloyd, vec dtype, weight dtype, permute)
    # vertex ids randomly permuted (seeded): the planted clusters give memory
    # no locality the method could not know about
    "sbm1m": (1_000_000, 10, 36, 4, 4, 30, 30, "f32", "f32", True),
    # the generator's order: cluster i holds vertices [i n/k, (i+1) n/k)
    "sbm1m-contig": (1_000_000, 10, 36, 4, 4, 30, 30, "f32", "f32", False),
    "sbm1m-bf16": (1_000_000, 10, 36, 4, 4, 30, 30, "bf16", "bf16", True),
    "sbm1k": (1000, 5, None, None, 3, 20, 20, "f64", None, False),
    # precision form on a k-NN graph: 70,000 points of 10 isotropic Gaussians
    # in 784 dimensions (means N(0, 4I)), symmetrised 10-NN graph with weights
    # exp(-d^2 / median d^2), weights and vectors in BF16 (a stand-in for the
    # MNIST-sized inputs of the paper's real-world experiments)
    "knn70k-bf16": (70_000, 10, None, None, 4, 40, 30, "bf16", "bf16", False),
}


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def make_graph(name, dev):
    """(host Graph, device indptr, indices, weights-or-None, planted labels)."""
    import torch
    import synth
    n, k, din, dout, l, t, lloyd, vec, wdt, permute = WORKLOADS[name]
    if name.startswith("knn"):
        from paper_2310_10939_amd import fsc
        X_h, lab = synth.gaussian_mixture(n // k, k, 784, seed=0)
        X = torch.from_numpy(X_h).to(dev)
        fsc.knn_graph(X, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ip, ix, w = fsc.knn_graph(X, 10)   # the graph the timed steps use
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        data = w.to(torch.bfloat16)
        # the oracle's input: the same graph definition computed with torch
        # ops on the same points, its weights rounded to BF16 as the device's
        rip, rix, rw, _ = synth.knn_mixture_device(n // k, k, 784, seed=0, device=dev)
        g = synth.Graph(n, rip.cpu().numpy(), rix.cpu().numpy(), None, lab)
        g.data = rw.to(torch.bfloat16).double().cpu().numpy()
        g.info = {"builder": "fsc_knn_graph (exact 10-NN search on the FP32 matrix cores, symmetrised)",
                  "knn_graph_ms": round(ms, 2),
                  "vs_torch_graph": synth.graph_agreement((ip, ix, w), (rip, rix, rw))}
        return g, ip, ix, data, torch.from_numpy(lab.astype(np.int32)).to(dev)
    g = synth.sbm(n, k, 0.5, 0.01, seed=0) if din is None else \
        synth.sbm_by_degree(n, k, din, dout, seed=0, permute=permute)
    ip = torch.from_numpy(g.indptr).to(dev)
    ix = torch.from_numpy(g.indices).to(dev)
    data = None
    if wdt is not None:
        tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[wdt]
        data = torch.ones(g.nnz, dtype=tdt, device=dev)   # unit weights, stored
        g.data = None
    return g, ip, ix, data, torch.from_numpy(g.labels.astype(np.int32)).to(dev)


def spmm_bytes(n, nnz, l, vec, wdt, stats=True):
    """Algorithmic bytes of one power step: col + val per nonzero, the row
    pointer, one read and one write of the padded n x l block, 1/(2d), and
    the FP64 degree read by the statistics epilogue.  Gathers of Z rows are
    counted once (the block stays cache-resident)."""
    LH = 1 if l <= 1 else 2 if l <= 2 else 4 if l <= 4 else 8
    se = {"f64": 8, "f32": 4, "bf16": 2}[vec]
    sv = {None: 0, "f64": 8, "f32": 4, "bf16": 2}[wdt]
    ha = 8 if vec == "f64" else 4
    return nnz * (4 + sv) + (n + 1) * 8 + 2 * n * LH * se + n * ha + (n * 8 if stats else 0)


def pattern_bytes(n, nnz, l, vec):
    """The same without the stored weights (a unit-weight graph needs only
    its pattern)."""
    return spmm_bytes(n, nnz, l, vec, None)


def oracle_report(g, k, l, t, lloyd, seed, E_gpu, labels_gpu):
    """The FP64 oracle's whole FastSpectralCluster (Algorithm 2) on the same
    graph, seed and sizes: timed with every host thread its numpy/scipy
    calls may use and again with one, then compared with the GPU's embedding
    (per-column and element-wise relative error) and labels (ARI)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import fsc_oracle as o

    def run():
        t0 = time.perf_counter()
        lab, _, E = o.fast_spectral_cluster(g.n, g.indptr, g.indices, g.data, k, l, t, seed, lloyd)
        return time.perf_counter() - t0, lab, E

    nproc = len(os.sched_getaffinity(0))
    pools = threadpool_info()
    threads = max([p.get("num_threads", 1) for p in pools] or [1])
    print(f"oracle: whole run with up to {threads} threads", file=sys.stderr, flush=True)
    dt_all, lab_o, E_o = run()
    print(f"oracle: {dt_all:.1f} s; again on one thread", file=sys.stderr, flush=True)
    with threadpool_limits(1):
        dt_1, _, _ = run()
    E_gpu = np.asarray(E_gpu, dtype=np.float64)
    col = float(np.max(np.linalg.norm(E_gpu - E_o, axis=0) / np.linalg.norm(E_o, axis=0)))
    rms = np.sqrt(np.mean(E_o * E_o, axis=0))
    elem = float(np.max(np.abs(E_gpu - E_o) / (np.abs(E_o) + 1e-3 * rms[None, :])))
    evi = g.nnz * l * t
    base = {"value": evi / dt_all, "unit": "EVI/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole FP64 oracle FastSpectralCluster on the full graph (t={t} power steps, "
                      f"k-means++ and {lloyd} Lloyd steps), {dt_all:.1f} s with up to {threads} BLAS threads "
                      f"(its sparse products run on one); {dt_1:.1f} s on one thread",
            "seconds": round(dt_all, 2), "value_1thread": evi / dt_1, "seconds_1thread": round(dt_1, 2),
            "nproc": nproc}
    parity = {"fp64_rel_err": col, "fp64_elem_err": elem, "elem_err_floor": "1e-3 x column rms",
              "ari_vs_oracle": round(float(o.ari(labels_gpu, lab_o)), 6)}
    return base, parity


def bench_batched(args):
    """512 SBM graphs (n in [1000, 200000], k in [2, 20], degree in [8, 64]
    with in/out ratio 9:1, fp32 unit weights, l = ceil(log2 k) + 1,
    t = ceil(3 ln n)) clustered by one fsc_cluster_batched call per step."""
    import torch
    import synth
    from paper_2310_10939_amd import fsc
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    params = synth.batched_sbm_params(512, seed=0)
    t_gen = time.perf_counter()
    graphs, planted = [], []
    for p in params:
        ip, ix, lab = synth.sbm_device(p["n"], p["k"], p["deg_in"], p["deg_out"], p["seed"], device=dev)
        graphs.append((ip, ix, torch.ones(ix.numel(), dtype=torch.float32, device=dev)))
        planted.append(lab)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    ks = [p["k"] for p in params]
    ls = [p["l"] for p in params]
    ts = [p["t"] for p in params]
    nnz = [g[1].numel() for g in graphs]
    evi = sum(z * l * t for z, l, t in zip(nnz, ls, ts))
    # autotune the tile shape once per degree class on a representative graph
    tuned = {}
    for cls_lo, cls_hi in ((0, 12), (12, 24), (24, 48), (48, 1e9)):
        cand = [i for i, p in enumerate(params) if cls_lo <= nnz[i] / p["n"] < cls_hi]
        if cand:
            i = max(cand, key=lambda j: params[j]["n"])
            tuned[f"deg<{cls_hi:g}"] = fsc.autotune(*graphs[i], ls[i], steps=5)
    seed = 0
    for _ in range(args.warmup):
        fsc.cluster_batched(graphs, ks, ls, ts, seed, kmeans_iters=30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        labels, off = fsc.cluster_batched(graphs, ks, ls, ts, seed, kmeans_iters=30)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    # the plain single-graph path over the same graphs, for comparison
    ms_loop, ari_plain, ari_planted = None, [], []
    if not args.no_plain_loop:
        for i in range(2):
            fsc.cluster(*graphs[i], ks[i], ls[i], ts[i], seed + i, kmeans_iters=30)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = [fsc.cluster(*graphs[i], ks[i], ls[i], ts[i], seed + i, kmeans_iters=30) for i in range(len(graphs))]
        torch.cuda.synchronize()
        ms_loop = (time.perf_counter() - t0) * 1e3
    for i in range(len(graphs)):
        lb = labels[off[i]:off[i + 1]]
        if ms_loop is not None:
            ari_plain.append(float(fsc.ari(lb, plain[i], ks[i], ks[i])))
        ari_planted.append(float(fsc.ari(lb, planted[i], ks[i], ks[i])))
    res = {
        "metric": METRIC, "value": evi / (ms_step / 1e3), "unit": "EVI/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded SBM, device-generated)",
        "config": {"workload": "batched512", "graphs": len(graphs), "sum_n": sum(p["n"] for p in params),
                   "sum_nnz": sum(nnz), "evi_per_step": evi, "lloyd_steps": 30, "parallelism": "single GPU"},
        "plain_loop_ms": ms_loop, "speedup_vs_plain_loop": ms_loop / ms_step if ms_loop else None,
        "ari_vs_plain": {"min": min(ari_plain), "mean": float(np.mean(ari_plain)),
                         "below_0.99": int(sum(a < 0.99 for a in ari_plain))} if ari_plain else None,
        "ari_vs_planted": {"min": min(ari_planted), "mean": float(np.mean(ari_planted))},
        "autotuned": tuned, "graph_generation_s": round(t_gen, 1),
    }
    print(json.dumps(res))
    return 0


def copy_probe(mb=512, reps=5):
    """A plain device copy of known size, to calibrate the HBM byte counters."""
    import torch
    x = torch.empty(mb * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": x.numel() * 4, "copy_probe_bytes_written": y.numel() * 4,
                      "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sbm1m", choices=sorted(WORKLOADS) + ["batched512"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-plain-loop", action="store_true",
                    help="batched512: skip the single-graph loop run for comparison (for kernel traces)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        return 2
    import torch
    if args.copy_probe:
        copy_probe()
        return 0
    if args.workload == "batched512":
        return bench_batched(args)
    from paper_2310_10939_amd import fsc

    n, k, din, dout, l, t, lloyd, vec, wdt, permute = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    g, ip, ix, data, planted = make_graph(args.workload, dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    seed = 0

    def step(**kw):
        return fsc.cluster(ip, ix, data, k, l, t, seed, kmeans_iters=lloyd, vec_dtype=vec, traces=True, **kw)

    LH = 1 if l <= 1 else 2 if l <= 2 else 4 if l <= 4 else 8
    slab_kb = fsc.tuning()["slab_kb"]
    row_bytes = LH * {"f64": 8, "f32": 4, "bf16": 2}[vec]
    S = 1
    while slab_kb > 0 and S * 2 * row_bytes <= slab_kb * 1024:
        S *= 2
    slab = vec != "f64" and slab_kb > 0 and g.n > S   # the library's rule for the column-slab form
    # a graph whose steps run the tile kernel gets its tile shape autotuned
    # once, before the timed region (the slab form has no tile shape to tune)
    tuned = None if slab else fsc.autotune(ip, ix, data, l, steps=5)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fsc.timing_enable(True)
    fsc.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, spmm_ms = fsc.timing_read()
    fsc.timing_enable(False)
    labels, sq, ray = out
    ari = float(fsc.ari(labels, planted, k, k))
    ms_step = (t1 - t0) * 1e3 / args.steps
    nnz = int(ix.numel())   # the graph the steps run on
    evi = nnz * l * t
    value = evi / (ms_step / 1e3)

    avg_ms = spmm_ms / max(launches, 1)
    bytes_launch = spmm_bytes(g.n, nnz, l, vec, wdt)
    achieved = bytes_launch / (avg_ms / 1e3) / 1e9
    traffic = None
    if os.path.exists(COUNTERS):
        c = json.load(open(COUNTERS))
        if c.get("kernel_hash") == kernel_hash() and c.get("workload") == args.workload:
            traffic = c.get("hbm_bytes_per_launch")
    kname = ("slab_kernel<StepOp> (one power step, column-slab form)" if slab
             else "tile_kernel<StepOp> (one power step)")
    pat = pattern_bytes(g.n, nnz, l, vec)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "avg_launch_us": round(avg_ms * 1e3, 2),
                "launches": launches, "algorithmic_bytes_per_launch": bytes_launch,
                "pattern_only_bytes_per_launch": pat,
                "frac_pattern_only": round(pat / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    knn = args.workload.startswith("knn")
    res = {
        "metric": METRIC, "value": value, "unit": "EVI/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": vec,
        "data": "synthetic (seeded Gaussian mixture, 10-NN graph)" if knn else "synthetic (seeded SBM)",
        "config": {"workload": args.workload, "n": g.n, "nnz": nnz, "k": k, "l": l, "t": t,
                   "lloyd_steps": lloyd, "weights": wdt or "unit (implicit)", "vertex_order":
                   "mixture components contiguous" if knn else
                   ("permuted" if permute else "planted clusters contiguous"), "parallelism": "single GPU"},
        "ari_vs_planted": round(ari, 6),
        "spmm_ms_per_step": spmm_ms / args.steps,
        "roofline": roofline,
        "graph_generation_s": round(t_gen, 1),
    }
    if getattr(g, "info", None):
        res["graph"] = g.info
    if tuned is not None:
        res["autotuned"] = tuned
    if not args.no_cpu_baseline:
        # one more call outside the timed region, same seed (same labels),
        # for its embedding
        lab_e, E_gpu, _, _ = step(return_embedding=True)
        torch.cuda.synchronize()
        res["cpu_baseline"], parity = oracle_report(g, k, l, t, lloyd, seed, E_gpu.float().cpu().numpy(),
                                                    lab_e.cpu().numpy())
        res.update(parity)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
