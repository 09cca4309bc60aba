"""Ten-trial accuracy and time report in the style of the paper's Table 1.

Each method runs `--trials` times on one fixed synthetic graph, with method
seeds 0, 1, ...; each trial's labels are scored against the planted clusters
with ARI and NMI (the two accuracy scores of Sec. 4.2, both computed by the
library's kernels) and timed with HIP events around the one library call
(after one untimed call that warms the context's workspace).  The report gives
mean +- standard deviation (population, over the trials) per method.

Methods:
  fsc        the plain method (Algorithm 2), l = ceil(log2 k), t as named by
             the workload
  fsc-l+1    the same with one more vector than log2 k
  pm-k       PM with k vectors (the comparison method of Sec. 4: k power
             vectors and one SVD), for k <= 8, same t
  k-eigs     the k leading eigenvectors of M (Sec. 4's "k Eigenvectors"), by
             subspace iteration: 4 rounds of t steps, for k <= 8
  logk-eigs  the same with l = ceil(log2 k) eigenvectors ("log(k) Eigenvectors")
  learned    the learned polynomial filter with the shipped parameters and the
             plain method as its fallback (SBM workloads only: the filter was
             trained on SBM graphs); the row names how many trials fell back

Usage: python -m paper_2310_10939_amd.report --workload sbm1m --trials 10
       [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# name: (kind, n, k, mean in-cluster degree, mean cross degree, t, permuted) for
# SBM graphs; the kNN entry is 70,000 points of 10 Gaussians in 784 dims
EIG_CYCLES = 4

WORKLOADS = {
    "sbm1m": ("sbm", 1_000_000, 10, 36, 4, 30, True),
    "sbm1m-k8": ("sbm", 1_000_000, 8, 36, 4, 30, True),
    "sbm100k": ("sbm", 100_000, 10, 36, 4, 25, True),
    "sbm100k-k50": ("sbm", 100_000, 50, 36, 4, 25, True),
    "knn70k": ("knn", 70_000, 10, None, None, 40, False),
}


def make(name, dev):
    import torch
    import synth
    kind, n, k, din, dout, t, permute = WORKLOADS[name]
    if kind == "knn":
        from paper_2310_10939_amd import fsc
        X, lab = synth.gaussian_mixture(n // k, k, 784, seed=0)
        ip, ix, w = fsc.knn_graph(torch.from_numpy(X).to(dev), 10)
        return ip, ix, w.contiguous(), torch.from_numpy(lab.astype(np.int32)).to(dev), k, t
    g = synth.sbm_by_degree(n, k, din, dout, seed=0, permute=permute)
    ip = torch.from_numpy(g.indptr).to(dev)
    ix = torch.from_numpy(g.indices).to(dev)
    return ip, ix, None, torch.from_numpy(g.labels.astype(np.int32)).to(dev), k, t


def run(name, trials, methods=None):
    import torch
    from paper_2310_10939_amd import fsc
    dev = torch.device("cuda", 0)
    ip, ix, w, truth, k, t = make(name, dev)
    l = max(1, math.ceil(math.log2(k)))
    params = None
    runs = {
        "fsc": lambda s: fsc.cluster(ip, ix, w, k, l, t, s),
        "fsc-l+1": lambda s: fsc.cluster(ip, ix, w, k, l + 1, t, s),
    }
    if k <= 8:
        runs["pm-k"] = lambda s: fsc.cluster_pmk(ip, ix, w, k, t, s)[0]
        runs["k-eigs"] = lambda s: fsc.cluster_eigs(ip, ix, w, k, k, EIG_CYCLES, t, s)[0]
    runs["logk-eigs"] = lambda s: fsc.cluster_eigs(ip, ix, w, k, min(l, 8), EIG_CYCLES, t, s)[0]
    if WORKLOADS[name][0] == "sbm":
        from paper_2310_10939_amd.train_filter import PARAMS_FILE
        params = torch.from_numpy(np.load(PARAMS_FILE)).to(dev)
        fallbacks = []

        def learned(s):
            lab, _, used = fsc.cluster_filtered(ip, ix, w, k, l, s, params=params, fallback_t=t)
            fallbacks.append(bool(used))
            return lab
        runs["learned"] = learned
    rows = {}
    for m, fn in runs.items():
        if methods and m not in methods:
            continue
        fn(1000)
        torch.cuda.synchronize()
        ari, nmi, ms = [], [], []
        for s in range(trials):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            lab = fn(s)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
            ari.append(float(fsc.ari(lab, truth, k, k)))
            nmi.append(float(fsc.nmi(lab, truth, k, k)))
        rows[m] = {"ari": ari, "nmi": nmi, "ms": ms}
        if m == "learned":
            rows[m]["fallbacks"] = int(sum(fallbacks[-trials:]))
    return {"workload": name, "n": int(ip.numel() - 1), "nnz": int(ix.numel()), "k": k, "l": l, "t": t,
            "trials": trials, "methods": rows}


def summary(res):
    """Markdown table: mean +- std of ARI, NMI and milliseconds per method."""
    def ms(v):
        a = np.asarray(v, dtype=np.float64)
        return a.mean(), a.std()
    lines = ["| workload | method | ARI | NMI | time (ms) |", "|---|---|---|---|---|"]
    for m, r in res["methods"].items():
        (am, asd), (nm, nsd), (tm, tsd) = ms(r["ari"]), ms(r["nmi"]), ms(r["ms"])
        name = m if "fallbacks" not in r else f"{m} (fell back {r['fallbacks']} of {len(r['ari'])})"
        lines.append(f"| {res['workload']} | {name} | {am:.4f} ± {asd:.4f} | {nm:.4f} ± {nsd:.4f} | "
                     f"{tm:.2f} ± {tsd:.2f} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", action="append", choices=sorted(WORKLOADS))
    ap.add_argument("--trials", type=int, default=10)
    ap.add_argument("--method", action="append")
    ap.add_argument("--json")
    a = ap.parse_args(argv)
    out = []
    for name in a.workload or ["sbm1m"]:
        res = run(name, a.trials, a.method)
        print(summary(res), flush=True)
        out.append(res)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
