"""Trains the MLP of the learned polynomial-filter form on the GPU.

Training data: degree-corrected SBM graphs (n uniform in [1e5, 2e6], k in
[2, 50], mean degree log-uniform in [8, 64], power-law degree propensities
with exponent uniform in [2.2, 8], in-cluster fraction in [0.85, 0.95], unit
weights), generated on the device.  For each graph the library's
kernels run the plain method (t = ceil(3 ln n) PowerMethod steps,
l = ceil(log2 k) + 1, k-means) for its labels, then the Chebyshev basis, the
within-cluster and total scatter matrices of the filtered embedding under
those labels, and the features (fsc_filter_stats); only these statistics are
kept.  The MLP is then trained by full-batch Adam on the normalised k-means
cost with the library's forward/backward/Adam kernels (fsc_mlp_train).
Held-out graphs measure the gain: ARI of the learned filter against the plain
method and the planted clusters, next to the same head with no network (the
fixed interval the training starts from), the fixed filter gamma^8 (8 plain
steps, the same budget of sparse products) and the per-graph optimum of the
loss, and wall times.

Usage: python -m paper_2310_10939_amd.train_filter --graphs 2000 --heldout 100
       --out <params.npy> --report <report.json>
The shipped parameters (filter_mlp_params.npy) come from this command with
its defaults; filter_mlp_report.json is their report.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PARAMS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "filter_mlp_params.npy")
LAYERS = [(9, 128), (128, 128), (128, 128), (128, 2)]
# Chebyshev coefficients c_1..c_8 of gamma^8 on [0, 1]: C(16, 8 - j) / 2^15
GAMMA8 = [11440 / 32768, 8008 / 32768, 4368 / 32768, 1820 / 32768, 560 / 32768, 120 / 32768, 16 / 32768,
          1 / 32768]
# the interval [a, b] the training starts from (about 0.5 +- 1/sqrt(20), the
# bulk of M for a random graph of mean degree 20)
INIT_A, INIT_B = 0.2, 0.72


def init_params(seed):
    """He-uniform weights, zero biases; the output layer's weights scaled by
    0.01 and its biases set so that every graph starts near the filter of
    [INIT_A, INIT_B] (alpha = log(b - a), beta = log(1 - b))."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (i, o) in enumerate(LAYERS):
        lim = np.sqrt(6.0 / i)
        w = rng.uniform(-lim, lim, size=(o, i))
        b = np.zeros(o)
        if li == len(LAYERS) - 1:
            w *= 0.01
            b = np.array([np.log(INIT_B - INIT_A), np.log(1.0 - INIT_B)])
        parts += [w.ravel(), b]
    return np.concatenate(parts).astype(np.float32)


def fixed_head_params(seed=0):
    """Parameters whose output layer ignores the features: every graph gets
    the filter of [INIT_A, INIT_B] (the head with no network)."""
    p = init_params(seed)
    w_out = LAYERS[-1][0] * LAYERS[-1][1]
    p[-(w_out + LAYERS[-1][1]):-LAYERS[-1][1]] = 0.0
    return p


def load_params(path=PARAMS_FILE, device="cuda"):
    import torch
    p = np.load(path, allow_pickle=False).astype(np.float32)
    return torch.from_numpy(p).to(device)


def collect(specs, device, log=print):
    """Training statistics of each graph (all on the device)."""
    import torch
    import synth
    from . import fsc
    F, W, T = [], [], []
    t0 = time.perf_counter()
    for i, s in enumerate(specs):
        ip, ix, _ = synth.learned_graph(s, device=device)
        f, w, tt, _ = fsc.filter_stats(ip, ix, None, s["k"], s["l"], s["t"], s["seed"])
        F.append(f)
        W.append(w)
        T.append(tt)
        del ip, ix
        if (i + 1) % 50 == 0 or i + 1 == len(specs):
            torch.cuda.synchronize()
            log(f"stats {i + 1}/{len(specs)} graphs, {time.perf_counter() - t0:.1f} s")
    return torch.stack(F), torch.stack(W), torch.stack(T)


def train(F, W, T, steps, lr, seed, log=print):
    import torch
    from . import fsc
    p = torch.from_numpy(init_params(seed)).to(F.device)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    traces = []
    done = 0
    for phase_steps, phase_lr in ((steps * 2 // 3, lr), (steps - steps * 2 // 3, lr * 0.3)):
        tr = fsc.mlp_train(p, m, v, F, W, T, phase_steps, phase_lr, first_step=done + 1)
        traces.append(tr)
        done += phase_steps
        torch.cuda.synchronize()
        log(f"train {done}/{steps} steps, loss {float(tr[0]):.4f} -> {float(tr[-1]):.4f}")
    return p, torch.cat(traces)


def ratio_optimum(W, T):
    """Per-graph coefficients c_1..c_8 minimising c^T W c / c^T T c (the best
    any degree-8 filter can do on that graph's loss): the generalised
    eigenvector of the smallest eigenvalue, scaled so p(1) = sum c = 1, and
    that eigenvalue.  Host FP64."""
    Li = np.linalg.inv(np.linalg.cholesky(T))
    lam, V = np.linalg.eigh(Li @ W @ Li.T)
    x = Li.T @ V[:, 0]
    return x[1:] / x.sum(), float(lam[0])


def heldout_loss(p, F, W, T):
    from . import fsc
    loss, _ = fsc.mlp_loss_grad(p, F, W, T)
    return float(loss[0])


def evaluate(p, specs, device, stats=None, log=print):
    """ARI against the plain method (and the planted clusters) of the learned
    filter, of the same head with no network, of the fixed gamma^8 filter
    and of the per-graph optimum of the loss, with wall times."""
    import torch
    import synth
    from . import fsc
    g8 = torch.tensor(GAMMA8, dtype=torch.float32, device=device)
    ph = torch.from_numpy(fixed_head_params()).to(device)
    rows = []
    for i, s in enumerate(specs):
        ip, ix, lab = synth.learned_graph(s, device=device)
        k, l, t, seed = s["k"], s["l"], s["t"], s["seed"]
        fsc.cluster(ip, ix, None, k, l, t, seed)   # warm the workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = fsc.cluster(ip, ix, None, k, l, t, seed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # the plain method with another seed: how far two runs of it agree
        reseeded = fsc.cluster(ip, ix, None, k, l, t, seed + 7919)
        fsc.cluster_filtered(ip, ix, None, k, l, seed, params=p)   # warm the filter's workspace
        torch.cuda.synchronize()
        t1f = time.perf_counter()
        learned, coef, used, diag = fsc.cluster_filtered(ip, ix, None, k, l, seed, params=p, diagnostics=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fixed, _, _, diag8 = fsc.cluster_filtered(ip, ix, None, k, l, seed, coeffs=g8, diagnostics=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        guarded, _, used_g = fsc.cluster_filtered(ip, ix, None, k, l, seed, params=p, fallback_t=t)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        head, _, used_h, diagh = fsc.cluster_filtered(ip, ix, None, k, l, seed, params=ph, diagnostics=True)
        # normalised k-means cost of the plain embedding, for calibration
        _, E, Cn = fsc.cluster(ip, ix, None, k, l, t, seed, return_embedding=True, return_centres=True)
        Eh = E.double().cpu().numpy()
        lab_p = plain.cpu().numpy()
        keep = np.diff(ip.cpu().numpy()) > 0
        Ek, lk = Eh[keep], lab_p[keep]
        cost_plain = float(((Ek - Cn.double().cpu().numpy()[lk]) ** 2).sum() / ((Ek - Ek.mean(0)) ** 2).sum())
        dg, d8 = diag.cpu().numpy(), diag8.cpu().numpy()
        extra = {}
        if stats is not None:
            Fi, Wi, Ti = (x[i].double().cpu().numpy() for x in stats)
            c_opt, loss_opt = ratio_optimum(Wi, Ti)
            best, _, _ = fsc.cluster_filtered(ip, ix, None, k, l, seed,
                                              coeffs=torch.tensor(c_opt, dtype=torch.float32, device=device))
            c_l = coef.double().cpu().numpy()
            full = np.concatenate([[1.0 - c_l.sum()], c_l])
            extra = dict(loss_optimum=loss_opt, loss_learned=float(full @ Wi @ full / (full @ Ti @ full)),
                         ari_opt_vs_plain=float(fsc.ari(best, plain, k, k)))
        if stats is not None:
            ch = fsc.cluster_filtered(ip, ix, None, k, l, seed, params=ph)[1].double().cpu().numpy()
            full = np.concatenate([[1.0 - ch.sum()], ch])
            extra["loss_head"] = float(full @ Wi @ full / (full @ Ti @ full))
        rows.append(dict(n=s["n"], k=k, l=l, t=t, deg=s["deg"], alpha=s["alpha"], in_frac=s["in_frac"], **extra,
                         ari_learned_vs_plain=float(fsc.ari(learned, plain, k, k)),
                         ari_fixed8_vs_plain=float(fsc.ari(fixed, plain, k, k)),
                         ari_plain_vs_planted=float(fsc.ari(plain, lab, k, k)),
                         ari_plain_reseeded_vs_plain=float(fsc.ari(reseeded, plain, k, k)),
                         ari_learned_vs_planted=float(fsc.ari(learned, lab, k, k)),
                         ari_fixed8_vs_planted=float(fsc.ari(fixed, lab, k, k)),
                         ari_guarded_vs_plain=float(fsc.ari(guarded, plain, k, k)),
                         ari_guarded_vs_planted=float(fsc.ari(guarded, lab, k, k)),
                         ari_head_vs_plain=float(fsc.ari(head, plain, k, k)),
                         ari_head_vs_planted=float(fsc.ari(head, lab, k, k)),
                         fallback=used, fallback_head=used_h, ms_plain=(t1 - t0) * 1e3, ms_learned=(t2 - t1f) * 1e3,
                         ms_fixed8=(t3 - t2) * 1e3, ms_guarded=(t4 - t3) * 1e3,
                         rho_learned=float(dg[0]), rho_8=float(dg[1]), cost_learned=float(dg[2]),
                         cost_fixed8=float(d8[2]), cost_head=float(diagh.cpu().numpy()[2]), cost_plain=cost_plain))
        if (i + 1) % 10 == 0 or i + 1 == len(specs):
            log(f"eval {i + 1}/{len(specs)}")
    return rows


def summarize(rows):
    keys = [k for k in rows[0] if k.split("_")[0] in ("ari", "ms", "loss", "rho", "cost")]
    out = {k: float(np.mean([r[k] for r in rows])) for k in keys}
    out["fallback_rate"] = float(np.mean([r["fallback"] for r in rows]))
    out["fallback_rate_head"] = float(np.mean([r["fallback_head"] for r in rows]))
    out["graphs"] = len(rows)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", type=int, default=2000)
    ap.add_argument("--heldout", type=int, default=100)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=PARAMS_FILE)
    ap.add_argument("--report", default=None)
    ap.add_argument("--eval-only", action="store_true", help="evaluate the saved parameters (--out)")
    ap.add_argument("--stats-out", default=None, help="save the collected statistics (.npz) and stop")
    args = ap.parse_args(argv)
    import torch
    import synth
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    def log(msg):
        print(msg, flush=True)

    test_specs = synth.learned_params(args.heldout, 100000)
    if args.eval_only:
        stats_t = collect(test_specs, dev, log)
        p = load_params(args.out, dev)
        rows = evaluate(p, test_specs, dev, stats_t, log)
        report = {"heldout_graphs": args.heldout, "heldout_loss": heldout_loss(p, *stats_t),
                  "heldout_loss_fixed_head": heldout_loss(torch.from_numpy(fixed_head_params()).to(dev), *stats_t),
                  "summary": summarize(rows), "rows": rows}
        if args.report:
            with open(args.report, "w") as fh:
                json.dump(report, fh, indent=1)
        log(json.dumps({k: v for k, v in report.items() if k != "rows"}))
        return 0
    train_specs = synth.learned_params(args.graphs, 0)
    F, W, T = collect(train_specs, dev, log)
    stats_t = collect(test_specs, dev, log)
    if args.stats_out:
        np.savez(args.stats_out, F=F.cpu().numpy(), W=W.cpu().numpy(), T=T.cpu().numpy(),
                 Ft=stats_t[0].cpu().numpy(), Wt=stats_t[1].cpu().numpy(), Tt=stats_t[2].cpu().numpy(),
                 specs=json.dumps(train_specs), test_specs=json.dumps(test_specs))
        return 0
    p, trace = train(F, W, T, args.steps, args.lr, args.seed, log)
    np.save(args.out, p.cpu().numpy())
    rows = evaluate(p, test_specs, dev, stats_t, log)
    report = {"train_graphs": args.graphs, "heldout_graphs": args.heldout, "steps": args.steps,
              "train_loss_first": float(trace[0]), "train_loss_last": float(trace[-1]),
              "heldout_loss": heldout_loss(p, *stats_t),
              "heldout_loss_identity_init": heldout_loss(torch.from_numpy(init_params(args.seed)).to(dev),
                                                         *stats_t),
              "heldout_loss_fixed_head": heldout_loss(torch.from_numpy(fixed_head_params()).to(dev), *stats_t),
              "summary": summarize(rows), "rows": rows}
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    log(json.dumps({k: v for k, v in report.items() if k != "rows"}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
