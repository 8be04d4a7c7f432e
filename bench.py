#!/usr/bin/env python3
"""Benchmark of the exact t-SNE hot path on one MI355X.

Workload: 65,536 points in D=50 from the 32-component anisotropic Gaussian
mixture (synthetic stand-in for the paper's GMM data sets), perplexity 50,
2-D map from N(0, 1e-4 I), 1,000 iterations with exaggeration 12 and momentum
0.5 before iteration 250, then 1 and 0.8, learning rate 200.

One timed step is one complete pass of the hot path over that input, with X
already resident in HBM: input affinities (centring, FP64-MFMA distances,
per-row bisection, symmetric packed P), the 1,000 exact-gradient iterations
(force pass + FP64 reduction + update), and the final KL cost. ``value`` is
end-to-end iterations per second over the timed steps.

Prints one JSON line (stdout). Diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(x_full, perplexity, n_target, iters_target, n_sample=8192, iters_sample=100):
    """Time the FP64 oracle on a bounded sample of the same workload.

    The oracle runs the affinities and ``iters_sample`` iterations on the first
    ``n_sample`` points; both stages are O(n^2) per pass, so the time is scaled
    by (n_target / n_sample)^2 and to ``iters_target`` iterations.
    """
    import numpy as np

    import oracle
    from paper_1812_09869_amd import synth

    xs = np.ascontiguousarray(x_full[:n_sample])
    y0 = synth.embedding_init(n_sample, seed=synth.SEEDS["init_aniso"]).astype(np.float64)
    t0 = time.perf_counter()
    st = oracle.calibrate(xs, perplexity)
    P = oracle.joint_p(xs, st)
    t_aff = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.run(P, y0, iters_sample)
    t_it = (time.perf_counter() - t0) / iters_sample
    scale = (n_target / n_sample) ** 2
    total = (t_aff + iters_target * t_it) * scale
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": iters_target / total,
        "unit": "iters/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"FP64 oracle on the first {n_sample} points of the same mixture: affinities "
                   f"+ {iters_sample} iterations ({t_aff:.2f} s + {iters_sample * t_it:.2f} s), "
                   f"scaled by (N/{n_sample})^2 to N={n_target} and to {iters_target} "
                   f"iterations"),
        "iter_s_at_sample": t_it,
        "affinity_s_at_sample": t_aff,
    }


def measured_traffic(n):
    """HBM bytes per force launch from the committed counter summary, if it was
    taken on the current force-kernel source at this size (else None)."""
    import hashlib

    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "force_n65536_traffic.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(root, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if n != 65536 or hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--iters", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1812_09869_amd import _lib, synth
    from paper_1812_09869_amd.tsne import Schedule

    _lib.load()
    n, d, perp = args.n, 50, 50.0
    x_np, _ = synth.gmm_aniso(n)
    y0_np = synth.embedding_init(n, seed=synth.SEEDS["init_aniso"])
    dev = torch.device("cuda:0")
    x = torch.from_numpy(x_np).to(dev)
    y0 = torch.from_numpy(y0_np).to(dev)
    ws = _lib.new_workspace(n, d)
    y = torch.empty_like(y0)
    u = torch.empty_like(y0)
    g = torch.empty_like(y0)
    cost = torch.zeros(2, dtype=torch.float64, device=dev)
    sched = Schedule()
    log(f"[bench] n={n} d={d} perplexity={perp} iters={args.iters} workspace "
        f"{ws.numel() / 2**30:.2f} GiB")

    def one_step(events=None):
        y.copy_(y0)
        u.zero_()
        g.fill_(1.0)
        if events is not None:
            events["aff"].append((torch.cuda.Event(enable_timing=True),
                                  torch.cuda.Event(enable_timing=True)))
            events["aff"][-1][0].record()
        _lib.affinities(x, perp, ws)
        if events is not None:
            events["aff"][-1][1].record()
        for t in range(args.iters):
            alpha, mu, eta = sched(t)
            if events is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
            _lib.forces(ws, n, y)
            if events is not None:
                e1.record()
                events["force"].append((e0, e1))
            _lib.update(ws, n, y, u, g, alpha, mu, eta, sched.min_gain, True)
        _lib.cost(ws, n, y, cost)

    for w in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    status = _lib.sync_status(ws)
    if status != 0:
        log(f"[bench] device status {status} after warmup")
        sys.exit(1)

    events = {"aff": [], "force": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        one_step(events)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    status = _lib.sync_status(ws)
    kl, cnorm = (float(v) for v in cost.cpu())
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s; final KL {kl:.6f} C_norm "
        f"{cnorm:.6f}; status {status}")
    if status != 0:
        sys.exit(1)

    force_ms = float(np.mean([a.elapsed_time(b) for a, b in events["force"]]))
    aff_ms = float(np.mean([a.elapsed_time(b) for a, b in events["aff"]]))
    ms_per_step = elapsed * 1e3 / args.steps
    iters_total = args.iters * args.steps
    value = iters_total / elapsed
    p_bytes = 4.0 * n * (n - 1) / 2.0  # FP32 P read once per unordered pair
    achieved = p_bytes / (force_ms * 1e-3) / 1e9
    steady_ms = (ms_per_step - aff_ms) / args.iters

    out = {
        "metric": "exact t-SNE iters/s at N=65k (FP32 vs BF16 dist) at oracle KL tol; "
                  "surrogate pts/s",
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"anisotropic 32-component GMM, N={n}, D={d}, perplexity {perp:g}, "
                         f"{args.iters} iterations (exaggeration 12 / momentum 0.5 before 250, "
                         f"then 1 / 0.8; learning rate 200); affinities + iterations + cost "
                         f"per step"),
            "n": n,
            "d": d,
            "perplexity": perp,
            "iterations_per_step": args.iters,
            "dist_mode": "fp64",
        },
        "roofline": {
            "kernel": "k_force",
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic(n),
            "algorithmic_bytes_per_launch": p_bytes,
            "avg_launch_ms": force_ms,
        },
        "steady_iters_per_s": 1e3 / steady_ms,
        "affinity_ms": aff_ms,
        "force_ms": force_ms,
        "pair_interactions_per_s": n * (n - 1) / 2.0 * 1e3 / steady_ms,
        "final_kl": kl,
        "final_cnorm": cnorm,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(x_np, perp, n, args.iters)
        log(f"[bench] cpu baseline {out['cpu_baseline']['value']:.4g} iters/s "
            f"({out['cpu_baseline']['cores']} threads)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
