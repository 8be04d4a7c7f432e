#!/usr/bin/env python3
"""Benchmark of the exact t-SNE hot path on one MI355X.

Workload: 65,536 points in D=50 from the 32-component anisotropic Gaussian
mixture (synthetic stand-in for the paper's GMM data sets), perplexity 50,
2-D map from N(0, 1e-4 I), 1,000 iterations with exaggeration 12 and momentum
0.5 before iteration 250, then 1 and 0.8, learning rate 200.

One timed step is one complete pass of the hot path over that input, with X
already resident in HBM: input affinities (centring, the locality order,
MFMA distances in the chosen mode -- by default the compensated BF16 mode,
which holds P to the FP64 oracle within the per-step gates -- per-row search
for beta, symmetric packed P), the 1,000 exact-gradient iterations (force
pass + FP64 reduction + update), and the final KL cost. ``value`` is
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
FORCE_SAMPLE = 10  # every 10th force pass of the timed steps is timed with events


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n=None):
    """Thread count of the OpenMP runtime the oracle runs on (sets it if n is given)."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def cpu_baseline(x_full, perplexity, n_target, iters_target, n_sample=8192, iters_sample=100,
                 n_one=4096, iters_one=20):
    """Time the FP64 oracle on bounded samples of the same workload.

    On all host threads: the affinities and ``iters_sample`` iterations on the
    first ``n_sample`` points. On one thread: the affinities and ``iters_one``
    iterations on the first ``n_one`` points. Both stages are O(n^2) per pass,
    so each time is scaled by (n_target / n)^2 and to ``iters_target``
    iterations. Also the whole 2,000-point, 500-iteration workload on all
    threads, unscaled.
    """
    import numpy as np

    import oracle
    from paper_1812_09869_amd import synth

    def sample(n, iters):
        xs = np.ascontiguousarray(x_full[:n])
        y0 = synth.embedding_init(n, seed=synth.SEEDS["init_aniso"]).astype(np.float64)
        t0 = time.perf_counter()
        st = oracle.calibrate(xs, perplexity)
        P = oracle.joint_p(xs, st)
        t_aff = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.run(P, y0, iters)
        t_it = (time.perf_counter() - t0) / iters
        scale = (n_target / n) ** 2
        return t_aff, t_it, iters_target / ((t_aff + iters_target * t_it) * scale)

    oracle._load()
    threads = _omp_threads()
    t_aff, t_it, rate = sample(n_sample, iters_sample)
    _omp_threads(1)
    t_aff1, t_it1, rate1 = sample(n_one, iters_one)
    _omp_threads(threads)
    xs, _ = synth.plain_small()
    t0 = time.perf_counter()
    P = oracle.joint_p(xs, oracle.calibrate(xs, 30.0))
    oracle.run(P, synth.embedding_init(xs.shape[0], synth.SEEDS["init_small"]), 500)
    t_small = time.perf_counter() - t0
    return {
        "value": rate,
        "unit": "iters/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 oracle on the first {n_sample} points of the same mixture: affinities "
                   f"+ {iters_sample} iterations ({t_aff:.2f} s + {iters_sample * t_it:.2f} s), "
                   f"scaled by (N/{n_sample})^2 to N={n_target} and to {iters_target} "
                   f"iterations"),
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
        "iter_s_at_sample": t_it,
        "affinity_s_at_sample": t_aff,
        "one_thread": {
            "value": rate1,
            "unit": "iters/s",
            "sample": (f"first {n_one} points: affinities + {iters_one} iterations "
                       f"({t_aff1:.2f} s + {iters_one * t_it1:.2f} s), scaled by "
                       f"(N/{n_one})^2 and to {iters_target} iterations"),
        },
        "plain_small_full_run_s": t_small,
        "plain_small_full_run": ("the 2,000-point, 10-D, perplexity-30 workload in full "
                                 "(affinities + 500 iterations), all threads"),
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


PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X FP32 vector, published (counts packed dual-FP32 issue)
PEAK_FP32_VALU_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz
FLOP_REPULSION = 17  # per unordered pair: dy (2), 1 + |dy|^2 (4), 1/q (1), w^2 (1), Z (1), row and column w^2 dy (8)
FLOP_ATTRACTION = 9  # per pair in a tile with nonzero P: p w (1), row and column p w dy (8)


def tile_pairs(ws, n):
    """(all unordered pairs, pairs in tiles whose stored P is not all zero,
    fraction of all-zero tiles) of a problem, from its exported tile flags."""
    from paper_1812_09869_amd import _lib

    T = 256
    nb = (n + T - 1) // T
    _, flags = _lib.export_order(ws, n)
    flags = flags.cpu().numpy()
    sizes = [min(T, n - b * T) for b in range(nb)]
    pairs_nz = 0.0
    tile = 0
    for i in range(nb):
        for j in range(i, nb):
            if flags[tile]:
                pairs_nz += sizes[i] * (sizes[i] - 1) / 2.0 if i == j else sizes[i] * sizes[j]
            tile += 1
    return n * (n - 1) / 2.0, pairs_nz, float((flags == 0).mean())


def force_roofline(ws, n, force_ms):
    """Roofline record of the force pass.

    Every unordered pair pays the repulsive terms on the vector ALUs; pairs in
    tiles whose stored P is all zero skip the P read and the attractive terms.
    The pass is bound by FP32 vector issue (the P stream of the nonzero tiles
    overlaps it), so the record is an ALU one: algorithmic FP32 flops per
    launch over the launch time, against the published FP32 vector peak.
    """
    from paper_1812_09869_amd import _lib

    pairs_total, pairs_nz, zero_frac = tile_pairs(ws, n)
    flops = FLOP_REPULSION * pairs_total + FLOP_ATTRACTION * pairs_nz
    achieved = flops / (force_ms * 1e-3) / 1e12
    p_bytes = 4.0 * pairs_nz
    traffic = measured_traffic(n)
    return {
        "kernel": "force pass: k_force_full (tiles with P) concurrent with k_force_zero (all-zero tiles)",
        "bound": "alu",
        "achieved": achieved,
        "peak": PEAK_FP32_VALU_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_VALU_TFLOPS,
        "traffic": traffic,
        "algorithmic_flops_per_launch": flops,
        "flops_per_pair": {"repulsion": FLOP_REPULSION, "attraction": FLOP_ATTRACTION},
        "pairs_per_launch": pairs_total,
        "pairs_in_nonzero_tiles": pairs_nz,
        "zero_tile_fraction": zero_frac,
        "frac_of_nonpacked_fp32_peak": achieved / PEAK_FP32_VALU_NONPACKED_TFLOPS,
        "p_bytes_per_launch": p_bytes,
        "p_stream_gbs": p_bytes / (force_ms * 1e-3) / 1e9,
        "p_stream_frac_of_hbm_peak": p_bytes / (force_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "avg_launch_ms": force_ms,
    }


MODES = ["fp64", "fp32", "fp16x3", "bf16x3", "fp16", "bf16"]


def precision_leg(x, lab, n, d, perp, iters, steady_ms):
    """Affinity time and per-step error of every distance mode at the benchmark size.

    Errors are taken against the FP64 mode (which the parity tests hold to the
    FP64 oracle at ~1e-7 at this size): P on 32 sampled rows (relative
    Frobenius, and the largest entry error over the largest entry), the
    gradient (alpha = 1) and the KL at a fixed clustered map. A mode meets the
    per-step gates if both P errors are <= 1e-5 and the gradient <= 1e-4.
    """
    import numpy as np
    import torch

    from paper_1812_09869_amd import _lib, synth

    ws = _lib.new_workspace(n, d, max(MODES, key=lambda m: _lib.workspace_bytes(n, d, m)))
    rng = np.random.Generator(np.random.PCG64(12))
    rows = np.sort(rng.choice(n, 32, replace=False))
    y = torch.from_numpy(synth.clustered_state(lab, seed=31, spread=30.0)).cuda()
    gbuf = torch.empty_like(y)
    cost = torch.zeros(2, dtype=torch.float64, device="cuda")
    res, ref = {}, None
    for mode in MODES:
        times = []
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            _lib.affinities(x, perp, ws, dist_mode=mode)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        if _lib.sync_status(ws) != 0:
            res[mode] = {"status": _lib.sync_status(ws)}
            continue
        prow = torch.cat([_lib.export_p_rows(ws, n, int(r), 1) for r in rows]).double().cpu()
        _lib.gradient(ws, n, y, 1.0, gbuf)
        g = gbuf.double().cpu()
        _lib.cost(ws, n, y, cost)
        kl = float(cost[0].cpu())
        if ref is None:
            ref = (prow, g, kl)
        pe = float(torch.linalg.norm(prow - ref[0]) / torch.linalg.norm(ref[0]))
        pm = float((prow - ref[0]).abs().max() / ref[0].max())
        ge = float(torch.linalg.norm(g - ref[1]) / torch.linalg.norm(ref[1]))
        ke = abs(kl - ref[2]) / ref[2]
        aff = min(times)
        res[mode] = {
            "affinity_ms": aff,
            "p_rel_vs_fp64": pe,
            "p_maxrel_vs_fp64": pm,
            "grad_rel_vs_fp64": ge,
            "kl_rel_vs_fp64": ke,
            "end_to_end_iters_per_s": iters / ((aff + iters * steady_ms) * 1e-3),
            "meets_step_gates": bool(pe <= 1e-5 and pm <= 1e-5 and ge <= 1e-4),
        }
        log(f"[bench] mode {mode:7s} affinities {aff:7.2f} ms  P {pe:.2e} (max {pm:.2e})  "
            f"grad {ge:.2e}  KL {ke:.2e}")
    del ws
    return res


def monitor_leg(ws, n, y0, iters, sched, every=50):
    """One more run of the benchmark trajectory, outside the timed steps, with
    the run log every ``every`` iterations: KL and C_norm (Eqs. 5 and 9, from
    tsne_cost), Z and the gradient norm of that iteration (from tsne_step),
    and the diagonal of the map's bounding box (the embedding size monitor)."""
    import torch

    from paper_1812_09869_amd import _lib

    y = y0.clone()
    u = torch.zeros_like(y)
    g = torch.ones_like(y)
    grad = torch.empty_like(y)
    z = torch.zeros(1, dtype=torch.float64, device=y.device)
    cost = torch.zeros(2, dtype=torch.float64, device=y.device)
    log_rows = []
    for t in range(iters):
        alpha, mu, eta = sched(t)
        want = (t + 1) % every == 0
        _lib.step(ws, n, y, u, g, alpha, mu, eta, sched.min_gain, True,
                  grad if want else None, z if want else None)
        if want:
            _lib.cost(ws, n, y, cost)
            ext = (y.max(dim=0).values - y.min(dim=0).values).double()
            log_rows.append({"t": t + 1, "kl": float(cost[0]), "cnorm": float(cost[1]),
                             "z": float(z[0]), "grad_norm": float(torch.linalg.norm(grad.double())),
                             "box_diagonal": float(torch.linalg.norm(ext))})
    return log_rows


def knn_overlap(x, y, rows, k=10):
    """Mean over the query rows of |kNN_k in x  intersect  kNN_k in y| / k
    (Euclidean, self excluded): an evaluation metric of a map, in torch on the
    device (FP64 distances of the query rows to all points)."""
    import torch

    q = torch.as_tensor(rows, device=x.device, dtype=torch.long)

    def nbrs(a):
        a = a.double()
        d = torch.cdist(a[q], a)
        d[torch.arange(q.numel(), device=a.device), q] = float("inf")
        return torch.topk(d, k, dim=1, largest=False).indices

    nx, ny = nbrs(x), nbrs(y)
    common = (nx.unsqueeze(2) == ny.unsqueeze(1)).any(dim=2).sum(dim=1)
    return float(common.double().mean() / k)


def surrogate_leg(x_train, y_train, perp, n_new=1 << 20, n_eval=65536, epochs=100, batch=1024):
    """Train the surrogate on the exact embedding, time inference on n_new new
    points of the same mixture, and judge it on the first n_eval of them: KL and
    10-NN overlap of (1) its map, (2) that map after 100 exact refinement
    iterations (exaggeration 1, momentum 0.8, learning rate 200), (3) exact
    t-SNE from a random start (1,000 iterations, standard schedule)."""
    import numpy as np
    import torch

    from paper_1812_09869_amd import synth
    from paper_1812_09869_amd.surrogate import Surrogate
    from paper_1812_09869_amd.tsne import ExactTSNE, Schedule

    net = Surrogate(x_train.shape[1], 256, seed=synth.SEEDS["surrogate_init"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.fit(x_train, y_train, epochs=epochs, batch=batch)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"[surrogate] trained {epochs} epochs in {t_train:.2f} s, loss {losses[0]:.4f} -> "
        f"{losses[-1]:.4f}")
    xn_np, _ = synth.gmm_aniso(n_new, sample_seed=synth.SEEDS["surrogate_new"])
    xn = torch.from_numpy(xn_np).cuda()
    out = torch.empty((n_new, 2), device="cuda")
    net.predict(xn, out)  # warm-up
    times = []
    for _ in range(5):  # five samples of 20 back-to-back passes over the 1M points
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            net.predict(xn, out)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 20)
    inf_ms = float(np.median(times))
    log(f"[surrogate] inference on {n_new} points: {inf_ms:.3f} ms "
        f"({n_new / inf_ms * 1e3:.3e} points/s)")
    xe = xn[:n_eval].contiguous()
    ye = out[:n_eval].clone()
    model = ExactTSNE(xe, perp)
    kl_net = float(model.cost(ye).cpu()[0])
    refine = Schedule(switch=0, exaggeration=1.0, mom_late=0.8)
    st = model.init_state(ye)
    model.run(st, 100, sched=refine)
    kl_ref = float(model.cost(st[0]).cpu()[0])
    st0 = model.init_state(torch.from_numpy(synth.embedding_init(n_eval, seed=5002)).cuda())
    kl_rand, t = {}, 0
    for t_end in list(range(50, 1001, 50)):
        model.run(st0, t_end - t, start=t)
        t = t_end
        kl_rand[t_end] = float(model.cost(st0[0]).cpu()[0])
    rows = np.arange(0, n_eval, n_eval // 1024)
    ov = {k: knn_overlap(xe, v, rows, 10)
          for k, v in (("surrogate", ye), ("refined_100", st[0]), ("exact_1000", st0[0]))}
    reach = next((t for t, v in sorted(kl_rand.items()) if v <= kl_ref), None)
    res = {
        "points_per_s": n_new / inf_ms * 1e3,
        "inference_ms_1m_points": inf_ms,
        "train_s": t_train,
        "train_loss_first_last": [losses[0], losses[-1]],
        "kl_surrogate": kl_net,
        "kl_refined_100": kl_ref,
        "kl_random_start_100": kl_rand[100],
        "kl_exact_1000": kl_rand[1000],
        "knn10_overlap": ov,
        "gain_at_100_iterations": kl_rand[100] - kl_ref,
        "random_start_iterations_to_reach_refined_kl": reach,
        "fallback_refinement_needed": bool(kl_net > 1.05 * kl_rand[1000]),
        "eval": f"first {n_eval} of {n_new} new points; 10-NN overlap on {rows.size} query rows",
    }
    log(f"[surrogate] {res}")
    return res


def batched_leg(sweeps=500):
    """The 64-problem workload (N ~ U{1000..20000}, D in {10, 50}, perplexity 30):
    affinities of every problem, then `sweeps` batched iterations (one launch
    per phase for all problems), timed with HIP events."""
    import torch

    from paper_1812_09869_amd import synth
    from paper_1812_09869_amd.tsne import BatchedTSNE

    data = [synth.batch_problem(p) for p in range(64)]
    xs = [torch.from_numpy(x).cuda() for x, _, _ in data]
    y0s = [torch.from_numpy(synth.embedding_init(x.shape[0], seed=4100 + p)).cuda()
           for p, (x, _, _) in enumerate(data)]
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record()
    batch = BatchedTSNE([(x, perp) for x, (_, _, perp) in zip(xs, data)])
    e[1].record()
    batch.init_states(y0s)
    batch.run(sweeps)
    e[2].record()
    torch.cuda.synchronize()
    status = max(m.status() for m in batch.models)
    counts = [tile_pairs(m.ws, m.n) for m in batch.models]
    pairs = sum(c[0] for c in counts)
    pairs_nz = sum(c[1] for c in counts)
    flops = FLOP_REPULSION * pairs + FLOP_ATTRACTION * pairs_nz
    sweep_ms = e[1].elapsed_time(e[2]) / sweeps
    res = {
        "problems": len(batch.models),
        "points": int(sum(m.n for m in batch.models)),
        "affinities_ms": e[0].elapsed_time(e[1]),
        "sweeps": sweeps,
        "sweep_ms": sweep_ms,
        "total_s": e[0].elapsed_time(e[2]) * 1e-3,
        "problem_iterations_per_s": len(batch.models) * 1e3 / sweep_ms,
        "pair_interactions_per_s": pairs * 1e3 / sweep_ms,
        "pairs_in_nonzero_tiles_fraction": pairs_nz / pairs,
        "p_bytes_per_sweep": 4.0 * pairs_nz,
        "fp32_tflops": flops / (sweep_ms * 1e-3) / 1e12,
        "status": status,
    }
    log(f"[batched] {res}")
    return res


def ptsne_leg(epochs=10):
    """The parallel scheme on the stand-in for the paper's rounds figure: 60,000
    points in D=30, 120 threads, 2 layers (z = 1,000), perplexity 400,
    momentum 0.8, 32 iterations per epoch, start map uniform in the unit disk.
    One untimed epoch, then `epochs` epochs timed with HIP events on the
    caller's stream (each epoch: mix, 120 partial affinities, 32 batched
    iterations, 120 partial costs, pool, monitors)."""
    import math

    import torch

    from paper_1812_09869_amd import synth
    from paper_1812_09869_amd.tsne import PTSNE

    n, threads, layers, perp = 60000, 120, 2, 400.0
    x, _ = synth.digits_like(n)
    y0 = synth.disk_init(n, synth.SEEDS["pt_init"])
    orders = torch.from_numpy(synth.epoch_orders(n, epochs + 1, synth.SEEDS["pt_orders"])).cuda()
    pt = PTSNE(torch.from_numpy(x).cuda(), threads, layers, perp, momentum=0.8)
    pt.init_maps(torch.from_numpy(y0).cuda())
    pt.epoch(orders[0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for e in range(1, epochs + 1):
        mon = pt.epoch(orders[e])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / epochs
    z = [n // threads * layers] * threads  # n divisible by threads here
    pairs = sum(k * (k - 1) / 2.0 for k in z) * pt.iters
    res = {
        "workload": "digits stand-in: N=60000, D=30, 10 anisotropic components; 120 threads, "
                    "2 layers (z=1000), perplexity 400, momentum 0.8",
        "iterations_per_epoch": pt.iters,
        "epochs_per_round": math.isqrt(n),
        "epochs_timed": epochs,
        "ms_per_epoch": ms,
        "round_s": ms * math.isqrt(n) * 1e-3,
        "partial_pair_interactions_per_s": pairs * 1e3 / ms,
        "monitors_last_epoch": {"mean_partial_cnorm": float(mon[0]),
                                "mean_layer_size": float(mon[1])},
        "status": pt.status(),
    }
    log(f"[ptsne] {res}")
    return res


def pakde_leg(y, perp=100.0, grid=512, reps=5):
    """paKDE of the benchmark's final map: bandwidths by the perplexity search
    on the map (perplexity 100, the paper's paKDE setting for its 7-D mixture),
    then the raster estimator on a grid x grid raster over the map's box plus
    a margin of 5% on each side. Each step timed with HIP events (mean of
    `reps`). The raster's unit of work is one (cell, point) kernel term: a
    squared distance (2 sub, 1 FMA), the scaled exponent (1 mul, 1 exp2) and
    the weighted sum (1 FMA)."""
    import torch

    from paper_1812_09869_amd import _lib

    n = y.shape[0]
    y = y.contiguous()
    lo = y.min(dim=0).values.double().cpu().numpy()
    hi = y.max(dim=0).values.double().cpu().numpy()
    pad = 0.05 * (hi - lo)
    lo, hi = lo - pad, hi + pad
    cx, cy = (hi[0] - lo[0]) / grid, (hi[1] - lo[1]) / grid
    ws = _lib.kde_new_workspace(n, device=y.device)
    beta = torch.empty(n, dtype=torch.float64, device=y.device)
    f = torch.empty((grid, grid), dtype=torch.float32, device=y.device)
    _lib.kde_bandwidths(y, perp, ws, beta)
    _lib.kde_raster(y, beta, lo[0], lo[1], cx, cy, grid, grid, f)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        _lib.kde_bandwidths(y, perp, ws, beta)
    ev[1].record()
    for _ in range(reps):
        _lib.kde_raster(y, beta, lo[0], lo[1], cx, cy, grid, grid, f)
    ev[2].record()
    torch.cuda.synchronize()
    bw_ms = ev[0].elapsed_time(ev[1]) / reps
    r_ms = ev[1].elapsed_time(ev[2]) / reps
    terms = float(n) * grid * grid
    res = {
        "n": n, "perplexity": perp, "raster": [grid, grid],
        "bandwidths_ms": bw_ms, "raster_ms": r_ms,
        "raster_terms_per_s": terms * 1e3 / r_ms,
        "raster_fp32_tflops": 7.0 * terms / (r_ms * 1e-3) / 1e12,
        "mass": float(f.double().sum()),
        "status": _lib.sync_status(ws),
    }
    log(f"[pakde] {res}")
    return res


def dissim_leg(x, perp=50.0, n=16384, reps=3):
    """Affinities from a given dissimilarity matrix against the same affinities
    from the points: the first n points of the benchmark mixture, their
    Euclidean distances as an n x n FP32 matrix (1 GiB at n = 16,384, built on
    the device by torch before timing), each path timed with HIP events (mean
    of `reps` after one untimed call). The dissimilarity path reads the
    matrix once (4 n^2 bytes) in place of the MFMA contraction."""
    import torch

    from paper_1812_09869_amd import _lib

    xs = x[:n].contiguous()
    dis = torch.cdist(xs.double(), xs.double()).float().contiguous()
    ws = _lib.new_workspace(n, xs.shape[1], device=xs.device)
    wsd = _lib.new_workspace(n, 1, device=xs.device)
    _lib.affinities(xs, perp, ws, reorder=False)
    _lib.affinities_dissim(dis, perp, wsd)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        _lib.affinities(xs, perp, ws, reorder=False)
    ev[1].record()
    for _ in range(reps):
        _lib.affinities_dissim(dis, perp, wsd)
    ev[2].record()
    torch.cuda.synchronize()
    pts_ms = ev[0].elapsed_time(ev[1]) / reps
    dis_ms = ev[1].elapsed_time(ev[2]) / reps
    a = _lib.export_p_rows(ws, n, 0, 256)
    b = _lib.export_p_rows(wsd, n, 0, 256)
    res = {"n": n, "d": int(xs.shape[1]), "perplexity": perp,
           "points_affinities_ms": pts_ms, "dissimilarity_affinities_ms": dis_ms,
           "p_rows_rel_diff": float((a - b).norm() / a.norm()),
           "status": max(_lib.sync_status(ws), _lib.sync_status(wsd))}
    log(f"[dissim] {res}")
    del dis, ws, wsd
    torch.cuda.empty_cache()
    return res


def implicit_leg(x, perp=50.0, iters=10, modes=("fp64", "fp32", "bf16x3", "bf16")):
    """Implicit P on the benchmark workload (N = 65,536, D = 50, perplexity
    50) in each distance mode: workspace size against the stored-P one, and
    the time of one iteration (every pass recomputes the nonzero tiles of P,
    buffer by buffer: the mode's MFMA distances with Eq. 3 in their epilogue,
    then the force body; the all-zero tiles take the repulsion-only body),
    mean of `iters` after one untimed. Here the mode sets the iteration rate,
    unlike the stored path; bf16x3 is the mode that keeps the per-step
    parity gates."""
    import torch

    from paper_1812_09869_amd import _lib, synth
    from paper_1812_09869_amd.tsne import ExactTSNE

    n, d = x.shape
    nb = (n + 255) // 256
    flop = float(d) * 256 * 256 * nb * (nb + 1)  # 2 d per (row, column) pair of the block rows
    res = {"n": n, "d": d, "stored_workspace_gb": _lib.workspace_bytes(n, d) / 1e9,
           "distance_flop_per_pass": flop, "modes": {}}
    y0 = torch.from_numpy(synth.embedding_init(n, seed=17)).to(x.device)
    for mode in modes:
        model = ExactTSNE(x, perp, dist_mode=mode, implicit=True)
        state = model.init_state(y0)
        model.run(state, 1, start=300)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        model.run(state, iters, start=301)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / iters
        res["modes"][mode] = {"workspace_gb": float(model.ws.numel()) / 1e9,
                              "ms_per_iteration": ms, "iters_per_s": 1e3 / ms,
                              "distance_tflops_over_pass": flop / (ms * 1e-3) / 1e12,
                              "status": model.status()}
        log(f"[implicit] {mode}: {res['modes'][mode]}")
        del model
        torch.cuda.empty_cache()
    return res


def precision_report(n=262144, d=128, perp=50.0):
    """Time and error of every distance mode at N=262,144, D=128 (the 10-D
    subspace mixture), against the FP64 mode: beta of every row, P on 24
    sampled rows (relative Frobenius and largest-entry error), the gradient and
    the KL at a fixed clustered map. The FP64 mode itself is held to the
    oracle by the tests (tests/test_gpu_large.py runs every mode against the
    oracle's statistics of all rows at 98,304 points of the same mixture).
    Prints one JSON line."""
    import numpy as np
    import torch

    from paper_1812_09869_amd import _lib, synth

    x_np, lab = synth.subspace(n, d=d)
    x = torch.from_numpy(x_np).cuda()
    rng = np.random.Generator(np.random.PCG64(5))
    prow = np.sort(rng.choice(n, 24, replace=False))
    ws = _lib.new_workspace(n, d, max(MODES, key=lambda m: _lib.workspace_bytes(n, d, m)))
    y = torch.from_numpy(synth.clustered_state(lab, seed=41, spread=60.0)).cuda()
    gbuf = torch.empty_like(y)
    cost = torch.zeros(2, dtype=torch.float64, device="cuda")
    out, ref = {}, None
    for mode in MODES:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.affinities(x, perp, ws, dist_mode=mode)
        e1.record()
        torch.cuda.synchronize()
        status = _lib.sync_status(ws)
        beta = _lib.export_rowstats(ws, n)[0].cpu().numpy()
        p = torch.cat([_lib.export_p_rows(ws, n, int(i), 1) for i in prow]).double().cpu()
        _lib.gradient(ws, n, y, 1.0, gbuf)
        g = gbuf.double().cpu()
        _lib.cost(ws, n, y, cost)
        kl = float(cost[0].cpu())
        if ref is None:
            ref = (beta, p, g, kl)
        pe = float(torch.linalg.norm(p - ref[1]) / torch.linalg.norm(ref[1]))
        pm = float((p - ref[1]).abs().max() / ref[1].max())
        ge = float(torch.linalg.norm(g - ref[2]) / torch.linalg.norm(ref[2]))
        out[mode] = {
            "status": status,
            "affinity_ms": e0.elapsed_time(e1),
            "beta_maxrel_vs_fp64": float((np.abs(beta - ref[0]) / ref[0]).max()),
            "p_rel_vs_fp64": pe,
            "p_maxrel_vs_fp64": pm,
            "grad_rel_vs_fp64": ge,
            "kl_rel_vs_fp64": abs(kl - ref[3]) / ref[3],
            "kl": kl,
            "meets_step_gates": bool(pe <= 1e-5 and pm <= 1e-5 and ge <= 1e-4),
        }
        log(f"[precision] {mode}: {out[mode]}")
    print(json.dumps({"workload": f"10-D subspace mixture, N={n}, D={d}, perplexity {perp:g}",
                      "modes": out}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--iters", type=int, default=1000)
    ap.add_argument("--dist-mode", default="bf16x3",
                    help="distance mode of the timed affinities (default: the compensated BF16 "
                         "mode, which meets the per-step parity gates)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the per-distance-mode affinity timing and error leg")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-problem batched leg")
    ap.add_argument("--no-pakde", action="store_true",
                    help="skip the paKDE leg (bandwidths and raster of the final map)")
    ap.add_argument("--no-implicit", action="store_true",
                    help="skip the implicit-P leg")
    ap.add_argument("--no-dissim", action="store_true",
                    help="skip the given-dissimilarity affinity leg")
    ap.add_argument("--no-ptsne", action="store_true",
                    help="skip the parallel-scheme (ptSNE) leg")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate training / inference / evaluation leg")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 64-problem batched leg (prints its JSON object)")
    ap.add_argument("--batched-sweeps", type=int, default=500,
                    help="sweeps of the batched leg")
    ap.add_argument("--ptsne-only", action="store_true",
                    help="only run the parallel-scheme leg (prints its JSON object)")
    ap.add_argument("--ptsne-epochs", type=int, default=10,
                    help="timed epochs of the parallel-scheme leg")
    ap.add_argument("--precision-report", action="store_true",
                    help="only run the per-mode error report at N=262,144, D=128")
    ap.add_argument("--implicit-large", action="store_true",
                    help="only run the implicit-P leg at N=262,144, D=128 (the 10-D subspace "
                         "mixture), where a stored P would take 142 GB")
    args = ap.parse_args()
    if args.precision_report:
        precision_report()
        return
    if args.implicit_large:
        import torch

        from paper_1812_09869_amd import synth
        xl, _ = synth.subspace(262144, d=128)
        res = implicit_leg(torch.from_numpy(xl).cuda(), 50.0, iters=5, modes=("fp64", "bf16x3", "bf16"))
        res["workload"] = "10-D subspace mixture, N=262144, D=128, perplexity 50"
        print(json.dumps(res), flush=True)
        return
    if args.ptsne_only:
        print(json.dumps(ptsne_leg(args.ptsne_epochs)), flush=True)
        return
    if args.batched_only:
        print(json.dumps(batched_leg(args.batched_sweeps)), flush=True)
        return
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
    x_np, lab_np = synth.gmm_aniso(n)
    y0_np = synth.embedding_init(n, seed=synth.SEEDS["init_aniso"])
    dev = torch.device("cuda:0")
    x = torch.from_numpy(x_np).to(dev)
    y0 = torch.from_numpy(y0_np).to(dev)
    ws = _lib.new_workspace(n, d, args.dist_mode)
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
        _lib.affinities(x, perp, ws, dist_mode=args.dist_mode)
        if events is not None:
            events["aff"][-1][1].record()
        for t in range(args.iters):
            alpha, mu, eta = sched(t)
            if events is not None and t % FORCE_SAMPLE == 0:
                # the force pass of every FORCE_SAMPLE-th iteration is timed on
                # its own (events on the stream it runs on); the others run as
                # one tsne_step call
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                _lib.forces(ws, n, y)
                e1.record()
                events["force"].append((e0, e1))
                _lib.update(ws, n, y, u, g, alpha, mu, eta, sched.min_gain, True)
            else:
                _lib.step(ws, n, y, u, g, alpha, mu, eta, sched.min_gain, True)
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
    steady_ms = (ms_per_step - aff_ms) / args.iters
    rl = force_roofline(ws, n, force_ms)
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
            "dist_mode": args.dist_mode,
        },
        "roofline": rl,
        "steady_iters_per_s": 1e3 / steady_ms,
        "affinity_ms": aff_ms,
        "force_ms": force_ms,
        "pair_interactions_per_s": n * (n - 1) / 2.0 * 1e3 / steady_ms,
        "final_kl": kl,
        "final_cnorm": cnorm,
    }
    out["run_log"] = monitor_leg(ws, n, y0, args.iters, sched)
    if not args.no_pakde:
        out["pakde"] = pakde_leg(y.clone())
    if not args.no_surrogate:
        y_exact = y.clone()
        out["surrogate"] = surrogate_leg(x, y_exact, perp)
    if not args.no_precision or not args.no_batched or not args.no_ptsne:
        del ws
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = batched_leg(args.batched_sweeps)
        torch.cuda.empty_cache()
    if not args.no_ptsne:
        out["ptsne"] = ptsne_leg(args.ptsne_epochs)
        torch.cuda.empty_cache()
    if not args.no_dissim:
        out["dissim"] = dissim_leg(x)
    if not args.no_implicit:
        out["implicit"] = implicit_leg(x, perp)
    if not args.no_precision:
        torch.cuda.empty_cache()
        out["dist_modes"] = precision_leg(x, lab_np, n, d, perp, args.iters, steady_ms)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(x_np, perp, n, args.iters)
        log(f"[bench] cpu baseline {out['cpu_baseline']['value']:.4g} iters/s "
            f"({out['cpu_baseline']['cores']} threads)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
