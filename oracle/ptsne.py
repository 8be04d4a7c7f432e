"""FP64 oracle of the parallel scheme (ptSNE), section "Parallelized implementation".

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the
smoke check and the benchmark's CPU-baseline leg are its only users.

The scheme, as the paper states it:
  * the n points are split into ``threads`` elementary chunks; thread k runs
    a partial t-SNE on ``layers`` chunks, k, k+1, ..., k+layers-1 (cyclic),
    so each chunk is shared by ``layers`` successive threads and each point
    has one position per layer (subsections "threads" and "layers");
  * thread size z = n * layers / threads (subsection "thread-size");
  * an epoch is: the master mixes the data and defines the chunks, every
    worker runs its partial t-SNE for a short run, the master pools the
    partial solutions (subsection "epochs");
  * a round is floor(sqrt(n)) epochs of ceil(sqrt(z)) iterations (subsection
    "rounds"; the rounding is fixed by the paper's own examples: 244 epochs
    at n = 60,000 and 32 iterations at z = 1,000 in the rounds figure, 547
    epochs at n = 300,000 in the computation-time discussion);
  * the start map is uniform in the unit disk; each partial t-SNE uses the
    paper's own optimiser (Eq. 11, momentum as an external constant, no
    exaggeration);
  * monitors: the average of the partial t-SNEs' pseudo-normalised costs
    (Eq. 9), and the embedding size, the diagonal of the map's box, averaged
    over the layers (section "Comparison of t-SNE and ptSNE").

Readings where the paper points to a supplement it does not include:
  * mixing: a fresh random order of the points per epoch (an input: the
    caller draws it); chunk c is the c-th contiguous piece of that order,
    chunks differ in size by at most one, the larger ones first;
  * the layer of a thread's chunk is its position in the thread: chunk
    (k + l) mod T enters thread k at its points' layer-l positions, and
    thread k's result for that chunk is written back to layer l. Every
    layer of every point is thus read and written by exactly one thread per
    epoch;
  * every partial t-SNE starts with zero momentum state; its affinities are
    those of its own points (Eqs. 1-3 with the given perplexity); the map is
    not re-centred (the gradient sums to zero, so the mean stays put).
"""
from __future__ import annotations

import math

import numpy as np

from . import calibrate, cost, embedding_size, joint_p, step_range


def epochs_per_round(n: int) -> int:
    """floor(sqrt(n)) epochs per round (subsection "rounds")."""
    return math.isqrt(n)


def iterations_per_epoch(z: float) -> int:
    """ceil(sqrt(z)) iterations per epoch (subsection "rounds")."""
    return int(math.ceil(math.sqrt(z) - 1e-12))


def thread_size(n: int, threads: int, layers: int) -> float:
    """z = n * layers / threads (subsection "thread-size")."""
    return n * layers / threads


def chunk_bounds(n: int, threads: int) -> np.ndarray:
    """Start offsets of the ``threads`` chunks in the epoch's order (threads + 1 entries)."""
    q, r = divmod(n, threads)
    sizes = np.array([q + (1 if c < r else 0) for c in range(threads)], dtype=np.int64)
    return np.concatenate([[0], np.cumsum(sizes)])


def thread_chunks(threads: int, layers: int, k: int) -> list[int]:
    """Chunks of thread k: k, k+1, ..., k+layers-1, cyclic (subsection "layers")."""
    return [(k + l) % threads for l in range(layers)]


def thread_members(order: np.ndarray, threads: int, layers: int, k: int):
    """(point indices, layer of each point) of thread k for an epoch with ``order``."""
    b = chunk_bounds(order.shape[0], threads)
    idx, lay = [], []
    for l, c in enumerate(thread_chunks(threads, layers, k)):
        pts = order[b[c]:b[c + 1]]
        idx.append(pts)
        lay.append(np.full(pts.shape[0], l, dtype=np.int64))
    return np.concatenate(idx).astype(np.int64), np.concatenate(lay)


def epoch(x, maps, order, threads: int, layers: int, perplexity: float, iters: int,
          momentum: float):
    """One epoch: mix (start maps from the layers), run every partial t-SNE for
    ``iters`` iterations of Eqs. 10-11, pool the results back into the layers.

    x: n x d; maps: layers x n x 2 (FP64, updated copy returned); order: the
    epoch's permutation of 0..n-1. Returns (maps, mean partial C_norm, mean
    layer size, per-thread C_norm).
    """
    x = np.asarray(x, dtype=np.float64)
    maps = np.array(maps, dtype=np.float64)
    out = maps.copy()
    costs = []
    for k in range(threads):
        idx, lay = thread_members(order, threads, layers, k)
        xk = x[idx]
        P = joint_p(xk, calibrate(xk, perplexity))
        y = np.ascontiguousarray(maps[lay, idx])
        u = np.zeros_like(y)
        for _ in range(iters):
            step_range(P, y, u, mu=momentum, alpha=1.0, recentre=False)
        costs.append(cost(P, y)[1])
        out[lay, idx] = y
    sizes = [embedding_size(out[l]) for l in range(layers)]
    return out, float(np.mean(costs)), float(np.mean(sizes)), np.array(costs)


def run(x, y0, orders, threads: int, layers: int, perplexity: float, iters: int,
        momentum: float):
    """Epochs over the given orders from the start map y0 (all layers equal).
    Returns (maps, list of (mean cost, mean size) per epoch)."""
    maps = np.repeat(np.asarray(y0, dtype=np.float64)[None], layers, axis=0)
    mon = []
    for order in orders:
        maps, c, s, _ = epoch(x, maps, order, threads, layers, perplexity, iters, momentum)
        mon.append((c, s))
    return maps, mon
