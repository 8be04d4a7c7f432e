"""Pins of the parallel-scheme oracle (section "Parallelized implementation").

The chunk and round bookkeeping is checked against the paper's own worked
numbers (tests/golden/ptsne_paper_examples.json, each entry citing its
passage); the epoch itself against invariants: every (point, layer) is
carried by exactly one thread, an epoch without iterations gives back the
maps it started from, and one thread with one layer is the plain iteration.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import ptsne
from paper_1812_09869_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "ptsne_paper_examples.json")))


def test_layers_example_from_paper():
    g = GOLD["layers_example"]
    got = [[c + 1 for c in ptsne.thread_chunks(g["threads"], g["layers"], k)]
           for k in range(g["threads"])]
    assert got == g["chunks_1based"]


def test_round_sizes_from_paper():
    g = GOLD["rounds_digits"]
    z = ptsne.thread_size(g["n"], g["threads"], g["layers"])
    assert z == g["z"]
    assert ptsne.epochs_per_round(g["n"]) == g["epochs"]
    assert ptsne.iterations_per_epoch(z) == g["iterations"]
    h = GOLD["large_n"]
    assert ptsne.epochs_per_round(h["n"]) == h["epochs"]
    for t, l, z in h["setups"]:
        assert ptsne.thread_size(h["n"], t, l) == z
    d = GOLD["dwt1005"]
    for l, f in zip(d["layers"], d["fraction"]):
        assert ptsne.thread_size(d["n"], d["threads"], l) / d["n"] == pytest.approx(f)


def test_iterations_round_up_exact_squares():
    assert ptsne.iterations_per_epoch(400) == 20
    assert ptsne.iterations_per_epoch(401) == 21
    assert ptsne.epochs_per_round(400) == 20
    assert ptsne.epochs_per_round(399) == 19


@pytest.mark.parametrize("n,threads,layers", [(100, 7, 3), (64, 4, 4), (10, 10, 1), (33, 5, 2)])
def test_every_point_once_per_layer(n, threads, layers):
    order = np.random.Generator(np.random.PCG64(n)).permutation(n)
    seen = np.zeros((layers, n), dtype=np.int64)
    total = 0
    for k in range(threads):
        idx, lay = ptsne.thread_members(order, threads, layers, k)
        assert len(set(idx.tolist())) == idx.shape[0]  # no point twice in a thread
        np.add.at(seen, (lay, idx), 1)
        total += idx.shape[0]
    assert np.all(seen == 1)
    assert total == n * layers
    b = ptsne.chunk_bounds(n, threads)
    sizes = np.diff(b)
    assert sizes.max() - sizes.min() <= 1 and sizes.sum() == n


def test_epoch_without_iterations_gives_back_the_maps():
    x, _ = synth.plain_small(120, seed=31)
    maps = np.stack([synth.disk_init(120, 32 + l).astype(np.float64) for l in range(2)])
    order = np.random.Generator(np.random.PCG64(33)).permutation(120)
    out, c, s, costs = ptsne.epoch(x, maps, order, 4, 2, 10.0, 0, 0.8)
    assert np.array_equal(out, maps)
    assert s == pytest.approx(np.mean([oracle.embedding_size(m) for m in maps]), rel=1e-15)
    assert costs.shape == (4,) and np.all(costs > 0.9)  # a random map: C_norm close to 1


def test_one_thread_one_layer_is_the_plain_iteration():
    """T = L = 1: the single partial t-SNE holds every point, so an epoch is
    ``iters`` steps of Eqs. 10-11 on the whole set (in the order's row order)."""
    x, _ = synth.plain_small(150, seed=41)
    y0 = synth.disk_init(150, 42).astype(np.float64)
    order = np.random.Generator(np.random.PCG64(43)).permutation(150)
    out, c, _, _ = ptsne.epoch(x, y0[None], order, 1, 1, 12.0, 5, 0.7)
    P = oracle.joint_p(x, oracle.calibrate(x, 12.0))
    y, u = y0.copy(), np.zeros_like(y0)
    for _ in range(5):
        oracle.step_range(P, y, u, mu=0.7, recentre=False)
    np.testing.assert_allclose(out[0], y, rtol=1e-9, atol=1e-12)
    assert c == pytest.approx(oracle.cost(P, y)[1], rel=1e-9)


def test_epochs_lower_the_global_cost():
    """A few epochs of the scheme lower the cost of the whole set (Eq. 9)."""
    x, _ = synth.plain_small(400, seed=51)
    y0 = synth.disk_init(400, 52)
    orders = synth.epoch_orders(400, 4, 53)
    P = oracle.joint_p(x, oracle.calibrate(x, 15.0))
    c0 = oracle.cost(P, y0.astype(np.float64))[1]
    maps, mon = ptsne.run(x, y0, orders, 4, 2, 15.0, 15, 0.8)
    c1 = oracle.cost(P, maps[0])[1]
    assert c1 < c0 - 0.05, (c0, c1)
    assert mon[-1][1] > mon[0][1] * 0.5  # the map keeps a nonzero size
