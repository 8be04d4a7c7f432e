"""Implicit P (recomputed block row by block row in every pass) on the GPU.

Each element's distance is the contraction the stored path forms for it, in
the workspace's mode, and Eq. 3 is the same arithmetic, so P is bitwise that
of the stored path; the force pass splits off the same all-zero tiles and
runs the same tile bodies, and the cost pass the same tile sums, so
gradients, Z, costs and maps are bitwise those of the stored path too (the
tests below check equality). Gates against the oracle (FP64 mode) are those
of the stored path: gradient relative L2 <= 1e-4, Z relative <= 1e-6, KL
relative <= 1e-5, map after three steps <= 1e-4. The reduced distance modes
are checked against the stored path of the same mode (their distance to the
oracle is the precision report's).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1812_09869_amd import _lib, synth
from paper_1812_09869_amd.tsne import ExactTSNE

pytestmark = pytest.mark.gpu

# n = 3: one tile, nearly all padding; n = 257: two block rows, the second
# holding one point (a ragged tail in both the row and the column direction)
CASES = [(3, 2, 1.5, "gauss"), (255, 3, 10.0, "gauss"), (257, 5, 20.0, "gauss"),
         (600, 50, 30.0, "aniso"), (1300, 10, 30.0, "small")]


def _data(n, d, gen, seed):
    if gen == "small":
        return synth.plain_small(n, seed=seed)
    if gen == "aniso":
        return synth.gmm_aniso(n, sample_seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal((n, d)) * 2.0).astype(np.float32), rng.integers(0, 4, n)


@pytest.mark.parametrize("n,d,perp,gen", CASES, ids=lambda v: str(v))
def test_implicit_matches_oracle_and_stored(n, d, perp, gen):
    x, lab = _data(n, d, gen, 300 + n)
    print(f"\n[implicit] n={n} d={d}", flush=True)
    P = oracle.joint_p(x, oracle.calibrate(x, perp))
    xt = torch.from_numpy(x).cuda()
    imp = ExactTSNE(xt, perp, implicit=True)
    sto = ExactTSNE(xt, perp)
    # same affinity stage: identical row statistics
    for a, b in zip(imp.rowstats(), sto.rowstats()):
        assert torch.equal(a, b)
    y = synth.clustered_state(lab, seed=9)
    yt = torch.from_numpy(y).cuda()
    for alpha in (1.0, 12.0):
        g_ref, z_ref = oracle.gradient(P, y.astype(np.float64), alpha)
        gi, zi = imp.gradient(yt, alpha)
        gi, zi = gi.cpu().numpy().astype(np.float64), float(zi.cpu()[0])
        gs, _ = sto.gradient(yt, alpha)
        gs = gs.cpu().numpy().astype(np.float64)
        rel = np.linalg.norm(gi - g_ref) / np.linalg.norm(g_ref)
        rel_s = np.linalg.norm(gi - gs) / np.linalg.norm(gs)
        print(f"  alpha {alpha}: gradient rel {rel:.2e} (vs stored {rel_s:.2e}), Z rel "
              f"{abs(zi - z_ref) / z_ref:.2e}")
        assert rel <= 1e-4 and rel_s == 0.0 and abs(zi - z_ref) <= 1e-6 * z_ref
    kl_ref, cn_ref = oracle.cost(P, y.astype(np.float64))
    out = imp.cost(yt).cpu().numpy()
    assert abs(out[0] - kl_ref) <= 1e-5 * abs(kl_ref) and abs(out[1] - cn_ref) <= 1e-6
    y0 = synth.embedding_init(n, seed=11)
    st = imp.init_state(torch.from_numpy(y0).cuda())
    imp.run(st, 3)
    yr, _, _ = oracle.run(P, y0.astype(np.float64), 3)
    rel = np.linalg.norm(st[0].cpu().numpy() - yr) / np.linalg.norm(yr)
    print(f"  map after 3 steps rel {rel:.2e}")
    assert rel <= 1e-4
    assert imp.status() == 0 and sto.status() == 0


def test_modes_are_not_mixed():
    """A stored-P entry point on an implicit workspace, and the reverse, are
    refused on the device (TSNE_E_STATE) instead of reading the wrong buffer."""
    x, _ = synth.plain_small(600, seed=5)
    xt = torch.from_numpy(x).cuda()
    y = torch.from_numpy(synth.embedding_init(600, seed=6)).cuda()
    g = torch.empty_like(y)
    imp = ExactTSNE(xt, 20.0, implicit=True)
    _lib.gradient(imp.ws, 600, y, 1.0, g)
    assert _lib.sync_status(imp.ws) == 7
    sto = ExactTSNE(xt, 20.0)
    _lib.gradient_implicit(sto.ws, 600, 10, y, 1.0, g)
    assert _lib.sync_status(sto.ws) == 7
    # the right kind of workspace with the wrong input dimension is refused too
    imp2 = ExactTSNE(xt, 20.0, implicit=True)
    _lib.gradient_implicit(imp2.ws, 600, 11, y, 1.0, g)
    assert _lib.sync_status(imp2.ws) == 7


@pytest.mark.parametrize("mode", ["fp32", "bf16", "fp16x3"])
def test_reduced_modes_match_stored(mode):
    """Implicit P in a reduced distance mode: the row statistics, gradient, Z,
    cost and map after three steps of the stored path of that mode, bitwise."""
    n, perp = 1300, 30.0
    x, lab = synth.gmm_aniso(n, sample_seed=77)
    print(f"\n[implicit] mode={mode} n={n} d={x.shape[1]}", flush=True)
    xt = torch.from_numpy(x).cuda()
    imp = ExactTSNE(xt, perp, dist_mode=mode, implicit=True)
    sto = ExactTSNE(xt, perp, dist_mode=mode)
    for a, b in zip(imp.rowstats(), sto.rowstats()):
        assert torch.equal(a, b)
    yt = torch.from_numpy(synth.clustered_state(lab, seed=9)).cuda()
    gi, zi = imp.gradient(yt, 1.0)
    gi, zi = gi.clone(), float(zi.cpu()[0])
    gs, zs = sto.gradient(yt, 1.0)
    zs = float(zs.cpu()[0])
    rel = (torch.linalg.norm(gi - gs) / torch.linalg.norm(gs)).item()
    print(f"  gradient rel vs stored {rel:.2e}, Z rel {abs(zi - zs) / zs:.2e}")
    assert torch.equal(gi, gs) and zi == zs
    ci = imp.cost(yt).cpu().numpy().copy()
    cs = sto.cost(yt).cpu().numpy()
    assert np.array_equal(ci, cs)
    y0 = torch.from_numpy(synth.embedding_init(n, seed=11)).cuda()
    si, ss = imp.init_state(y0), sto.init_state(y0)
    imp.run(si, 3)
    sto.run(ss, 3)
    rel = (torch.linalg.norm(si[0] - ss[0]) / torch.linalg.norm(ss[0])).item()
    print(f"  map after 3 steps rel vs stored {rel:.2e}")
    assert all(torch.equal(a, b) for a, b in zip(si, ss))
    assert imp.status() == 0 and sto.status() == 0


def test_wrong_mode_is_refused():
    """An implicit workspace used with another distance mode is refused on the
    device before its buffers are read (the reduced modes' operands sit past
    the end of an FP64 workspace)."""
    x, _ = synth.plain_small(600, seed=5)
    xt = torch.from_numpy(x).cuda()
    y = torch.from_numpy(synth.embedding_init(600, seed=6)).cuda()
    g = torch.empty_like(y)
    f64 = ExactTSNE(xt, 20.0, implicit=True)
    _lib.gradient_implicit(f64.ws, 600, 10, y, 1.0, g, dist_mode="bf16")
    assert _lib.sync_status(f64.ws) == 7
    b16 = ExactTSNE(xt, 20.0, dist_mode="bf16", implicit=True)
    _lib.gradient_implicit(b16.ws, 600, 10, y, 1.0, g, dist_mode="fp64")
    assert _lib.sync_status(b16.ws) == 7
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    b16b = ExactTSNE(xt, 20.0, dist_mode="bf16", implicit=True)
    _lib.cost_implicit(b16b.ws, 600, 10, y, out, dist_mode="fp32")
    assert _lib.sync_status(b16b.ws) == 7


@pytest.mark.parametrize("mode", ["fp64", "bf16"])
def test_benchmark_size_matches_stored(mode):
    """The benchmark workload (N = 65,536, D = 50, perplexity 50): 17 buffers
    of tiles, three quarters of them all zero and skipped after the affinity
    stage. Implicit P against the stored path of the same mode, bitwise: row
    statistics, gradient, Z, cost, and the state after ten steps of the
    benchmark schedule."""
    n = 65536
    x, lab = synth.gmm_aniso(n)
    print(f"\n[implicit] benchmark size, mode={mode}", flush=True)
    xt = torch.from_numpy(x).cuda()
    imp = ExactTSNE(xt, 50.0, dist_mode=mode, implicit=True)
    sto = ExactTSNE(xt, 50.0, dist_mode=mode)
    for a, b in zip(imp.rowstats(), sto.rowstats()):
        assert torch.equal(a, b)
    yt = torch.from_numpy(synth.clustered_state(lab, seed=3, spread=30.0)).cuda()
    gi, zi = imp.gradient(yt, 1.0)
    gi, zi = gi.clone(), float(zi.cpu()[0])
    gs, zs = sto.gradient(yt, 1.0)
    zs = float(zs.cpu()[0])
    rel = (torch.linalg.norm(gi - gs) / torch.linalg.norm(gs)).item()
    print(f"  gradient rel vs stored {rel:.2e}, Z rel {abs(zi - zs) / zs:.2e}", flush=True)
    assert torch.equal(gi, gs) and zi == zs
    ci = imp.cost(yt).cpu().numpy().copy()
    cs = sto.cost(yt).cpu().numpy()
    assert np.array_equal(ci, cs)
    y0 = torch.from_numpy(synth.embedding_init(n, seed=17)).cuda()
    si, ss = imp.init_state(y0), sto.init_state(y0)
    imp.run(si, 10)
    sto.run(ss, 10)
    rel = (torch.linalg.norm(si[0] - ss[0]) / torch.linalg.norm(ss[0])).item()
    print(f"  map after 10 steps rel vs stored {rel:.2e}", flush=True)
    assert all(torch.equal(a, b) for a, b in zip(si, ss))
    assert imp.status() == 0 and sto.status() == 0


@pytest.mark.parametrize("mode", ["fp64", "bf16"])
def test_no_reorder_matches_stored(mode):
    """Implicit P without the locality order (the caller's order is the
    internal one; the FP64 operands are the identity copy of the centred X),
    over three block rows: bitwise the stored path of the same mode."""
    n = 600
    x, lab = synth.gmm_aniso(n, sample_seed=91)
    print(f"\n[implicit] no reorder, mode={mode}, n={n}", flush=True)
    xt = torch.from_numpy(x).cuda()
    imp = ExactTSNE(xt, 30.0, dist_mode=mode, implicit=True, reorder=False)
    sto = ExactTSNE(xt, 30.0, dist_mode=mode, reorder=False)
    for a, b in zip(imp.rowstats(), sto.rowstats()):
        assert torch.equal(a, b)
    yt = torch.from_numpy(synth.clustered_state(lab, seed=9)).cuda()
    gi, zi = imp.gradient(yt, 1.0)
    gi, zi = gi.clone(), float(zi.cpu()[0])
    gs, zs = sto.gradient(yt, 1.0)
    assert torch.equal(gi, gs) and zi == float(zs.cpu()[0])
    y0 = torch.from_numpy(synth.embedding_init(n, seed=12)).cuda()
    si, ss = imp.init_state(y0), sto.init_state(y0)
    imp.run(si, 3)
    sto.run(ss, 3)
    assert all(torch.equal(a, b) for a, b in zip(si, ss))
    assert imp.status() == 0 and sto.status() == 0
