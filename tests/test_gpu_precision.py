"""Precision path: reduced-precision distance contractions against the FP64 oracle.

Every mode must give a valid P (symmetric, summing to 1, zero diagonal, every
row calibrated), and its error against the FP64 oracle must sit inside its
bound.

* The plain modes (fp32, fp16, bf16) keep the cancellation of
  |x|^2 + |y|^2 - 2 x.y: with u the unit roundoff of the operands or of the
  FP32 accumulator (BF16 2^-9, FP16 2^-12, FP32 2^-24), the distance error is
  of order u |x|^2 and the relative error of p_ij beta times that. Their
  bounds are those estimates for the test data times about 10; they do not
  meet the per-step gates.
* The x3 modes (three exact-accumulate slices, compensated FP32 combine) are
  held to the per-step gates themselves: P within 1e-5 (relative Frobenius
  and largest entry error over the largest entry) and the gradient within
  1e-4 relative L2.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1812_09869_amd import _lib, synth
from paper_1812_09869_amd.tsne import ExactTSNE

pytestmark = pytest.mark.gpu

# (mode, bound on the relative Frobenius error of P, bound on the gradient rel-L2,
#  bound on the largest entry error over the largest entry, or None)
MODES = [
    ("fp64", 1e-5, 1e-4, 1e-5),
    ("fp16x3", 1e-5, 1e-4, 1e-5),
    ("bf16x3", 1e-5, 1e-4, 1e-5),
    ("fp32", 2e-4, 2e-4, None),
    ("fp16", 2e-2, 2e-2, None),
    ("bf16", 2e-1, 2e-1, None),
]

WORKLOADS = {
    "small": lambda: (*synth.plain_small(2000), 30.0),
    "subspace": lambda: (*synth.subspace(1500, d=128), 50.0),
}


@pytest.fixture(scope="module", params=list(WORKLOADS))
def ref(request):
    x, lab, perp = WORKLOADS[request.param]()
    print(f"\n[workload] {request.param} n={x.shape[0]} d={x.shape[1]}", flush=True)
    st = oracle.calibrate(x, perp)
    P = oracle.joint_p(x, st)
    y = synth.clustered_state(lab, seed=5)
    g_ref, _ = oracle.gradient(P, y.astype(np.float64), 1.0)
    kl_ref, _ = oracle.cost(P, y.astype(np.float64))
    return dict(name=request.param, x=x, perp=perp, P=P, y=y, g_ref=g_ref, kl_ref=kl_ref)


@pytest.mark.parametrize("mode,p_bound,g_bound,max_bound", MODES, ids=[m[0] for m in MODES])
def test_mode_errors(ref, mode, p_bound, g_bound, max_bound):
    x, P = ref["x"], ref["P"]
    n = x.shape[0]
    model = ExactTSNE(torch.from_numpy(x).cuda(), ref["perp"], dist_mode=mode)
    assert model.status() == 0
    pg = model.p_rows(0, n).cpu().numpy().astype(np.float64)
    assert np.array_equal(pg, pg.T) and np.all(np.diag(pg) == 0)
    psum = _lib.export_scalars(model.ws, n)[0]
    assert abs(psum - 1.0) <= 1e-5
    fro = np.linalg.norm(pg - P) / np.linalg.norm(P)
    mx = np.abs(pg - P).max() / P.max()
    g, _ = model.gradient(torch.from_numpy(ref["y"]).cuda(), 1.0)
    grel = np.linalg.norm(g.cpu().numpy() - ref["g_ref"]) / np.linalg.norm(ref["g_ref"])
    kl = float(model.cost(torch.from_numpy(ref["y"]).cuda()).cpu()[0])
    klrel = abs(kl - ref["kl_ref"]) / ref["kl_ref"]
    print(f"  {ref['name']:9s} {mode:7s} P fro {fro:.2e} max {mx:.2e} | grad {grel:.2e} | "
          f"KL {klrel:.2e}")
    assert fro <= p_bound and grel <= g_bound
    if max_bound is not None:
        assert mx <= max_bound
    assert klrel <= max(p_bound, 1e-5)


# Sizes and widths at the edges of the x3 kernels: a 3-point problem, ragged
# last row blocks (255, 257, 300 points), one coordinate, and widths one past
# a 32-wide slice block (33, 65: a second, almost empty K step).
EDGES = [(3, 2, 1.5), (255, 1, 10.0), (257, 33, 20.0), (300, 65, 30.0), (600, 64, 30.0)]


@pytest.mark.parametrize("mode", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("n,d,perp", EDGES, ids=[f"n{n}-d{d}" for n, d, _ in EDGES])
def test_x3_edges_against_oracle(n, d, perp, mode):
    rng = np.random.Generator(np.random.PCG64(1000 + n + d))
    x = (rng.standard_normal((n, d)) * 4.0 + 20.0).astype(np.float32)  # offset: cancellation
    st = oracle.calibrate(x, perp)
    P = oracle.joint_p(x, st)
    y = synth.embedding_init(n, seed=3) * 100.0
    g_ref, _ = oracle.gradient(P, y.astype(np.float64), 1.0)
    model = ExactTSNE(torch.from_numpy(x).cuda(), perp, dist_mode=mode)
    assert model.status() == 0
    pg = model.p_rows(0, n).cpu().numpy().astype(np.float64)
    assert np.array_equal(pg, pg.T) and np.all(np.diag(pg) == 0)
    fro = np.linalg.norm(pg - P) / np.linalg.norm(P)
    mx = np.abs(pg - P).max() / P.max()
    g, _ = model.gradient(torch.from_numpy(y).cuda(), 1.0)
    grel = np.linalg.norm(g.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    print(f"\n  n={n} d={d} {mode}: P fro {fro:.2e} max {mx:.2e} | grad {grel:.2e}")
    assert fro <= 1e-5 and mx <= 1e-5 and grel <= 1e-4
