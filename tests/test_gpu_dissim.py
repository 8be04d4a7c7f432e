"""Affinities from given dissimilarities on the GPU against the FP64 oracle.

The dissimilarity takes the place of ||x_i - x_j|| (its square enters Eq. 1);
the cases are Euclidean distances of points (ragged sizes) and hop distances
on a 1,005-node cylinder mesh, the stand-in for the paper's dwt1005 set. Gates
are those of the point input: ||dP||_F / ||P||_F <= 1e-5, max |dP| / max P <=
1e-5, |H_i - ln u| <= 1e-5, gradient relative L2 <= 1e-4.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

import oracle
from paper_1812_09869_amd import _lib, synth
from paper_1812_09869_amd.tsne import ExactTSNE

pytestmark = pytest.mark.gpu


def _cases():
    out = []
    for n, d, perp in [(257, 5, 12.0), (600, 10, 30.0)]:
        x = np.random.Generator(np.random.PCG64(n)).standard_normal((n, d)) * 3.0
        out.append(pytest.param(f"euclid{n}", np.sqrt(cdist(x, x, "sqeuclidean")).astype(np.float32),
                                perp, id=f"euclid{n}"))
    out.append(pytest.param("mesh1005", synth.mesh_graph_distances(), 50.0, id="mesh1005"))
    return out


@pytest.mark.parametrize("name,dis,perp", _cases())
def test_dissimilarity_affinities_and_gradient(name, dis, perp):
    n = dis.shape[0]
    print(f"\n[dissim] {name} n={n} perplexity={perp}", flush=True)
    st = oracle.calibrate_dissim(dis, perp)
    P = oracle.joint_p_dissim(dis, st)
    model = ExactTSNE.from_dissimilarities(torch.from_numpy(dis).cuda(), perp)
    assert model.status() == 0
    pg = model.p_rows(0, n).cpu().numpy().astype(np.float64)
    _, _, _, H, ev = (t.cpu().numpy() for t in model.rowstats())
    fro = np.linalg.norm(pg - P) / np.linalg.norm(P)
    mx = np.abs(pg - P).max() / np.abs(P).max()
    print(f"  P rel-Frobenius {fro:.2e} max-rel {mx:.2e}")
    assert fro <= 1e-5 and mx <= 1e-5
    assert np.array_equal(pg, pg.T) and np.all(ev > 0)
    assert np.abs(H - math.log(perp)).max() <= 1e-5
    y = synth.disk_init(n, 5) * 10.0
    g_ref, _ = oracle.gradient(P, y.astype(np.float64), 1.0)
    g, _ = model.gradient(torch.from_numpy(y).cuda(), 1.0)
    rel = np.linalg.norm(g.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    print(f"  gradient rel {rel:.2e}")
    assert rel <= 1e-4


def test_negative_dissimilarity_is_flagged():
    dis = synth.mesh_graph_distances(5, 8)
    dis[3, 7] = -1.0
    model = ExactTSNE.from_dissimilarities(torch.from_numpy(dis).cuda(), 5.0)
    assert model.status() == 5  # TSNE_E_NONFINITE


def test_benchmark_size_euclidean():
    """The benchmark's dissimilarity leg: Euclidean distances of the first 16,384 points
    of the benchmark mixture (D = 50) given as a 1 GiB FP32 matrix. The bandwidths of 64
    sampled points against the oracle's search on the points (relative <= 1e-5), and
    eight sampled rows of P against the path from the points (max |dP| / max P <= 1e-5)."""
    n = 16384
    x, _ = synth.gmm_aniso(n)
    xt = torch.from_numpy(x).cuda()
    dis = torch.cdist(xt.double(), xt.double()).float().contiguous()  # FP64, then rounded
    print(f"\n[dissim] n={n}, matrix {dis.numel() * 4 / 2**30:.2f} GiB", flush=True)
    m_d = ExactTSNE.from_dissimilarities(dis, 50.0)
    del dis
    torch.cuda.empty_cache()
    m_x = ExactTSNE(xt, 50.0)
    rng = np.random.Generator(np.random.PCG64(16))
    rows = rng.choice(n, 64, replace=False)
    ref = oracle.calibrate(x.astype(np.float64), 50.0, rows=rows).beta
    beta = m_d.rowstats()[0].cpu().numpy()[rows]
    rb = np.abs(beta - ref) / ref
    print(f"  beta (64 sampled points) max-rel {rb.max():.2e}", flush=True)
    assert rb.max() <= 1e-5
    worst = 0.0
    for r in rng.choice(n - 1, 8, replace=False):
        pd = m_d.p_rows(int(r), 1).cpu().numpy()
        px = m_x.p_rows(int(r), 1).cpu().numpy()
        worst = max(worst, float(np.abs(pd - px).max() / px.max()))
    print(f"  P rows (8 sampled) max |dP| / max P {worst:.2e}", flush=True)
    assert worst <= 1e-5
    assert m_d.status() == 0 and m_x.status() == 0
