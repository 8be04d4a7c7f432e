"""Pins of the paKDE oracle (section "Perplexity-adaptive Kernel Density Estimation").

Each kernel (beta_j / pi) exp(-beta_j |c - y_j|^2) is a bivariate Gaussian
density, so a fine raster that covers the map holds total mass 1; one
isolated kernel evaluated at its own centre is (S / n) beta_j / pi; the
raster moves and scales with the map (beta scales as 1 / s^2); a mirrored map
gives a mirrored raster. The bandwidths come from the perplexity search,
pinned in test_oracle_pins.py; here the 2-D form is checked by brute-force
entropy.
"""
import math

import numpy as np
import pytest

from oracle import pakde
from paper_1812_09869_amd import synth


def _map(n=120, seed=3):
    lab = np.random.Generator(np.random.PCG64(seed)).integers(0, 4, n)
    return synth.clustered_state(lab, seed=seed + 1, spread=6.0).astype(np.float64)


def test_bandwidth_entropy_brute_force():
    y = _map()
    beta = pakde.bandwidths(y, 10.0)
    for j in (0, 17, 99):
        d = ((y - y[j]) ** 2).sum(axis=1)
        d = np.delete(d, j)
        p = np.exp(-beta[j] * (d - d.min()))
        p /= p.sum()
        assert -(p * np.log(p + 1e-300)).sum() == pytest.approx(math.log(10.0), abs=1e-9)


def test_raster_mass_is_one():
    y = _map()
    beta = pakde.bandwidths(y, 10.0)
    h = 1.0 / math.sqrt(beta.max())  # narrowest kernel
    lo, hi = y.min(axis=0) - 12.0 / math.sqrt(beta.min()), y.max(axis=0) + 12.0 / math.sqrt(beta.min())
    c = h / 6.0
    gx, gy = int((hi[0] - lo[0]) / c) + 1, int((hi[1] - lo[1]) / c) + 1
    f = pakde.raster(y, beta, lo[0], lo[1], c, c, gx, gy)
    assert f.sum() == pytest.approx(1.0, abs=1e-6)


def test_isolated_kernel_at_its_centre():
    """Three points far apart on a line: at a cell centred on a point the
    other kernels vanish and f = (S / n) beta_j / pi."""
    y = np.array([[0.0, 0.0], [1000.0, 0.0], [2000.0, 0.0]])
    beta = np.array([0.5, 2.0, 1.0])
    f = pakde.raster(y, beta, 999.95, -0.05, 0.1, 0.1, 1, 1)  # one cell centred on y_1
    assert f[0, 0] == pytest.approx(0.01 / 3 * 2.0 / math.pi, rel=1e-14)


def test_raster_follows_translation_and_scale():
    y = _map(60, 7)
    beta = pakde.bandwidths(y, 8.0)
    f = pakde.raster(y, beta, -20.0, -20.0, 0.5, 0.5, 80, 80)
    g = pakde.raster(y + [3.0, -2.0], beta, -17.0, -22.0, 0.5, 0.5, 80, 80)
    np.testing.assert_allclose(g, f, rtol=1e-10, atol=1e-18)
    s = 2.5
    beta_s = pakde.bandwidths(s * y, 8.0)
    np.testing.assert_allclose(beta_s, beta / s ** 2, rtol=1e-7)
    fs = pakde.raster(s * y, beta_s, -20.0 * s, -20.0 * s, 0.5 * s, 0.5 * s, 80, 80)
    np.testing.assert_allclose(fs, f, rtol=1e-6, atol=1e-14)


def test_mirrored_map_mirrors_the_raster():
    y = _map(50, 9)
    beta = pakde.bandwidths(y, 6.0)
    f = pakde.raster(y, beta, -20.0, -20.0, 0.8, 0.8, 50, 50)
    g = pakde.raster(y * [-1.0, 1.0], beta, -20.0, -20.0, 0.8, 0.8, 50, 50)
    np.testing.assert_allclose(g, f[:, ::-1], rtol=1e-10, atol=1e-18)


def test_spot_cells_equal_the_raster():
    """raster_at (spot checks on rasters too large to form) gives the raster's values at
    the chosen cells, corners and ragged last row and column included."""
    y = _map(70, 11)
    beta = pakde.bandwidths(y, 9.0)
    f = pakde.raster(y, beta, -18.0, -21.0, 0.7, 0.6, 53, 47)
    rng = np.random.Generator(np.random.PCG64(4))
    cells = np.concatenate([np.stack([rng.integers(0, 47, 40), rng.integers(0, 53, 40)], 1),
                            [[0, 0], [46, 52], [0, 52], [46, 0]]])
    got = pakde.raster_at(y, beta, -18.0, -21.0, 0.7, 0.6, cells)
    np.testing.assert_allclose(got, f[cells[:, 0], cells[:, 1]], rtol=1e-12, atol=1e-300)
