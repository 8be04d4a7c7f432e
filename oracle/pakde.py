"""FP64 oracle of the perplexity-adaptive kernel density estimate (paKDE),
section "Perplexity-adaptive Kernel Density Estimation".

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The estimator is the sample smoothing estimator with locally scaled bivariate
Gaussian kernels:
  f(c) = (S / n) sum_j h_j^{-2} K((c - y_j) / h_j),
  K_j = (1 / pi) exp(-beta_j |c - y_j|^2),  h_j^2 = 2 sigma_j^2 = 1 / beta_j,
so that f(c) = (S / n) sum_j (beta_j / pi) exp(-beta_j |c - y_j|^2), evaluated
at the centres c of a regular raster with cells of area S. beta_j comes from
the same perplexity search as the input affinities (Eqs. 1-2), run on the
2-D map: the squared map distances |y_j - y_k|^2 in place of |x_j - x_k|^2.

Readings: the raster is the caller's (origin, cell sizes, cell counts), each
cell evaluated at its centre; f(c) is the probability mass of the cell (the
factor S), so the raster sums to about 1 when it covers the map.
"""
from __future__ import annotations

import numpy as np

from . import calibrate


def bandwidths(y, perplexity: float) -> np.ndarray:
    """beta_j of every map point: the perplexity search on the 2-D map (Eqs. 1-2)."""
    return calibrate(np.asarray(y, dtype=np.float64), perplexity).beta


def cell_centres(x0: float, y0: float, cx: float, cy: float, gx: int, gy: int):
    """Centres of a gy x gx raster whose cell (v, u) spans
    [x0 + u cx, x0 + (u + 1) cx] x [y0 + v cy, y0 + (v + 1) cy]."""
    u = x0 + (np.arange(gx) + 0.5) * cx
    v = y0 + (np.arange(gy) + 0.5) * cy
    return np.meshgrid(u, v)  # each gy x gx


def raster(y, beta, x0: float, y0: float, cx: float, cy: float, gx: int, gy: int) -> np.ndarray:
    """f(c) on the raster (gy x gx), the sum over points taken in point order."""
    y = np.asarray(y, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    n = y.shape[0]
    cu, cv = cell_centres(x0, y0, cx, cy, gx, gy)
    f = np.zeros((gy, gx))
    for j in range(n):
        f += (beta[j] / np.pi) * np.exp(-beta[j] * ((cu - y[j, 0]) ** 2 + (cv - y[j, 1]) ** 2))
    return f * (cx * cy / n)


def raster_at(y, beta, x0: float, y0: float, cx: float, cy: float, cells) -> np.ndarray:
    """f(c) at the centres of the given cells (v, u) of the same raster, for
    spot checks where the whole raster is too large: the same sum as
    raster(), over the points in point order."""
    y = np.asarray(y, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.int64)
    cu = x0 + (cells[:, 1] + 0.5) * cx
    cv = y0 + (cells[:, 0] + 0.5) * cy
    f = np.zeros(cells.shape[0])
    for j in range(y.shape[0]):
        f += (beta[j] / np.pi) * np.exp(-beta[j] * ((cu - y[j, 0]) ** 2 + (cv - y[j, 1]) ** 2))
    return f * (cx * cy / y.shape[0])


def pakde(y, perplexity: float, x0, y0, cx, cy, gx, gy):
    """(beta, raster) of the paKDE of a 2-D map."""
    beta = bandwidths(y, perplexity)
    return beta, raster(y, beta, x0, y0, cx, cy, gx, gy)
