"""Seeded synthetic inputs for the exact t-SNE hot path.

This module only draws random numbers. It holds none of the method's
arithmetic, so both the FP64 CPU oracle and the HIP path can take their
inputs from it without sharing any computation.

The paper evaluates on Gaussian-mixture data sets of its own (the GMMx family,
section "data sets") that are not distributed; the mixtures below stand in for
them. Every generator uses numpy's ``Generator(PCG64(seed))``, draws in FP64
and casts once to FP32, which is the precision the GPU path receives.

Workloads (sizes and recipes):

* ``plain_small``: N=2,000, D=10, 8 isotropic unit-variance components with 250
  points each, means ~ N(0, 25 I), shuffled; perplexity 30.
* ``gmm_aniso``: N=65,536 (any N may be asked for), D=50, 32 components with
  Dirichlet(1) weights and multinomial counts, means ~ N(0, 25 I), covariance
  Q diag(lambda) Q^T with Q Haar-orthogonal and lambda log-uniform in
  [0.1, 10]; shuffled; perplexity 50.
* ``subspace``: N=262,144, D=128, a 64-component unit-covariance mixture in a
  10-D subspace (means ~ N(0, 25 I_10), equal weights), embedded by a Haar
  orthonormal 128x10 basis plus isotropic noise of std 0.05; perplexity 50.
* ``batch_problem(p)``: problem p of the 64-instance batch: N ~ U{1000..20000},
  D in {10, 50}, K ~ U{4..16} isotropic equal-weight components; perplexity 30.
* ``embedding_init``: initial 2-D map ~ N(0, 1e-4 I), i.e. std 0.01.
* ``disk_init``: initial map of the parallel scheme, uniform in the unit disk
  (section "Parallelized implementation").
* ``epoch_orders``: one random permutation of the points per epoch (the
  master's mixing draw of the parallel scheme).
* ``mesh_graph_distances``: stand-in for the paper's dwt1005 set (a 3-D mesh
  given as shortest-path distances between its 1,005 nodes): a closed
  cylinder mesh of 15 x 67 nodes with grid edges, hop-count shortest paths.
* ``digits_like``: stand-in for the whitened 30-D digits set of the paper's
  rounds figure: N=60,000, D=30, 10 anisotropic components (Dirichlet(5)
  weights, means ~ N(0, 25 I), covariance log-uniform in [0.1, 10] along Haar
  axes); run with 120 threads, 2 layers and perplexity 400.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Mixture",
    "plain_small",
    "gmm_aniso_mixture",
    "gmm_aniso",
    "subspace",
    "batch_problem",
    "embedding_init",
    "clustered_state",
    "disk_init",
    "epoch_orders",
    "digits_like",
    "mesh_graph_distances",
    "SEEDS",
]

# Fixed seeds of the standard workloads.
SEEDS = {
    "plain_small": 1001,
    "gmm_aniso": 1002,
    "subspace": 1003,
    "init_small": 2001,
    "init_aniso": 2002,
    "surrogate_new": 5001,
    "surrogate_init": 6001,
    "digits_like": 1005,
    "pt_init": 2005,
    "pt_orders": 3005,
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _haar_orthogonal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Haar-distributed matrix with orthonormal columns (QR of a Gaussian, sign-fixed)."""
    a = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(a)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


@dataclass
class Mixture:
    """Parameters of a Gaussian mixture: weights, means and covariance factors.

    A sample of component k is ``means[k] + factors[k] @ z`` with z ~ N(0, I).
    """

    weights: np.ndarray  # (K,)
    means: np.ndarray  # (K, D)
    factors: np.ndarray  # (K, D, D)

    def sample(self, rng: np.random.Generator, n: int, counts: np.ndarray | None = None):
        k = self.weights.shape[0]
        d = self.means.shape[1]
        if counts is None:
            counts = rng.multinomial(n, self.weights)
        labels = np.repeat(np.arange(k), counts)
        x = np.empty((n, d), dtype=np.float64)
        row = 0
        for c in range(k):
            m = int(counts[c])
            if m == 0:
                continue
            z = rng.standard_normal((m, d))
            x[row:row + m] = self.means[c] + z @ self.factors[c].T
            row += m
        perm = rng.permutation(n)
        return x[perm], labels[perm]


def plain_small(n: int = 2000, seed: int = SEEDS["plain_small"]):
    """N points in D=10 from 8 isotropic unit-variance components of equal size."""
    rng = _rng(seed)
    k, d = 8, 10
    means = rng.standard_normal((k, d)) * 5.0
    base, extra = divmod(n, k)
    counts = np.full(k, base, dtype=np.int64)
    counts[:extra] += 1
    mix = Mixture(np.full(k, 1.0 / k), means, np.broadcast_to(np.eye(d), (k, d, d)).copy())
    x, lab = mix.sample(rng, n, counts)
    return x.astype(np.float32), lab


def gmm_aniso_mixture(seed: int = SEEDS["gmm_aniso"], k: int = 32, d: int = 50) -> Mixture:
    """The 32-component anisotropic mixture in D=50 (parameters only)."""
    rng = _rng(seed)
    w = rng.dirichlet(np.ones(k))
    means = rng.standard_normal((k, d)) * 5.0
    factors = np.empty((k, d, d))
    for c in range(k):
        q = _haar_orthogonal(rng, d, d)
        lam = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=d))
        factors[c] = q * np.sqrt(lam)  # Q diag(sqrt(lambda)): covariance Q diag(lambda) Q^T
    return Mixture(w, means, factors)


def gmm_aniso(n: int = 65536, seed: int = SEEDS["gmm_aniso"], sample_seed: int | None = None):
    """N points from the anisotropic 32-component mixture.

    The mixture parameters always come from ``seed``; the sample comes from
    ``sample_seed`` (default: a stream derived from ``seed``), so that fresh
    points from the same mixture can be drawn.
    """
    mix = gmm_aniso_mixture(seed)
    rng = _rng(seed * 7919 + 17 if sample_seed is None else sample_seed)
    x, lab = mix.sample(rng, n)
    return x.astype(np.float32), lab


def subspace(n: int = 262144, seed: int = SEEDS["subspace"], d: int = 128, sub: int = 10,
             k: int = 64, noise: float = 0.05):
    """Mixture of 64 unit-covariance components on a random 10-D subspace plus noise."""
    rng = _rng(seed)
    means = rng.standard_normal((k, sub)) * 5.0
    basis = _haar_orthogonal(rng, d, sub)
    lab = rng.integers(0, k, size=n)
    z = means[lab] + rng.standard_normal((n, sub))
    x = z @ basis.T + noise * rng.standard_normal((n, d))
    return x.astype(np.float32), lab


def batch_problem(p: int):
    """Problem p (0..63) of the 64-instance batch; returns (x, labels, perplexity)."""
    rng = _rng(4000 + p)
    n = int(rng.integers(1000, 20001))
    d = int(rng.choice([10, 50]))
    k = int(rng.integers(4, 17))
    means = rng.standard_normal((k, d)) * 5.0
    lab = rng.integers(0, k, size=n)
    x = means[lab] + rng.standard_normal((n, d))
    return x.astype(np.float32), lab, 30.0


def embedding_init(n: int, seed: int) -> np.ndarray:
    """Initial 2-D map, N(0, 1e-4 I) (std 0.01), cast to FP32."""
    rng = _rng(seed)
    return (rng.standard_normal((n, 2)) * 0.01).astype(np.float32)


def clustered_state(labels: np.ndarray, seed: int, spread: float = 8.0, jitter: float = 1.0):
    """A synthetic mid-run 2-D map: each cluster at a random centre plus jitter.

    Used as a state from which gradients are compared; it has the structure of
    an embedding after early exaggeration (separated blobs), without running
    any optimiser.
    """
    rng = _rng(seed)
    k = int(labels.max()) + 1
    centres = rng.standard_normal((k, 2)) * spread
    y = centres[labels] + jitter * rng.standard_normal((labels.shape[0], 2))
    return y.astype(np.float32)


def disk_init(n: int, seed: int) -> np.ndarray:
    """Initial 2-D map uniform in the disk of radius 1, cast to FP32."""
    rng = _rng(seed)
    r = np.sqrt(rng.uniform(0.0, 1.0, n))
    a = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.stack([r * np.cos(a), r * np.sin(a)], axis=1).astype(np.float32)


def epoch_orders(n: int, epochs: int, seed: int) -> np.ndarray:
    """``epochs`` independent random permutations of 0..n-1 (int32, epochs x n)."""
    rng = _rng(seed)
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)


def digits_like(n: int = 60000, seed: int = SEEDS["digits_like"], k: int = 10, d: int = 30):
    """N points from a 10-component anisotropic mixture in D=30."""
    rng = _rng(seed)
    w = rng.dirichlet(np.full(k, 5.0))
    means = rng.standard_normal((k, d)) * 5.0
    factors = np.empty((k, d, d))
    for c in range(k):
        q = _haar_orthogonal(rng, d, d)
        lam = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=d))
        factors[c] = q * np.sqrt(lam)
    x, lab = Mixture(w, means, factors).sample(rng, n)
    return x.astype(np.float32), lab


def mesh_graph_distances(around: int = 15, along: int = 67) -> np.ndarray:
    """Shortest-path (hop) distances on a cylinder mesh of around x along nodes
    (edges to the grid neighbours, wrapping around); FP32, n x n, n = 1,005."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path
    n = around * along
    idx = np.arange(n).reshape(along, around)
    rows = np.concatenate([idx.ravel(), idx[:-1].ravel()])
    cols = np.concatenate([np.roll(idx, -1, axis=1).ravel(), idx[1:].ravel()])
    g = coo_matrix((np.ones(rows.shape[0]), (rows, cols)), shape=(n, n))
    return shortest_path(g, directed=False, unweighted=True).astype(np.float32)
