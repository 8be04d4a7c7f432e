"""FP64 CPU oracle of the exact t-SNE hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only users. The product package never imports this
module, and this module imports nothing from the product package.

Each function restates the part of the method it follows; the arithmetic
itself lives in ``tsne_oracle.c`` (and ``mlp_oracle.c`` for the surrogate
network), in double precision.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_d = ctypes.c_double

DEFAULT_TOL = 1e-12
DEFAULT_MAX_ITER = 200


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path):
        _build.build()
    lib = ctypes.CDLL(path)
    sig = {
        "orc_sqdist": (None, [_f64p, _i64, _i32, _f64p]),
        "orc_calibrate": (None, [_f64p, _i64, _i32, _d, ctypes.c_void_p, _i64, ctypes.c_int, _d,
                                 _f64p, _f64p, _f64p, _f64p, _i32p]),
        "orc_joint_p": (None, [_f64p, _i64, _i32, _f64p, _f64p, _f64p, _f64p]),
        "orc_calibrate_dissim": (None, [_f64p, _i64, _d, ctypes.c_int, _d, _f64p, _f64p, _f64p,
                                        _f64p, _i32p]),
        "orc_joint_p_dissim": (None, [_f64p, _i64, _f64p, _f64p, _f64p, _f64p]),
        "orc_p_entries": (None, [_f64p, _i64, _i32, _i64p, _i64p, _i64, _f64p, _f64p, _f64p,
                                 _f64p, _f64p, _f64p, _f64p]),
        "orc_p_rows": (None, [_f64p, _i64, _i32, _i64p, _i64, _f64p, _f64p, _f64p, _f64p]),
        "orc_p_entropy_term": (_d, [_f64p, _i64]),
        "orc_gradient_rows": (None, [_f64p, _i64, _f64p, _i64p, _i64, _d, _d, _f64p]),
        "orc_kl_rows": (None, [_f64p, _i64, _f64p, _i64p, _i64, _d, _f64p]),
        "orc_z": (_d, [_f64p, _i64]),
        "orc_gradient": (None, [_f64p, _i64, _f64p, _d, _f64p, ctypes.POINTER(_d)]),
        "orc_repulsion_rows": (None, [_f64p, _i64, _i64p, _i64, _d, _f64p]),
        "orc_cost": (None, [_f64p, _i64, _f64p, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
        "orc_step": (None, [_f64p, _i64, _f64p, _f64p, _f64p, _d, _d, _d, _d, ctypes.c_int,
                            ctypes.c_void_p, ctypes.c_void_p]),
        "orc_adaptive_eta": (_d, [_f64p, _i64]),
        "orc_embedding_size": (_d, [_f64p, _i64]),
        "orc_step_range": (None, [_f64p, _i64, _f64p, _f64p, _d, _d, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
        "orc_knn_overlap": (_d, [_f64p, _i64, _i32, _f64p, _i64p, _i64, ctypes.c_int]),
        "orc_mlp_param_count": (_i64, [ctypes.c_int, ctypes.c_int]),
        "orc_bf16_round": (None, [_f64p, _i64, _f64p]),
        "orc_mlp_forward": (None, [_f64p, ctypes.c_int, ctypes.c_int, _f64p, _f64p, _f64p, _i64,
                                   ctypes.c_int, _f64p]),
        "orc_mlp_gradient": (_d, [_f64p, ctypes.c_int, ctypes.c_int, _f64p, _f64p, _f64p, _f64p,
                                  _i64, ctypes.c_int, _f64p]),
        "orc_adam": (None, [_f64p, _f64p, _f64p, _f64p, _i64, _d, _d, _d, _d, ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# --------------------------------------------------------------------------
# Input similarities and calibration (Eqs. 1-2)
# --------------------------------------------------------------------------

def sqdist(x) -> np.ndarray:
    """Full matrix of squared Euclidean distances, direct-difference form."""
    x = _f64(x)
    n, d = x.shape
    out = np.empty((n, n), dtype=np.float64)
    _load().orc_sqdist(x, n, d, out)
    return out


@dataclass
class RowStats:
    beta: np.ndarray  # Gaussian precision per row (Eq. 1)
    m: np.ndarray  # row minimum of d_ij, j != i (shift of the exponent)
    S: np.ndarray  # sum_{j != i} exp(-beta (d_ij - m)) at the returned beta
    H: np.ndarray  # entropy of p_{.|i} in nats at the returned beta
    iters: np.ndarray  # evaluations used; negative if the row did not converge


def calibrate(x, perplexity: float, rows=None, max_iter: int = DEFAULT_MAX_ITER,
              tol: float = DEFAULT_TOL) -> RowStats:
    """Per-row bisection on beta so that H(p_{.|i}) = ln(perplexity) (Eqs. 1-2).

    ``rows`` limits the work to the listed rows (distances are recomputed per
    row, nothing of size n^2 is stored); outputs follow the order of ``rows``.
    """
    x = _f64(x)
    n, d = x.shape
    if rows is None:
        nr, rp = n, None
    else:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nr, rp = rows.shape[0], rows.ctypes.data_as(ctypes.c_void_p)
    beta, m, S, H = (np.empty(nr) for _ in range(4))
    iters = np.empty(nr, dtype=np.int32)
    _load().orc_calibrate(x, n, d, float(perplexity), rp, nr, int(max_iter), float(tol),
                          beta, m, S, H, iters)
    return RowStats(beta, m, S, H, iters)


# --------------------------------------------------------------------------
# Joint P (Eq. 3)
# --------------------------------------------------------------------------

def joint_p(x, st: RowStats) -> np.ndarray:
    """Full square P, p_ij = (p_{j|i} + p_{i|j}) / (2n), zero diagonal."""
    x = _f64(x)
    n, d = x.shape
    out = np.empty((n, n), dtype=np.float64)
    _load().orc_joint_p(x, n, d, _f64(st.beta), _f64(st.m), _f64(st.S), out)
    return out


def calibrate_dissim(dis, perplexity: float, max_iter: int = DEFAULT_MAX_ITER,
                     tol: float = DEFAULT_TOL) -> RowStats:
    """Row calibration (Eqs. 1-2) from a given n x n dissimilarity matrix; the
    dissimilarity stands for ||x_i - x_j||, so its square enters Eq. 1."""
    dis = _f64(dis)
    n = dis.shape[0]
    beta, m, S, H = (np.empty(n) for _ in range(4))
    iters = np.empty(n, dtype=np.int32)
    _load().orc_calibrate_dissim(dis, n, float(perplexity), int(max_iter), float(tol), beta, m, S,
                                 H, iters)
    return RowStats(beta, m, S, H, iters)


def joint_p_dissim(dis, st: RowStats) -> np.ndarray:
    """Full square P of Eq. 3 from a dissimilarity matrix and its row statistics."""
    dis = _f64(dis)
    n = dis.shape[0]
    out = np.empty((n, n), dtype=np.float64)
    _load().orc_joint_p_dissim(dis, n, _f64(st.beta), _f64(st.m), _f64(st.S), out)
    return out


def p_entries(x, ii, jj, st_i: RowStats, st_j: RowStats) -> np.ndarray:
    """Entries p_{ii[k], jj[k]} from the statistics of their two rows."""
    x = _f64(x)
    n, d = x.shape
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    out = np.empty(ii.shape[0])
    _load().orc_p_entries(x, n, d, ii, jj, ii.shape[0], _f64(st_i.beta), _f64(st_i.m),
                          _f64(st_i.S), _f64(st_j.beta), _f64(st_j.m), _f64(st_j.S), out)
    return out


def p_rows(x, rows, st: RowStats) -> np.ndarray:
    """Rows of P (Eq. 3) for the listed points, from the statistics of every
    row (``st`` indexed by point); (len(rows), n)."""
    x = _f64(x)
    n, d = x.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.shape[0], n))
    _load().orc_p_rows(x, n, d, rows, rows.shape[0], _f64(st.beta), _f64(st.m), _f64(st.S), out)
    return out


def p_entropy_term(P) -> float:
    """sum_{p > 0} p ln p over i != j (the constant part of Eq. 5)."""
    P = _f64(P)
    return _load().orc_p_entropy_term(P, P.shape[0])


# --------------------------------------------------------------------------
# Output side: Z, gradient, cost, update (Eqs. 4-6, 9, 10)
# --------------------------------------------------------------------------

def z(y) -> float:
    """Z = sum_{k != l} (1 + ||y_k - y_l||^2)^{-1} (denominator of Eq. 4)."""
    y = _f64(y)
    return _load().orc_z(y, y.shape[0])


def gradient(P, y, alpha: float = 1.0):
    """Eq. 6 with early exaggeration alpha on p_ij; returns (g, Z)."""
    P, y = _f64(P), _f64(y)
    g = np.empty_like(y)
    zz = _d()
    _load().orc_gradient(P, y.shape[0], y, float(alpha), g, ctypes.byref(zz))
    return g, zz.value


def repulsion_rows(y, rows, Z: float) -> np.ndarray:
    """-4 sum_j w_ij^2 (y_i - y_j) / Z for the listed rows (Eq. 6 at alpha = 0)."""
    y = _f64(y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.shape[0], 2))
    _load().orc_repulsion_rows(y, y.shape[0], rows, rows.shape[0], float(Z), out)
    return out


def gradient_rows(prows, y, rows, alpha: float, Z: float) -> np.ndarray:
    """Eq. 6 for the listed rows from their rows of P and the global Z."""
    prows, y = _f64(prows), _f64(y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.shape[0], 2))
    _load().orc_gradient_rows(prows, y.shape[0], y, rows, rows.shape[0], float(alpha), float(Z),
                              out)
    return out


def kl_rows(prows, y, rows, Z: float) -> np.ndarray:
    """Per-row shares sum_j p_ij ln(p_ij / q_ij) of the KL (Eq. 5) for the listed rows."""
    prows, y = _f64(prows), _f64(y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0])
    _load().orc_kl_rows(prows, y.shape[0], y, rows, rows.shape[0], float(Z), out)
    return out


def cost(P, y):
    """(KL of Eq. 5, pseudo-normalised cost of Eq. 9) with the true P."""
    P, y = _f64(P), _f64(y)
    kl, cn = _d(), _d()
    _load().orc_cost(P, y.shape[0], y, ctypes.byref(kl), ctypes.byref(cn))
    return kl.value, cn.value


@dataclass
class StepParams:
    alpha: float  # early exaggeration on p_ij
    mu: float  # momentum
    eta: float  # learning rate
    min_gain: float = 0.01
    recentre: bool = True


def schedule(t: int, switch: int = 250, exaggeration: float = 12.0, eta: float = 200.0):
    """Exaggeration 12 and momentum 0.5 before iteration ``switch``, then 1 and 0.8."""
    early = t < switch
    return StepParams(alpha=exaggeration if early else 1.0, mu=0.5 if early else 0.8, eta=eta)


def step(P, y, u, gains, prm: StepParams, want_grad: bool = False):
    """One update of (Y, U, G) in place (Eq. 10, descent reading, gains); returns (g, Z)."""
    for a in (y, u, gains):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    n = y.shape[0]
    g = np.empty_like(y) if want_grad else None
    zz = _d()
    _load().orc_step(_f64(P), n, y, u, gains, prm.alpha, prm.mu, prm.eta, prm.min_gain,
                     int(prm.recentre),
                     g.ctypes.data_as(ctypes.c_void_p) if g is not None else None,
                     ctypes.cast(ctypes.pointer(zz), ctypes.c_void_p))
    return g, zz.value


def run(P, y0, iters: int, start: int = 0, state=None, sched=schedule):
    """Run ``iters`` updates from Y0 (U = 0, G = 1) or from ``state`` = (Y, U, G)."""
    if state is None:
        y = _f64(y0).copy()
        u = np.zeros_like(y)
        gains = np.ones_like(y)
    else:
        y, u, gains = (np.array(a, dtype=np.float64) for a in state)
    P = _f64(P)
    for t in range(start, start + iters):
        step(P, y, u, gains, sched(t))
    return y, u, gains


def adaptive_eta(y) -> float:
    """Eq. 11: ln(n - 1) (Y_max - Y_min) / 2, Y_max - Y_min the larger coordinate range."""
    y = _f64(y)
    return _load().orc_adaptive_eta(y, y.shape[0])


def embedding_size(y) -> float:
    """Diagonal of the box spanned by the map (the embedding-size monitor)."""
    y = _f64(y)
    return _load().orc_embedding_size(y, y.shape[0])


def step_range(P, y, u, mu: float, alpha: float = 1.0, recentre: bool = True,
               want_grad: bool = False):
    """One update of (Y, U) in place with the paper's optimiser (Eqs. 10-11,
    descent reading, no gains); returns (g, Z, eta)."""
    for a in (y, u):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    n = y.shape[0]
    g = np.empty_like(y) if want_grad else None
    zz, ee = _d(), _d()
    _load().orc_step_range(_f64(P), n, y, u, float(alpha), float(mu), int(recentre),
                           g.ctypes.data_as(ctypes.c_void_p) if g is not None else None,
                           ctypes.cast(ctypes.pointer(zz), ctypes.c_void_p),
                           ctypes.cast(ctypes.pointer(ee), ctypes.c_void_p))
    return g, zz.value, ee.value


def knn_overlap(x, y, rows, k: int = 10) -> float:
    """Mean |kNN_k in X  intersect  kNN_k in Y| / k over the query rows (ties: lower index)."""
    x, y = _f64(x), _f64(y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    return _load().orc_knn_overlap(x, x.shape[0], x.shape[1], y, rows, rows.shape[0], int(k))


# --------------------------------------------------------------------------
# Surrogate network (not in the paper): 50 -> 256 -> 256 -> 2, ReLU, MSE
# --------------------------------------------------------------------------

def bf16_round(a) -> np.ndarray:
    """Round to bfloat16 (nearest even, through float), returned as float64."""
    a = _f64(a)
    out = np.empty_like(a)
    _load().orc_bf16_round(a.ravel(), a.size, out.ravel())
    return out


def mlp_param_count(d_in: int = 50, hidden: int = 256) -> int:
    return int(_load().orc_mlp_param_count(d_in, hidden))


def mlp_forward(params, x, mean, invstd, hidden: int = 256, emulate: bool = False):
    """out = W3 relu(W2 relu(W1 (x - mean) invstd + b1) + b2) + b3, rows of x."""
    x = _f64(x)
    B, d_in = x.shape
    out = np.empty((B, 2))
    _load().orc_mlp_forward(_f64(params), d_in, hidden, _f64(mean), _f64(invstd), x, B,
                            int(emulate), out)
    return out


def mlp_gradient(params, x, y, mean, invstd, hidden: int = 256, emulate: bool = False):
    """(loss, packed gradient) of L = (1/2B) sum |out - y|^2."""
    x = _f64(x)
    B, d_in = x.shape
    g = np.empty(mlp_param_count(d_in, hidden))
    loss = _load().orc_mlp_gradient(_f64(params), d_in, hidden, _f64(mean), _f64(invstd), x,
                                    _f64(y), B, int(emulate), g)
    return loss, g


def adam(p, g, m, v, lr, beta1, beta2, eps, t):
    """One Adam step (t is 1-based), in place on p, m, v (float64 arrays)."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().orc_adam(p, _f64(g), m, v, p.shape[0], lr, beta1, beta2, eps, int(t))
