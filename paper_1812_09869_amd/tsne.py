"""Exact t-SNE driver over the C ABI (state handling and schedule only).

``ExactTSNE`` owns a workspace, fills it with the affinities of X and runs
the exact gradient iteration on the GPU. Every computation is a call into
libtsne355; this module only allocates tensors and chooses per-iteration
parameters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import _lib


def paper_schedule(momentum: float = 0.8) -> "Schedule":
    """The paper's own optimiser (section "Internal parametric configuration"):
    no early exaggeration, a constant external momentum and the learning rate
    of Eq. 11 computed on the device from the extent of the map."""
    return Schedule(switch=0, exaggeration=1.0, mom_early=momentum, mom_late=momentum,
                    learning_rate=0.0, lr_rule="range")


@dataclass
class Schedule:
    """Early exaggeration and momentum switch at ``switch``; constant learning rate.

    Defaults: exaggeration 12 and momentum 0.5 before iteration 250, then 1
    and 0.8; learning rate 200; gains floored at 0.01.
    """

    switch: int = 250
    exaggeration: float = 12.0
    mom_early: float = 0.5
    mom_late: float = 0.8
    learning_rate: float = 200.0
    min_gain: float = 0.01
    lr_rule: str = "gains"  # "range": the learning rate of Eq. 11, no gains

    def __call__(self, t: int):
        early = t < self.switch
        return (self.exaggeration if early else 1.0, self.mom_early if early else self.mom_late,
                self.learning_rate)


class ExactTSNE:
    def __init__(self, x: torch.Tensor, perplexity: float, dist_mode="fp64", max_bisect: int = 200,
                 tol_h: float = 1e-6, ws: torch.Tensor | None = None, reorder: bool = True,
                 implicit: bool = False):
        """implicit: keep no P and recompute it in every pass (in dist_mode)."""
        if x.dim() != 2:
            raise ValueError("x must be n x d")
        self.n, self.d = x.shape
        self.perplexity = float(perplexity)
        self.implicit = bool(implicit)
        self.dist_mode = dist_mode
        if ws is None:
            ws = (_lib.new_workspace_implicit(self.n, self.d, device=x.device, dist_mode=dist_mode)
                  if implicit else _lib.new_workspace(self.n, self.d, dist_mode, device=x.device))
        self.ws = ws
        _lib.affinities(x, perplexity, self.ws, dist_mode, max_bisect, tol_h, reorder, implicit)
        self._z = torch.zeros(1, dtype=torch.float64, device=x.device)
        self._cost = torch.zeros(2, dtype=torch.float64, device=x.device)

    @classmethod
    def from_dissimilarities(cls, dis: torch.Tensor, perplexity: float, max_bisect: int = 200,
                             tol_h: float = 1e-6):
        """Affinities from an n x n dissimilarity matrix (device FP32) instead
        of points; the iteration is the same."""
        self = cls.__new__(cls)
        self.n, self.d = dis.shape[0], 1
        self.implicit = False
        self.dist_mode = "fp64"
        self.perplexity = float(perplexity)
        self.ws = _lib.new_workspace(self.n, 1, "fp64", device=dis.device)
        _lib.affinities_dissim(dis.contiguous(), perplexity, self.ws, max_bisect, tol_h)
        self._z = torch.zeros(1, dtype=torch.float64, device=dis.device)
        self._cost = torch.zeros(2, dtype=torch.float64, device=dis.device)
        return self

    def init_state(self, y0: torch.Tensor):
        y = y0.detach().to(dtype=torch.float32).contiguous().clone()
        return y, torch.zeros_like(y), torch.ones_like(y)

    def step(self, t: int, state, sched: Schedule, grad_out=None, z_out=None):
        y, u, g = state
        alpha, mu, eta = sched(t)
        if self.implicit:
            _lib.step_implicit(self.ws, self.n, self.d, y, u, g, alpha, mu, eta, sched.min_gain,
                               True, grad_out, z_out, lr_rule=sched.lr_rule,
                               dist_mode=self.dist_mode)
        else:
            _lib.step(self.ws, self.n, y, u, g, alpha, mu, eta, sched.min_gain, True, grad_out,
                      z_out, lr_rule=sched.lr_rule)

    def run(self, state, iters: int, start: int = 0, sched: Schedule | None = None):
        sched = sched or Schedule()
        for t in range(start, start + iters):
            self.step(t, state, sched)
        return state

    def gradient(self, y: torch.Tensor, alpha: float = 1.0):
        g = torch.empty_like(y)
        if self.implicit:
            _lib.gradient_implicit(self.ws, self.n, self.d, y, alpha, g, self._z,
                                   dist_mode=self.dist_mode)
        else:
            _lib.gradient(self.ws, self.n, y, alpha, g, self._z)
        return g, self._z

    def cost(self, y: torch.Tensor):
        """Device tensor [KL, C_norm]."""
        if self.implicit:
            _lib.cost_implicit(self.ws, self.n, self.d, y, self._cost, dist_mode=self.dist_mode)
        else:
            _lib.cost(self.ws, self.n, y, self._cost)
        return self._cost

    def status(self) -> int:
        return _lib.sync_status(self.ws)

    def check(self):
        _lib.check_status(self.ws)

    def rowstats(self):
        return _lib.export_rowstats(self.ws, self.n)

    def p_rows(self, row0: int, nrows: int):
        return _lib.export_p_rows(self.ws, self.n, row0, nrows)


class BatchedTSNE:
    """Independent exact t-SNE problems advanced together (one launch per phase).

    ``problems`` is a list of (x, perplexity); each gets its own workspace and
    affinities. ``run`` advances all of them with the same schedule.
    """

    def __init__(self, problems, dist_mode="fp64"):
        self.models = [ExactTSNE(x, perp, dist_mode=dist_mode) for x, perp in problems]
        self.states = None
        self._arr = None
        self._bws = None

    def init_states(self, y0s):
        self.states = [m.init_state(y0) for m, y0 in zip(self.models, y0s)]
        self._arr = _lib.batch_problems([(m.ws, m.n, *st) for m, st in zip(self.models,
                                                                            self.states)])
        self._bws = _lib.batch_plan(self._arr, device=self.models[0].ws.device)
        return self.states

    def step(self, t: int, sched: Schedule):
        alpha, mu, eta = sched(t)
        _lib.batch_step(self._arr, self._bws, alpha, mu, eta, sched.min_gain, True,
                        lr_rule=sched.lr_rule)

    def run(self, iters: int, start: int = 0, sched: Schedule | None = None):
        sched = sched or Schedule()
        for t in range(start, start + iters):
            self.step(t, sched)
        return self.states


class PTSNE:
    """The parallel scheme (ptSNE) over the C ABI: partial t-SNEs on shared
    chunks, run for short epochs and pooled into ``layers`` maps.

    Every epoch is one ``tsne_pt_epoch`` call (mix, affinities, batched
    iterations with the rate of Eq. 11, monitors, pool, all on the device);
    this class only allocates and passes the per-epoch order.
    """

    def __init__(self, x: torch.Tensor, threads: int, layers: int, perplexity: float,
                 momentum: float = 0.8, iters: int = 0, dist_mode="fp64", reorder: bool = False):
        if x.dim() != 2:
            raise ValueError("x must be n x d")
        self.x = x.contiguous()
        self.n, self.d = x.shape
        self.opts = _lib.pt_opts(threads, layers, perplexity, momentum, iters, dist_mode, reorder)
        self.ws = _lib.pt_new_workspace(self.n, self.d, self.opts, device=x.device)
        _lib.pt_init(self.n, self.d, self.opts, self.ws)
        self.iters = _lib.pt_iterations(self.n, self.opts)
        self.epochs_per_round = int(math.isqrt(self.n))
        self.monitors = torch.zeros(2, dtype=torch.float64, device=x.device)
        self.maps = None

    def init_maps(self, y0: torch.Tensor):
        """Every layer starts at the same map y0 (n x 2)."""
        y0 = y0.detach().to(device=self.x.device, dtype=torch.float32)
        self.maps = y0.unsqueeze(0).repeat(self.opts.layers, 1, 1).contiguous()
        return self.maps

    def epoch(self, order: torch.Tensor):
        """One epoch with the given permutation (int32 device tensor of n);
        returns the device monitors {mean partial C_norm, mean layer size}."""
        _lib.pt_epoch(self.x, self.opts, order, self.maps, self.ws, self.monitors)
        return self.monitors

    def status(self) -> int:
        return _lib.pt_sync_status(self.n, self.d, self.opts, self.ws)


def pakde(y: torch.Tensor, perplexity: float, x0: float, y0: float, cx: float, cy: float,
          gx: int, gy: int):
    """Perplexity-adaptive KDE of a map (n x 2 device FP32): returns (beta, f),
    f the gy x gx raster of cell masses. Both steps run on the device."""
    n = y.shape[0]
    y = y.contiguous()
    ws = _lib.kde_new_workspace(n, device=y.device)
    beta = torch.empty(n, dtype=torch.float64, device=y.device)
    _lib.kde_bandwidths(y, perplexity, ws, beta)
    f = torch.empty((gy, gx), dtype=torch.float32, device=y.device)
    _lib.kde_raster(y, beta, x0, y0, cx, cy, gx, gy, f)
    if _lib.sync_status(ws) != 0:
        raise _lib.TsneError(_lib.sync_status(ws), "paKDE bandwidth search flagged a device condition")
    return beta, f
