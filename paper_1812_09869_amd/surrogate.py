"""Learned surrogate of the exact embedding (not in the paper).

A 50 -> 256 -> 256 -> 2 ReLU network is trained on the (x, y) pairs that the
exact path produced, then maps new points straight to the embedding. Every
forward pass, gradient and Adam step runs in libtsne355 (BF16 MFMA with FP32
accumulation for the wide layers). Exact t-SNE remains the fallback (a short
refinement seeded from the network's map) and the reference its error is
measured against.

Host-side bookkeeping only: input standardisation statistics and target
scaling are computed once on the training set (numpy, FP64); after training
the target scaling is folded into the output layer, so that ``predict`` is a
single library call.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib


class Surrogate:
    def __init__(self, d_in: int = 50, hidden: int = 256, seed: int = 6001, device="cuda"):
        self.d_in, self.hidden, self.device = d_in, hidden, torch.device(device)
        self.count = _lib.mlp_param_count(d_in, hidden)
        rng = np.random.Generator(np.random.PCG64(seed))
        H = hidden
        parts = [
            rng.standard_normal(H * d_in) * np.sqrt(2.0 / d_in), np.zeros(H),  # He-normal, ReLU
            rng.standard_normal(H * H) * np.sqrt(2.0 / H), np.zeros(H),
            rng.standard_normal(2 * H) * np.sqrt(1.0 / H), np.zeros(2),
        ]
        p = np.concatenate(parts).astype(np.float32)
        assert p.size == self.count
        self.params = torch.from_numpy(p).to(self.device)
        self.mean = torch.zeros(d_in, device=self.device)
        self.invstd = torch.ones(d_in, device=self.device)
        self._fwd_ws = None

    def _slices(self):
        H, d = self.hidden, self.d_in
        o_w3 = H * d + H + H * H + H
        return o_w3, o_w3 + 2 * H

    def fit(self, x: torch.Tensor, y: torch.Tensor, epochs: int = 100, batch: int = 1024,
            lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
            seed: int = 6002, log_every: int = 0):
        """Adam on L = (1/2B) sum |net(x) - (y - mean y) / rms(y)|^2; returns per-epoch losses."""
        n = x.shape[0]
        xh = x.detach().cpu().double().numpy()
        yh = y.detach().cpu().double().numpy()
        mu, sd = xh.mean(axis=0), xh.std(axis=0)
        sd[sd == 0] = 1.0
        self.mean = torch.from_numpy(mu.astype(np.float32)).to(self.device)
        self.invstd = torch.from_numpy((1.0 / sd).astype(np.float32)).to(self.device)
        ymean = yh.mean(axis=0)
        yrms = float(np.sqrt(((yh - ymean) ** 2).sum(axis=1).mean()))
        ys = torch.from_numpy(((yh - ymean) / yrms).astype(np.float32)).to(self.device)
        xs = x.detach().to(self.device, torch.float32).contiguous()
        ws = _lib.mlp_new_workspace(self.d_in, self.hidden, batch, True, self.device)
        grad = torch.empty_like(self.params)
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        rng = np.random.Generator(np.random.PCG64(seed))
        losses, t = [], 0
        nb = n // batch
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(self.device)
            acc = torch.zeros(1, dtype=torch.float64, device=self.device)
            for b in range(nb):
                idx = perm[b * batch:(b + 1) * batch]
                _lib.mlp_gradient(self.params, self.d_in, self.hidden, self.mean, self.invstd, xs,
                                  ys, idx, batch, grad, loss, ws)
                t += 1
                _lib.mlp_adam(self.params, grad, m, v, lr, beta1, beta2, eps, t)
                acc += loss
            losses.append(float(acc.cpu()[0]) / nb)
            if log_every and (ep + 1) % log_every == 0:
                print(f"[surrogate] epoch {ep + 1}: loss {losses[-1]:.5f}", flush=True)
        # fold the target scaling into the output layer: out = rms * out_s + mean
        o_w3, o_b3 = self._slices()
        p = self.params.cpu().double().numpy()
        p[o_w3:o_b3] *= yrms
        p[o_b3:o_b3 + 2] = p[o_b3:o_b3 + 2] * yrms + ymean
        self.params = torch.from_numpy(p.astype(np.float32)).to(self.device)
        return losses

    def predict(self, x: torch.Tensor, out: torch.Tensor | None = None, chunk: int = 65536):
        n = x.shape[0]
        if out is None:
            out = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        if self._fwd_ws is None:
            self._fwd_ws = _lib.mlp_new_workspace(self.d_in, self.hidden, chunk, False,
                                                  self.device)
        _lib.mlp_forward(self.params, self.d_in, self.hidden, self.mean, self.invstd, x, out,
                         self._fwd_ws)
        return out
