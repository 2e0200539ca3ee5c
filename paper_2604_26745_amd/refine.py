"""Learned refinement for the safeguarded Deep Gauss-Newton loop.

The learned step G_k : (u_k, s_k) -> u~ of Sec. 3 sits outside the kernels:
the LM solver (``pget.Plan.lm_solve``) calls it after every accepted step
and keeps its proposal only when the safeguard of Prop. 3.2 / Alg. 2 holds
(evaluated on the device).  This module holds

* ``RefineCNN``: the encoder-decoder network of the paper's CNN figure --
  two encoders (u and s, 2 -> 8 -> 16 -> 32 channels, ReLU(conv) each), their
  sum, a decoder (32 -> 32 -> 16 -> 8 ReLU(conv), then conv to 2), a
  bias-free 5x5 convolution L(s), and the output ReLU(u + dec * L(s)).  The
  paper names 5x5 kernels and 28 104 parameters, which cannot both hold for
  these channel counts (5x5 everywhere gives 75 070); the reading here uses
  3x3 kernels in encoders and decoder and 5x5 for L: 27 198 parameters.
  Inputs are scaled by their upper bounds (by default emission 1 and
  attenuation 0.14 /mm, the scanner phantoms' ranges) and the output scaled
  back; pixels outside the field-of-view disk are 0.
* ``collect_steps``: the LM step s_k = LMA(u_k) for a set of samples, i.e.
  the first accepted step of an LM solve started at u_k (Alg. 1).
* ``train_stage``: one network of Alg. 1 (Adam with weight decay, mean
  squared error to the ground truth, inputs and targets rotated together by
  a random angle in [-5, 5] degrees per sample and epoch).
* ``train_networks``: Alg. 1 for k = 0 .. K-1.
* ``deep_gn_solve``: Alg. 2 through the solver's hook, G_k for the k-th
  accepted step (the last network for later ones).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import pget


def _torch():
    import torch
    return torch


def build_cnn(f_max: float = 1.0, mu_max: float = 0.14, mask: Optional[np.ndarray] = None):
    torch = _torch()
    nn = torch.nn

    def enc():
        return nn.Sequential(
            nn.Conv2d(2, 8, 3, padding=1), nn.ReLU(),
            nn.Conv2d(8, 16, 3, padding=1), nn.ReLU(),
            nn.Conv2d(16, 32, 3, padding=1), nn.ReLU())

    class RefineCNN(nn.Module):
        def __init__(self):
            super().__init__()
            self.enc_u = enc()
            self.enc_s = enc()
            self.dec = nn.Sequential(
                nn.Conv2d(32, 32, 3, padding=1), nn.ReLU(),
                nn.Conv2d(32, 16, 3, padding=1), nn.ReLU(),
                nn.Conv2d(16, 8, 3, padding=1), nn.ReLU(),
                nn.Conv2d(8, 2, 3, padding=1))
            self.L = nn.Conv2d(2, 2, 5, padding=2, bias=False)
            self.register_buffer("scale", torch.tensor([f_max, mu_max], dtype=torch.float32).view(1, 2, 1, 1))
            m = torch.ones(1, 1, 1, 1) if mask is None else torch.tensor(mask, dtype=torch.float32)[None, None]
            self.register_buffer("mask", m)

        def forward(self, u, s):
            """u, s: (B, 2, N, N) physical units -> u~ (B, 2, N, N)."""
            un, sn = u / self.scale, s / self.scale
            d = self.dec(self.enc_u(un) + self.enc_s(sn))
            out = torch.relu(un + d * self.L(sn))
            return out * self.scale * self.mask

    return RefineCNN()


def n_params(model) -> int:
    return sum(p.numel() for p in model.parameters() if p.requires_grad)


def rotate(x, angles_deg):
    """Rotate each image of (B, C, N, N) about its centre (bilinear, zero fill)."""
    torch = _torch()
    th = torch.as_tensor(angles_deg, dtype=x.dtype, device=x.device) * (math.pi / 180.0)
    c, s = torch.cos(th), torch.sin(th)
    z = torch.zeros_like(c)
    A = torch.stack([torch.stack([c, -s, z], -1), torch.stack([s, c, z], -1)], 1)
    grid = torch.nn.functional.affine_grid(A, list(x.shape), align_corners=False)
    return torch.nn.functional.grid_sample(x, grid, mode="bilinear", padding_mode="zeros", align_corners=False)


def collect_steps(plan: "pget.Plan", ys, us, params: "pget.SolverParams", max_tries: int = 6):
    """s_k = LMA(u_k) for every sample: the first accepted step of an LM
    solve from u_k (at most max_tries outer iterations; zero if none is
    accepted).  us: list of (f, mu) device tensors.  Returns a list of
    (s_f, s_mu) tensors."""
    torch = _torch()
    steps = []
    for y, (f, mu) in zip(ys, us):
        got = []

        def capture(f_, mu_, sf, sm):
            if not got:
                got.append((sf.clone(), sm.clone()))
            return f_ + sf, mu_ + sm          # the LM point itself: kept, and the solve stops
        prm = pget.SolverParams(**{**params.__dict__, "max_outer": max_tries, "tol": 1e30, "replay": None})
        plan.lm_solve(y, f, mu, prm, hook=capture)
        steps.append(got[0] if got else (torch.zeros_like(f), torch.zeros_like(mu)))
    return steps


def train_stage(model, U, S, Ut, epochs: int = 60, batch: int = 16, lr: float = 2e-3,
                weight_decay: float = 1e-6, max_rot: float = 5.0, seed: int = 0, log=None):
    """One network of Alg. 1.  U, S, Ut: (n, 2, N, N) device tensors
    (iterates, LM steps, ground truths)."""
    torch = _torch()
    g = torch.Generator(device="cpu").manual_seed(seed)
    opt = torch.optim.Adam(model.parameters(), lr=lr, weight_decay=weight_decay)
    n = U.shape[0]
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g)
        tot = 0.0
        for i in range(0, n, batch):
            idx = perm[i:i + batch].to(U.device)
            ang = (torch.rand(idx.numel(), generator=g) * 2.0 - 1.0) * max_rot
            u, s, t = (rotate(X[idx], ang) for X in (U, S, Ut))
            loss = torch.mean((model(u, s) - t) ** 2)
            opt.zero_grad()
            loss.backward()
            opt.step()
            tot += float(loss) * idx.numel()
        if log and (ep + 1) % max(1, epochs // 4) == 0:
            log("  epoch %d loss %.3e" % (ep + 1, tot / n))
    return model


@dataclass
class TrainReport:
    n_params: int = 0
    loss_before: List[float] = field(default_factory=list)
    loss_after: List[float] = field(default_factory=list)


def train_networks(plan, ys, u0s, truths, params, K: int = 3, epochs: int = 60, mask=None, log=None,
                   seed: int = 0, f_max: float = 1.0, mu_max: float = 0.14) -> Tuple[list, TrainReport]:
    """Alg. 1: for k = 0..K-1 collect s_k = LMA(u_k), train G_k on
    ((u_k, s_k); u_dagger), and move every sample to u_{k+1} = G_k(u_k, s_k)."""
    torch = _torch()
    us = [(f.clone(), mu.clone()) for f, mu in u0s]
    Ut = torch.stack([torch.stack(t) for t in truths]).float()
    models, rep = [], TrainReport()
    for k in range(K):
        steps = collect_steps(plan, ys, us, params)
        U = torch.stack([torch.stack(u) for u in us])
        S = torch.stack([torch.stack(s) for s in steps])
        torch.manual_seed(seed + k)
        model = build_cnn(f_max, mu_max, mask=mask).to(U.device)
        rep.n_params = n_params(model)
        with torch.no_grad():
            rep.loss_before.append(float(torch.mean((U + S - Ut) ** 2)))
        train_stage(model, U, S, Ut, epochs=epochs, seed=seed + k, log=log)
        model.eval()
        with torch.no_grad():
            out = torch.cat([model(U[i:i + 16], S[i:i + 16]) for i in range(0, U.shape[0], 16)])
            rep.loss_after.append(float(torch.mean((out - Ut) ** 2)))
        if log:
            log("stage %d: mse of the LM point %.3e, of G_k %.3e" % (k, rep.loss_before[-1], rep.loss_after[-1]))
        us = [(out[i, 0].contiguous(), out[i, 1].contiguous()) for i in range(out.shape[0])]
        models.append(model)
    return models, rep


def deep_gn_solve(plan, y, f0, mu0, params, models: Sequence, stats: Optional[dict] = None):
    """Alg. 2: the LM solve with G_k offered after the k-th accepted step."""
    torch = _torch()
    calls = [0]

    def hook(f, mu, sf, sm):
        k = min(calls[0], len(models) - 1)
        calls[0] += 1
        with torch.no_grad():
            out = models[k](torch.stack([f, mu])[None], torch.stack([sf, sm])[None])[0]
        return out[0].contiguous(), out[1].contiguous()

    f, mu, rb = plan.lm_solve(y, f0, mu0, params, hook=hook)
    if stats is not None:
        stats["hook_calls"] = calls[0]
    return f, mu, rb
