"""Training the learned proposal from trajectories of the plain sampler.

Data: for beads picked at random, the 60 features at cycle t and the
displacement r(t + K) - r(t) after K further SCMF cycles of the plain move
(``soma_collect_training``).  The network fits a Gaussian to that
displacement (negative log-likelihood, ``soma_train_step``); used as a
Metropolis-Hastings proposal it moves a bead further per attempt than the
plain local move, while the acceptance test keeps the sampled distribution
exact.  Every step runs in the library's kernels; torch only owns the
buffers, and batches are contiguous slices of the collected data (samples of
a round are already random beads).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import soma as C

LAYOUT = {"shift": 0, "scale": 60, "w1": 120, "b1": 3960, "w2": 4024, "b2": 8120,
          "w3": 8184, "b3": 8568, "size": 8576}


def _stream():
    return torch.cuda.current_stream().cuda_stream


def collect(melt, n_per_round: int, lag: int, rounds: int, move=C.SOMA_MOVE_LOCAL,
            first_round: int = 0, frozen_field: bool = False, species=C.SOMA_ALL_SPECIES):
    """(features [rounds*n, 60], displacements [rounds*n, 3]) on the device: each
    round records n random beads, runs `lag` SCMF cycles with `move` (sweeps
    without field refresh if `frozen_field`), and records their displacements.
    `species` restricts the beads to one species (per-species networks)."""
    n = n_per_round
    feats = torch.empty((rounds * n, 60), dtype=torch.float32, device="cuda")
    disp = torch.empty((rounds * n, 3), dtype=torch.float32, device="cuda")
    r0 = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    s = _stream()
    for k in range(rounds):
        f_ptr = feats.data_ptr() + k * n * 60 * 4
        d_ptr = disp.data_ptr() + k * n * 3 * 4
        C.soma_collect_training(melt.handle, n, first_round + k, 0, f_ptr, r0.data_ptr(), 0, 0, s,
                                species)
        if frozen_field:
            melt.sweep(lag, move)
        else:
            melt.cycle(lag, move)
        C.soma_collect_training(melt.handle, n, first_round + k, 1, 0, r0.data_ptr(), d_ptr, 0, s,
                                species)
    return feats, disp


def init_params(features: torch.Tensor, seed: int = 0, out_gain: float = 0.01,
                stats_rows: int = 65536) -> torch.Tensor:
    """Random weights; standardisation constants (mean, 1/std per feature) from the
    first `stats_rows` samples (host statistics of the training data)."""
    gen = np.random.default_rng(seed)
    L = LAYOUT
    p = np.zeros(L["size"], np.float32)
    sample = features[:stats_rows].cpu().numpy().astype(np.float64)
    mean = sample.mean(0)
    std = sample.std(0)
    p[L["shift"]:L["shift"] + 60] = mean
    p[L["scale"]:L["scale"] + 60] = 1.0 / np.maximum(std, 1e-6)
    p[L["w1"]:L["w1"] + 3840] = gen.standard_normal(3840) / math.sqrt(60)
    p[L["w2"]:L["w2"] + 4096] = gen.standard_normal(4096) / math.sqrt(64)
    p[L["w3"]:L["w3"] + 384] = gen.standard_normal(384) * out_gain / math.sqrt(64)
    return torch.from_numpy(p).cuda()


class Trainer:
    """Adam state and workspace for ``soma_train_step`` over one data set."""

    def __init__(self, params: torch.Tensor, *, lr=3e-3, mu_max=1.0, sigma_min=0.02,
                 sigma_max=1.0, max_waves=512):
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.ws_bytes = C.soma_train_workspace_bytes(max_waves)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.opts = C.soma_train_opts(lr, 0.9, 0.999, 1e-8, mu_max, math.log(sigma_min),
                                      math.log(sigma_max), 1, max_waves)
        self.step = 0

    def run(self, features: torch.Tensor, targets: torch.Tensor, *, steps: int,
            batch: int = 4096, seed: int = 0, loss_every: int = 1):
        """`steps` Adam steps on contiguous batches in a seeded order; returns the
        losses of every `loss_every`-th step (host floats)."""
        n_batches = features.shape[0] // batch
        assert n_batches >= 1, "fewer samples than one batch"
        order = np.random.default_rng(seed).permutation(n_batches)
        s = _stream()
        out = []
        for k in range(steps):
            b = int(order[k % n_batches])
            self.step += 1
            record = (k % loss_every) == 0 or k == steps - 1
            C.soma_train_step(features.data_ptr() + b * batch * 60 * 4,
                              targets.data_ptr() + b * batch * 3 * 4, batch,
                              self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                              self.step, self.opts, self.ws.data_ptr(), self.ws_bytes, 0,
                              self.loss.data_ptr() if record else 0, s)
            if record:
                out.append(float(self.loss.item()))
        return out


def train(params, features, targets, *, steps, batch=4096, lr=3e-3, mu_max=1.0,
          sigma_min=0.02, sigma_max=1.0, seed=0, max_waves=512, loss_every=1):
    """Convenience: a fresh Trainer for `steps` Adam steps."""
    t = Trainer(params, lr=lr, mu_max=mu_max, sigma_min=sigma_min, sigma_max=sigma_max,
                max_waves=max_waves)
    return t.run(features, targets, steps=steps, batch=batch, seed=seed, loss_every=loss_every)
