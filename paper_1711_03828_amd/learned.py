"""Training the learned proposal from trajectories of the plain sampler.

Data: at sweep t, the 60 features of randomly chosen beads (``soma_features``)
and, K SCMF cycles later, the displacement of the same beads.  The network
learns a Gaussian for that displacement (negative log-likelihood); used as a
Metropolis-Hastings proposal it moves beads further per attempt than the
plain local move while the acceptance test keeps the sampled distribution
exact.  All device work runs through the C ABI (``soma_features``,
``soma_train_step``); torch only holds the buffers.
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


def collect(melt, n_per_round: int, lag: int, rounds: int, seed: int = 0, move=C.SOMA_MOVE_LOCAL):
    """(features [rounds*n, 60], displacements [rounds*n, 3]) from plain SCMF cycles."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    n_chains = sum(melt.cfg.species[i].n_chains for i in range(melt.cfg.n_species))
    feats, disp = [], []
    pos = melt.pos
    for _ in range(rounds):
        chains = torch.randint(0, n_chains, (n_per_round,), generator=g, dtype=torch.int64)
        beads = torch.empty_like(chains)
        # bead index within the chain's species
        first_bead = torch.empty_like(chains)
        off_chain, off_bead = 0, 0
        for i in range(melt.cfg.n_species):
            sp = melt.cfg.species[i]
            sel = (chains >= off_chain) & (chains < off_chain + sp.n_chains)
            nsel = int(sel.sum())
            beads[sel] = torch.randint(0, sp.n, (nsel,), generator=g, dtype=torch.int64)
            first_bead[sel] = off_bead + (chains[sel] - off_chain) * sp.n
            off_chain += sp.n_chains
            off_bead += sp.n_chains * sp.n
        idx = (first_bead + beads).cuda()
        c32 = chains.to(torch.int32).cuda()
        b32 = beads.to(torch.int32).cuda()
        f = torch.empty((n_per_round, 60), dtype=torch.float32, device="cuda")
        C.soma_features(melt.handle, c32.data_ptr(), b32.data_ptr(), n_per_round, f.data_ptr(),
                        _stream())
        r0 = pos[idx].clone()
        melt.cycle(lag, move)
        disp.append(pos[idx] - r0)
        feats.append(f)
    return torch.cat(feats), torch.cat(disp)


def init_params(features: torch.Tensor, seed: int = 0, out_gain: float = 0.01) -> torch.Tensor:
    """Random weights with standardisation constants from the data (device tensor)."""
    gen = np.random.default_rng(seed)
    L = LAYOUT
    p = np.zeros(L["size"], np.float32)
    mean = features.mean(0).cpu().numpy()
    std = features.std(0).cpu().numpy()
    p[L["shift"]:L["shift"] + 60] = mean
    p[L["scale"]:L["scale"] + 60] = 1.0 / np.maximum(std, 1e-6)
    p[L["w1"]:L["w1"] + 3840] = gen.standard_normal(3840) / math.sqrt(60)
    p[L["w2"]:L["w2"] + 4096] = gen.standard_normal(4096) / math.sqrt(64)
    p[L["w3"]:L["w3"] + 384] = gen.standard_normal(384) * out_gain / math.sqrt(64)
    return torch.from_numpy(p).cuda()


def train(params: torch.Tensor, features: torch.Tensor, targets: torch.Tensor, *, steps: int,
          batch: int = 4096, lr: float = 3e-3, mu_max=1.0, sigma_min=0.02, sigma_max=1.0,
          seed: int = 0, max_waves: int = 256):
    """Adam on mini-batches; returns the per-step losses (host list)."""
    n = features.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws_bytes = C.soma_train_workspace_bytes(max_waves)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    opts = C.soma_train_opts(lr, 0.9, 0.999, 1e-8, mu_max, math.log(sigma_min),
                             math.log(sigma_max), 1, max_waves)
    losses = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).cuda()
        fb = features[idx].contiguous()
        tb = targets[idx].contiguous()
        C.soma_train_step(fb.data_ptr(), tb.data_ptr(), fb.shape[0], params.data_ptr(),
                          m.data_ptr(), v.data_ptr(), step, opts, ws_ptr, ws_bytes, 0,
                          loss.data_ptr(), _stream())
        losses.append(loss)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    return [float(x) for x in losses]
