"""A melt on one GPU: torch tensors own the device buffers, the C ABI does the work.

``Melt`` derives the model constants from a workload description (Re0 in grid
units, chain lengths, chiN, kappaN) and holds the buffers and the handle:

* k0 = 3 (N_ref - 1) / Re0^2, so that the ideal chain has b0^2 = 3/k0 =
  Re0^2/(N_ref - 1) (Sec. 2.1, after Eq. (9));
* local half-width a = a_frac * b0; smart-MC step A = smc_frac * Re0^2 / N_ref.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import soma as C


def make_config(w, *, seed=None, replica=0, set_order=0, origin_mode=1, p_learn=0.0,
                mu_max=1.0, sigma_min=0.02, sigma_max=1.0) -> C.soma_config:
    cfg = C.soma_config()
    cfg.nx, cfg.ny, cfg.nz = (int(v) for v in w.grid)
    cfg.n_species = len(w.species)
    for i, s in enumerate(w.species):
        cfg.species[i].n_chains = s.n_chains
        cfg.species[i].n = s.n
        cfg.species[i].n_a = s.n_a
        cfg.species[i].k0 = float(np.float32(3.0 * (w.n_ref - 1) / w.re_cells ** 2))
    cfg.n_ref = w.n_ref
    cfg.chi_n = w.chi_n
    cfg.kappa_n = w.kappa_n
    b0 = w.re_cells / math.sqrt(w.n_ref - 1)
    cfg.local_a = float(np.float32(w.a_frac * b0))
    cfg.smc_a = float(np.float32(w.smc_frac * w.re_cells ** 2 / w.n_ref))
    cfg.seed = w.seed if seed is None else seed
    cfg.replica = replica
    cfg.count_width = w.count_width
    cfg.set_order = set_order
    cfg.origin_mode = origin_mode
    cfg.p_learn = p_learn
    cfg.mu_max = mu_max
    cfg.log_sigma_min = math.log(sigma_min)
    cfg.log_sigma_max = math.log(sigma_max)
    return cfg


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Melt:
    """Buffers + handle for one melt on one device."""

    def __init__(self, cfg: C.soma_config, positions: torch.Tensor | None = None,
                 device="cuda", stream=None):
        self.cfg = cfg
        pos_b, cnt_b, om_b, ws_b = C.soma_buffer_sizes(cfg)
        self.n_beads = pos_b // 12
        self.n_cells = cfg.nx * cfg.ny * cfg.nz
        if positions is None:
            self.pos = torch.empty((self.n_beads, 3), dtype=torch.float32, device=device)
        else:
            assert positions.shape == (self.n_beads, 3) and positions.dtype == torch.float32
            self.pos = positions.to(device).contiguous()
        cdt = torch.int32 if cfg.count_width == 16 else torch.int64
        self.counts = torch.empty(self.n_cells, dtype=cdt, device=device)
        self.omega = torch.empty((2, self.n_cells), dtype=torch.float32, device=device)
        self.n_types = 2
        self.workspace = torch.empty(ws_b, dtype=torch.uint8, device=device)
        self.buf = C.soma_buffers(self.pos.data_ptr(), pos_b, self.counts.data_ptr(), cnt_b,
                                  self.omega.data_ptr(), om_b, self.workspace.data_ptr(), ws_b)
        self.handle = C.soma_init_system(cfg, self.buf, positions is None, _stream(stream))

    def sweep(self, n_sweeps=1, move_kind=C.SOMA_MOVE_LOCAL, stream=None):
        C.soma_mc_sweep(self.handle, n_sweeps, move_kind, _stream(stream))

    def set_proposal(self, params: torch.Tensor, species=C.SOMA_ALL_SPECIES, stream=None):
        """Install the learned proposal's FP32 parameter blob (a device tensor) for
        one species or all."""
        assert params.dtype == torch.float32 and params.numel() == C.NET_PARAMS
        C.soma_set_proposal(self.handle, params.contiguous().data_ptr(), _stream(stream),
                            species)

    def update_fields(self, stream=None):
        C.soma_update_fields(self.handle, _stream(stream))

    def rebuild_histogram(self, stream=None):
        C.soma_rebuild_histogram(self.handle, _stream(stream))

    def cycle(self, n=1, move_kind=C.SOMA_MOVE_LOCAL, stream=None):
        """n SCMF cycles: the sweep, then the field refresh (per chain subset when
        sub-steps are set)."""
        C.soma_cycle(self.handle, n, move_kind, _stream(stream))

    def sync_fields(self, stream=None):
        """After writing self.omega directly: rebuild the copies the sweeps read."""
        C.soma_sync_fields(self.handle, _stream(stream))

    def keep_grad_field(self, on: bool = True, stream=None):
        """Keep the (omega, grad omega) float4 field for smart-MC moves (allocates
        32 B per cell), or drop it."""
        if on:
            self.grad = torch.empty((2, self.n_cells, 4), dtype=torch.float32,
                                    device=self.pos.device)
            C.soma_set_grad_field(self.handle, self.grad.data_ptr(), self.grad.numel() * 4,
                                  _stream(stream))
        else:
            C.soma_set_grad_field(self.handle, 0, 0, _stream(stream))
            self.grad = None

    def set_substeps(self, k: int):
        """Field refreshes per cycle (k interleaved chain subsets)."""
        C.soma_set_substeps(self.handle, k)

    def observables(self, stream=None, raise_on_flag=True) -> C.soma_obs:
        return C.soma_observables(self.handle, _stream(stream), raise_on_flag)

    @property
    def sweep_index(self) -> int:
        return C.soma_get_sweep(self.handle)

    @sweep_index.setter
    def sweep_index(self, v: int):
        C.soma_set_sweep(self.handle, v, _stream(None))

    def capture_cycle(self, cycles: int, move_kind=C.SOMA_MOVE_LOCAL):
        """Record `cycles` SCMF cycles into a HIP graph (replayed by run_cycle)."""
        C.soma_capture_cycle(self.handle, cycles, move_kind)

    def run_cycle(self, n_launches: int = 1, stream=None):
        C.soma_run_cycle(self.handle, n_launches, _stream(stream))

    def autotune(self, cycles: int, move_kind=C.SOMA_MOVE_LOCAL, cache_path=None, stream=None):
        return C.soma_autotune(self.handle, cycles, move_kind, cache_path, _stream(stream))

    def set_external(self, ext=None, forbid=None, stream=None):
        """External fields: ext a device float32 tensor [2, n_cells] (or None),
        forbid a device int32/uint32 tensor of packed impenetrable-cell bits (or
        None).  The melt keeps references to both."""
        self.ext, self.forbid = ext, forbid
        C.soma_set_external(self.handle, ext.data_ptr() if ext is not None else None,
                            ext.numel() * 4 if ext is not None else 0,
                            forbid.data_ptr() if forbid is not None else None,
                            forbid.numel() * 4 if forbid is not None else 0, _stream(stream))

    def set_architecture(self, words, species: int = 0, stream=None):
        """General molecular architecture of a species (numpy uint32 array in the
        32-bit format), or None for a linear chain."""
        C.soma_set_architecture(self.handle, species, words, _stream(stream))

    def set_hamiltonian(self, form: int, stream=None):
        """Interaction term: 1 = chiN phi_A phi_B (default), 0 = -chiN/4 (phi_A - phi_B)^2."""
        C.soma_set_hamiltonian(self.handle, form, _stream(stream))

    def set_types(self, chi_n, stream=None):
        """n_t bead types with the symmetric matrix chi_n (n_t x n_t, chi_ij N):
        count and field buffers with a plane per type pair and per type
        replace the two-type ones; the histogram and fields are rebuilt."""
        chi = np.asarray(chi_n, dtype=np.float32)
        n_t = chi.shape[0]
        planes = (n_t + 1) // 2
        cdt = self.counts.dtype
        counts = torch.zeros(planes * self.n_cells, dtype=cdt, device=self.pos.device)
        omega = torch.empty((n_t, self.n_cells), dtype=torch.float32, device=self.pos.device)
        C.soma_set_types(self.handle, n_t, chi, counts.data_ptr(),
                         counts.numel() * counts.element_size(), omega.data_ptr(),
                         omega.numel() * 4, _stream(stream))
        self.counts, self.omega, self.n_types = counts, omega, n_t

    def type_counts(self, stream=None):
        """Total count of every bead type in the kept histogram."""
        return C.soma_type_counts(self.handle, self.n_types, _stream(stream))

    def set_scheme(self, scheme: int):
        """Iteration order of local moves: C.SOMA_SCHEME_SET or C.SOMA_SCHEME_MOLECULE."""
        C.soma_set_scheme(self.handle, scheme)

    def set_histogram(self, mode: int):
        """Count updates of SET sweeps: C.SOMA_HIST_DIRECT or C.SOMA_HIST_BINNED."""
        C.soma_set_histogram(self.handle, mode)

    def choose_scheme(self, cycles: int, stream=None):
        """Times both orders and keeps the faster; returns (scheme, [ms SET, ms MOLECULE])."""
        return C.soma_choose_scheme(self.handle, cycles, _stream(stream))

    def counts_planes(self) -> np.ndarray:
        """Unpack the packed counts to uint32 [n_types, n_cells] on the host."""
        n_t = self.n_types
        c = self.counts.cpu().numpy().reshape(-1, self.n_cells)
        if self.cfg.count_width == 16:
            u = c.view(np.uint32)
            lo, hi = u & 0xFFFF, u >> 16
        else:
            u = c.view(np.uint64)
            lo, hi = u & 0xFFFFFFFF, u >> 32
        out = np.empty((2 * u.shape[0], self.n_cells), np.uint32)
        out[0::2], out[1::2] = lo, hi
        return out[:n_t]

    def close(self):
        if self.handle:
            C.soma_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several melts swept by one launch per sweep (and per field refresh)."""

    def __init__(self, melts, stream=None):
        self.melts = list(melts)   # the melts must outlive the batch
        handles = [m.handle for m in self.melts]
        ws_b = C.soma_batch_workspace_size(handles)
        self.workspace = torch.empty(ws_b, dtype=torch.uint8, device=self.melts[0].pos.device)
        self.handle = C.soma_batch_create(handles, self.workspace.data_ptr(), ws_b,
                                          _stream(stream))

    def set_launch(self, mode: int, grid_blocks: int = 0):
        C.soma_batch_set_launch(self.handle, mode, grid_blocks)

    def set_histogram(self, mode: int):
        C.soma_batch_set_histogram(self.handle, mode)

    def sweep(self, n_sweeps=1, move_kind=C.SOMA_MOVE_LOCAL, stream=None):
        C.soma_batch_sweep(self.handle, n_sweeps, move_kind, _stream(stream))

    def update_fields(self, stream=None):
        C.soma_batch_update_fields(self.handle, _stream(stream))

    def cycle(self, n=1, move_kind=C.SOMA_MOVE_LOCAL, stream=None):
        C.soma_batch_cycle(self.handle, n, move_kind, _stream(stream))

    def set_substeps(self, k: int, stream=None):
        C.soma_batch_set_substeps(self.handle, k, _stream(stream))

    def capture_cycle(self, cycles: int, move_kind=C.SOMA_MOVE_LOCAL):
        C.soma_batch_capture_cycle(self.handle, cycles, move_kind)

    def run_cycle(self, n_launches: int = 1, stream=None):
        C.soma_batch_run_cycle(self.handle, n_launches, _stream(stream))

    def autotune(self, cycles: int, move_kind=C.SOMA_MOVE_LOCAL, cache_path=None, stream=None):
        return C.soma_batch_autotune(self.handle, cycles, move_kind, cache_path, _stream(stream))

    def close(self):
        if self.handle:
            C.soma_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
