"""ctypes binding of the C ABI in ``include/soma.h`` (argument marshalling only).

Every function here has the name of the C entry point it calls; all work runs
in the HIP library ``libsoma_hip.so``.  Device memory comes from PyTorch
tensors (``tensor.data_ptr()``); streams are HIP streams
(``torch.cuda.current_stream().cuda_stream``).  If the library has not been
built this module raises on import -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsoma_hip.so")

SOMA_OK = 0
SOMA_E_INVAL = -1
SOMA_E_HIP = -2
SOMA_E_SIZE = -3
SOMA_E_UNSUPPORTED = -4
SOMA_E_DEVICE_FLAG = -5

SOMA_MOVE_LOCAL = 0
SOMA_MOVE_SMC = 1
SOMA_MOVE_MIXED = 2
SOMA_MOVE_GIBBS = 3
SOMA_SCHEME_SET = 0
SOMA_SCHEME_MOLECULE = 1
SOMA_HIST_DIRECT = 0
SOMA_HIST_BINNED = 1
SOMA_NOALLOC_TRAIN_WAVES = 128
SOMA_FLAG_POSITION = 1
SOMA_FLAG_NETWORK = 2
SOMA_ALL_SPECIES = 0xFFFFFFFF
NET_PARAMS = 8576
SOMA_MAX_SPECIES = 8
SOMA_MAX_BEADS_PER_CHAIN = 128


class soma_species(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_uint32), ("n", ctypes.c_uint32),
                ("n_a", ctypes.c_uint32), ("k0", ctypes.c_float)]


class soma_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_uint32), ("ny", ctypes.c_uint32), ("nz", ctypes.c_uint32),
                ("n_species", ctypes.c_uint32),
                ("species", soma_species * SOMA_MAX_SPECIES),
                ("n_ref", ctypes.c_uint32), ("chi_n", ctypes.c_float),
                ("kappa_n", ctypes.c_float), ("local_a", ctypes.c_float),
                ("smc_a", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("count_width", ctypes.c_uint32),
                ("set_order", ctypes.c_uint32), ("origin_mode", ctypes.c_uint32),
                ("p_learn", ctypes.c_float), ("mu_max", ctypes.c_float),
                ("log_sigma_min", ctypes.c_float), ("log_sigma_max", ctypes.c_float)]


class soma_buffers(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("pos_bytes", ctypes.c_uint64),
                ("counts", ctypes.c_void_p), ("counts_bytes", ctypes.c_uint64),
                ("omega", ctypes.c_void_p), ("omega_bytes", ctypes.c_uint64),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64)]


class soma_obs(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_uint64), ("n_beads", ctypes.c_uint64),
                ("n_chains", ctypes.c_uint64), ("count_a", ctypes.c_uint64),
                ("count_b", ctypes.c_uint64), ("accepted", ctypes.c_uint64 * 4),
                ("attempted", ctypes.c_uint64 * 4), ("re2_sum", ctypes.c_double),
                ("rg2_sum", ctypes.c_double), ("b2_sum", ctypes.c_double),
                ("e_bond", ctypes.c_double), ("e_field", ctypes.c_double),
                ("h_nb", ctypes.c_double), ("error_flags", ctypes.c_uint32),
                ("counts_conserved", ctypes.c_uint32)]


class soma_train_opts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("mu_max", ctypes.c_float),
                ("log_sigma_min", ctypes.c_float), ("log_sigma_max", ctypes.c_float),
                ("apply", ctypes.c_uint32), ("max_waves", ctypes.c_uint32)]


class soma_tune(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("grid_blocks", ctypes.c_uint32),
                ("ms_per_cycle", ctypes.c_float), ("candidates", ctypes.c_uint32),
                ("cycles_run", ctypes.c_uint32), ("from_cache", ctypes.c_uint32),
                ("hist_mode", ctypes.c_uint32), ("block_threads", ctypes.c_uint32)]


class SomaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"soma error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with "
                      "`python -m paper_1711_03828_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_u32, _u64, _i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
_pu64 = ctypes.POINTER(ctypes.c_uint64)
_pu32 = ctypes.POINTER(ctypes.c_uint32)

_SIGS = {
    "soma_buffer_sizes": ([ctypes.POINTER(soma_config), _pu64, _pu64, _pu64, _pu64], _i32),
    "soma_workspace_size": ([ctypes.POINTER(soma_config), _pu64], _i32),
    "soma_init_system": ([ctypes.POINTER(soma_config), ctypes.POINTER(soma_buffers), _u32, _P,
                          ctypes.POINTER(_P)], _i32),
    "soma_mc_sweep": ([_P, _u32, _u32, _P], _i32),
    "soma_update_fields": ([_P, _P], _i32),
    "soma_rebuild_histogram": ([_P, _P], _i32),
    "soma_set_sweep_blocks": ([_P, _u32], _i32),
    "soma_set_histogram": ([_P, _u32], _i32),
    "soma_set_sweep_threads": ([_P, _u32], _i32),
    "soma_probe_atomics": ([_P, _u64, _u64, _u32, _u32, _P], _i32),
    "soma_set_self_term": ([_P, _u32], _i32),
    "soma_set_scheme": ([_P, _u32], _i32),
    "soma_set_hamiltonian": ([_P, _u32, _P], _i32),
    "soma_set_types": ([_P, _u32, _P, _P, _u64, _P, _u64, _P], _i32),
    "soma_type_counts": ([_P, _pu64, _u32, _P], _i32),
    "soma_set_architecture": ([_P, _u32, _P, _u32, _P], _i32),
    "soma_set_external": ([_P, _P, _u64, _P, _u64, _P], _i32),
    "soma_choose_scheme": ([_P, _u32, _P, ctypes.POINTER(_u32), ctypes.POINTER(ctypes.c_float)],
                           _i32),
    "soma_observables": ([_P, ctypes.POINTER(soma_obs), _P], _i32),
    "soma_check": ([_P, _pu32, _P], _i32),
    "soma_get_sweep": ([_P, _pu64], _i32),
    "soma_set_sweep": ([_P, _u64, _P], _i32),
    "soma_set_substeps": ([_P, _u32], _i32),
    "soma_set_grad_field": ([_P, _P, _u64, _P], _i32),
    "soma_sync_fields": ([_P, _P], _i32),
    "soma_cycle": ([_P, _u32, _u32, _P], _i32),
    "soma_batch_set_substeps": ([_P, _u32, _P], _i32),
    "soma_batch_cycle": ([_P, _u32, _u32, _P], _i32),
    "soma_capture_cycle": ([_P, _u32, _u32], _i32),
    "soma_run_cycle": ([_P, _u32, _P], _i32),
    "soma_autotune": ([_P, _u32, _u32, ctypes.c_char_p, _P, ctypes.POINTER(soma_tune)], _i32),
    "soma_batch_workspace_size": ([ctypes.POINTER(_P), _u32, _pu64], _i32),
    "soma_batch_create": ([ctypes.POINTER(_P), _u32, _P, _u64, _P, ctypes.POINTER(_P)], _i32),
    "soma_batch_set_launch": ([_P, _u32, _u32], _i32),
    "soma_batch_set_histogram": ([_P, _u32], _i32),
    "soma_batch_sweep": ([_P, _u32, _u32, _P], _i32),
    "soma_batch_update_fields": ([_P, _P], _i32),
    "soma_batch_capture_cycle": ([_P, _u32, _u32], _i32),
    "soma_batch_run_cycle": ([_P, _u32, _P], _i32),
    "soma_batch_autotune": ([_P, _u32, _u32, ctypes.c_char_p, _P, ctypes.POINTER(soma_tune)],
                            _i32),
    "soma_batch_destroy": ([_P], None),
    "soma_density_hist": ([ctypes.POINTER(soma_config), _P, _P, _P], _i32),
    "soma_field_from_counts": ([ctypes.POINTER(soma_config), _P, _P, _P], _i32),
    "soma_init_positions": ([ctypes.POINTER(soma_config), _P, _P], _i32),
    "soma_net_bytes": ([], ctypes.c_uint64),
    "soma_prepare_net": ([_P, _P, _P], _i32),
    "soma_set_proposal": ([_P, _u32, _P, _P], _i32),
    "soma_mlp_forward": ([_P, _P, _u32, _P, _P], _i32),
    "soma_features": ([_P, _P, _P, _u32, _P, _P], _i32),
    "soma_collect_training": ([_P, _u32, _u32, _u32, _u32, _P, _P, _P, _P, _P], _i32),
    "soma_train_workspace_bytes": ([_u32], ctypes.c_uint64),
    "soma_train_step": ([_P, _P, _u32, _P, _P, _P, _u32, ctypes.POINTER(soma_train_opts), _P,
                         _u64, _P, _P, _P], _i32),
    "soma_train_step_noalloc": ([_P, _P, _u32, _P, _P, _P, _u32, ctypes.POINTER(soma_train_opts),
                                 _P, _P, _P], _i32),
    "soma_sq_workspace_bytes": ([_P], ctypes.c_uint64),
    "soma_structure_factor": ([_P, _P, _u64, _P, _P], _i32),
    "soma_sq_shells": ([_P, _u32, _u32, _u32, _u32, _P, _P, _P, _pu32], _i32),
    "soma_sq_plane_shells": ([_P, _u32, _u32, _u32, _P, _P, _P, _pu32], _i32),
    "soma_destroy": ([_P], None),
    "soma_last_error": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def soma_last_error() -> str:
    return _lib.soma_last_error().decode()


def _check(rc: int) -> int:
    if rc != SOMA_OK:
        raise SomaError(rc, soma_last_error())
    return rc


def soma_buffer_sizes(cfg: soma_config):
    v = [ctypes.c_uint64() for _ in range(4)]
    _check(_lib.soma_buffer_sizes(ctypes.byref(cfg), *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def soma_workspace_size(cfg: soma_config) -> int:
    v = ctypes.c_uint64()
    _check(_lib.soma_workspace_size(ctypes.byref(cfg), ctypes.byref(v)))
    return v.value


def soma_init_system(cfg: soma_config, buf: soma_buffers, init_positions: bool, stream: int):
    h = ctypes.c_void_p()
    _check(_lib.soma_init_system(ctypes.byref(cfg), ctypes.byref(buf), int(init_positions),
                                 ctypes.c_void_p(stream), ctypes.byref(h)))
    return h


def soma_mc_sweep(h, n_sweeps: int, move_kind: int, stream: int) -> None:
    _check(_lib.soma_mc_sweep(h, n_sweeps, move_kind, ctypes.c_void_p(stream)))


def soma_update_fields(h, stream: int) -> None:
    _check(_lib.soma_update_fields(h, ctypes.c_void_p(stream)))


def soma_set_sweep_blocks(h, blocks: int) -> None:
    _check(_lib.soma_set_sweep_blocks(h, blocks))


def soma_set_histogram(h, mode: int) -> None:
    _check(_lib.soma_set_histogram(h, mode))


def soma_set_sweep_threads(h, threads: int) -> None:
    _check(_lib.soma_set_sweep_threads(h, threads))


def soma_set_self_term(h, on: int) -> None:
    _check(_lib.soma_set_self_term(h, on))


def soma_probe_atomics(words_ptr: int, n_words: int, n_updates: int, mode: int, seed: int,
                       stream) -> None:
    _check(_lib.soma_probe_atomics(ctypes.c_void_p(words_ptr), n_words, n_updates, mode, seed,
                                   ctypes.c_void_p(stream)))


def soma_set_external(h, ext_ptr, ext_bytes: int, forbid_ptr, forbid_bytes: int, stream) -> None:
    _check(_lib.soma_set_external(h, ext_ptr, ext_bytes, forbid_ptr, forbid_bytes, stream))


def soma_set_architecture(h, species: int, words, stream) -> None:
    """words: numpy uint32 architecture array (host), or None for a linear chain."""
    import numpy as np
    if words is None:
        _check(_lib.soma_set_architecture(h, species, None, 0, stream))
        return
    w = np.ascontiguousarray(words, dtype=np.uint32)
    _check(_lib.soma_set_architecture(h, species, w.ctypes.data, w.size, stream))


def soma_set_hamiltonian(h, form: int, stream) -> None:
    _check(_lib.soma_set_hamiltonian(h, form, stream))


def soma_set_types(h, n_types: int, chi_n, counts_ptr: int, counts_bytes: int, omega_ptr: int,
                   omega_bytes: int, stream) -> None:
    """chi_n: host n_types x n_types matrix of chi_ij N (symmetric)."""
    import numpy as np
    chi = np.ascontiguousarray(chi_n, dtype=np.float32).reshape(n_types, n_types)
    _check(_lib.soma_set_types(h, n_types, chi.ctypes.data, counts_ptr, counts_bytes, omega_ptr,
                               omega_bytes, stream))


def soma_type_counts(h, n_types: int, stream):
    out = (ctypes.c_uint64 * n_types)()
    _check(_lib.soma_type_counts(h, out, n_types, stream))
    return [int(x) for x in out]


def soma_set_scheme(h, scheme: int) -> None:
    _check(_lib.soma_set_scheme(h, scheme))


def soma_choose_scheme(h, cycles: int, stream):
    """Returns (chosen scheme, [ms per cycle SET, MOLECULE])."""
    chosen = _u32()
    ms = (ctypes.c_float * 2)()
    _check(_lib.soma_choose_scheme(h, cycles, stream, ctypes.byref(chosen), ms))
    return chosen.value, [ms[0], ms[1]]


def soma_rebuild_histogram(h, stream: int) -> None:
    _check(_lib.soma_rebuild_histogram(h, ctypes.c_void_p(stream)))


def soma_observables(h, stream: int, raise_on_flag: bool = True) -> soma_obs:
    out = soma_obs()
    rc = _lib.soma_observables(h, ctypes.byref(out), ctypes.c_void_p(stream))
    if rc != SOMA_OK and (raise_on_flag or rc != SOMA_E_DEVICE_FLAG):
        raise SomaError(rc, soma_last_error())
    return out


def soma_check(h, stream: int) -> int:
    f = ctypes.c_uint32()
    rc = _lib.soma_check(h, ctypes.byref(f), ctypes.c_void_p(stream))
    if rc not in (SOMA_OK, SOMA_E_DEVICE_FLAG):
        raise SomaError(rc, soma_last_error())
    return f.value


def soma_get_sweep(h) -> int:
    v = ctypes.c_uint64()
    _check(_lib.soma_get_sweep(h, ctypes.byref(v)))
    return v.value


def soma_set_sweep(h, sweep: int, stream: int = 0) -> None:
    _check(_lib.soma_set_sweep(h, sweep, ctypes.c_void_p(stream)))


def soma_sync_fields(h, stream: int) -> None:
    _check(_lib.soma_sync_fields(h, ctypes.c_void_p(stream)))


def soma_set_grad_field(h, grad_ptr: int, grad_bytes: int, stream: int) -> None:
    _check(_lib.soma_set_grad_field(h, ctypes.c_void_p(grad_ptr) if grad_ptr else None,
                                    grad_bytes, ctypes.c_void_p(stream)))


def soma_set_substeps(h, k: int) -> None:
    _check(_lib.soma_set_substeps(h, k))


def soma_cycle(h, n_cycles: int, move_kind: int, stream: int) -> None:
    _check(_lib.soma_cycle(h, n_cycles, move_kind, ctypes.c_void_p(stream)))


def soma_batch_set_substeps(b, k: int, stream: int) -> None:
    _check(_lib.soma_batch_set_substeps(b, k, ctypes.c_void_p(stream)))


def soma_batch_cycle(b, n_cycles: int, move_kind: int, stream: int) -> None:
    _check(_lib.soma_batch_cycle(b, n_cycles, move_kind, ctypes.c_void_p(stream)))


def soma_capture_cycle(h, cycles: int, move_kind: int) -> None:
    _check(_lib.soma_capture_cycle(h, cycles, move_kind))


def soma_run_cycle(h, n_launches: int, stream: int) -> None:
    _check(_lib.soma_run_cycle(h, n_launches, ctypes.c_void_p(stream)))


def _path(p):
    return None if p is None else os.fsencode(p)


def soma_autotune(h, cycles: int, move_kind: int, cache_path, stream: int) -> soma_tune:
    out = soma_tune()
    _check(_lib.soma_autotune(h, cycles, move_kind, _path(cache_path), ctypes.c_void_p(stream),
                              ctypes.byref(out)))
    return out


def _handles(handles):
    arr = (_P * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                for h in handles])
    return arr


def soma_batch_workspace_size(handles) -> int:
    v = ctypes.c_uint64()
    _check(_lib.soma_batch_workspace_size(_handles(handles), len(handles), ctypes.byref(v)))
    return v.value


def soma_batch_create(handles, ws_ptr: int, ws_bytes: int, stream: int):
    b = ctypes.c_void_p()
    _check(_lib.soma_batch_create(_handles(handles), len(handles), ctypes.c_void_p(ws_ptr),
                                  ws_bytes, ctypes.c_void_p(stream), ctypes.byref(b)))
    return b


def soma_batch_set_launch(b, mode: int, grid_blocks: int) -> None:
    _check(_lib.soma_batch_set_launch(b, mode, grid_blocks))


def soma_batch_set_histogram(b, mode: int) -> None:
    _check(_lib.soma_batch_set_histogram(b, mode))


def soma_batch_sweep(b, n_sweeps: int, move_kind: int, stream: int) -> None:
    _check(_lib.soma_batch_sweep(b, n_sweeps, move_kind, ctypes.c_void_p(stream)))


def soma_batch_update_fields(b, stream: int) -> None:
    _check(_lib.soma_batch_update_fields(b, ctypes.c_void_p(stream)))


def soma_batch_capture_cycle(b, cycles: int, move_kind: int) -> None:
    _check(_lib.soma_batch_capture_cycle(b, cycles, move_kind))


def soma_batch_run_cycle(b, n_launches: int, stream: int) -> None:
    _check(_lib.soma_batch_run_cycle(b, n_launches, ctypes.c_void_p(stream)))


def soma_batch_autotune(b, cycles: int, move_kind: int, cache_path, stream: int) -> soma_tune:
    out = soma_tune()
    _check(_lib.soma_batch_autotune(b, cycles, move_kind, _path(cache_path),
                                    ctypes.c_void_p(stream), ctypes.byref(out)))
    return out


def soma_batch_destroy(b) -> None:
    if b:
        _lib.soma_batch_destroy(b)


def soma_density_hist(cfg: soma_config, pos_ptr: int, counts_ptr: int, stream: int) -> None:
    _check(_lib.soma_density_hist(ctypes.byref(cfg), ctypes.c_void_p(pos_ptr),
                                  ctypes.c_void_p(counts_ptr), ctypes.c_void_p(stream)))


def soma_field_from_counts(cfg: soma_config, counts_ptr: int, omega_ptr: int, stream: int) -> None:
    _check(_lib.soma_field_from_counts(ctypes.byref(cfg), ctypes.c_void_p(counts_ptr),
                                       ctypes.c_void_p(omega_ptr), ctypes.c_void_p(stream)))


def soma_init_positions(cfg: soma_config, pos_ptr: int, stream: int) -> None:
    _check(_lib.soma_init_positions(ctypes.byref(cfg), ctypes.c_void_p(pos_ptr),
                                    ctypes.c_void_p(stream)))


def soma_net_bytes() -> int:
    return int(_lib.soma_net_bytes())


def soma_prepare_net(params_ptr: int, net_ptr: int, stream: int) -> None:
    _check(_lib.soma_prepare_net(ctypes.c_void_p(params_ptr), ctypes.c_void_p(net_ptr),
                                 ctypes.c_void_p(stream)))


def soma_set_proposal(h, params_ptr: int, stream: int, species: int = SOMA_ALL_SPECIES) -> None:
    _check(_lib.soma_set_proposal(h, species, ctypes.c_void_p(params_ptr), ctypes.c_void_p(stream)))


def soma_mlp_forward(net_ptr: int, features_ptr: int, n: int, z_ptr: int, stream: int) -> None:
    _check(_lib.soma_mlp_forward(ctypes.c_void_p(net_ptr), ctypes.c_void_p(features_ptr), n,
                                 ctypes.c_void_p(z_ptr), ctypes.c_void_p(stream)))


def soma_features(h, chains_ptr: int, beads_ptr: int, n: int, out_ptr: int, stream: int) -> None:
    _check(_lib.soma_features(h, ctypes.c_void_p(chains_ptr), ctypes.c_void_p(beads_ptr), n,
                              ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream)))


def soma_collect_training(h, n: int, round_: int, phase: int, features_ptr: int, r0_ptr: int,
                          dr_ptr: int, picked_ptr: int, stream: int,
                          species: int = SOMA_ALL_SPECIES) -> None:
    vp = lambda x: ctypes.c_void_p(x) if x else None
    _check(_lib.soma_collect_training(h, species, n, round_, phase, vp(features_ptr),
                                      vp(r0_ptr), vp(dr_ptr), vp(picked_ptr),
                                      ctypes.c_void_p(stream)))


def soma_sq_workspace_bytes(h) -> int:
    return int(_lib.soma_sq_workspace_bytes(h))


def soma_structure_factor(h, ws_ptr: int, ws_bytes: int, sq_ptr: int, stream: int) -> None:
    _check(_lib.soma_structure_factor(h, ctypes.c_void_p(ws_ptr), ws_bytes,
                                      ctypes.c_void_p(sq_ptr), ctypes.c_void_p(stream)))


def soma_sq_shells(sq_host, grid, n_shells: int):
    """Shell average of a host float64 array (C-contiguous, n_cells):
    (q_mid, s_avg, count, peak) as numpy arrays and an int."""
    import numpy as np
    sq_host = np.ascontiguousarray(sq_host, dtype=np.float64)
    q = np.zeros(n_shells)
    s = np.zeros(n_shells)
    c = np.zeros(n_shells, np.uint64)
    peak = ctypes.c_uint32()
    nx, ny, nz = (int(v) for v in grid)
    _check(_lib.soma_sq_shells(sq_host.ctypes.data, nx, ny, nz, n_shells, q.ctypes.data,
                               s.ctypes.data, c.ctypes.data, ctypes.byref(peak)))
    return q, s, c, peak.value


def soma_sq_plane_shells(sq_host, grid, n_shells: int):
    """In-plane (m_z = 0) shell average of a host float64 S(q) array of a film:
    (q_mid, s_avg, count, peak)."""
    import numpy as np
    nx, ny, _ = (int(v) for v in grid)
    plane = np.ascontiguousarray(np.asarray(sq_host, dtype=np.float64).ravel()[:nx * ny])
    q = np.zeros(n_shells)
    s = np.zeros(n_shells)
    c = np.zeros(n_shells, np.uint64)
    peak = ctypes.c_uint32()
    _check(_lib.soma_sq_plane_shells(plane.ctypes.data, nx, ny, n_shells, q.ctypes.data,
                                     s.ctypes.data, c.ctypes.data, ctypes.byref(peak)))
    return q, s, c, peak.value


def soma_train_workspace_bytes(max_waves: int) -> int:
    return int(_lib.soma_train_workspace_bytes(max_waves))


def soma_train_step(features_ptr, targets_ptr, n, params_ptr, m_ptr, v_ptr, step,
                    opts: soma_train_opts, ws_ptr, ws_bytes, grad_ptr, loss_ptr, stream) -> None:
    vp = lambda x: ctypes.c_void_p(x) if x else None
    _check(_lib.soma_train_step(vp(features_ptr), vp(targets_ptr), n, vp(params_ptr), vp(m_ptr),
                                vp(v_ptr), step, ctypes.byref(opts), vp(ws_ptr), ws_bytes,
                                vp(grad_ptr), vp(loss_ptr), ctypes.c_void_p(stream)))


def soma_train_step_noalloc(features_ptr, targets_ptr, n, params_ptr, m_ptr, v_ptr, step,
                            opts: soma_train_opts, grad_ptr, loss_ptr, stream) -> None:
    vp = lambda x: ctypes.c_void_p(x) if x else None
    _check(_lib.soma_train_step_noalloc(vp(features_ptr), vp(targets_ptr), n, vp(params_ptr),
                                        vp(m_ptr), vp(v_ptr), step, ctypes.byref(opts),
                                        vp(grad_ptr), vp(loss_ptr), ctypes.c_void_p(stream)))


def soma_destroy(h) -> None:
    if h:
        _lib.soma_destroy(h)
