"""The C-ABI library loads and exports every function include/soma.h declares,
and the ctypes mirrors of its structs match the C layout (CPU only)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "soma.h")
LIB = os.path.join(ROOT, "paper_1711_03828_amd", "libsoma_hip.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(soma_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("soma_init_system", "soma_mc_sweep", "soma_update_fields", "soma_observables",
              "soma_density_hist", "soma_workspace_size", "soma_last_error", "soma_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n


def test_struct_layout_matches_ctypes(tmp_path):
    from paper_1711_03828_amd import soma as C
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "soma.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(soma_species), sizeof(soma_config),
         sizeof(soma_buffers), sizeof(soma_obs), offsetof(soma_config, seed));
  printf("%zu %zu %zu\n", offsetof(soma_obs, re2_sum), offsetof(soma_obs, error_flags),
         offsetof(soma_config, origin_mode));
  printf("%zu %zu %zu %zu\n", sizeof(soma_train_opts), offsetof(soma_train_opts, apply),
         sizeof(soma_tune), offsetof(soma_tune, from_cache));
  return 0;
}''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    exp = [ctypes.sizeof(C.soma_species), ctypes.sizeof(C.soma_config),
           ctypes.sizeof(C.soma_buffers), ctypes.sizeof(C.soma_obs),
           C.soma_config.seed.offset, C.soma_obs.re2_sum.offset, C.soma_obs.error_flags.offset,
           C.soma_config.origin_mode.offset, ctypes.sizeof(C.soma_train_opts),
           C.soma_train_opts.apply.offset, ctypes.sizeof(C.soma_tune),
           C.soma_tune.from_cache.offset]
    assert got == exp


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_config_validation_without_gpu():
    """Host-side checks run before any device call."""
    from paper_1711_03828_amd import soma as C
    import synth
    from paper_1711_03828_amd.melt import make_config
    cfg = make_config(synth.C2_LARGE)
    pos_b, cnt_b, om_b, ws_b = C.soma_buffer_sizes(cfg)
    assert pos_b == 12 * 134217728 and cnt_b == 8 * 384 * 384 * 192 and om_b == 8 * 384 * 384 * 192
    assert ws_b >= 256
    cfg.count_width = 12
    with pytest.raises(C.SomaError) as e:
        C.soma_buffer_sizes(cfg)
    assert e.value.code == C.SOMA_E_INVAL
    cfg = make_config(synth.C1_SMALL)
    cfg.species[0].n = 300
    with pytest.raises(C.SomaError) as e:
        C.soma_buffer_sizes(cfg)
    assert e.value.code == C.SOMA_E_UNSUPPORTED
