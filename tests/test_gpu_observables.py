"""Statistical parity of observables: the device against the oracle.

Each protocol of synth.OBS_PROTOCOLS (the 1024-chain melt with local,
smart-MC and bond-Gibbs moves; a 256-chain melt at the bead density of the
262k-chain study with local and learned moves) is run on the device from
twelve seeds of its own and on the oracle from twelve other seeds
(tests/golden/observable_stats.json, written by make_observable_stats.py,
which calls only the oracle), so the two samples are independent.  Both
sides start from the Philox init distribution and are compared at equal
cycles (the melts are still ordering: the ensemble at a given cycle is what
must agree).

Bars: the mean over seeds of <Re^2>, <Rg^2> (averaged over the sampled
cycles), the acceptance rate and S(q) at the peak shell agree within 3 sigma,
sigma^2 = s_dev^2/n_dev + s_orc^2/n_orc from the seed-to-seed spreads; the
peak shell of the seed-averaged shell profile is the same on both sides.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from tests.gpu_helpers import flush

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "observable_stats.json")


def _device_sq(m, C):
    ws_b = C.soma_sq_workspace_bytes(m.handle)
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    sq = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    C.soma_structure_factor(m.handle, ws.data_ptr(), ws_b, sq.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return sq.cpu().numpy()


def run_device(p, seed):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt, make_config
    w = p.workload
    learned = p.move == "learned"
    m = Melt(make_config(w, seed=seed, p_learn=1.0 if learned else 0.0, sigma_max=1.0))
    kind = {"local": C.SOMA_MOVE_LOCAL, "smc": C.SOMA_MOVE_SMC, "gibbs": C.SOMA_MOVE_GIBBS,
            "learned": C.SOMA_MOVE_MIXED}[p.move]
    kidx = {"local": 0, "smc": 1, "gibbs": 3, "learned": 2}[p.move]
    if learned:
        m.set_proposal(torch.from_numpy(synth.designed_net_params()).cuda())
    re2, rg2 = [], []
    acc0 = None
    for cyc in range(p.cycles):
        m.cycle(1, kind)
        if cyc + 1 == p.first:
            o = m.observables()
            acc0 = (o.accepted[kidx], o.attempted[kidx])
        if cyc + 1 >= p.first and (cyc + 1 - p.first) % p.every == 0:
            o = m.observables()
            re2.append(o.re2_sum / w.n_chains / w.re_cells ** 2)
            rg2.append(o.rg2_sum / w.n_chains / w.re_cells ** 2)
    o = m.observables()
    assert o.error_flags == 0 and o.counts_conserved == 1
    acc = (o.accepted[kidx] - acc0[0]) / (o.attempted[kidx] - acc0[1])
    assert o.attempted[kidx] - acc0[1] == (p.cycles - p.first) * w.n_beads
    sq = _device_sq(m, C)
    _, mean, _, peak = C.soma_sq_shells(sq, w.grid, p.n_shells)
    m.close()
    return dict(re2=float(np.mean(re2)), rg2=float(np.mean(rg2)), acc=float(acc),
                sq_shells=[float(v) for v in mean], peak=int(peak))


def _golden():
    with open(GOLDEN) as f:
        return {e["protocol"]["name"]: e["runs"] for e in json.load(f)["protocols"]}


def _agree(name, what, dev, orc):
    dev, orc = np.asarray(dev, float), np.asarray(orc, float)
    sig = math.sqrt(dev.var(ddof=1) / dev.size + orc.var(ddof=1) / orc.size)
    diff = dev.mean() - orc.mean()
    flush(f"{name:16s} {what:6s} device {dev.mean():.6g} oracle {orc.mean():.6g}  "
          f"diff/sigma {diff / sig if sig > 0 else 0.0:+.2f}")
    assert abs(diff) <= 3.0 * sig, (name, what, diff, sig)


@pytest.mark.parametrize("p", synth.OBS_PROTOCOLS, ids=[p.name for p in synth.OBS_PROTOCOLS])
def test_observables_agree_with_oracle(p):
    golden = _golden()[p.name]
    assert [r["seed"] for r in golden] == list(synth.OBS_SEEDS_ORACLE)
    dev = [run_device(p, s) for s in synth.OBS_SEEDS_DEVICE]
    for what in ("re2", "rg2", "acc"):
        _agree(p.name, what, [r[what] for r in dev], [r[what] for r in golden])
    prof_d = np.mean([r["sq_shells"] for r in dev], axis=0)
    prof_o = np.mean([r["sq_shells"] for r in golden], axis=0)
    pk_d = 1 + int(np.argmax(prof_d[1:]))
    pk_o = 1 + int(np.argmax(prof_o[1:]))
    flush(p.name, "peak shell of the mean profile: device", pk_d, "oracle", pk_o,
          "per-seed peaks", [r["peak"] for r in dev], [r["peak"] for r in golden])
    assert pk_d == pk_o
    _agree(p.name, "S(q*)", [r["sq_shells"][pk_o] for r in dev],
           [r["sq_shells"][pk_o] for r in golden])
