"""The stored oracle statistics of the observable-parity test are current.

tests/golden/observable_stats.json is written by make_observable_stats.py
(oracle only).  Checked here: the stored protocols equal synth.OBS_PROTOCOLS
and the oracle's seeds, and re-running one seed of the cheapest protocol
reproduces its stored numbers exactly (the oracle is deterministic).
"""
import importlib.util
import json
import os

import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _script():
    spec = importlib.util.spec_from_file_location(
        "make_observable_stats", os.path.join(HERE, "golden", "make_observable_stats.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_stored_protocols_are_current():
    mod = _script()
    with open(mod.OUT) as f:
        stored = json.load(f)["protocols"]
    assert [e["protocol"] for e in stored] == [mod.protocol_key(p) for p in synth.OBS_PROTOCOLS]
    for e in stored:
        assert [r["seed"] for r in e["runs"]] == list(synth.OBS_SEEDS_ORACLE)


def test_one_seed_reproduces(orc):
    mod = _script()
    with open(mod.OUT) as f:
        stored = {e["protocol"]["name"]: e["runs"] for e in json.load(f)["protocols"]}
    p = next(p for p in synth.OBS_PROTOCOLS if p.name == "c4dens_local")
    got = mod.run_oracle(p, synth.OBS_SEEDS_ORACLE[0], 4)
    exp = stored["c4dens_local"][0]
    for k in ("re2", "rg2", "acc", "peak"):
        assert got[k] == pytest.approx(exp[k], rel=1e-12, abs=0), k
