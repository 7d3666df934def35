"""Writes observable_stats.json: the oracle's side of the statistical parity
test of observables (per seed: mean Re^2 and Rg^2 over the sampled cycles in
units of Re0^2, acceptance over the sampled window, S(q) shell means and peak
after the last cycle), for every protocol in synth.OBS_PROTOCOLS and the
oracle's seeds synth.OBS_SEEDS_ORACLE.  Calls only the oracle.

    python tests/golden/make_observable_stats.py [threads]
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import Species  # noqa: E402
from oracle import analysis as A  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "observable_stats.json")
HEAD = dict(m_max=1.0, lo=math.log(0.02), hi=0.0)


def protocol_key(p) -> dict:
    w = p.workload
    return dict(name=p.name, grid=list(w.grid), species=[[s.n_chains, s.n, s.n_a] for s in w.species],
                chi_n=w.chi_n, kappa_n=w.kappa_n, re_cells=w.re_cells, n_ref=w.n_ref,
                a_frac=w.a_frac, smc_frac=w.smc_frac, move=p.move, cycles=p.cycles,
                first=p.first, every=p.every, n_shells=p.n_shells)


def run_oracle(p, seed: int, threads: int) -> dict:
    w = p.workload
    sp = Species(*[(s.n_chains, s.n, s.n_a) for s in w.species][0])
    k0 = np.float32(3.0 * (w.n_ref - 1) / w.re_cells ** 2)
    a = np.float32(w.a_frac * w.re_cells / math.sqrt(w.n_ref - 1))
    A_smc = np.float32(w.smc_frac * w.re_cells ** 2 / w.n_ref)
    inv_rho = np.float32(w.n_cells / w.n_beads)
    pos = oracle.init_chains(sp, w.grid, bond_sigma=np.float32(1.0 / math.sqrt(float(k0))),
                             seed=seed, origin_mode=1).reshape(-1, 3).copy()

    def field(pp):
        return oracle.field_f32(oracle.density_hist(pp, [sp], w.grid), inv_rho,
                                np.float32(w.chi_n), np.float32(w.kappa_n))

    omega = field(pos)
    params = synth.designed_net_params() if p.move == "learned" else None
    re2, rg2 = [], []
    acc = 0
    for cyc in range(p.cycles):
        if p.move == "learned":
            n_acc, _, bad, _, _ = oracle.mc_sweep_mixed(pos, sp, omega, w.grid, k0=k0,
                                                        n_ref=w.n_ref, local_a=a, p_learn=1.0,
                                                        params=params, **HEAD, seed=seed,
                                                        sweep=cyc, threads=threads)
            assert bad == 0
        else:
            kind = {"local": oracle.MOVE_LOCAL, "smc": oracle.MOVE_SMC,
                    "gibbs": oracle.MOVE_GIBBS}[p.move]
            n_acc, _ = oracle.mc_sweep(pos, sp, omega, w.grid, k0=k0, n_ref=w.n_ref,
                                       move_kind=kind, step=A_smc if p.move == "smc" else a,
                                       seed=seed, sweep=cyc, threads=threads)
        omega = field(pos)
        if cyc + 1 > p.first:
            acc += int(n_acc)
        if cyc + 1 >= p.first and (cyc + 1 - p.first) % p.every == 0:
            r, g, _ = oracle.chain_observables(pos, sp.n_chains, sp.n)
            re2.append(r.mean() / w.re_cells ** 2)
            rg2.append(g.mean() / w.re_cells ** 2)
    counts = oracle.density_hist(pos, [sp], w.grid)
    sq = A.structure_factor(counts, w.grid, w.n_ref, w.n_beads)
    _, mean, _, peak = A.sq_shells(sq, w.grid, p.n_shells)
    return dict(seed=seed, re2=float(np.mean(re2)), rg2=float(np.mean(rg2)),
                acc=acc / ((p.cycles - p.first) * w.n_beads), sq_shells=[float(v) for v in mean],
                peak=int(peak))


def main(threads: int = 8):
    oracle.build()
    out = dict(note="oracle side of the statistical parity test; written by "
                    "tests/golden/make_observable_stats.py", protocols=[])
    for p in synth.OBS_PROTOCOLS:
        t = time.time()
        runs = [run_oracle(p, s, threads) for s in synth.OBS_SEEDS_ORACLE]
        out["protocols"].append(dict(protocol=protocol_key(p), runs=runs))
        print(p.name, f"{time.time() - t:.1f} s", "re2", np.mean([r["re2"] for r in runs]),
              "acc", np.mean([r["acc"] for r in runs]), "peaks", [r["peak"] for r in runs],
              flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
