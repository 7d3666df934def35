"""Benchmark of the SCMF hot path on one MI355X.

A step is one SCMF cycle (Sec. 2.2) of the whole melt: one MC sweep of every
bead with the fields held fixed (histogram of the final positions fused into
the sweep), then the field refresh from that histogram.  The default workload
is the 134M-bead diblock melt (4,194,304 A16B16 chains, 384x384x192 cells,
chiN = 20, kappaN = 50, 32-bit counts), initialised on the device; inputs are
resident in HBM before timing starts.

Prints one JSON line: bead-moves/s of the whole job, the roofline of the
dominant kernel (mc_sweep, HIP-event timed on the stream it runs on, against
its algorithmic bytes) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "bead MC moves/s and uncorrelated samples/s, plain vs learned proposal, 1 GPU"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0      # dense BF16 matrix cores (no sparsity)
# the learned proposal's network 60 -> 64 -> 64 -> 6: 2 flop per weight
FLOP_FORWARD = 2 * (60 * 64 + 64 * 64 + 64 * 6)                      # 16,640
# training per sample: forward, errors back through layers 3 and 2, weight gradients
FLOP_TRAIN_SAMPLE = FLOP_FORWARD + 2 * (6 * 64 + 64 * 64) + FLOP_FORWARD   # 42,240


def algorithmic_bytes(w):
    """Bytes one sweep launch must move: every bead's position read and written
    (2 x 12 B), every cell's two field values read (8 B) and its packed count
    word read and written by the histogram (2 x 4 or 2 x 8 B)."""
    cw = 4 if w.count_width == 16 else 8
    per_bead = 24
    per_cell = 8 + 2 * cw
    return per_bead * w.n_beads + per_cell * w.n_cells, per_bead, per_cell


def field_bytes(w):
    cw = 4 if w.count_width == 16 else 8
    return (cw + 8) * w.n_cells   # counts read, two fields written


# Sources the sweep kernels and their launches are built from.
SWEEP_SOURCES = ("paper_1711_03828_amd/csrc/soma_api.hip",
                 "paper_1711_03828_amd/csrc/soma_bins.hpp",
                 "paper_1711_03828_amd/csrc/soma_device.hpp",
                 "paper_1711_03828_amd/csrc/soma_mlp.hpp",
                 "paper_1711_03828_amd/csrc/soma_sweep.hpp")


def kernel_source_digest() -> str:
    """SHA-1 of the sweep kernels' sources, to tell whether stored counters still apply."""
    import hashlib
    h = hashlib.sha1()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(w, move: str, launch: dict):
    """HBM bytes per sweep (the sweep kernel, plus the bin-apply kernel when the
    count updates are binned) from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (scaled by the copy-kernel calibration), or None if the kernel
    sources changed since it was taken or no record covers this workload and
    launch shape (histogram mode, block size, grid)."""
    path = os.path.join(ROOT, "profiles", f"mc_sweep_{move}_diblock_4M_N32_traffic.json")
    if w.name != "diblock_4M_N32_grid384x384x192" or not os.path.exists(path):
        return None
    with open(path) as fh:
        recs = json.load(fh).get("records", [])
    digest = kernel_source_digest()
    for rec in recs:
        if rec["kernel_source_sha1"] == digest and rec["launch"] == launch:
            return rec["traffic_bytes"]
    return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_cycles(w, grid, n_chains, seconds, threads, *, learned=None, max_cycles=None):
    """SCMF cycles of the oracle (sweep + histogram + fields) on n_chains chains
    of w's species on `grid`, for about `seconds` (or max_cycles).  learned:
    (params, p_learn) for mixed sweeps with the oracle's FP64 network.
    Returns (bead moves per second, cycles, beads)."""
    import numpy as np

    import oracle
    from oracle import Species

    s0 = w.species[0]
    k0 = np.float32(3.0 * (w.n_ref - 1) / w.re_cells ** 2)
    a = np.float32(w.a_frac * w.re_cells / math.sqrt(w.n_ref - 1))
    n_beads = n_chains * s0.n
    n_cells = grid[0] * grid[1] * grid[2]
    inv_rho = np.float32(n_cells / n_beads)
    sp = Species(n_chains, s0.n, s0.n_a)
    pos = oracle.init_chains(sp, grid, bond_sigma=np.float32(1 / math.sqrt(float(k0))),
                             seed=w.seed, origin_mode=1)

    def fields():
        return oracle.field_f32(oracle.density_hist(pos, [sp], grid), inv_rho,
                                np.float32(w.chi_n), np.float32(w.kappa_n))
    omega = fields()
    cycles = 0
    t0 = time.perf_counter()
    while True:
        if learned is None:
            oracle.mc_sweep(pos, sp, omega, grid, k0=k0, n_ref=w.n_ref, step=a, seed=w.seed,
                            sweep=cycles, threads=threads)
        else:
            params, p_learn = learned
            oracle.mc_sweep_mixed(pos, sp, omega, grid, k0=k0, n_ref=w.n_ref, local_a=a,
                                  p_learn=p_learn, params=params, m_max=1.0,
                                  lo=math.log(0.02), hi=math.log(1.0), bf16_mode=False,
                                  seed=w.seed, sweep=cycles, threads=threads)
        omega = fields()
        cycles += 1
        dt = time.perf_counter() - t0
        if (max_cycles is not None and cycles >= max_cycles) or \
                (max_cycles is None and dt > seconds):
            break
    return n_beads * cycles / dt, cycles, n_beads


def cpu_baseline(w, seconds: float):
    """The oracle as it stands, OpenMP over chains on the host cores (the
    paper's own CPU scheme), on bounded samples:
      * a slab of the benchmark melt (same density, chemistry and moves),
        all host threads: the reported value;
      * the 1024-chain melt in full (100 cycles), one thread;
      * a slab of the 262,144-chain learned-proposal melt with local moves and
        with learned moves (the oracle's FP64 network, a random network of the
        same shape), all host threads.
    Cycles = sweep + histogram + fields, timed per call, excluding set-up."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    nx, ny, nz = w.grid
    slab_z = max(1, min(nz, 12))
    n_chains = max(1, int(round(w.species[0].n_chains * slab_z / nz)))
    value, cycles, n_beads = _oracle_cycles(w, (nx, ny, slab_z), n_chains, seconds, threads)
    out = {"value": value, "unit": "bead-moves/s", "cores": threads, "kind": "oracle",
           "sample": (f"{cycles} SCMF cycles (local moves + histogram + fields) of a "
                      f"{nx}x{ny}x{slab_z}-cell slab of the same melt: {n_chains} chains, "
                      f"{n_beads} beads, same density/chiN/kappaN"),
           "cpu_model": _cpu_model(), "nproc": os.cpu_count()}
    c1 = synth.C1_SMALL
    v1, cyc1, nb1 = _oracle_cycles(c1, c1.grid, c1.species[0].n_chains, 0.0, 1, max_cycles=100)
    out["single_thread_c1"] = {"value": v1, "unit": "bead-moves/s", "cores": 1,
                               "sample": f"{c1.name} in full: {cyc1} cycles, {nb1} beads"}
    c4 = synth.C4_MEDIUM
    z4 = 6
    n4 = int(round(c4.species[0].n_chains * z4 / c4.grid[2]))
    vp, cp, nb4 = _oracle_cycles(c4, (c4.grid[0], c4.grid[1], z4), n4, seconds / 5, threads)
    params = synth.mlp_params(1, out_gain=0.3)
    vl, cl, _ = _oracle_cycles(c4, (c4.grid[0], c4.grid[1], z4), n4, seconds / 2, threads,
                               learned=(params, 1.0), max_cycles=None)
    out["c4_slab"] = {"sample": f"{c4.grid[0]}x{c4.grid[1]}x{z4}-cell slab of {c4.name}: "
                                f"{n4} chains, {nb4} beads", "cores": threads,
                      "plain_bead_moves_per_s": vp, "plain_cycles": cp,
                      "learned_bead_moves_per_s": vl, "learned_cycles": cl,
                      "learned_network": "60-64-64-6 MLP in FP64 (the oracle's), random "
                                         "weights, every move learned (p_learn = 1)"}
    return out


def _re_vectors(melt, n):
    x = melt.pos.view(-1, n, 3)
    return (x[:, -1] - x[:, 0]).double()


def learned_leg(p_learn: float, equil_cycles: int, substeps: int, lag: int = 64,
                n_rep: int = 8, side: int = 32, tau_scale: float = 1.0,
                train_steps: int = 3000, self_term: int = 1):
    """Plain vs learned proposal on the 262,144-chain melt (96^3 cells, chiN 25).

    1. Training data from the plain sampler: 10 rounds of 2^20 random beads,
       features at cycle t and displacement after `lag` further plain cycles
       (10,485,760 samples), collected and trained on the device.  (Measured:
       learned moves only (p_learn = 1) decorrelate faster than a 9:1 mixture
       with the local move, and lags of 64-128 cycles beat 256 and 512, whose
       larger moves are accepted less often; lag 64 leaves the smallest shift of
       <Re^2> against the plain sampler.)
    2. Bead-moves/s of both samplers on the full melt (HIP events, graph-replayed
       SCMF cycles).  The learned sampler runs `substeps` chain subsets per cycle
       with a field refresh after each: its moves are large, and the
       quasi-instantaneous field approximation needs few beads moved between two
       refreshes to give the plain sampler's observables (end-to-end distance).
    3. The melt equilibrated with the learned sampler for `equil_cycles` cycles
       and the network fine-tuned on plain trajectories from that state
       (4 x 2^20 samples).
    4. tau_int and <Re^2> of the plain, learned and (as context) bond-Gibbs
       samplers from n_rep independent replicas of a side^3-cell melt at the
       same density and chiN (replica_statistics): discarded transients of
       about 3 tau_int, measured runs of about 50 tau_int, seed-to-seed
       standard errors.  Uncorrelated samples/s = n_chains * cycles/s /
       (2 tau_int), cycles/s of the full melt from step 2.  The bond-Gibbs
       proposal draws each bead from its law given its bonded neighbours and
       is accepted on the field term alone.
    With self_term = 1 every sampler (steps 2-4) charges a cell-changing move
    the bead's own share of the grid Hamiltonian's change (soma_set_self_term):
    the samplers' <Re^2> then agree within a few standard errors, where without
    it moves that change cell more often (the learned and bond-Gibbs ones) end
    up more or less stretched than the plain sampler's chains.
    """
    import torch

    from paper_1711_03828_amd import learned
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt, make_config

    w = synth.C4_MEDIUM
    t0 = time.perf_counter()
    melt = Melt(make_config(w, p_learn=p_learn))
    melt.cycle(50)
    feats, disp = learned.collect(melt, 1 << 20, lag, 10)
    params = learned.init_params(feats, seed=1)
    tr = learned.Trainer(params, lr=3e-3)
    losses = tr.run(feats, disp, steps=train_steps, batch=8192, loss_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_samples = int(feats.shape[0])
    stream = torch.cuda.current_stream()
    # matrix-core roofline of a training step (batch 8192, lr 0 on a copy of
    # the network): forward, back-propagation to the first hidden layer and
    # the weight gradients, 42,240 flop per sample
    probe = learned.Trainer(params.clone(), lr=0.0)
    probe.run(feats, disp, steps=5, batch=8192, loss_every=5)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    probe.run(feats, disp, steps=50, batch=8192, loss_every=50)
    e1.record(stream)
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / 50
    del probe, feats, disp
    melt.set_proposal(params)
    C.soma_set_self_term(melt.handle, self_term)
    out = {"workload": w.name, "p_learn": p_learn, "self_term": self_term,
           "training": {"samples": n_samples, "lag_cycles": lag, "adam_steps": train_steps,
                        "batch": 8192, "loss_first": losses[0], "loss_last": losses[-1],
                        "seconds_collect_and_train": t_train}}
    flop_train = 8192 * FLOP_TRAIN_SAMPLE
    out["roofline_train_step"] = {
        "bound": "mfma", "achieved": flop_train / (train_ms * 1e-3) / 1e12,
        "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": flop_train / (train_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, "traffic": None,
        "kernel": "mlp_grad_kernel + mlp_adam_kernel", "ms_per_step": train_ms,
        "flop_per_step": flop_train, "flop_per_sample": FLOP_TRAIN_SAMPLE}
    rates = {}
    ksub = {"plain": 1, "learned": substeps, "gibbs": substeps}
    tuned = {}
    for name, kind in (("plain", C.SOMA_MOVE_LOCAL), ("learned", C.SOMA_MOVE_MIXED),
                       ("gibbs", C.SOMA_MOVE_GIBBS)):
        melt.set_substeps(ksub[name])
        # launch shape per sampler (results do not depend on it); 4 cycles per
        # candidate, as their times lie within a few per cent of each other
        t = melt.autotune(4, kind)
        tuned[name] = {"hist_mode": "binned" if t.hist_mode else "direct",
                       "block_threads": t.block_threads, "grid_blocks": t.grid_blocks}
        melt.capture_cycle(10, kind)
        melt.run_cycle(2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        melt.run_cycle(5)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 50
        rates[name] = 1e3 / ms
        out[name] = {"ms_per_cycle": ms, "bead_moves_per_s": w.n_beads * 1e3 / ms,
                     "substeps": ksub[name], "launch": tuned[name]}
    # matrix-core roofline of the mixed sweep: every learned move evaluates the
    # network at r and at r' (2 x 16,640 flop); sweeps with the fields frozen,
    # HIP events on the launch stream
    melt.set_substeps(1)
    melt.autotune(4, C.SOMA_MOVE_MIXED)
    melt.sweep(2, C.SOMA_MOVE_MIXED)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    melt.sweep(10, C.SOMA_MOVE_MIXED)
    e1.record(stream)
    torch.cuda.synchronize()
    mixed_ms = e0.elapsed_time(e1) / 10
    flop_sweep = w.n_beads * p_learn * 2 * FLOP_FORWARD
    out["roofline_mixed_sweep"] = {
        "bound": "mfma", "achieved": flop_sweep / (mixed_ms * 1e-3) / 1e12,
        "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": flop_sweep / (mixed_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, "traffic": None,
        "kernel": "mc_sweep_mixed_kernel", "kernel_ms": mixed_ms, "flop_per_launch": flop_sweep,
        "flop_per_learned_move": 2 * FLOP_FORWARD}
    obs = melt.observables()
    out["learned"]["acceptance"] = obs.accepted[2] / max(1, obs.attempted[2])
    out["plain"]["acceptance"] = obs.accepted[0] / max(1, obs.attempted[0])
    out["gibbs"]["acceptance"] = obs.accepted[3] / max(1, obs.attempted[3])

    # equilibrate the full melt with the learned sampler, then fine-tune on
    # plain trajectories from that state
    melt.set_substeps(substeps)
    melt.capture_cycle(100, C.SOMA_MOVE_MIXED)
    melt.run_cycle(max(1, equil_cycles // 100))
    melt.set_substeps(1)
    C.soma_set_self_term(melt.handle, 0)    # training targets: the paper's plain sampler
    feats, disp = learned.collect(melt, 1 << 20, lag, 4, first_round=1000)
    tune = learned.Trainer(params, lr=1e-3)
    tl = tune.run(feats, disp, steps=2000, batch=8192, loss_every=500)
    del feats, disp
    melt.set_proposal(params)
    out["training"]["fine_tune"] = {"samples": 4 << 20, "adam_steps": 2000,
                                    "loss_first": tl[0], "loss_last": tl[-1],
                                    "after_learned_cycles": equil_cycles}
    melt.close()
    if tau_scale > 0:
        out["statistics"] = replica_statistics(params, substeps, p_learn, rates, n_rep, side,
                                               tau_scale, self_term=self_term)
    return out


def _c4_subsystem(side: int):
    """The learned-proposal melt's chemistry and density (262,144 A16B16 chains
    on 96^3 cells: 9.48 beads per cell, chiN 25, kappaN 50) in a box of side^3
    cells."""
    w = synth.C4_MEDIUM
    n = int(round(w.species[0].n_chains * side ** 3 / w.n_cells))
    return synth.Workload(f"diblock_{n}_N32_grid{side}", (side, side, side),
                          (synth.SpeciesSpec(n, 32, 16),), w.re_cells, w.n_ref, w.chi_n,
                          w.kappa_n, w.count_width)


# Per sampler, in the order run: (move kind, chain subsets per cycle, cycles
# per frame, frames discarded, frames measured).  Run lengths aim at >= 3
# tau_int discarded and >= 50 tau_int measured for the tau_int these replicas
# show with the self term (about 1,100 cycles learned with 8 refreshes, 21,000
# to 40,000 plain depending on the start, 480 bond-Gibbs); the JSON states the
# ratio actually reached.  The learned sampler runs first, from the common
# start it made; the plain run follows from the learned one's end state, the
# bond-Gibbs run from the plain one's.
def _replica_plan(C, substeps: int, scale: float):
    def n(x):
        return max(20, int(round(x * scale)))
    # transients of more than 3 tau_int at the tau_int these samplers show on
    # this melt (about 1,700, 72,000 and 550 cycles; the plain and learned
    # estimates still grow with the run length), runs of 40-55 tau_int
    return {"learned": (C.SOMA_MOVE_MIXED, substeps, 20, n(280), n(3900)),
            "plain": (C.SOMA_MOVE_LOCAL, 1, 400, n(580), n(7600)),
            "gibbs": (C.SOMA_MOVE_GIBBS, substeps, 10, n(180), n(2900))}


def replica_statistics(params, substeps: int, p_learn: float, rates: dict, n_rep: int,
                       side: int, scale: float, plan=None, self_term: int = 0):
    """tau_int and <Re^2> of each sampler from independent replicas.

    n_rep replicas (independent Philox streams: replica index r) of the
    learned-proposal melt's chemistry at its density in a side^3-cell box, all
    in one batched launch.  A common start (learned-sampler cycles from the
    Gaussian walks: its stationary <Re^2> is near the plain sampler's, while
    the bond-Gibbs sampler's lies about 8% lower), then per sampler a
    discarded transient and a measured run; frames of every second chain's
    end-to-end vector every few cycles.  Per replica: tau_int
    (Sokal window over its chains' pooled autocorrelation) and <Re^2>; means
    and standard errors over the replicas (seed-to-seed spread).  Uncorrelated
    samples/s use the full melt's cycle rate (`rates`, cycles/s) and the
    replicas' tau_int; the learned/plain gain carries the propagated seed
    errors, and the shift of <Re^2> between samplers is given in units of its
    standard error."""
    import numpy as np
    import torch

    from paper_1711_03828_amd import analysis
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch, Melt, make_config

    w = _c4_subsystem(side)
    nch = w.species[0].n_chains
    n_obs = (nch + 1) // 2          # end-to-end vectors of every second chain
    melts = [Melt(make_config(w, replica=r, p_learn=p_learn)) for r in range(n_rep)]
    for m in melts:
        m.set_proposal(params)
        C.soma_set_self_term(m.handle, self_term)
    batch = Batch(melts)
    t0 = time.perf_counter()
    equil = max(100, int(round(20000 * scale)) // 100 * 100)
    batch.set_substeps(substeps)
    batch.capture_cycle(100, C.SOMA_MOVE_MIXED)
    batch.run_cycle(equil // 100)
    out = {"workload": (f"{n_rep} replicas (independent Philox streams) of {w.name}: "
                        f"{nch} A16B16 chains on {side}^3 cells, the density and chiN of the "
                        f"262,144-chain melt; one batched launch; end-to-end vectors of "
                        f"every second chain"),
           "common_start_learned_cycles": equil, "self_term": self_term}
    kidx = {C.SOMA_MOVE_LOCAL: 0, C.SOMA_MOVE_MIXED: 2, C.SOMA_MOVE_GIBBS: 3}
    plan = plan or _replica_plan(C, substeps, scale)
    for name, (kind, ksub, fc, discard, frames) in plan.items():
        batch.set_substeps(ksub)
        batch.capture_cycle(fc, kind)
        batch.run_cycle(discard)
        o0 = [m.observables() for m in melts]
        re = torch.empty((frames, n_rep, n_obs, 3), dtype=torch.float32, device="cuda")
        for f in range(frames):
            batch.run_cycle(1)
            for r, m in enumerate(melts):
                x = m.pos.view(nch, 32, 3)[::2]
                re[f, r] = x[:, -1] - x[:, 0]
        o1 = [m.observables() for m in melts]
        k = kidx[kind]
        acc = (sum(b.accepted[k] - a.accepted[k] for a, b in zip(o0, o1)) /
               max(1, sum(b.attempted[k] - a.attempted[k] for a, b in zip(o0, o1))))
        re_np = re.cpu().numpy().astype(np.float64)
        del re
        taus, re2s = [], []
        for r in range(n_rep):
            series = re_np[:, r].reshape(frames, -1)
            t_frames, _ = analysis.tau_int(series)
            taus.append(t_frames * fc)
            re2s.append(float((re_np[:, r] ** 2).sum(-1).mean()) / w.re_cells ** 2)
        taus, re2s = np.array(taus), np.array(re2s)
        tau = float(taus.mean())
        tau_err = float(taus.std(ddof=1) / math.sqrt(n_rep))
        out[name] = {"tau_int_cycles": tau, "tau_int_err_cycles": tau_err,
                     "tau_int_replicas": [round(float(t), 2) for t in taus],
                     "re2_over_re02": float(re2s.mean()),
                     "re2_err": float(re2s.std(ddof=1) / math.sqrt(n_rep)),
                     "re2_replicas": [round(float(v), 5) for v in re2s],
                     "discarded_cycles": discard * fc, "measured_cycles": frames * fc,
                     "discarded_over_tau": discard * fc / tau,
                     "measured_over_tau": frames * fc / tau,
                     "cycles_per_frame": fc, "substeps": ksub, "acceptance": acc,
                     "uncorrelated_samples_per_s":
                         synth.C4_MEDIUM.n_chains * rates[name] / (2.0 * tau)}
        print(f"# replicas {name}: tau_int {tau:.1f} +- {tau_err:.1f} cycles, <Re^2>/Re0^2 "
              f"{re2s.mean():.4f} +- {out[name]['re2_err']:.4f}, run {frames * fc / tau:.1f} tau",
              file=sys.stderr, flush=True)
    batch.close()
    for m in melts:
        m.close()

    def ratio(a, b):
        g = out[a]["uncorrelated_samples_per_s"] / out[b]["uncorrelated_samples_per_s"]
        rel = math.hypot(out[a]["tau_int_err_cycles"] / out[a]["tau_int_cycles"],
                         out[b]["tau_int_err_cycles"] / out[b]["tau_int_cycles"])
        shift = ((out[a]["re2_over_re02"] - out[b]["re2_over_re02"]) /
                 math.hypot(out[a]["re2_err"], out[b]["re2_err"]))
        return g, g * rel, shift

    if not all(k in out for k in ("learned", "plain", "gibbs")):
        return out
    g, ge, sh = ratio("learned", "plain")
    out["gain_learned_over_plain"] = g
    out["gain_err"] = ge
    out["re2_shift_learned_vs_plain_sigma"] = sh
    # the gain counts as one at equal observable accuracy only if <Re^2> agrees
    # within three standard errors
    out["gain_at_equal_accuracy"] = g if abs(sh) < 3.0 else None
    g2, ge2, sh2 = ratio("gibbs", "plain")
    out["gain_gibbs_over_plain"] = g2
    out["gain_gibbs_err"] = ge2
    out["re2_shift_gibbs_vs_plain_sigma"] = sh2
    g3, ge3, sh3 = ratio("learned", "gibbs")
    out["learned_over_gibbs"] = g3
    out["learned_over_gibbs_err"] = ge3
    out["seconds"] = time.perf_counter() - t0
    return out


def batched_leg(cycles: int):
    """64 uneven replicas (chains log-uniform on 2048..262144, N in {16, 32, 64},
    chiN 10..40): autotuned batched launch, graph-replayed SCMF cycles, against
    the same cycles run melt by melt."""
    import torch

    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch, Melt, make_config

    reps = synth.c3_replicas()
    melts = [Melt(make_config(w, replica=i)) for i, w in enumerate(reps)]
    n_beads = sum(w.n_beads for w in reps)
    batch = Batch(melts)
    tune = batch.autotune(3, C.SOMA_MOVE_LOCAL)
    batch.capture_cycle(10, C.SOMA_MOVE_LOCAL)
    batch.run_cycle(1)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    batch.run_cycle(cycles // 10)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (cycles // 10 * 10)
    # the same cycles melt by melt (one launch per melt and kernel), in the
    # histogram mode the batch was tuned to
    for m in melts:
        m.set_histogram(tune.hist_mode)
    e0.record(stream)
    for m in melts:
        m.cycle(10)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / 10
    obs = [m.observables() for m in melts]
    acc = sum(o.accepted[0] for o in obs) / max(1, sum(o.attempted[0] for o in obs))
    batch.close()
    for m in melts:
        m.close()
    return {"workload": f"{len(reps)} replicas, {n_beads} beads, "
                        f"{sum(w.n_cells for w in reps)} cells",
            "ms_per_cycle": ms, "bead_moves_per_s": n_beads * 1e3 / ms,
            "ms_per_cycle_unbatched": ms_single,
            "speedup_vs_unbatched": ms_single / ms,
            "tuned": {"mode": tune.mode, "grid_blocks": tune.grid_blocks,
                      "hist_mode": "binned" if tune.hist_mode else "direct",
                      "candidates": tune.candidates, "cycles_run": tune.cycles_run},
            "acceptance": acc}


def scheme_leg(cycles: int):
    """The two iteration orders of local moves (Sec. 3.1.2) over system size, as in
    the weak-scaling study of Sec. 5.2: homopolymer melts of N = 64 at
    sqrt(Nbar) = 128 (8192 beads per Re0^3, Delta L = Re0/6, kappaN = 50) with
    n = 2^7 .. 2^17 chains in a cube of side round(6 (n/128)^(1/3)) cells.  Each
    order is autotuned (launch grid), then runs graph-replayed SCMF cycles (10
    per graph) from the same initial state; bead moves per second per order
    and size."""
    import torch

    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt, make_config

    stream = torch.cuda.current_stream()
    rows = []
    for e in range(7, 18, 2):
        n = 1 << e
        side = int(round(6 * (n / 128) ** (1 / 3)))
        w = synth.Workload(f"homopolymer_N64_n{n}", (side, side, side),
                           (synth.SpeciesSpec(n, 64, 64),), 6.0, 64, 0.0, 50.0, 16)
        row = {"chains": n, "beads": w.n_beads, "grid": side}
        for name, scheme in (("set", C.SOMA_SCHEME_SET), ("molecule", C.SOMA_SCHEME_MOLECULE)):
            m = Melt(make_config(w))
            m.set_scheme(scheme)
            tune = m.autotune(3)
            m.capture_cycle(10, C.SOMA_MOVE_LOCAL)
            m.run_cycle(2)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            m.run_cycle(cycles // 10)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (cycles // 10 * 10)
            obs = m.observables()
            row[name] = {"ms_per_cycle": ms, "bead_moves_per_s": w.n_beads * 1e3 / ms,
                         "grid_blocks": tune.grid_blocks,
                         "acceptance": obs.accepted[0] / max(1, obs.attempted[0])}
            m.close()
        row["set_over_molecule"] = row["set"]["bead_moves_per_s"] / row["molecule"]["bead_moves_per_s"]
        print(f"# schemes n={n}: SET {row['set']['bead_moves_per_s']:.3e}, molecule "
              f"{row['molecule']['bead_moves_per_s']:.3e} moves/s", file=sys.stderr, flush=True)
        rows.append(row)
    return {"workload": "homopolymer N=64, sqrt(Nbar)=128, n=2^7..2^17 chains",
            "cycles": cycles // 10 * 10, "sizes": rows}


def arch_leg(cycles: int):
    """General molecular architectures (Sec. 3.2.1): the 262,144-chain A16B16 melt
    swept by the linear kernel and, given as an architecture, by the
    general-architecture kernel (same bits, the cost of generality), a melt
    of 6-arm stars (31 monomers, arms of 5, A core half) and a melt of ABC
    triblocks (three bead types, Sec. 2.1) at the same density.
    Graph-replayed SCMF cycles."""
    import numpy as np
    import torch

    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt, make_config

    stream = torch.cuda.current_stream()

    def timed(m):
        m.capture_cycle(10)
        m.run_cycle(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        m.run_cycle(cycles // 10)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / (cycles // 10 * 10)

    out = {}
    w = synth.C4_MEDIUM
    for name, arch in (("linear_kernel", False), ("architecture_kernel", True)):
        m = Melt(make_config(w))
        if arch:
            m.set_architecture(synth.linear_architecture(32, 16))
        ms = timed(m)
        out[name] = {"workload": w.name, "ms_per_cycle": ms, "bead_moves_per_s": w.n_beads * 1e3 / ms}
        m.close()
    n, bonds = synth.star_bonds(6, 5)
    types = [0] + [0 if (i - 1) % 5 < 2 else 1 for i in range(1, n)]
    n_chains = w.n_beads // n
    ws = synth.Workload("star6x5_melt_grid96", w.grid, (synth.SpeciesSpec(n_chains, n, 0),),
                        6.0, 32, w.chi_n, w.kappa_n, 16)
    k0 = 3.0 * 31 / 36.0
    pos = torch.from_numpy(synth.tree_walks(7, n_chains, n, bonds, w.grid, 1 / math.sqrt(k0)))
    m = Melt(make_config(ws), positions=pos)
    m.set_architecture(synth.encode_architecture(n, types, bonds))
    ms = timed(m)
    obs = m.observables()
    out["star_melt"] = {"workload": ws.name, "molecules": n_chains, "n_beads": ws.n_beads,
                        "ms_per_cycle": ms, "bead_moves_per_s": ws.n_beads * 1e3 / ms,
                        "acceptance": obs.accepted[0] / max(1, obs.attempted[0]),
                        "counts_conserved": obs.counts_conserved}
    m.close()
    # ABC triblock terpolymer A11 B10 C11: three types, fields from a chi_ij N matrix
    n = 32
    types = [0] * 11 + [1] * 10 + [2] * 11
    bonds = [(i, i + 1) for i in range(n - 1)]
    chi = [[0.0, w.chi_n, 2.0 * w.chi_n], [w.chi_n, 0.0, w.chi_n], [2.0 * w.chi_n, w.chi_n, 0.0]]
    wt = synth.Workload("abc_triblock_A11B10C11_grid96", w.grid,
                        (synth.SpeciesSpec(w.n_beads // n, n, 0),), 6.0, 32, w.chi_n, w.kappa_n, 16)
    m = Melt(make_config(wt))
    m.set_types(chi)
    m.set_architecture(synth.encode_architecture(n, types, bonds))
    ms_t = timed(m)
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        m.update_fields()
    e1.record(stream)
    torch.cuda.synchronize()
    field_ms = e0.elapsed_time(e1) / reps
    obs = m.observables()
    per_type = m.type_counts()
    field_bytes = wt.n_cells * (2 * 4 + 3 * 4)   # two packed u32 count planes read, three fields written
    out["abc_triblock_melt"] = {
        "workload": wt.name, "n_types": 3, "chi_n_matrix": chi, "n_beads": wt.n_beads,
        "ms_per_cycle": ms_t, "bead_moves_per_s": wt.n_beads * 1e3 / ms_t,
        "field_refresh_ms": field_ms, "field_refresh_GBs": field_bytes / field_ms / 1e6,
        "acceptance": obs.accepted[0] / max(1, obs.attempted[0]),
        "type_counts": per_type, "counts_conserved": obs.counts_conserved}
    m.close()
    print(f"# architectures: linear {out['linear_kernel']['ms_per_cycle']:.3f} ms, as architecture "
          f"{out['architecture_kernel']['ms_per_cycle']:.3f} ms, stars {ms:.3f} ms, ABC triblock "
          f"{ms_t:.3f} ms per cycle (3-type field {field_ms * 1e3:.1f} us)",
          file=sys.stderr, flush=True)
    return out


def film_leg(kind: str, lateral_re: float, cycles: int):
    """The thin-film workloads of Sec. 5.6 on one GPU: diblocks of N = 100 at
    sqrt(Nbar) = 85.7 (Delta L = Re0/6, kappaN = 50), lamella-forming (f = 0.5,
    chiN = 17, film thickness 1.2 Re0) or cylinder-forming (f = 0.75, chiN = 28,
    0.75 Re0), lateral size lateral_re x lateral_re Re0 (periodic), between two
    impenetrable, non-preferential walls (one plane of cells each).  Disordered
    start (Gaussian walks folded into the film) quenched to chiN; graph-replayed
    SCMF cycles; the in-plane structure factor S(q_par) at the end and the
    domain spacing 2 pi / q* it implies."""
    import numpy as np
    import torch

    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt, make_config

    f, chi_n, lz_re = (0.5, 17.0, 1.2) if kind == "lam" else (0.75, 28.0, 0.75)
    n, re = 100, 6.0
    side = int(round(lateral_re * re))
    inner = int(round(lz_re * re))
    nz = inner + 2
    n_chains = int(round(85.7 * n / re ** 3 * side * side * inner / n))
    w = synth.Workload(f"film_{kind}_{lateral_re:g}Re0_N100", (side, side, nz),
                       (synth.SpeciesSpec(n_chains, n, int(round(f * n))),), re, n, chi_n, 50.0, 16)
    t0 = time.perf_counter()
    m = Melt(make_config(w))
    z = m.pos.view(-1, 3)[:, 2]            # fold every z into the film interior [1, nz - 1)
    t = torch.remainder(z - 1.0, 2.0 * inner)
    z.copy_(1.0 + torch.where(t < inner, t, 2.0 * inner - t))
    z.clamp_(1.0, float(np.nextafter(np.float32(nz - 1), np.float32(0))))
    m.rebuild_histogram()
    forbid = torch.from_numpy(synth.pack_mask(synth.wall_cells(w.grid, [0, nz - 1]))
                              .view(np.int32)).cuda()
    m.set_external(None, forbid)
    tune = m.autotune(2)
    m.capture_cycle(10)
    m.run_cycle(1)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    m.run_cycle(cycles // 10)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (cycles // 10 * 10)
    obs = m.observables()
    ws = torch.empty(C.soma_sq_workspace_bytes(m.handle), dtype=torch.uint8, device="cuda")
    sq = torch.empty(w.n_cells, dtype=torch.float64, device="cuda")
    C.soma_structure_factor(m.handle, ws.data_ptr(), ws.numel(), sq.data_ptr(),
                            stream.cuda_stream)
    q, mean, cnt, peak = C.soma_sq_plane_shells(sq.cpu().numpy(), w.grid, side // 2)
    z = m.pos.view(-1, 3)[:, 2]
    zc = torch.remainder(torch.floor(z), nz)
    in_walls = int(((zc == 0) | (zc == nz - 1)).sum().item())
    m.close()
    print(f"# film {kind}: {w.n_beads} beads, {ms:.3f} ms per cycle, S(q_par) peak shell {peak}",
          file=sys.stderr, flush=True)
    return {"workload": w.name, "n_beads": w.n_beads, "n_chains": n_chains,
            "grid": list(w.grid), "f": f, "chi_n": chi_n, "cycles": cycles // 10 * 10,
            "ms_per_cycle": ms, "bead_moves_per_s": w.n_beads * 1e3 / ms,
            "grid_blocks": tune.grid_blocks, "setup_s": t_setup,
            "acceptance": obs.accepted[0] / max(1, obs.attempted[0]),
            "beads_in_walls": in_walls, "counts_conserved": obs.counts_conserved,
            "sq_peak_shell": peak, "q_star": float(q[peak]),
            "spacing_over_re0": float(2 * math.pi / q[peak] / re) if peak else None}


def blend_leg(rate_cycles: int, tau_frames: int, frame_cycles: int, plain_mult: int,
              equil_cycles: int, tau_scale: float, substeps: int, p_learn: float = 1.0,
              lag: int = 64):
    """Ternary blend replicas (32 melts of A16B16 diblocks with A16 and B16
    homopolymers, chiN 15..35): one network per species trained on the blend's
    own plain trajectories, used inside graph-captured batched cycles.

    Rates at full size (about 4.2e7 beads); tau_int of the diblocks' end-to-end
    vectors and the S(q) peak shell of every replica on a copy scaled by
    `tau_scale` in chains (same density and chemistry), with the diblocks' <Re^2>.
    The learned sampler runs `substeps` field refreshes per cycle."""
    import numpy as np
    import torch

    from paper_1711_03828_amd import analysis, learned
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch, Melt, make_config

    def build(reps):
        melts = [Melt(make_config(w, replica=i, p_learn=p_learn)) for i, w in enumerate(reps)]
        return melts, Batch(melts)

    out = {}
    # training data from the full-size blend: per species, 2^15 beads per replica and round
    reps = synth.c5_replicas()
    melts, batch = build(reps)
    batch.cycle(20)
    n_round, rounds = 1 << 15, 4
    data = {sp: (torch.empty((len(melts) * rounds * n_round, 60), device="cuda"),
                 torch.empty((len(melts) * rounds * n_round, 3), device="cuda")) for sp in range(3)}
    r0 = torch.empty((len(melts), 3, n_round, 3), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    batch.capture_cycle(lag, C.SOMA_MOVE_LOCAL)
    for k in range(rounds):
        for i, m in enumerate(melts):
            for sp in range(3):
                off = ((k * len(melts)) + i) * n_round
                C.soma_collect_training(m.handle, n_round, k, 0, data[sp][0][off].data_ptr(),
                                        r0[i, sp].data_ptr(), 0, 0, s, species=sp)
        batch.run_cycle(1)
        for i, m in enumerate(melts):
            for sp in range(3):
                off = ((k * len(melts)) + i) * n_round
                C.soma_collect_training(m.handle, n_round, k, 1, 0, r0[i, sp].data_ptr(),
                                        data[sp][1][off].data_ptr(), 0, s, species=sp)
    nets = []
    for sp in range(3):
        params = learned.init_params(data[sp][0], seed=10 + sp)
        losses = learned.train(params, data[sp][0], data[sp][1], steps=2000, batch=8192,
                               loss_every=500)
        nets.append(params)
        out[f"species{sp}_loss"] = [losses[0], losses[-1]]
    del data
    for m in melts:
        for sp in range(3):
            m.set_proposal(nets[sp], species=sp)
    n_beads = sum(w.n_beads for w in reps)
    stream = torch.cuda.current_stream()
    ksub = {"plain": 1, "learned": substeps}
    for name, kind in (("plain", C.SOMA_MOVE_LOCAL), ("learned", C.SOMA_MOVE_MIXED)):
        batch.set_substeps(ksub[name])
        batch.capture_cycle(10, kind)
        batch.run_cycle(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        batch.run_cycle(rate_cycles // 10)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (rate_cycles // 10 * 10)
        out[name] = {"ms_per_cycle": ms, "bead_moves_per_s": n_beads * 1e3 / ms,
                     "substeps": ksub[name]}
    out["workload"] = f"{len(reps)} blend replicas, {n_beads} beads"
    batch.close()
    for m in melts:
        m.close()
    # tau_int and S(q) peaks on the scaled copy
    sreps = synth.c5_replicas(scale=tau_scale)
    melts, batch = build(sreps)
    for m in melts:
        for sp in range(3):
            m.set_proposal(nets[sp], species=sp)
    batch.set_substeps(substeps)
    batch.capture_cycle(frame_cycles, C.SOMA_MOVE_MIXED)
    batch.run_cycle(max(1, equil_cycles // frame_cycles))
    ws = [torch.empty(C.soma_sq_workspace_bytes(m.handle), dtype=torch.uint8, device="cuda")
          for m in melts]
    for name, kind, mult in (("learned", C.SOMA_MOVE_MIXED, 1), ("plain", C.SOMA_MOVE_LOCAL,
                                                                  plain_mult)):
        batch.set_substeps(ksub[name])
        batch.capture_cycle(frame_cycles * mult, kind)
        series = []
        for f in range(tau_frames):
            batch.run_cycle(1)
            series.append(torch.cat([_re_vectors_species(m, w) for m, w in zip(melts, sreps)]))
        xs = torch.stack(series)
        re2 = float((xs ** 2).sum(-1).mean()) / 36.0
        tau, window = analysis.tau_int(xs.reshape(tau_frames, -1).cpu().numpy())
        tau *= frame_cycles * mult
        peaks = []
        for m, w, wsb in zip(melts, sreps, ws):
            sq = torch.empty(w.n_cells, dtype=torch.float64, device="cuda")
            C.soma_structure_factor(m.handle, wsb.data_ptr(), wsb.numel(), sq.data_ptr(), s)
            torch.cuda.synchronize()
            _, mean, _, peak = C.soma_sq_shells(sq.cpu().numpy(), w.grid, 16)
            peaks.append(int(peak))
        out[name].update({"tau_int_cycles": tau, "window_frames": window,
                          "diblock_re2_over_re02": re2,
                          "uncorrelated_samples_per_s":
                              sum(w.species[0].n_chains for w in reps) * 1e3 /
                              out[name]["ms_per_cycle"] / (2.0 * tau),
                          "sq_peak_shells": peaks})
        print(f"# blend {name}: tau_int {tau:.1f} cycles, S(q) peaks {peaks[:8]}",
              file=sys.stderr, flush=True)
    out["gain_uncorrelated_samples_per_s"] = (out["learned"]["uncorrelated_samples_per_s"] /
                                              out["plain"]["uncorrelated_samples_per_s"])
    out["tau_workload"] = (f"the same 32 replicas with {tau_scale:g} of the chains "
                           f"({sum(w.n_beads for w in sreps)} beads); diblock end-to-end vectors")
    batch.close()
    for m in melts:
        m.close()
    return out


def _re_vectors_species(melt, w):
    """End-to-end vectors of the first species' chains (the diblocks)."""
    sp = w.species[0]
    x = melt.pos[:sp.n_chains * sp.n].view(sp.n_chains, sp.n, 3)
    return (x[:, -1] - x[:, 0]).double()


def copy_bandwidth():
    """Device-to-device copy bandwidth (read + write bytes per second) of a 4 GiB
    working set (HBM) and a 128 MiB one (resident in the 256 MB Infinity Cache),
    the measured denominators beside the datasheet peak."""
    import torch
    out = {}
    for name, nbytes, reps in (("hbm_4GiB", 4 << 30, 5), ("mall_128MiB", 128 << 20, 50)):
        src = torch.ones(nbytes // 8, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = 2 * src.numel() * 4 / (ms * 1e-3) / 1e9
        del src, dst
    out["unit"] = "GB/s"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c4"])
    ap.add_argument("--move", default="local", choices=["local", "smc"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the plain-vs-learned proposal comparison")
    ap.add_argument("--p-learn", type=float, default=1.0,
                    help="probability of the learned move per bead (else the local move)")
    ap.add_argument("--learned-substeps", type=int, default=8,
                    help="chain subsets (field refreshes) per cycle for the learned and "
                         "bond-Gibbs samplers of the 262,144-chain melt")
    ap.add_argument("--blend-substeps", type=int, default=2,
                    help="chain subsets per cycle for the blend leg's learned sampler")
    ap.add_argument("--no-self-term", action="store_true",
                    help="the learned-proposal leg's samplers without the single-bead self "
                         "term of cell-changing moves (the paper's SCMF)")
    ap.add_argument("--replicas", type=int, default=8,
                    help="independent replicas for tau_int and <Re^2> of each sampler")
    ap.add_argument("--replica-side", type=int, default=32,
                    help="cells per side of a replica (the learned-proposal melt's density)")
    ap.add_argument("--tau-scale", type=float, default=1.0,
                    help="scales the replica runs' lengths (1: about 50 tau_int measured; "
                         "0: no replica runs)")
    ap.add_argument("--train-steps", type=int, default=3000,
                    help="Adam steps of the first training of the learned proposal")
    ap.add_argument("--tau-frames", type=int, default=400,
                    help="frames per tau_int run of the blend leg")
    ap.add_argument("--frame-cycles", type=int, default=50,
                    help="cycles between frames of the blend leg's learned run")
    ap.add_argument("--equil-cycles", type=int, default=20000,
                    help="learned-sampler cycles before the tau_int runs")
    ap.add_argument("--plain-frame-mult", type=int, default=8,
                    help="the blend leg's plain frames are this many times further apart")
    ap.add_argument("--no-blend", action="store_true",
                    help="skip the ternary-blend batched learned-proposal measurement")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-replica batched measurement")
    ap.add_argument("--no-schemes", action="store_true",
                    help="skip the SET vs molecule-parallel comparison over system size")
    ap.add_argument("--learned-lag", type=int, default=64,
                    help="plain cycles between a training sample's features and its target")
    ap.add_argument("--no-arch", action="store_true",
                    help="skip the general-architecture measurement")
    ap.add_argument("--film", choices=["lam", "hex"], default="lam",
                    help="thin-film workload: lamella- or cylinder-forming diblocks")
    ap.add_argument("--film-lateral", type=float, default=200.0,
                    help="lateral film size in Re0 (the paper's films: 200)")
    ap.add_argument("--no-second-film", action="store_true",
                    help="skip the cylinder-forming film after the lamella-forming one")
    ap.add_argument("--film-cycles", type=int, default=2500,
                    help="SCMF cycles of the film run after the quench (0: skip the film)")
    ap.add_argument("--launch", default="auto",
                    help="launch shape of the main leg's sweeps: 'auto' (autotuned) or "
                         "HIST,THREADS,GRID, e.g. binned,128,0 (HIST: direct or binned; "
                         "GRID 0: one block per tile group)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the SCMF path here runs on a single "
              "device (--gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.launch != "auto":
        parts = args.launch.split(",")
        if (len(parts) != 3 or parts[0] not in ("direct", "binned")
                or not all(p.isdigit() for p in parts[1:])):
            ap.error("--launch: 'auto' or HIST,THREADS,GRID (HIST direct or binned)")

    import torch

    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt, make_config

    w = {"c1": synth.C1_SMALL, "c2": synth.C2_LARGE, "c4": synth.C4_MEDIUM}[args.workload]
    move = C.SOMA_MOVE_LOCAL if args.move == "local" else C.SOMA_MOVE_SMC
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    melt = Melt(make_config(w))            # device-side Gaussian-walk init + fields
    torch.cuda.synchronize()
    print(f"# initialised {w.name}: {w.n_beads} beads, {w.n_cells} cells", file=sys.stderr,
          flush=True)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        melt.sweep(1, move)
        melt.update_fields()
    # launch shape: histogram mode x block size x grid, timed on real cycles
    # (results do not depend on it), or the one named by --launch
    if args.launch == "auto":
        tune_main = melt.autotune(3, move)
    else:
        hist, threads, blocks = args.launch.split(",")
        tune_main = types.SimpleNamespace(
            hist_mode=C.SOMA_HIST_BINNED if hist == "binned" else C.SOMA_HIST_DIRECT,
            block_threads=int(threads), grid_blocks=int(blocks), candidates=0)
        melt.set_histogram(tune_main.hist_mode)
        C.soma_set_sweep_threads(melt.handle, tune_main.block_threads)
        C.soma_set_sweep_blocks(melt.handle, tune_main.grid_blocks)
    torch.cuda.synchronize()
    print(f"# tuned: histogram {'binned' if tune_main.hist_mode else 'direct'}, "
          f"{tune_main.block_threads} threads, grid {tune_main.grid_blocks}, "
          f"{tune_main.candidates} candidates", file=sys.stderr, flush=True)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        melt.sweep(1, move)
        e1.record(stream)
        melt.update_fields()
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweep_ms = sum(e0.elapsed_time(e1) for e0, e1, _ in ev) / args.steps
    field_ms = sum(e1.elapsed_time(e2) for _, e1, e2 in ev) / args.steps
    obs = melt.observables()
    k = 0 if move == C.SOMA_MOVE_LOCAL else 1
    acc = obs.accepted[k] / max(1, obs.attempted[k])
    print(f"# sweep {sweep_ms:.4f} ms, field {field_ms:.4f} ms, acceptance {acc:.4f}, "
          f"<Re^2>/Re0^2 {obs.re2_sum / w.n_chains / w.re_cells ** 2:.4f}, "
          f"conserved {obs.counts_conserved}", file=sys.stderr, flush=True)

    ms_per_step = wall * 1e3 / args.steps
    value = w.n_beads * args.steps / wall
    launch = {"hist_mode": "binned" if tune_main.hist_mode else "direct",
              "block_threads": tune_main.block_threads, "grid_blocks": tune_main.grid_blocks}
    nbytes, per_bead, per_cell = algorithmic_bytes(w)
    achieved = nbytes / (sweep_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "bead-moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_beads": w.n_beads, "n_chains": w.n_chains,
                   "grid": list(w.grid), "chi_n": w.chi_n, "kappa_n": w.kappa_n,
                   "move": args.move, "count_width": w.count_width,
                   "step": "1 MC sweep (fused histogram) + field update"},
        "launch": dict(launch, candidates=tune_main.candidates),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(w, args.move, launch),
                     "kernel": (f"mc_sweep_{args.move}_kernel" +
                                (" + bin_apply_kernel" if tune_main.hist_mode else "")),
                     "kernel_ms": sweep_ms,
                     "algorithmic_bytes": nbytes,
                     "bytes_per_bead": per_bead, "bytes_per_cell": per_cell},
        "field_update": {"ms": field_ms,
                         "achieved_GBs": field_bytes(w) / (field_ms * 1e-3) / 1e9},
        "acceptance": acc,
    }
    # histogram atomic rate: a sweep issues two count atomics per bead that changes
    # cell; counted for one more sweep by comparing the cells before and after it
    grid_t = torch.tensor(w.grid, dtype=torch.float64, device=melt.pos.device)

    def cells():
        return torch.remainder(torch.floor(melt.pos.view(-1, 3).double()), grid_t)

    before = cells()
    melt.sweep(1, move)
    changed = int((cells() != before).any(dim=1).sum().item())
    del before
    # against a from-scratch recount: one atomic per bead (before aggregation)
    melt.rebuild_histogram()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        melt.rebuild_histogram()
    e1.record(stream)
    torch.cuda.synchronize()
    recount_ms = e0.elapsed_time(e1) / 3
    # the device's scattered-update rates over an array the size of this melt's
    # counts, with as many updates as the sweep's direct histogram issues
    probe = torch.zeros(melt.counts.numel() * melt.counts.element_size() // 4,
                        dtype=torch.int32, device="cuda")
    probe_rates = {}
    for mode, name in ((0, "atomic_random"), (1, "atomic_local"), (2, "store_random")):
        C.soma_probe_atomics(probe.data_ptr(), probe.numel(), 2 * changed, mode, 1,
                             stream.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for rep in range(3):
            C.soma_probe_atomics(probe.data_ptr(), probe.numel(), 2 * changed, mode, 2 + rep,
                                 stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        probe_rates[name] = {"per_s": 2 * changed / (ms * 1e-3), "ms": ms}
    del probe
    result["atomics"] = {"per_sweep": 2 * changed, "per_s": 2 * changed / (sweep_ms * 1e-3),
                         "probe": probe_rates,
                         "beads_changing_cell": changed / w.n_beads,
                         "hist_mode": "binned" if tune_main.hist_mode else "direct",
                         "recount_ms": recount_ms,
                         "recount_beads_per_s": w.n_beads / (recount_ms * 1e-3),
                         "recount": "binned: a reservation atomic per (wave, brick), the "
                                    "updates added brick by brick in LDS"}
    if args.move == "local":
        # the molecule-parallel order (Sec. 3.1.2, scheme 1) on the same melt
        melt.set_scheme(C.SOMA_SCHEME_MOLECULE)
        tune = melt.autotune(2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        melt.cycle(10)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_mol = e0.elapsed_time(e1) / 10
        result["molecule_order"] = {"ms_per_cycle": ms_mol,
                                    "bead_moves_per_s": w.n_beads * 1e3 / ms_mol,
                                    "grid_blocks": tune.grid_blocks}
        melt.set_scheme(C.SOMA_SCHEME_SET)
        C.soma_set_sweep_blocks(melt.handle, 0)
    melt.close()
    # the second move kind of this workload: smart-MC, with the kept gradient field
    melt = Melt(make_config(w))
    melt.keep_grad_field()
    smc = {}
    for _ in range(2):
        melt.cycle(1, C.SOMA_MOVE_SMC)
    tune_smc = melt.autotune(2, C.SOMA_MOVE_SMC)
    smc["launch"] = {"hist_mode": "binned" if tune_smc.hist_mode else "direct",
                     "block_threads": tune_smc.block_threads}
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    melt.sweep(10, C.SOMA_MOVE_SMC)
    e1.record(stream)
    for _ in range(10):
        melt.update_fields()
    e2.record(stream)
    torch.cuda.synchronize()
    smc["sweep_ms"] = e0.elapsed_time(e1) / 10
    smc["field_and_gradient_ms"] = e1.elapsed_time(e2) / 10
    smc["bead_moves_per_s"] = w.n_beads * 1e3 / (smc["sweep_ms"] + smc["field_and_gradient_ms"])
    obs = melt.observables()
    smc["acceptance"] = obs.accepted[1] / max(1, obs.attempted[1])
    result["smart_mc"] = smc
    # local and smart-MC moves 50/50: cycles of the two kinds alternating (the
    # composition of two kernels that each leave the distribution invariant)
    for _ in range(2):
        melt.cycle(1, C.SOMA_MOVE_LOCAL)
        melt.cycle(1, C.SOMA_MOVE_SMC)
    e0.record(stream)
    for _ in range(10):
        melt.cycle(1, C.SOMA_MOVE_LOCAL)
        melt.cycle(1, C.SOMA_MOVE_SMC)
    e1.record(stream)
    torch.cuda.synchronize()
    mix_ms = e0.elapsed_time(e1) / 20
    result["local_smc_mixture"] = {"ms_per_cycle": mix_ms,
                                   "bead_moves_per_s": w.n_beads * 1e3 / mix_ms,
                                   "cycles": 20, "order": "local and smart-MC cycles alternating"}
    melt.close()
    copy = copy_bandwidth()
    result["roofline"]["copy_bandwidth"] = copy
    result["roofline"]["frac_of_copy_hbm"] = achieved / copy["hbm_4GiB"]
    if not args.no_learned:
        result["learned_proposal"] = learned_leg(args.p_learn, args.equil_cycles,
                                                 args.learned_substeps, args.learned_lag,
                                                 args.replicas, args.replica_side,
                                                 args.tau_scale, args.train_steps,
                                                 0 if args.no_self_term else 1)
    if not args.no_batched:
        result["batched"] = batched_leg(50)
    if not args.no_schemes:
        result["schemes"] = scheme_leg(200)
    if not args.no_arch:
        result["architectures"] = arch_leg(200)
    if args.film_cycles > 0:
        result["film"] = film_leg(args.film, args.film_lateral, args.film_cycles)
        if args.film == "lam" and not args.no_second_film:   # the paper's second film system
            result["film_hex"] = film_leg("hex", args.film_lateral, args.film_cycles)
    if not args.no_blend:
        result["blend"] = blend_leg(50, args.tau_frames // 2, args.frame_cycles,
                                    args.plain_frame_mult, args.equil_cycles // 2, 1.0 / 16,
                                    args.blend_substeps, args.p_learn, args.learned_lag)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
