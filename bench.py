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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "bead MC moves/s and uncorrelated samples/s, plain vs learned proposal, 1 GPU"
HBM_PEAK_GBS = 8000.0


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


def kernel_source_digest() -> str:
    """SHA-1 of the HIP sources, to tell whether stored counters still apply."""
    import glob
    import hashlib
    h = hashlib.sha1()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1711_03828_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(w, move: str):
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (scaled by the copy-kernel calibration), or None if the kernel
    sources changed since it was taken or no summary covers this workload."""
    path = os.path.join(ROOT, "profiles", f"mc_sweep_{move}_diblock_4M_N32_traffic.json")
    if w.name != "diblock_4M_N32_grid384x384x192" or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha1") != kernel_source_digest():
        return None
    return rec["traffic_bytes"]


def cpu_baseline(w, seconds: float):
    """The oracle as it stands, OpenMP over chains on the host cores, on a
    slab of the same melt (same density, chemistry and moves)."""
    import numpy as np

    import oracle
    from oracle import Species

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    nx, ny, nz = w.grid
    slab_z = max(1, min(nz, 12))
    frac = slab_z / nz
    s0 = w.species[0]
    n_chains = max(1, int(round(s0.n_chains * frac)))
    sample = synth.Workload(w.name + "_slab", (nx, ny, slab_z),
                            (synth.SpeciesSpec(n_chains, s0.n, s0.n_a),), w.re_cells, w.n_ref,
                            w.chi_n, w.kappa_n, w.count_width, w.a_frac, w.smc_frac)
    k0 = np.float32(3.0 * (w.n_ref - 1) / w.re_cells ** 2)
    a = np.float32(w.a_frac * w.re_cells / math.sqrt(w.n_ref - 1))
    inv_rho = np.float32(sample.n_cells / sample.n_beads)
    sp = Species(n_chains, s0.n, s0.n_a)
    pos = oracle.init_chains(sp, sample.grid, bond_sigma=np.float32(1 / math.sqrt(float(k0))),
                             seed=w.seed, origin_mode=1)
    omega = oracle.field_f32(oracle.density_hist(pos, [sp], sample.grid), inv_rho,
                             np.float32(w.chi_n), np.float32(w.kappa_n))
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        oracle.mc_sweep(pos, sp, omega, sample.grid, k0=k0, n_ref=w.n_ref, step=a, seed=w.seed,
                        sweep=sweeps, threads=threads)
        omega = oracle.field_f32(oracle.density_hist(pos, [sp], sample.grid), inv_rho,
                                 np.float32(w.chi_n), np.float32(w.kappa_n))
        sweeps += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": sample.n_beads * sweeps / dt, "unit": "bead-moves/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"{sweeps} SCMF cycles (local moves + histogram + fields) of a "
                       f"{nx}x{ny}x{slab_z}-cell slab of the same melt: {n_chains} chains, "
                       f"{sample.n_beads} beads, same density/chiN/kappaN")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c4"])
    ap.add_argument("--move", default="local", choices=["local", "smc"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the SCMF path here runs on a single "
              "device (--gpus 1).", file=sys.stderr)
        sys.exit(2)

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
    torch.cuda.synchronize()

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
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(w, args.move),
                     "kernel": f"mc_sweep_{args.move}_kernel", "kernel_ms": sweep_ms,
                     "algorithmic_bytes": nbytes,
                     "bytes_per_bead": per_bead, "bytes_per_cell": per_cell},
        "field_update": {"ms": field_ms,
                         "achieved_GBs": field_bytes(w) / (field_ms * 1e-3) / 1e9},
        "acceptance": acc,
    }
    melt.close()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
