"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (written here, applied element by element on identical seeded inputs):
  * histogram: bit-exact (integers);
  * fields: bit-exact against the oracle's fixed FP32 operation order;
  * local moves, one sweep from identical state and fields: positions
    bit-identical (both sides compute r' = fma(a, v, r) in FP32) for every
    chain without an accept-decision mismatch; mismatches (FP32 vs FP64
    energies at the Metropolis threshold) at most 1e-6 of the attempted moves,
    rounded up;
  * smart-MC and bond-Gibbs moves: positions within 1e-5 Re0 per coordinate, same
    mismatch bar;
  * initial walks: origins bit-exact, every bead within 1e-5 Re0;
  * observables: FP64 sums within 1e-9 relative.
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species
from tests.gpu_helpers import (constants, custom_config, device_config, flush,
                               stepwise_cycles, unpack_counts, walks_for)

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

RE = 6.0
TOL_POS = 1e-5 * RE


@pytest.fixture(scope="module")
def C():
    from paper_1711_03828_amd import soma
    return soma


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _gpu_hist(C, cfg, pos_np):
    pos = torch.from_numpy(pos_np).cuda()
    _, cnt_b, _, _ = C.soma_buffer_sizes(cfg)
    counts = torch.zeros(cnt_b // 4, dtype=torch.int32, device="cuda")
    C.soma_density_hist(cfg, pos.data_ptr(), counts.data_ptr(), _stream())
    torch.cuda.synchronize()
    return unpack_counts(counts.cpu().numpy(), cfg.count_width)


HIST_CASES = [
    ("diblock_1k_grid24_u16", (24, 24, 24), [Species(1024, 32, 16)], 16),
    ("ragged_species_u32", (11, 7, 9), [Species(37, 32, 16), Species(5, 16, 16),
                                        Species(3, 17, 0)], 32),
    ("ragged_species_u16", (13, 5, 3), [Species(3, 17, 5), Species(0, 32, 16),
                                        Species(29, 64, 20), Species(7, 1, 0)], 16),
]


@pytest.mark.parametrize("name,grid,species,width", HIST_CASES)
def test_density_hist_bit_exact(C, orc, name, grid, species, width):
    flush("case", name)
    n_beads = sum(s.n_chains * s.n for s in species)
    pos = synth.gaussian_walks(31, 1, max(n_beads, 1), grid, 1.3)[:n_beads]
    cfg = custom_config(grid, species, k0=2.5, n_ref=32, count_width=width)
    got = _gpu_hist(C, cfg, pos)
    exp = orc.density_hist(pos, species, grid)
    np.testing.assert_array_equal(got, exp)


def test_density_hist_boundary_positions(C, orc):
    grid = (24, 10, 7)
    pos = synth.boundary_positions(grid)
    sp = [Species(pos.shape[0], 1, 1)]
    cfg = custom_config(grid, sp, k0=2.5, n_ref=32)
    np.testing.assert_array_equal(_gpu_hist(C, cfg, pos), orc.density_hist(pos, sp, grid))


@pytest.mark.parametrize("width,n_cells", [(16, 24 ** 3), (32, 693), (16, 1001), (32, 5)])
def test_field_bit_exact(C, orc, width, n_cells):
    g = np.random.default_rng(n_cells)
    planes = g.integers(0, 40, size=(2, n_cells)).astype(np.uint32)
    planes[:, :3] = [[0, 7, 3], [0, 0, 3]]          # empty, pure A, balanced
    if width == 16:
        packed = (planes[0] | (planes[1] << 16)).astype(np.uint32).view(np.int32)
    else:
        packed = (planes[0].astype(np.uint64) | (planes[1].astype(np.uint64) << 32)).view(np.int64)
    grid = (n_cells, 1, 1)
    sp = [Species(n_cells // 4 + 1, 8, 4)]
    cfg = custom_config(grid, sp, k0=2.5, n_ref=32, chi_n=23.5, kappa_n=47.0, count_width=width)
    counts = torch.from_numpy(packed.copy()).cuda()
    omega = torch.empty((2, n_cells), dtype=torch.float32, device="cuda")
    C.soma_field_from_counts(cfg, counts.data_ptr(), omega.data_ptr(), _stream())
    torch.cuda.synchronize()
    inv_rho = np.float32(n_cells / (sp[0].n_chains * 8))
    exp = orc.field_f32(planes, inv_rho, np.float32(23.5), np.float32(47.0))
    np.testing.assert_array_equal(omega.cpu().numpy(), exp)
    # the stand-alone field leaves the counts untouched
    np.testing.assert_array_equal(counts.cpu().numpy(), packed)


def _both_sides(C, orc, w, seed, pos=None):
    """Device melt and oracle state from the same synthetic walks."""
    from paper_1711_03828_amd.melt import Melt
    k0, a, A, inv_rho = constants(w)
    if pos is None:
        pos = walks_for(w, seed)
    cfg = device_config(w)
    melt = Melt(cfg, positions=torch.from_numpy(pos))
    sp = [Species(s.n_chains, s.n, s.n_a) for s in w.species]
    counts = orc.density_hist(pos, sp, w.grid)
    omega = orc.field_f32(counts, inv_rho, np.float32(w.chi_n), np.float32(w.kappa_n))
    return melt, pos.copy(), omega, sp, (k0, a, A)


def test_init_fields_bit_exact(C, orc):
    w = synth.C1_SMALL
    melt, pos, omega, sp, _ = _both_sides(C, orc, w, 41)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(melt.omega.cpu().numpy(), omega)
    np.testing.assert_array_equal(melt.counts_planes(), orc.density_hist(pos, sp, w.grid))
    obs = melt.observables()
    assert obs.counts_conserved == 1 and obs.error_flags == 0
    assert obs.h_nb == pytest.approx(orc.h_nb(orc.density_hist(pos, sp, w.grid),
                                              w.n_cells / w.n_beads, w.chi_n, w.kappa_n,
                                              w.n_ref), rel=1e-9)


def _chain_mismatch(got, exp, n, tol):
    g = got.reshape(-1, n, 3).astype(np.float64)
    e = exp.reshape(-1, n, 3).astype(np.float64)
    return np.abs(g - e).reshape(g.shape[0], -1).max(axis=1) > tol


@pytest.mark.parametrize("kind", ["local", "smc", "gibbs"])
@pytest.mark.parametrize("wname", ["c1", "ragged"])
def test_one_sweep_parity(C, orc, kind, wname):
    if wname == "c1":
        w = synth.scaled(synth.C1_SMALL, 16384, (48, 48, 48))   # 524,288 beads
    else:
        w = synth.Workload("ragged", (17, 23, 9),
                           (synth.SpeciesSpec(301, 32, 16), synth.SpeciesSpec(77, 16, 16),
                            synth.SpeciesSpec(45, 17, 4), synth.SpeciesSpec(13, 64, 13)),
                           6.0, 32, 25.0, 50.0, 32)
    flush("case", wname, kind)
    melt, pos, omega, sp, (k0, a, A) = _both_sides(C, orc, w, 42)
    move = {"local": C.SOMA_MOVE_LOCAL, "smc": C.SOMA_MOVE_SMC, "gibbs": C.SOMA_MOVE_GIBBS}[kind]
    melt.sweep(1, move)
    torch.cuda.synchronize()
    got = melt.pos.cpu().numpy()
    acc_total = 0
    off = 0
    bad_chains = 0
    chain_base = 0
    for s in sp:
        seg = pos[off:off + s.n_chains * s.n]
        acc, _ = orc.mc_sweep(seg, s, omega, w.grid, k0=k0, n_ref=w.n_ref,
                              move_kind={"local": 0, "smc": 1, "gibbs": 3}[kind],
                              step=a if kind == "local" else A, seed=w.seed, sweep=0,
                              chain_base=chain_base, threads=8)
        acc_total += acc
        gseg = got[off:off + s.n_chains * s.n]
        if kind == "local":
            bad = _chain_mismatch(gseg, seg, s.n, 0.0)
        else:
            bad = _chain_mismatch(gseg, seg, s.n, TOL_POS)
        bad_chains += int(bad.sum())
        off += s.n_chains * s.n
        chain_base += s.n_chains
    moves = w.n_beads
    allowed = math.ceil(1e-6 * moves)
    flush("mismatched chains", bad_chains, "allowed", allowed, "moves", moves)
    assert bad_chains <= allowed
    # the histogram kept by the sweep is the histogram of the final positions
    # (exactly: the library's from-scratch recount of its positions agrees) ...
    hist_gpu = melt.counts_planes()
    cfg = device_config(w)
    np.testing.assert_array_equal(hist_gpu, _gpu_hist(C, cfg, got))
    # ... and differs from the oracle's own histogram only where a bead sits in a
    # different cell on the two sides (none for local moves without mismatches;
    # for smart MC a bead within 1e-5 Re0 of a cell face)
    hist_ref = orc.density_hist(pos, sp, w.grid)
    cells_differ = int((np.floor(got.astype(np.float64)) != np.floor(pos.astype(np.float64)))
                       .any(axis=1).sum())
    if kind == "local" and bad_chains == 0:
        assert cells_differ == 0
    assert int((hist_gpu != hist_ref).sum()) <= 2 * cells_differ
    obs = melt.observables()
    kidx = {"local": 0, "smc": 1, "gibbs": 3}[kind]
    assert obs.attempted[kidx] == moves
    assert abs(int(obs.accepted[kidx]) - int(acc_total)) <= allowed
    assert obs.counts_conserved == 1  # conservation of the init histogram


def test_cycles_parity_c1(C, orc):
    """Ten SCMF cycles (sweep, histogram, field) on the 1024-chain melt, each
    cycle compared in full from the device's own state: histogram and fields
    bit-exact before and after, positions bit-identical per chain (at most
    ceil(1e-6 x moves) chains with a threshold mismatch per cycle)."""
    w = synth.C1_SMALL
    melt, pos, omega, sp, (k0, a, A) = _both_sides(C, orc, w, 43)
    inv_rho = constants(w)[3]

    def sweep(p, om, cyc):
        orc.mc_sweep(p, sp[0], om, w.grid, k0=k0, n_ref=w.n_ref, step=a, seed=w.seed,
                     sweep=cyc, threads=8)

    def field_of(counts):
        return orc.field_f32(counts, inv_rho, np.float32(w.chi_n), np.float32(w.kappa_n))

    stepwise_cycles(melt, orc, sp, w.grid, 10, sweep, field_of, n_per_chain=32)


def test_init_positions_parity(C, orc):
    w = synth.Workload("init", (40, 24, 17),
                       (synth.SpeciesSpec(500, 32, 16), synth.SpeciesSpec(77, 16, 16)),
                       6.0, 32, 20.0, 50.0, 16)
    for mode in (0, 1):
        cfg = device_config(w, origin_mode=mode)
        pos = torch.empty((w.n_beads, 3), dtype=torch.float32, device="cuda")
        C.soma_init_positions(cfg, pos.data_ptr(), _stream())
        torch.cuda.synchronize()
        got = pos.cpu().numpy()
        off = 0
        base = 0
        for s in w.species:
            exp = orc.init_chains(Species(s.n_chains, s.n, s.n_a), w.grid,
                                  bond_sigma=np.float32(1 / math.sqrt(cfg.species[0].k0)),
                                  seed=w.seed, chain_base=base, total_chains=w.n_chains,
                                  origin_mode=mode)
            g = got[off:off + s.n_chains * s.n]
            np.testing.assert_array_equal(g.reshape(-1, s.n, 3)[:, 0], exp.reshape(-1, s.n, 3)[:, 0])
            assert np.abs(g.astype(np.float64) - exp).max() < TOL_POS
            off += s.n_chains * s.n
            base += s.n_chains


def test_observables_match_oracle(C, orc):
    w = synth.C1_SMALL
    melt, pos, omega, sp, _ = _both_sides(C, orc, w, 44)
    obs = melt.observables()
    re2, rg2, b2 = orc.chain_observables(pos, 1024, 32)
    assert obs.re2_sum == pytest.approx(re2.sum(), rel=1e-9)
    assert obs.rg2_sum == pytest.approx(rg2.sum(), rel=1e-9)
    assert obs.b2_sum == pytest.approx(b2.sum(), rel=1e-9)
    k0 = constants(w)[0]
    assert obs.e_bond == pytest.approx(0.5 * float(k0) * b2.sum(), rel=1e-9)
    assert obs.e_field == pytest.approx(orc.field_energy(pos, sp[0], omega, w.grid, w.n_ref),
                                        rel=1e-9)
    assert obs.n_beads == 32768 and obs.n_chains == 1024 and obs.sweeps == 0


def test_resume_is_bit_exact(C):
    from paper_1711_03828_amd.melt import Melt
    w = synth.C1_SMALL
    pos0 = walks_for(w, 45)
    cfg = device_config(w)
    m1 = Melt(cfg, positions=torch.from_numpy(pos0))
    m1.cycle(4)
    m2 = Melt(cfg, positions=torch.from_numpy(pos0))
    m2.cycle(2)
    saved = m2.pos.cpu().numpy()
    m3 = Melt(cfg, positions=torch.from_numpy(saved))
    m3.sweep_index = 2
    m3.cycle(2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m1.pos.cpu().numpy(), m3.pos.cpu().numpy())
    np.testing.assert_array_equal(m1.omega.cpu().numpy(), m3.omega.cpu().numpy())


def test_nonfinite_position_raises_flag(C):
    from paper_1711_03828_amd.melt import Melt
    w = synth.scaled(synth.C1_SMALL, 64, (24, 24, 24))
    pos = walks_for(w, 46)
    pos[5] = [np.nan, 1.0, 2.0]
    m = Melt(device_config(w), positions=torch.from_numpy(pos))
    m.sweep(1)
    with pytest.raises(C.SomaError) as e:
        m.observables()
    assert e.value.code == C.SOMA_E_DEVICE_FLAG
    assert C.soma_check(m.handle, _stream()) & C.SOMA_FLAG_POSITION
    # the NaN bead is never moved, so the histogram stays that of the positions
    np.testing.assert_array_equal(m.counts_planes()[:, :].sum(), w.n_beads)


def test_invalid_configs_rejected(C):
    w = synth.C1_SMALL
    cfg = device_config(w)
    cfg.count_width = 8
    with pytest.raises(C.SomaError):
        C.soma_buffer_sizes(cfg)
    cfg = device_config(w)
    cfg.species[0].n = 129
    with pytest.raises(C.SomaError):
        C.soma_buffer_sizes(cfg)
