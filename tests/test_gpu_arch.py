"""GPU parity of general molecular architectures (Sec. 3.2.1 encoding, Sec.
3.1.2 independent sets) against the oracle.

Bars: a linear chain given as an architecture moves bit for bit as the linear
kernel (both set orders, several species, walls); stars, combs and odd rings
(three sets, shuffled order) match the oracle's sweep bit for bit per molecule
without an accept-decision mismatch (at most 1e-6 of the moves, rounded up);
the kept histogram equals the recount with the architecture's types; bond
observables sum over the bonds; ideal stars keep their closed forms on the
device; malformed arrays and unsupported combinations are refused.
"""
import math

import numpy as np
import pytest

import synth
from oracle import references
from tests.gpu_helpers import custom_config, flush

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

RE = 6.0


@pytest.fixture(scope="module")
def C():
    from paper_1711_03828_amd import soma
    return soma


def _cfg(grid, species, k0, **kw):
    from oracle import Species
    return custom_config(grid, [Species(*s) for s in species], k0=k0, n_ref=32, chi_n=20.0,
                         kappa_n=40.0, local_a=0.3, count_width=16, seed=123, **kw)


@pytest.mark.parametrize("set_order,substeps", [(0, 1), (1, 1), (0, 3)])
def test_linear_architecture_equals_linear_kernel(C, set_order, substeps):
    from paper_1711_03828_amd.melt import Melt
    grid = (20, 18, 10)
    species = [(300, 32, 16), (70, 17, 5), (40, 1, 1)]
    k0 = 2.5
    pos = np.concatenate([synth.film_walks(40 + i, n_c, n, grid, 0.6, 1.0, 9.0)
                          for i, (n_c, n, _) in enumerate(species)])
    mask = torch.from_numpy(synth.pack_mask(synth.wall_cells(grid, [0, 9])).view(np.int32)).cuda()
    runs = []
    for use_arch in (False, True):
        m = Melt(_cfg(grid, species, k0, set_order=set_order), positions=torch.from_numpy(pos))
        m.set_external(None, mask)
        if use_arch:
            for sp, (_, n, n_a) in enumerate(species):
                m.set_architecture(synth.linear_architecture(n, n_a), sp)
        m.set_substeps(substeps)
        m.cycle(4)
        torch.cuda.synchronize()
        obs = m.observables()
        runs.append((m.pos.cpu().numpy(), m.counts_planes(), m.omega.cpu().numpy(),
                     obs.accepted[0], obs.b2_sum, obs.counts_conserved))
        m.close()
    for x, y in zip(runs[0][:3], runs[1][:3]):
        np.testing.assert_array_equal(x, y)
    assert runs[0][3] == runs[1][3]
    assert runs[1][4] == pytest.approx(runs[0][4], rel=1e-12)
    assert runs[0][5] == 1 and runs[1][5] == 1


def _arch(kind):
    if kind == "star":
        n, bonds = synth.star_bonds(6, 5)
        types = [0] + [0 if (i - 1) % 5 < 2 else 1 for i in range(1, n)]
    elif kind == "comb":
        n, bonds = 24, [(i, i + 1) for i in range(11)] + [(i, 12 + i) for i in range(12)]
        types = [0] * 12 + [1] * 12
    else:
        n, bonds = synth.ring_bonds(15)
        types = [0] * 8 + [1] * 7
    return n, bonds, synth.encode_architecture(n, types, bonds)


@pytest.mark.parametrize("kind", ["star", "comb", "ring", "star_walls"])
def test_architecture_sweep_matches_oracle(C, orc, kind):
    from paper_1711_03828_amd.melt import Melt
    walls = kind.endswith("_walls")
    kind = kind.replace("_walls", "")
    n, bonds, words = _arch(kind)
    n_chains = 4000
    grid = (30, 30, 30)
    k0 = np.float32(2.0)
    pos = (synth.ring_walks(61, n_chains, n, grid, 1 / math.sqrt(float(k0))) if kind == "ring"
           else synth.tree_walks(61, n_chains, n, bonds, grid, 1 / math.sqrt(float(k0))))
    mask = None
    if walls:   # a wall plane at z = 0; start every monomer outside it
        z = pos[:, 2].astype(np.float64)
        pos[:, 2] = np.where(np.floor(z) % 30 == 0, z + 1.0, z).astype(np.float32)
        mask = synth.pack_mask(synth.wall_cells(grid, [0]))
    m = Melt(_cfg(grid, [(n_chains, n, 0)], k0), positions=torch.from_numpy(pos))
    if walls:
        m.set_external(None, torch.from_numpy(mask.view(np.int32)).cuda())
    m.set_architecture(words)
    counts = orc.density_hist_arch(pos, n_chains, words, grid)
    np.testing.assert_array_equal(m.counts_planes(), counts)
    n_free = grid[0] * grid[1] * (grid[2] - 1) if walls else grid[0] * grid[1] * grid[2]
    inv_rho = np.float32(n_free / (n_chains * n))
    omega = orc.field_f32(counts, inv_rho, np.float32(20.0), np.float32(40.0), None, mask)
    np.testing.assert_array_equal(m.omega.cpu().numpy(), omega)
    m.sweep(1, C.SOMA_MOVE_LOCAL)
    torch.cuda.synchronize()
    got = m.pos.cpu().numpy()
    ref = pos.copy()
    acc, _ = orc.mc_sweep_arch(ref, n_chains, words, omega, grid, k0=k0, n_ref=32,
                               step=np.float32(0.3), seed=123, sweep=0, threads=8, forbid=mask)
    if walls:
        zc = np.floor(got[:, 2].astype(np.float64)).astype(np.int64) % 30
        assert (zc != 0).all()
    bad = (got.reshape(n_chains, -1) != ref.reshape(n_chains, -1)).any(axis=1)
    allowed = math.ceil(1e-6 * n_chains * n)
    flush(kind, "mismatched molecules", int(bad.sum()), "allowed", allowed)
    assert bad.sum() <= allowed
    np.testing.assert_array_equal(m.counts_planes(), orc.density_hist_arch(got, n_chains, words, grid))
    obs = m.observables()
    assert obs.counts_conserved == 1
    assert abs(int(obs.accepted[0]) - int(acc)) <= n * allowed
    p = got.reshape(n_chains, n, 3).astype(np.float64)
    b2 = sum(((p[:, i] - p[:, j]) ** 2).sum() for i, j in bonds)
    assert obs.b2_sum == pytest.approx(b2, rel=1e-9)
    m.close()


def test_ideal_star_on_device(C):
    from paper_1711_03828_amd.melt import Melt
    arms, arm_len = 6, 5
    n, bonds = synth.star_bonds(arms, arm_len)
    words = synth.encode_architecture(n, [0] * n, bonds)
    k0 = float(np.float32(3.0 * 31 / RE ** 2))
    n_chains = 32768
    grid = (40, 40, 40)
    pos = synth.tree_walks(71, n_chains, n, bonds, grid, 1 / math.sqrt(k0))
    cfg = custom_config(grid, [__import__("oracle").Species(n_chains, n, n)], k0=k0, n_ref=32,
                        local_a=float(np.float32(0.1 * RE / math.sqrt(31))), count_width=16,
                        seed=5)
    m = Melt(cfg, positions=torch.from_numpy(pos))
    m.set_architecture(words)
    m.omega.zero_()
    m.sweep(20, C.SOMA_MOVE_LOCAL)
    obs = m.observables()
    torch.cuda.synchronize()
    a = float(np.float32(0.1 * RE / math.sqrt(31)))
    deg = np.zeros(n, int)
    for i, j in bonds:
        deg[i] += 1
        deg[j] += 1
    exp = sum(references.ideal_local_acceptance(g * k0 / 2, a)[0] for g in deg) / n
    rate = obs.accepted[0] / obs.attempted[0]
    flush("star acceptance", rate, "closed form", exp)
    assert abs(rate - exp) < 6 * math.sqrt(exp * (1 - exp) / obs.attempted[0]) + 1e-4
    # <b^2> per bond and arm-end to core distance
    b2_exp = 3 / k0 * (n - 1)
    assert abs(obs.b2_sum / n_chains - b2_exp) < 5 * math.sqrt(2 / 3 / (n - 1)) * b2_exp / math.sqrt(n_chains)
    p = m.pos.cpu().numpy().reshape(n_chains, n, 3).astype(np.float64)
    r2 = ((p[:, 0] - p[:, arm_len]) ** 2).sum(axis=1)
    assert abs(r2.mean() - 3 * arm_len / k0) < 4 * r2.std() / math.sqrt(n_chains)
    m.close()


def test_refusals(C):
    from paper_1711_03828_amd.melt import Melt
    m = Melt(_cfg((12, 12, 12), [(100, 8, 4)], 2.0, smc_a=0.05))
    with pytest.raises(C.SomaError):
        m.set_architecture(synth.linear_architecture(9, 4))      # N differs
    bad = synth.linear_architecture(8, 4)
    bad[4] = bad[4] & 0xFF000000                                  # one-sided bond
    with pytest.raises(C.SomaError):
        m.set_architecture(bad)
    m.set_architecture(synth.encode_architecture(*synth.ring_bonds(8)[:1], [0] * 8,
                                                 synth.ring_bonds(8)[1]))
    with pytest.raises(C.SomaError):
        m.sweep(1, C.SOMA_MOVE_SMC)
    m.set_scheme(C.SOMA_SCHEME_MOLECULE)
    with pytest.raises(C.SomaError):
        m.sweep(1, C.SOMA_MOVE_LOCAL)
    m.set_scheme(C.SOMA_SCHEME_SET)
    m.sweep(2, C.SOMA_MOVE_LOCAL)
    m.set_architecture(None)                                      # back to linear
    m.sweep(1, C.SOMA_MOVE_SMC)
    assert m.observables().counts_conserved == 1
    m.close()
