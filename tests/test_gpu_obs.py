"""GPU species amplitudes (eq. 3) and structure observables (pair histogram
by class, Sec. 5; radius of gyration, Sec. 6) against the CPU oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_1303_4523_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV).contiguous()


PRM = dict(a=25.0, gamma=4.5, sigma=3.0, dt=0.03, lam=0.65, k_bond=4.0, r0_bond=0.7, kappa=1.1, seed=23)
ENUF = dict(alpha=0.3, p=4, sigma=2.0, r_cut=3.0, lam=0.25)
TABLE = np.array([[25.0, 31.0, 27.5], [31.0, 22.0, 40.0], [27.5, 40.0, 26.0]])


def _system(L=8.0, chain=12, nq=80, seed=9):
    rs = np.random.default_rng(seed)
    n = int(round(3.0 * L ** 3))
    pos = rs.uniform(0.0, L, (n, 3))
    for i in range(1, chain):
        pos[i] = (pos[i - 1] + 0.7 * rs.normal(size=3) / math.sqrt(3)) % L
    vel = rs.normal(size=(n, 3))
    vel -= vel.mean(0)
    q = np.zeros(n)
    q[chain:chain + nq // 2] = 1.0
    q[chain + nq // 2:chain + nq] = -1.0
    bonds = np.array([(i, i + 1) for i in range(chain - 1)], dtype=np.int64)
    species = rs.integers(0, 3, n).astype(np.int32)
    species[:chain] = 1
    return pos, vel, q, bonds, species


def _dpd(L, q, bonds, precision="fp64"):
    from paper_1303_4523_amd.dpd import DPD
    e = dict(ENUF, M=wl.mesh_size(3.2 * L), Kc=int(0.8 * L))
    return DPD(L, q, PRM, bonds=bonds, enuf=e, precision=precision, device=0)


def _oracle_params(L, species):
    return dict(PRM, L=L, alpha=ENUF["alpha"], r_cut=ENUF["r_cut"], lambda_e=ENUF["lam"], Kc=int(0.8 * L),
                use_elec=1, species=species, a_table=TABLE)


def test_species_forces_and_steps_match_oracle():
    """Three species with distinct amplitudes: the force at step 0 and five
    steps of the trajectory agree with the oracle's typed DPD."""
    L = 8.0
    pos, vel, q, bonds, sp = _system(L)
    print(f"case: species L={L} N={len(q)}", flush=True)
    d = _dpd(L, q, bonds)
    d.set_species(sp, TABLE)
    tp, tv = _t(pos), _t(vel)
    F = torch.empty_like(tp)
    d.forces(tp, tv, F, step=0)
    F0 = F.cpu().numpy()
    d.run(tp, tv, F, 1, 5)
    st = d.status()
    gp, gv = tp.cpu().numpy(), tv.cpu().numpy()
    d.close()
    P = _oracle_params(L, sp)
    Fo, _ = oracle.dpd_forces(pos, vel, q, bonds, P, seed=PRM["seed"], step=0)
    e0 = np.linalg.norm(F0 - Fo) / np.linalg.norm(Fo)
    untyped, _ = oracle.dpd_forces(pos, vel, q, bonds, dict(P, species=None), seed=PRM["seed"], step=0)
    op, ov = pos.copy(), vel.copy()
    for s in range(1, 6):
        op, ov, Fo, _ = oracle.dpd_step(op, ov, Fo, q, bonds, P, seed=PRM["seed"], step=s)
    dp = gp - op
    dp -= L * np.round(dp / L)
    print(f"species: force rel rms {e0:.3e}; 5 steps max |dr| {np.abs(dp).max():.3e}")
    assert st == 0
    assert e0 < 1e-6
    assert np.linalg.norm(F0 - untyped) / np.linalg.norm(untyped) > 1e-3
    assert np.abs(dp).max() < 1e-6
    assert np.abs(gv - ov).max() < 1e-5


def test_species_batch_member_equals_alone():
    """A typed integrator stepped in a batch follows its lone trajectory bit
    for bit; set_species is refused while it is a member."""
    from paper_1303_4523_amd._lib import EnufError
    from paper_1303_4523_amd.batch import Batch
    L = 8.0
    pos, vel, q, bonds, sp = _system(L, seed=4)
    out = []
    for batched in (False, True):
        d = _dpd(L, q, bonds, precision="mixed")
        d.set_species(sp, TABLE)
        tp, tv = _t(pos), _t(vel)
        F = torch.empty_like(tp)
        d.forces(tp, tv, F, step=0)
        if batched:
            b = Batch("mixed", device=0)
            b.add(d, tp, tv, F, first_step=1)
            with pytest.raises(EnufError):
                d.set_species(sp, TABLE)
            b.run(6)
            torch.cuda.synchronize()
            b.close()
        else:
            d.run(tp, tv, F, 1, 6)
        torch.cuda.synchronize()
        out.append((tp.cpu().numpy(), tv.cpu().numpy(), d.status()))
        d.close()
    assert out[0][2] == 0 and out[1][2] == 0
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_set_species_rejects_bad_input():
    from paper_1303_4523_amd._lib import EnufError
    L = 8.0
    pos, vel, q, bonds, sp = _system(L)
    d = _dpd(L, q, bonds)
    bad = TABLE.copy()
    bad[0, 1] += 1.0
    with pytest.raises(EnufError):
        d.set_species(sp, bad)                         # not symmetric
    with pytest.raises(EnufError):
        d.set_species(np.full(len(q), 3), TABLE)       # species out of range
    with pytest.raises(EnufError):
        d.set_species(sp, np.ones((5, 5)))             # more than 4 species
    d.set_species(sp, np.array([[25.0]]))              # one species: plain a
    d.close()


def _hist_gpu(pos, sel, cls, ncls, L, r_max, nbins, samples=1):
    from paper_1303_4523_amd.observables import PairHistogram
    H = PairHistogram(len(pos), sel, cls, ncls, L, r_max, nbins, device=0)
    tp = _t(pos)
    for _ in range(samples):
        H.sample(tp)
    torch.cuda.synchronize()
    return H.counts()


def test_pair_histogram_set3_bitwise():
    """The set-3 electrolyte (N = 4000, 16 tiles): counts by class equal the
    oracle's exactly; two samples accumulate to twice the counts."""
    s = wl.electrolyte_set3()
    cls = np.where(s.q > 0, 1, np.where(s.q < 0, 2, 0)).astype(np.int32)
    print(f"case: histogram {s.meta['name']}", flush=True)
    g = _hist_gpu(s.pos, np.arange(s.N), cls, 3, s.L, 5.0, 100, samples=2)
    o = oracle.pair_histogram(s.pos, np.arange(s.N), cls, 3, s.L, 5.0, 100)
    assert np.array_equal(g, 2 * o)
    assert o.sum() > 0


def test_pair_histogram_subset_and_edges():
    """A ragged selection (1037 of 3000, unsorted, with repeats of classes)
    and a lattice whose distances fall exactly on bin edges: exact counts."""
    rs = np.random.default_rng(3)
    L = 9.0
    pos = rs.uniform(0.0, L, (3000, 3))
    sel = rs.permutation(3000)[:1037]
    cls = rs.integers(0, 4, 1037).astype(np.int32)
    print("case: histogram subset 1037/3000", flush=True)
    g = _hist_gpu(pos, sel, cls, 4, L, 4.4, 37)
    o = oracle.pair_histogram(pos, sel, cls, 4, L, 4.4, 37)
    assert np.array_equal(g, o)
    # lattice with integer spacing: r^2 = 1, 2, 3, 4 exactly, bins of 0.1
    n = 6
    gr = np.arange(n, dtype=np.float64)
    lat = np.stack(np.meshgrid(gr, gr, gr, indexing="ij"), -1).reshape(-1, 3) + 0.5
    lcls = (lat.astype(int).sum(1) % 2).astype(np.int32)
    print("case: histogram lattice edges", flush=True)
    g = _hist_gpu(lat, np.arange(len(lat)), lcls, 2, float(n), 2.5, 25)
    o = oracle.pair_histogram(lat, np.arange(len(lat)), lcls, 2, float(n), 2.5, 25)
    assert np.array_equal(g, o)
    # fewer than two selected particles: nothing counted
    assert _hist_gpu(pos, sel[:1], cls[:1], 4, L, 4.4, 37).sum() == 0


def test_pair_histogram_rejects_bad_sizes():
    from paper_1303_4523_amd._lib import EnufError
    from paper_1303_4523_amd.observables import PairHistogram
    pos = _t(np.zeros((10, 3)))
    with pytest.raises(EnufError):
        PairHistogram(10, np.arange(10), np.zeros(10), 4, 5.0, 2.0, 1000, device=0).sample(pos)  # 16000 bins
    with pytest.raises(EnufError):
        PairHistogram(10, np.arange(10), np.zeros(10), 1, 5.0, -1.0, 10, device=0).sample(pos)


def test_chain_rg2_matches_oracle():
    """Five 48-bead random-walk chains crossing the box boundary, one 2-bead
    chain: Rg^2 equals the oracle's (same operation order, no fused
    multiply-adds on either side)."""
    from paper_1303_4523_amd.observables import chain_rg2
    rs = np.random.default_rng(8)
    L = 7.5
    chains = [wl.random_walk(rs, 48, L, 0.7) for _ in range(5)]
    pos = np.vstack(chains + [rs.uniform(0, L, (100, 3))])
    beads = np.arange(5 * 48).reshape(5, 48)
    print("case: rg2 five chains", flush=True)
    out = chain_rg2(_t(pos), _t(beads, torch.int64), L).cpu().numpy()
    ref = oracle.chain_rg2(pos, beads, L)
    print(f"rg2 max rel diff {np.max(np.abs(out - ref) / ref):.3e}")
    assert np.allclose(out, ref, rtol=1e-14, atol=0)
    two = chain_rg2(_t(pos), _t(np.array([[0, 1]]), torch.int64), L).cpu().numpy()
    assert np.allclose(two, oracle.chain_rg2(pos, np.array([[0, 1]]), L), rtol=1e-14)
