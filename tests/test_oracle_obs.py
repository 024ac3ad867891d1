"""Pins of the oracle's structure observables: the pair-distance histogram
behind the radial distribution functions (Sec. 5) and the radius of gyration
of a chain (Sec. 6)."""
import math

import numpy as np

import oracle


def _rocksalt(n, a, off=0.25):
    """Simple cubic lattice of n^3 sites with spacing a; class = parity of
    i + j + k (unlike nearest neighbours, as in rock salt)."""
    g = np.arange(n)
    i, j, k = np.meshgrid(g, g, g, indexing="ij")
    pos = (np.stack([i, j, k], -1).reshape(-1, 3) + off) * a
    cls = ((i + j + k) % 2).reshape(-1)
    return pos, cls


def test_histogram_lattice_shells():
    """Periodic simple cubic lattice, 6^3 sites, spacing 1.03 (L = 6.18):
    each site has 6 neighbours at a, 12 at a sqrt 2, 8 at a sqrt 3 and 6 at 2a
    (then 24 at a sqrt 5 = 2.30, beyond r_max = 2.2).  Unordered pairs:
    216 x {6, 12, 8, 6} / 2; the first and third shells join unlike classes,
    the second and fourth like classes (half of them each)."""
    a, n = 1.03, 6
    pos, cls = _rocksalt(n, a)
    L = n * a
    h = oracle.pair_histogram(pos, np.arange(len(pos)), cls, 2, L, 2.2, 22)
    N = n ** 3
    want = np.zeros((2, 2, 22), dtype=np.uint64)
    want[0, 1, 10] = N * 6 // 2                                   # r = 1.03
    want[0, 0, 14] = want[1, 1, 14] = N * 12 // 4                  # r = 1.457
    want[0, 1, 17] = N * 8 // 2                                   # r = 1.784
    want[0, 0, 20] = want[1, 1, 20] = N * 6 // 4                   # r = 2.06
    assert np.array_equal(h, want)


def test_histogram_ideal_gas():
    """Uniform points: the expected count in a shell is
    pairs x (shell volume / V); the histogram over 40 shells agrees within
    5 standard deviations of a Poisson count in every shell."""
    rs = np.random.default_rng(11)
    L, n = 8.0, 1500
    pos = rs.uniform(0.0, L, (n, 3))
    nb, rmax = 40, 3.0
    h = oracle.pair_histogram(pos, np.arange(n), np.zeros(n, dtype=np.int32), 1, L, rmax, nb)[0, 0]
    edges = np.linspace(0.0, rmax, nb + 1)
    shell = 4.0 / 3.0 * math.pi * np.diff(edges ** 3)
    expect = n * (n - 1) / 2 * shell / L ** 3
    assert np.all(np.abs(h - expect) < 5.0 * np.sqrt(expect) + 3.0)


def test_histogram_selection_and_accumulation():
    """Only selected particles are counted, with the class given per
    selected entry, and calls accumulate; a selection of the whole lattice
    by two halves misses exactly the cross pairs."""
    a, n = 1.03, 6
    pos, cls = _rocksalt(n, a)
    L = n * a
    N = len(pos)
    full = oracle.pair_histogram(pos, np.arange(N), cls, 2, L, 2.2, 22)
    h1 = oracle.pair_histogram(pos, np.arange(N // 2), cls[:N // 2], 2, L, 2.2, 22)
    h2 = oracle.pair_histogram(pos, np.arange(N // 2, N), cls[N // 2:], 2, L, 2.2, 22)
    assert np.all(h1 + h2 <= full) and (h1 + h2).sum() < full.sum()
    # one class for everything: the shells collapse into [0, 0]
    one = oracle.pair_histogram(pos, np.arange(N), np.zeros(N, dtype=np.int32), 1, L, 2.2, 22)[0, 0]
    assert np.array_equal(one, full[0, 0] + full[0, 1] + full[1, 1])


def test_rg_straight_chain_across_the_boundary():
    """n beads spaced b on a line: Rg^2 = b^2 (n^2 - 1) / 12, also when the
    chain crosses the periodic boundary (wrapped coordinates)."""
    L, n, b = 7.0, 48, 0.7
    x = (5.0 + b * np.arange(n)) % L
    pos = np.stack([x, np.full(n, 1.0), np.full(n, 2.0)], 1)
    rg2 = oracle.chain_rg2(pos, np.arange(n), L)[0]
    assert abs(rg2 - b * b * (n * n - 1) / 12.0) < 1e-10


def test_rg_ring_and_invariance():
    """Beads on a circle of radius R: Rg^2 = R^2; a rigid shift of the whole
    chain (wrapped back into the box) and the reversal of the bead order
    leave it unchanged; two chains are evaluated independently."""
    L, n, R = 9.0, 40, 2.0
    t = 2.0 * math.pi * np.arange(n) / n
    pos = np.stack([4.0 + R * np.cos(t), 4.0 + R * np.sin(t), np.full(n, 3.0)], 1)
    shifted = (pos + np.array([6.5, -3.2, 7.7])) % L
    both = np.vstack([pos, shifted])
    beads = np.stack([np.arange(n), n + np.arange(n)[::-1]])
    rg2 = oracle.chain_rg2(both, beads, L)
    assert np.allclose(rg2, R * R, rtol=0, atol=1e-10)
