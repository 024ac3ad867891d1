"""Pins of the oracle's random numbers and DPD step (Sec. 2, Table 2)."""
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    """Philox4x64-10 against the published known-answer vectors."""
    with open(os.path.join(GOLD, "philox4x64_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) >= 3
    for row in rows:
        v = [int(x, 16) for x in row]
        out = oracle.philox4x64_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_philox4x32_known_answers():
    """Philox4x32-10 (the generator of theta_ij) against the published vectors."""
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) >= 3
    for row in rows:
        v = [int(x, 16) for x in row]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_philox_matches_numpy_bit_generator():
    """numpy.random.Philox is Philox4x64-10; it increments the counter before
    each block, so counter c - 1 yields the block of counter c."""
    rs = np.random.default_rng(3)
    for _ in range(20):
        c = [int(x) for x in rs.integers(1, 2 ** 63, 4)]
        k = [int(x) for x in rs.integers(0, 2 ** 63, 2)]
        bg = np.random.Philox(counter=[c[0] - 1] + c[1:], key=k)
        assert [int(x) for x in oracle.philox4x64_10(c, k)] == [int(x) for x in bg.random_raw(4)]


def test_theta_symmetric_zero_mean_unit_variance():
    """Sec. 2: theta_ij has zero mean and unit variance; theta_ij = theta_ji
    makes the random force pairwise antisymmetric."""
    vals = np.array([oracle.theta(42, s, i, i + 1 + (s % 7)) for s in range(200) for i in range(200)])
    assert abs(vals.mean()) < 0.02
    assert abs(vals.var() - 1.0) < 0.02
    assert vals.min() >= -math.sqrt(3.0) and vals.max() < math.sqrt(3.0)
    for (i, j) in [(0, 5), (17, 3), (1000, 999)]:
        assert oracle.theta(9, 4, i, j) == oracle.theta(9, 4, j, i)


def _dpd_box(n, L, seed, nq=0, chain=0):
    rs = np.random.default_rng(seed)
    pos = rs.uniform(0.0, L, (n, 3))
    vel = rs.normal(size=(n, 3))
    vel -= vel.mean(0)
    q = np.zeros(n)
    q[:nq // 2] = 1.0
    q[nq // 2:nq] = -1.0
    bonds = np.array([(i, i + 1) for i in range(chain - 1)], dtype=np.int64).reshape(-1, 2)
    for i in range(1, chain):   # bonded beads start close together
        pos[i] = (pos[i - 1] + 0.7 * rs.normal(size=3) / math.sqrt(3)) % L
    return pos, vel, q, bonds


BASE = dict(a=25.0, gamma=4.5, sigma=3.0, dt=0.03, lam=0.65, k_bond=4.0, r0_bond=0.7)


def test_dpd_forces_conserve_momentum():
    """eq. 2-7: every pair force is antisymmetric (theta_ij = theta_ji), so
    the total force is zero -- also with bonds and direct-Ewald electrostatics."""
    pos, vel, q, bonds = _dpd_box(300, 5.0, 1, nq=40, chain=10)
    P = dict(BASE, L=5.0, kappa=1.1, alpha=0.8, r_cut=2.5, lambda_e=0.25, Kc=8, use_elec=1)
    F, _ = oracle.dpd_forces(pos, vel, q, bonds, P, seed=7, step=3)
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).max()


def _potential(pos, q, bonds, P, E_elec):
    L = P["L"]
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    iu = np.triu_indices(len(pos), 1)
    rr = r[iu]
    Uc = 0.5 * P["a"] * ((1.0 - rr[rr < 1.0]) ** 2).sum()
    db = pos[bonds[:, 0]] - pos[bonds[:, 1]]
    db -= L * np.round(db / L)
    Ub = 0.5 * P["k_bond"] * ((np.sqrt((db ** 2).sum(1)) - P["r0_bond"]) ** 2).sum()
    return Uc + Ub + E_elec


def test_conservative_dynamics_conserve_energy():
    """Table 2 with gamma = sigma = 0 and lambda = 1/2 is plain velocity Verlet:
    the conservative force (eq. 3 with w^C = 1 - r), the bonds and the
    electrostatic force are gradients of U_C = a (1 - r)^2 / 2, the spring
    energy and the Ewald energy, so the total energy is conserved to O(dt^2)."""
    L = 4.0
    pos, vel, q, bonds = _dpd_box(150, L, 2, nq=16, chain=8)
    P = dict(BASE, L=L, gamma=0.0, sigma=0.0, dt=0.004, lam=0.5, kappa=1.1,
             alpha=1.0, r_cut=2.0, lambda_e=0.25, Kc=8, use_elec=1)
    F, Ee = oracle.dpd_forces(pos, vel, q, bonds, P, seed=1, step=0)
    E0 = _potential(pos, q, bonds, P, Ee) + 0.5 * (vel ** 2).sum()
    drift = []
    for s in range(1, 121):
        pos, vel, F, Ee = oracle.dpd_step(pos, vel, F, q, bonds, P, seed=1, step=s)
        drift.append(_potential(pos, q, bonds, P, Ee) + 0.5 * (vel ** 2).sum() - E0)
    assert np.abs(drift).max() < 2e-3 * abs(E0)


def test_thermostat_reaches_kT():
    """eq. 6: sigma^2 = 2 gamma kT makes the dissipative and random forces a
    thermostat at kT = 1 (the modified VV with lambda = 0.65 keeps the
    temperature within a few per cent at dt = 0.03)."""
    L = 4.64
    n = int(round(3 * L ** 3))
    pos, vel, q, bonds = _dpd_box(n, L, 3)
    vel *= 0.3  # start cold
    P = dict(BASE, L=L)
    F, _ = oracle.dpd_forces(pos, vel, q, bonds, P, seed=5, step=0)
    ke = []
    for s in range(1, 601):
        pos, vel, F, _ = oracle.dpd_step(pos, vel, F, q, bonds, P, seed=5, step=s)
        if s > 200:
            ke.append((vel ** 2).sum() / (3 * (n - 1)))
    assert abs(np.mean(ke) - 1.0) < 0.04


def test_one_step_worked_by_hand():
    """Table 2 on two beads with dissipation only, worked by hand.  Beads at
    x = 1.0 and 1.5 (y = z = 2, L = 10), velocities +1 and -1 along x, the
    force of the last step F = +2 and -2, dt = 0.1, gamma = 4.5,
    lambda = 0.65, a = sigma = 0:
      (0) predicted v0 = v + lambda dt F = +1.13 / -1.13
      (1) half kick   v  = v + dt F / 2   = +1.1 / -1.1
      (2) drift       x  = x + dt v       = 1.11 / 1.39, so r = 0.28
      (3-5) F^D on bead 0 = -gamma (1 - r)^2 (rhat . v0_01) rhat with
            rhat = -x, v0_01 = 2.26 x: magnitude 4.5 * 0.5184 * 2.26 =
            5.272128 along -x (bead 1: +x)
      (6) half kick   v  = 1.1 - 0.05 * 5.272128 = 0.8363936 / -0.8363936.
    Reading the half-kicked velocity (1.1) or the old one (1.0) in the
    dissipative force, or lambda = 1/2, would give 5.13216 or 4.6656."""
    L = 10.0
    pos = np.array([[1.0, 2.0, 2.0], [1.5, 2.0, 2.0]])
    vel = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    F0 = np.array([[2.0, 0.0, 0.0], [-2.0, 0.0, 0.0]])
    P = dict(BASE, L=L, a=0.0, gamma=4.5, sigma=0.0, dt=0.1, lam=0.65, k_bond=0.0, use_elec=0)
    p1, v1, F1, _ = oracle.dpd_step(pos, vel, F0, np.zeros(2), np.zeros((0, 2)), P, seed=3, step=1)
    assert np.allclose(p1, [[1.11, 2.0, 2.0], [1.39, 2.0, 2.0]], rtol=0, atol=1e-14)
    assert np.allclose(F1, [[-5.272128, 0.0, 0.0], [5.272128, 0.0, 0.0]], rtol=0, atol=1e-12)
    assert np.allclose(v1, [[0.8363936, 0.0, 0.0], [-0.8363936, 0.0, 0.0]], rtol=0, atol=1e-13)


def test_species_amplitudes_hand_computed():
    """eq. 3 with species-dependent amplitudes (a_ij = a_ii + 2.05 chi, Sec. 2):
    three beads on a line at x = 0, 0.5, 0.9 of species 0, 1, 2 with
    a_01 = 10, a_02 = 20, a_12 = 30 and no dissipation or noise.  Worked by
    hand: F_0 = -10 (0.5) - 20 (0.1) = -7, F_1 = 10 (0.5) - 30 (0.6) = -13,
    F_2 = 20 (0.1) + 30 (0.6) = 20 along x."""
    L = 10.0
    pos = np.array([[1.0, 2.0, 2.0], [1.5, 2.0, 2.0], [1.9, 2.0, 2.0]])
    tab = np.array([[1.0, 10.0, 20.0], [10.0, 2.0, 30.0], [20.0, 30.0, 3.0]])
    P = dict(BASE, L=L, gamma=0.0, sigma=0.0, k_bond=0.0, species=[0, 1, 2], a_table=tab)
    F, _ = oracle.dpd_forces(pos, np.zeros((3, 3)), np.zeros(3), np.zeros((0, 2)), P, seed=1, step=0)
    assert np.allclose(F[:, 0], [-7.0, -13.0, 20.0], rtol=0, atol=1e-12)
    assert np.all(F[:, 1:] == 0.0)


def test_species_reduce_to_one_amplitude():
    """A table whose every entry is a gives the single-species forces bit for
    bit, and relabelling the species with the table permuted alike changes
    nothing (the force depends on the pair's amplitude only)."""
    pos, vel, q, bonds = _dpd_box(200, 5.0, 3, chain=10)
    P = dict(BASE, L=5.0)
    F1, _ = oracle.dpd_forces(pos, vel, q, bonds, P, seed=5, step=2)
    sp = (np.arange(200) % 3).astype(np.int32)
    F2, _ = oracle.dpd_forces(pos, vel, q, bonds, dict(P, species=sp, a_table=np.full((3, 3), 25.0)),
                              seed=5, step=2)
    assert np.array_equal(F1, F2)
    tab = np.array([[25.0, 27.0, 31.0], [27.0, 26.0, 29.0], [31.0, 29.0, 24.0]])
    F3, _ = oracle.dpd_forces(pos, vel, q, bonds, dict(P, species=sp, a_table=tab), seed=5, step=2)
    perm = np.array([2, 0, 1])           # old species s becomes perm[s]
    tab2 = np.empty_like(tab)
    tab2[np.ix_(perm, perm)] = tab
    F4, _ = oracle.dpd_forces(pos, vel, q, bonds, dict(P, species=perm[sp], a_table=tab2), seed=5, step=2)
    assert np.array_equal(F3, F4)
    assert not np.allclose(F1, F3)
    assert np.abs(F3.sum(0)).max() < 1e-10 * np.abs(F3).max()
