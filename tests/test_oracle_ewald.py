"""Pins of the FP64 CPU oracle's Ewald sum against what the paper and the
mathematics fix (no GPU).  Each test names the passage it follows.

A plausible slip in the oracle -- a dropped term, a wrong sign, a transposed
operand, a wrong prefactor -- fails at least one of these:
  * lattice Madelung constants (real + reciprocal + self together, prefactors),
  * the closed-form energy of a periodic +-1 pair with Slater smearing (eq. 27),
  * Gauss's law for the Slater density (eq. 26) vs the real-space pair term,
  * the r -> 0 limits stated after eq. 28,
  * Ewald-free brute-force image sums,
  * zero net force, finite differences of the energy, alpha independence,
    translation and permutation invariance.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate, special

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _madelung():
    with open(os.path.join(GOLD, "madelung.json")) as f:
        return json.load(f)


# ---------------------------------------------------------------- lattices

def test_madelung_nacl():
    """Sec. 5, first test set: Madelung constant of a rock-salt crystal.
    8^3 ions alternating +-1 at unit spacing, L = 8, point charges."""
    n = 8
    g = np.array([(i, j, k) for i in range(n) for j in range(n) for k in range(n)], float)
    q = np.where(g.sum(1) % 2 == 0, 1.0, -1.0)
    r = oracle.ewald(g, q, float(n), 1.5, 24, 4.0, 0.0)
    m = -2.0 * r["E"] / len(q)
    assert abs(m - _madelung()["NaCl"]) < 1e-11
    assert np.abs(r["F"]).max() < 1e-12  # every ion sits at a centre of symmetry


def test_madelung_cscl():
    """Caesium-chloride lattice: Cs at cube corners, Cl at body centres;
    nearest-neighbour distance sqrt(3)/2 of the cube edge."""
    n = 6
    c = np.array([(i, j, k) for i in range(n) for j in range(n) for k in range(n)], float)
    pos = np.vstack([c, c + 0.5])
    q = np.concatenate([np.ones(len(c)), -np.ones(len(c))])
    r = oracle.ewald(pos, q, float(n), 2.0, 26, 3.0, 0.0)
    r0 = math.sqrt(3.0) / 2.0
    m = -r["E"] * r0 / len(c)
    assert abs(m - _madelung()["CsCl"]) < 1e-11


# ------------------------------------------------- Slater pair, closed form

def _b1(r, lam):
    x = r / lam
    return 1.0 - (1.0 + x) * math.exp(-2.0 * x)


def _pair_energy(L, d, lam, alpha, r_cut, Kc, direction=(1.0, 0.0, 0.0)):
    u = np.asarray(direction, float)
    u /= np.linalg.norm(u)
    c = np.array([L / 2, L / 2, L / 2])
    pos = np.vstack([c, c + d * u])
    q = np.array([1.0, -1.0])
    return oracle.ewald(pos, q, L, alpha, Kc, r_cut, lam)


@pytest.mark.parametrize("lam", [0.0, 0.25])
def test_periodic_pair_closed_form(lam):
    """eq. 27 + the Ewald sum: a neutral +-1 pair at separation d in a cubic
    box with tin-foil boundary conditions has
        E = -B1(d)/d - 2 pi d^2 / (3 L^3) + O(d^4 / L^5)
    (the 1/L Wigner terms of pair and self-images cancel for a neutral pair).
    The residual must shrink as L^-5."""
    d = 1.0
    res = {}
    for L, alpha, r_cut, Kc in [(10.0, 1.2, 5.0, 24), (20.0, 0.6, 10.0, 24), (40.0, 0.4, 15.0, 32)]:
        E = _pair_energy(L, d, lam, alpha, r_cut, Kc)["E"]
        b1 = _b1(d, lam) if lam > 0 else 1.0
        res[L] = E - (-b1 / d - 2.0 * math.pi * d * d / (3.0 * L ** 3))
    assert abs(res[10.0]) < 1e-4
    assert 20.0 < res[10.0] / res[20.0] < 45.0     # ~ 2^5
    assert 20.0 < res[20.0] / res[40.0] < 45.0
    assert abs(res[40.0]) < 1e-7


def test_coincident_pair_limit():
    """After eq. 28: as r -> 0 the smeared pair energy tends to q_i q_j / lambda
    and the force to zero.  A +-1 pair at the same point in a periodic box has
    no monopole or dipole, so its periodic energy is -1/lambda."""
    lam = 0.25
    r = _pair_energy(10.0, 0.0, lam, 1.2, 5.0, 24)
    assert abs(r["E"] - (-1.0 / lam)) < 1e-12
    assert np.abs(r["F"]).max() < 1e-12
    # point charges may not coincide
    with pytest.raises(oracle.OracleError):
        _pair_energy(10.0, 0.0, 0.0, 1.2, 5.0, 24)


def _slater_gauss(r, lam):
    """Potential and enclosed charge of the Slater density of eq. 26 (unit q),
    by quadrature of the density alone (shell theorem / Gauss's law):
        Q(r)   = int_0^r rho 4 pi s^2 ds,
        phi(r) = Q(r)/r + int_r^inf rho 4 pi s ds."""
    rho = lambda s: math.exp(-2.0 * s / lam) / (math.pi * lam ** 3)
    Q = integrate.quad(lambda s: rho(s) * 4 * math.pi * s * s, 0.0, r, epsabs=1e-15, epsrel=1e-13)[0]
    tail = integrate.quad(lambda s: rho(s) * 4 * math.pi * s, r, np.inf, epsabs=1e-15, epsrel=1e-13)[0]
    return Q / r + tail, Q


@pytest.mark.parametrize("r", [0.05, 0.2, 0.5, 1.0, 2.0, 2.9])
@pytest.mark.parametrize("lam", [0.25, 1.0 / 1.125])
def test_real_space_pair_vs_gauss_law(r, lam):
    """eq. 26-28 in the additive reading: the real-space pair term equals the
    potential of a Slater-smeared charge minus the erf long-range part that
    the reciprocal sum carries,  u(r) = phi_slater(r) - erf(alpha r)/r, and its
    radial force is  Q_enclosed(r)/r^2 - d/dr[erf(alpha r)/r]  (B2 = Q_enc)."""
    alpha, r_cut, L = 0.3, 3.0, 10.0
    pos = np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]])
    q = np.array([1.0, 1.0])
    F, Ee, Es = oracle.real_space(pos, q, L, alpha, r_cut, lam)
    phi, Q = _slater_gauss(r, lam)
    ar = alpha * r
    u_ref = phi - special.erf(ar) / r
    f_ref = Q / (r * r) - (special.erf(ar) / r ** 2 - 2 * alpha / math.sqrt(math.pi) * math.exp(-ar * ar) / r)
    assert abs(Ee - u_ref) < 1e-10 * max(1.0, abs(u_ref))
    # force on particle 0 points along -x for repulsion (it sits at smaller x)
    assert abs(-F[0, 0] - f_ref) < 1e-9 * max(1.0, abs(f_ref))
    assert abs(F[0, 0] + F[1, 0]) < 1e-14 and np.abs(F[:, 1:]).max() == 0.0


def test_b1_b2_values_at_paper_beta():
    """Sec. 4: B1, B2 at beta = R_c/lambda_e = 1.125 evaluated through the
    oracle's pair term at r = 1, 2, 3 and compared with Gauss's-law
    quadrature of eq. 26.  B2(3) = 0.964..., so the paper's remark that both
    factors are ~1 beyond 3 R_c holds only loosely for B2."""
    lam = 1.0 / 1.125
    alpha = 0.3
    for r in (1.0, 2.0, 2.99):
        pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        F, Ee, Es = oracle.real_space(pos, np.array([1.0, 1.0]), 10.0, alpha, 3.0, lam)
        B1 = r * Ee + special.erf(alpha * r)
        B2 = r * r * (-F[0, 0]) + (special.erf(alpha * r)
                                   - 2 * alpha * r / math.sqrt(math.pi) * math.exp(-(alpha * r) ** 2))
        phi, Q = _slater_gauss(r, lam)
        assert abs(B1 - r * phi) < 1e-10
        assert abs(B2 - Q) < 1e-10
    assert 0.96 < Q < 0.97  # B2 at r = 2.99


@pytest.mark.parametrize("r", [1e-9, 1e-7, 2.5e-5, 1e-3, 0.1249, 0.1251, 0.5])
def test_small_r_branch_vs_high_precision(r):
    """The series used below r = lambda/2 and the closed form above it both
    match a 50-digit evaluation of u(r) = [erfc(alpha r) - (1+x) e^{-2x}]/r and
    of -u'(r)/r (x = r/lambda)."""
    lam, alpha = 0.25, 0.3
    mpmath.mp.dps = 50
    R = mpmath.mpf(r)
    a = mpmath.mpf(alpha)
    lm = mpmath.mpf(lam)
    u = lambda s: (mpmath.erfc(a * s) - (1 + s / lm) * mpmath.exp(-2 * s / lm)) / s
    u_ref = float(u(R))
    f_ref = float(-mpmath.diff(u, R) / R)
    pos = np.array([[2.0, 2.0, 2.0], [2.0 + r, 2.0, 2.0]])
    F, Ee, Es = oracle.real_space(pos, np.array([1.0, -1.0]), 10.0, alpha, 3.0, lam)
    assert abs(-Ee - u_ref) < 1e-13 * abs(u_ref)
    # force on 0 = q0 q1 f d with d = r0 - r1 = -r x_hat; the separation itself
    # carries the rounding of 2 + r
    d = (2.0 + r) - 2.0
    f = F[0, 0] / d
    assert abs(f - f_ref) < 1e-12 * abs(f_ref) + 1e-15 * abs(f_ref) * 2.0 / r


# ------------------------------------------------ brute-force image sums

def _brute_energy(pos, q, L, nmax, lam=0.0):
    """Ewald-free reference: spherical-shell sum of q_i q_j B1(r)/r over all
    images |n| <= nmax (i = j excluded for n = 0), plus the tin-foil term
    -2 pi |sum q r|^2 / (3 V) (de Leeuw, Perram & Smith 1980)."""
    rng = np.arange(-nmax, nmax + 1)
    n = np.array(np.meshgrid(rng, rng, rng, indexing="ij")).reshape(3, -1).T
    n = n[(n ** 2).sum(1) <= nmax * nmax].astype(float) * L
    E = 0.0
    for i in range(len(q)):
        for j in range(len(q)):
            d = pos[i] - pos[j] + n
            r = np.sqrt((d ** 2).sum(1))
            if i == j:
                r = r[r > 0]
            pot = 1.0 / r if lam == 0.0 else (1.0 - (1.0 + r / lam) * np.exp(-2 * r / lam)) / r
            E += 0.5 * q[i] * q[j] * pot.sum()
    dip = (q[:, None] * pos).sum(0)
    return E - 2.0 * math.pi * (dip @ dip) / (3.0 * L ** 3)


@pytest.mark.parametrize("lam", [0.0, 0.03])
def test_brute_force_image_sum(lam):
    """eq. 15 summed directly (no Ewald split) converges to the oracle's
    total; the error falls roughly as nmax^-4."""
    rs = np.random.default_rng(7)
    pos = rs.uniform(0.0, 1.0, (4, 3))
    q = np.array([1.0, -1.0, 2.0, -2.0])
    Eo = oracle.ewald(pos, q, 1.0, 12.0, 24, 0.5, lam)["E"]
    e20 = abs(_brute_energy(pos, q, 1.0, 20, lam) - Eo)
    e40 = abs(_brute_energy(pos, q, 1.0, 40, lam) - Eo)
    assert e40 < 4e-6 * abs(Eo) + 4e-6
    assert e20 > 5.0 * e40


# ------------------------------------------------------------- invariants

def _random_system(n, L, seed, lam=0.25, zmax=1):
    rs = np.random.default_rng(seed)
    pos = rs.uniform(0.0, L, (n, 3))
    q = rs.choice(np.arange(1, zmax + 1), size=n).astype(float)
    q[n // 2:] *= -1.0
    q[-1] -= q.sum()
    return pos, q


def test_net_force_zero():
    """Newton's third law for the real-space pairs and Im(S* S) = 0 for the
    direct reciprocal sum: the net force vanishes to round-off."""
    pos, q = _random_system(200, 6.0, 1, zmax=2)
    r = oracle.ewald(pos, q, 6.0, 0.9, 10, 3.0, 0.25)
    scale = np.sqrt((r["F"] ** 2).sum())
    assert np.abs(r["F_real"].sum(0)).max() < 1e-12 * scale
    assert np.abs(r["F_recip"].sum(0)).max() < 1e-12 * scale


@pytest.mark.parametrize("lam", [0.0, 0.25])
def test_force_is_minus_gradient(lam):
    """eq. 22 and eq. 32 (as the exact gradient of eq. 31 with eq. 27): central
    differences of each energy component reproduce the matching force."""
    L, alpha, r_cut, Kc = 5.0, 0.9, 2.5, 8
    pos, q = _random_system(16, L, 3)
    h = 1e-5
    r0 = oracle.ewald(pos, q, L, alpha, Kc, r_cut, lam)
    for i in (0, 5, 11):
        for a in range(3):
            ep = pos.copy(); ep[i, a] += h
            em = pos.copy(); em[i, a] -= h
            rp = oracle.ewald(ep, q, L, alpha, Kc, r_cut, lam)
            rm = oracle.ewald(em, q, L, alpha, Kc, r_cut, lam)
            fk = -(rp["E_recip"] - rm["E_recip"]) / (2 * h)
            fr = -(rp["E_real"] - rm["E_real"]) / (2 * h)
            assert abs(fk - r0["F_recip"][i, a]) < 1e-6 * (1 + abs(fk))
            assert abs(fr - r0["F_real"][i, a]) < 1e-6 * (1 + abs(fr))


def test_alpha_independence():
    """Sec. 5: the converged electrostatic energy does not depend on alpha
    (erfc(alpha r_cut) < 1e-16 and exp(-pi^2 Kc^2/(alpha L)^2) < 1e-16)."""
    pos, q = _random_system(40, 10.0, 4, zmax=2)
    Es, Fs = [], []
    for alpha in (1.2, 1.4, 1.6, 1.8):
        Kc = int(math.ceil(alpha * 10.0 * math.sqrt(38.0) / math.pi)) + 1
        r = oracle.ewald(pos, q, 10.0, alpha, Kc, 5.0, 0.25)
        Es.append(r["E"])
        Fs.append(r["F"])
    for E, F in zip(Es[1:], Fs[1:]):
        assert abs(E - Es[0]) < 1e-11 * abs(Es[0])
        assert np.abs(F - Fs[0]).max() < 1e-10 * np.abs(Fs[0]).max()


def test_translation_and_permutation_invariance():
    L = 7.0
    pos, q = _random_system(60, L, 5)
    r0 = oracle.ewald(pos, q, L, 0.6, 8, 3.0, 0.25)
    shift = np.array([0.37, -2.9, 11.3])
    r1 = oracle.ewald(pos + shift, q, L, 0.6, 8, 3.0, 0.25)
    perm = np.random.default_rng(0).permutation(len(q))
    r2 = oracle.ewald(pos[perm], q[perm], L, 0.6, 8, 3.0, 0.25)
    for r in (r1, r2):
        assert abs(r["E"] - r0["E"]) < 1e-12 * abs(r0["E_real"])
    assert np.abs(r1["F"] - r0["F"]).max() < 1e-11
    assert np.abs(r2["F"] - r0["F"][perm]).max() < 1e-11


def test_selected_rows_match_full():
    pos, q = _random_system(80, 6.0, 6)
    full = oracle.ewald(pos, q, 6.0, 0.8, 8, 3.0, 0.25)
    sel = np.array([3, 17, 42, 79])
    part = oracle.ewald(pos, q, 6.0, 0.8, 8, 3.0, 0.25, sel=sel)
    assert np.array_equal(part["F"], full["F"][sel])
    assert math.isnan(part["E"])
