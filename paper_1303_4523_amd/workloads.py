"""Seeded synthetic inputs (positions, charges, chains, velocities).

This module is shared by the tests, the benchmark, the oracle checks and the
GPU path.  It holds none of the method's arithmetic: it only draws particle
configurations with NumPy's PCG64 generator.

Seeds: base 13034523; workload k uses base + k; replica / request r of a
multi-system workload adds 1000 r.

Shapes follow the paper's test systems (Table 3): uniform bulk electrolytes
in a periodic cube at DPD density 3 with a fraction of the beads carrying
+-1 (or z-valent) charges, and single polyelectrolyte chains built as random
walks of bond length 0.7 with counterions and added salt.
"""
from dataclasses import dataclass, field
import math

import numpy as np

BASE_SEED = 13034523


@dataclass
class System:
    L: float
    pos: np.ndarray              # (N, 3) float64, in [0, L)
    q: np.ndarray                # (N,) float64
    vel: np.ndarray = None       # (N, 3) float64 or None
    bonds: np.ndarray = None     # (nb, 2) int64 or None
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return len(self.q)

    @property
    def Nq(self):
        return int(np.count_nonzero(self.q))


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _velocities(rng, n, kT=1.0):
    v = rng.normal(0.0, math.sqrt(kT), size=(n, 3))
    v -= v.mean(axis=0)
    return v


def electrolyte(L, n_total, n_plus, n_minus, seed, z_plus=1.0, z_minus=-1.0,
                with_velocities=False):
    """Uniform beads; a seeded random subset carries charges."""
    rng = _rng(seed)
    pos = rng.uniform(0.0, L, size=(n_total, 3))
    perm = rng.permutation(n_total)
    q = np.zeros(n_total)
    q[perm[:n_plus]] = z_plus
    q[perm[n_plus:n_plus + n_minus]] = z_minus
    vel = _velocities(rng, n_total) if with_velocities else None
    return System(L=float(L), pos=pos, q=q, vel=vel,
                  meta=dict(seed=seed, n_plus=n_plus, n_minus=n_minus))


def random_walk(rng, n, L, step):
    start = rng.uniform(0.0, L, size=3)
    d = rng.normal(size=(n - 1, 3))
    d *= step / np.linalg.norm(d, axis=1, keepdims=True)
    chain = np.vstack([start, start + np.cumsum(d, axis=0)])
    return chain - L * np.floor(chain / L)


def polyelectrolyte(L, density, chain_len, charge_fraction, salt_per_volume, valency, seed,
                    bond_length=0.7, with_velocities=True):
    """One chain with evenly spaced -1 charges, +1 counterions, z:1 salt
    (round(salt_per_volume * V) cations at +z and z times as many -1 anions),
    neutral solvent filling the rest to the given density."""
    rng = _rng(seed)
    V = L ** 3
    n_total = int(round(density * V))
    n_chain_q = int(round(chain_len * charge_fraction))
    n_cat = int(round(salt_per_volume * V))
    n_an = valency * n_cat
    n_other = n_total - chain_len
    if n_chain_q + n_cat + n_an > n_other:
        raise ValueError("not enough beads for the requested ions")
    chain = random_walk(rng, chain_len, L, bond_length)
    rest = rng.uniform(0.0, L, size=(n_other, 3))
    pos = np.vstack([chain, rest])
    q = np.zeros(n_total)
    if n_chain_q > 0:
        idx = np.unique(np.round(np.linspace(0, chain_len - 1, n_chain_q)).astype(np.int64))
        if len(idx) < n_chain_q:  # dense case: fall back to the first beads
            idx = np.arange(n_chain_q)
        q[idx] = -1.0
    perm = chain_len + rng.permutation(n_other)
    k = 0
    q[perm[k:k + n_chain_q]] = 1.0          # counterions of the chain
    k += n_chain_q
    q[perm[k:k + n_cat]] = float(valency)   # salt cations
    k += n_cat
    q[perm[k:k + n_an]] = -1.0              # salt anions
    bonds = np.stack([np.arange(chain_len - 1), np.arange(1, chain_len)], axis=1).astype(np.int64)
    vel = _velocities(rng, n_total) if with_velocities else None
    return System(L=float(L), pos=pos, q=q, vel=vel, bonds=bonds,
                  meta=dict(seed=seed, chain_len=chain_len, charge_fraction=charge_fraction,
                            n_cat=n_cat, n_an=n_an, valency=valency))


# --------------------------------------------------------------------------
# Named workloads.  ENUF parameters: alpha = 0.3, r_cut = 3, lambda_e = 0.25,
# p = 4, sigma = 2, M = 3.2 L, Kc = 0.8 L (all in units of R_c).
# --------------------------------------------------------------------------

ENUF_DEFAULTS = dict(alpha=0.3, r_cut=3.0, lam=0.25, p=4, sigma=2.0)


def enuf_params(L, **over):
    M = int(round(3.2 * L))
    Kc = int(math.floor(0.8 * L + 1e-9))
    d = dict(ENUF_DEFAULTS, L=float(L), M=M, Kc=Kc)
    d.update(over)
    return d


def single_eval_small():
    """L = 10, N = 3000 uniform beads, 150 at +1 and 150 at -1; M = 32, Kc = 8."""
    s = electrolyte(10.0, 3000, 150, 150, BASE_SEED + 1)
    s.meta["enuf"] = enuf_params(10.0)
    s.meta["name"] = "single-eval L=10 N=3000 Nq=300"
    return s


BJERRUM_COUPLING = 13.87


def dpd_polyelectrolyte_24k():
    """L = 20 at density 3 (N = 24000): one 50-bead chain with charge fraction
    0.5 (25 beads at -1), 25 counterions at +1, 800 + 800 salt ions, neutral
    solvent; DPD a = 25, gamma = 4.5, sigma = 3, dt = 0.03, bonds k = 4 and
    r0 = 0.7, velocity-Verlet lambda = 0.65; ENUF M = 64, Kc = 16."""
    s = polyelectrolyte(20.0, 3.0, 50, 0.5, 0.1, 1, BASE_SEED + 2)
    s.meta["enuf"] = enuf_params(20.0)
    s.meta["dpd"] = dict(L=20.0, a=25.0, gamma=4.5, sigma=3.0, dt=0.03, lam=0.65,
                         k_bond=4.0, r0_bond=0.7, kappa=BJERRUM_COUPLING / (4.0 * math.pi))
    s.meta["name"] = "DPD L=20 N=24000 Nq=1650"
    return s


def n_sweep(L):
    """L in {10, 15, 20, 30, 40}: N = 3 L^3 uniform, 10 % charged (half +1)."""
    n = int(round(3 * L ** 3))
    nq = int(round(0.1 * n))
    s = electrolyte(float(L), n, nq // 2, nq // 2, BASE_SEED + 3 + 10 * int(L))
    s.meta["enuf"] = enuf_params(float(L))
    s.meta["name"] = f"N-sweep L={L} N={n} Nq={2 * (nq // 2)}"
    return s


def mesh_size(n):
    """Smallest even 2^a 3^b 5^c that is >= n (an FFT-friendly mesh)."""
    m = max(2, int(math.ceil(n - 1e-9)))
    while True:
        k = m
        for r in (2, 3, 5):
            while k % r == 0:
                k //= r
        if k == 1 and m % 2 == 0:
            return m
        m += 1


DPD_DEFAULTS = dict(a=25.0, gamma=4.5, sigma=3.0, dt=0.03, lam=0.65, k_bond=4.0, r0_bond=0.7,
                    kappa=BJERRUM_COUPLING / (4.0 * math.pi))


def replica(s, n_min=3000, n_max=48000, seed_base=BASE_SEED + 4):
    """Replica s of the batched workload: N log-uniform in [n_min, n_max] at
    density 3 (L = (N/3)^(1/3)); one 50-bead chain with charge fraction
    f = (0.1, 0.25, 0.5, 1.0)[s mod 4] and its +1 counterions; z:1 salt with
    z = (1, 2, 3)[(s div 4) mod 3] (0.1 cations per unit volume at +z and z
    times as many -1 anions); M = smallest even 2^a 3^b 5^c >= 3.2 L,
    Kc = min(floor(0.8 L), floor(M / 4))."""
    seed = seed_base + 1000 * s
    rng = _rng(seed)
    n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
    L = (n / 3.0) ** (1.0 / 3.0)
    f = (0.1, 0.25, 0.5, 1.0)[s % 4]
    z = (1, 2, 3)[(s // 4) % 3]
    sysm = polyelectrolyte(L, 3.0, 50, f, 0.1, z, seed + 1)
    M = mesh_size(3.2 * L)
    Kc = min(int(math.floor(0.8 * L + 1e-9)), M // 4)
    sysm.meta["enuf"] = enuf_params(L, M=M, Kc=Kc)
    sysm.meta["dpd"] = dict(DPD_DEFAULTS, L=L, seed=seed)
    sysm.meta["name"] = f"replica {s}: N={sysm.N} L={L:.3f} f={f} z={z} M={M} Kc={Kc}"
    return sysm


def batched_replicas(nsys=64):
    """The batched workload: nsys independent polyelectrolyte replicas."""
    return [replica(s) for s in range(nsys)]


def serving_request(r, n_min=3000, n_max=200000, seed_base=BASE_SEED + 5):
    """Request r of the serving stream: N log-uniform in [n_min, n_max] at
    density 3, a fraction c ~ U[0.05, 1] of the beads charged as
    n = round(c N / (1 + z)) cations at +z and z n anions at -1 (neutral),
    z uniform in {1, 2, 3}; no bonds; M = smallest even 2^a 3^b 5^c >= 3.2 L,
    Kc = min(floor(0.8 L), floor(M / 4))."""
    seed = seed_base + 1000 * r
    rng = _rng(seed)
    n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
    L = (n / 3.0) ** (1.0 / 3.0)
    c = rng.uniform(0.05, 1.0)
    z = int(rng.integers(1, 4))
    n_cat = int(round(c * n / (1 + z)))
    s = electrolyte(L, n, n_cat, z * n_cat, seed + 1, z_plus=float(z), z_minus=-1.0, with_velocities=True)
    M = mesh_size(3.2 * L)
    Kc = min(int(math.floor(0.8 * L + 1e-9)), M // 4)
    s.meta["enuf"] = enuf_params(L, M=M, Kc=Kc)
    s.meta["dpd"] = dict(DPD_DEFAULTS, L=L, seed=seed)
    s.meta["name"] = f"request {r}: N={n} L={L:.3f} c={c:.3f} z={z} M={M} Kc={Kc}"
    return s


def poisson_arrivals(n, rate, seed=BASE_SEED + 6):
    """n arrival times (seconds) of a Poisson stream with the given rate."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# --------------------------------------------------------------------------
# The paper's physics test systems (Table 3) with its DPD parameters (Table 1):
# density 4, a_ii = 78.67, gamma = 6.74, sigma = 3.67, dt = 0.02,
# lambda = 0.65, Slater decay length lambda_e = R_c / 1.125 (Sec. 4).  The
# ENUF parameters are not set here: the studies take them from the accuracy
# rule of eq. 29 (``params.choose``) with these r_cut and lambda_e.
# --------------------------------------------------------------------------

PAPER_DPD = dict(a=78.67, gamma=6.74, sigma=3.67, dt=0.02, lam=0.65, k_bond=64.0, r0_bond=0.7,
                 kappa=BJERRUM_COUPLING / (4.0 * math.pi))
PAPER_LAMBDA_E = 1.0 / 1.125
CHI_POLYMER_SOLVENT = 0.87
PAPER_R_CUT = 3.0


def electrolyte_set3(seed=BASE_SEED + 7, L=10.0, n_pairs=132):
    """Set 3 (Sec. 5, Table 3): N = 4000 beads at density 4 in (10 R_c)^3,
    132 cations (+1) and 132 anions (-1), 3736 neutral solvent beads."""
    n = int(round(4.0 * L ** 3))
    s = electrolyte(L, n, n_pairs, n_pairs, seed, with_velocities=True)
    s.meta["dpd"] = dict(PAPER_DPD, L=float(L), seed=seed)
    s.meta["name"] = f"electrolyte set 3: N={n} L={L} {n_pairs}+{n_pairs} ions"
    return s


def polyelectrolyte_set5(f, L=30.0, chain_len=48, seed=BASE_SEED + 8):
    """Set 5 (Sec. 6, Table 3): one chain of 48 beads at density 4 with a
    fraction f of its beads at -1 (evenly spaced), as many +1 counterions,
    neutral solvent; bonds K^S = 64, r_eq = 0.7; species 1 = chain beads,
    0 = everything else, a_01 = a_ii + 2.05 chi with chi = 0.87 (Sec. 2).
    The paper uses L = 30 (N = 108000); smaller boxes keep the same density."""
    s = polyelectrolyte(L, 4.0, chain_len, f, 0.0, 1, seed + int(round(1000 * f)), bond_length=0.7)
    s.meta["dpd"] = dict(PAPER_DPD, L=float(L), seed=seed + int(round(1000 * f)))
    species = np.zeros(s.N, dtype=np.int32)
    species[:chain_len] = 1
    a_ii = PAPER_DPD["a"]
    a_ps = a_ii + 2.05 * CHI_POLYMER_SOLVENT
    s.meta["species"] = species
    s.meta["a_table"] = np.array([[a_ii, a_ps], [a_ps, a_ii]])
    s.meta["chain"] = np.arange(chain_len, dtype=np.int64)
    s.meta["name"] = f"polyelectrolyte set 5: f={f} N={s.N} L={L}"
    return s
