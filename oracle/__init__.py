"""FP64 CPU oracle for ENUF-DPD electrostatics -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls anything here, and this
package imports nothing from the product.

Contents
--------
* ``ewald`` / ``real_space`` / ``recip_direct`` / ``self_energy``:
  the truncated Ewald sum of the paper (Sec. 3.1, eq. 16) with the reciprocal
  part summed directly over every integer wave vector 0 < |k| < Kc
  (eq. 18-24) and the real-space erfc term plus the additive Slater
  correction over minimum-image pairs with r < r_cut (eq. 27, 31).
* ``dpd_forces`` / ``dpd_step``: the modified velocity-Verlet DPD step of
  Table 2 with the pair forces of eq. 2-7, harmonic bonds and the
  electrostatic force above.
* ``pair_histogram`` / ``chain_rg2``: the pair-distance histogram by class
  behind the radial distribution functions (Sec. 5) and the radius of
  gyration of a chain (Sec. 6).
* ``philox4x32_10`` / ``theta``: the counter-based generator that supplies
  the random variable theta_ij (``philox4x64_10`` is kept and pinned too).
* ``nfft_mirror``: a NumPy re-statement of the NFFT reciprocal path (window
  spread, FFT, deconvolution, window-gradient gather) for checking GPU
  intermediates; it is not the parity target.

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _DPDParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("a", ctypes.c_double),
                ("gamma", ctypes.c_double), ("sigma", ctypes.c_double),
                ("dt", ctypes.c_double), ("lam", ctypes.c_double),
                ("k_bond", ctypes.c_double), ("r0_bond", ctypes.c_double),
                ("kappa", ctypes.c_double), ("alpha", ctypes.c_double),
                ("r_cut", ctypes.c_double), ("lambda_e", ctypes.c_double),
                ("Kc", ctypes.c_int), ("use_elec", ctypes.c_int),
                ("nspec", ctypes.c_int), ("species", ctypes.c_void_p),
                ("atab", ctypes.c_double * 16)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "enuf_oracle.c"))):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    d, i64, ip = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_real.argtypes = [i64, ip, ip, d, d, d, d, i64, ip, ip, ip]
    lib.oracle_real.restype = ctypes.c_int
    lib.oracle_recip.argtypes = [i64, ip, ip, d, d, ctypes.c_int, i64, ip, ip, ip]
    lib.oracle_recip.restype = ctypes.c_int
    lib.oracle_pair_histogram.argtypes = [i64, ip, i64, ip, ip, ctypes.c_int, d, d, ctypes.c_int, ip]
    lib.oracle_pair_histogram.restype = ctypes.c_int
    lib.oracle_chain_rg2.argtypes = [i64, ip, ctypes.c_int, ctypes.c_int, ip, d, ip]
    lib.oracle_chain_rg2.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_self.argtypes = [i64, ip, d]
    lib.oracle_self.restype = d
    lib.oracle_philox4x64_10.argtypes = [ip, ip, ip]
    lib.oracle_philox4x64_10.restype = None
    lib.oracle_philox4x32_10.argtypes = [ip, ip, ip]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_theta.argtypes = [ctypes.c_uint64, ctypes.c_uint64, i64, i64]
    lib.oracle_theta.restype = d
    lib.oracle_dpd_forces.argtypes = [i64, ip, ip, ip, i64, ip, ctypes.POINTER(_DPDParams),
                                      ctypes.c_uint64, ctypes.c_uint64, ip, ip]
    lib.oracle_dpd_forces.restype = ctypes.c_int
    lib.oracle_dpd_step.argtypes = [i64, ip, ip, ip, ip, i64, ip, ctypes.POINTER(_DPDParams),
                                    ctypes.c_uint64, ctypes.c_uint64, ip]
    lib.oracle_dpd_step.restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(st, what):
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


def real_space(pos, q, L, alpha, r_cut, lam, sel=None):
    """Real-space erfc term + Slater correction (eq. 27, 31).

    Returns (F, E_short, E_slater): E_short is the whole short-range energy
    (erfc term plus Slater correction, added pair by pair), E_slater the part
    of it due to the Slater correction.  With ``sel`` only the listed rows of
    F are computed and the energies are NaN.
    """
    lib = _load()
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    n = len(q)
    s = None if sel is None else np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    nout = n if s is None else len(s)
    F = np.zeros((nout, 3))
    E = np.zeros(2)
    st = lib.oracle_real(n, _ptr(pos), _ptr(q), L, alpha, r_cut, lam,
                         0 if s is None else len(s), _ptr(s), _ptr(F), _ptr(E))
    _check(st, "oracle_real")
    return F, float(E[0]), float(E[1])


def recip_direct(pos, q, L, alpha, Kc, sel=None):
    """Direct reciprocal sum over integer 0 < |k| < Kc (eq. 18-24): (F, E)."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    n = len(q)
    s = None if sel is None else np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    nout = n if s is None else len(s)
    F = np.zeros((nout, 3))
    E = np.zeros(1)
    st = lib.oracle_recip(n, _ptr(pos), _ptr(q), L, alpha, int(Kc),
                          0 if s is None else len(s), _ptr(s), _ptr(F), _ptr(E))
    _check(st, "oracle_recip")
    return F, float(E[0])


def num_threads():
    """OpenMP threads used by the oracle's parallel loops."""
    return int(_load().oracle_num_threads())


def set_threads(n):
    """OpenMP threads of the oracle's parallel loops started from the calling
    thread from now on."""
    _load().oracle_set_threads(int(n))


def self_energy(q, alpha):
    """Self term of eq. 16."""
    q = _f64(q)
    return float(_load().oracle_self(len(q), _ptr(q), alpha))


def ewald(pos, q, L, alpha, Kc, r_cut, lam, sel=None):
    """Full truncated Ewald energy and forces (Coulomb prefactor 1).

    Returns a dict with the energies ``E_real`` (whole short-range sum: erfc
    term plus Slater correction), ``E_slater`` (the Slater part of E_real,
    diagnostic), ``E_recip``, ``E_self``, the total ``E = E_real + E_recip +
    E_self`` (NaN when ``sel`` is given), and the forces ``F_real`` (erfc +
    Slater), ``F_recip`` and ``F``.
    """
    Fr, Ee, Es = real_space(pos, q, L, alpha, r_cut, lam, sel)
    Fk, Ek = recip_direct(pos, q, L, alpha, Kc, sel)
    Eself = self_energy(q, alpha)
    return dict(E_real=Ee, E_slater=Es, E_recip=Ek, E_self=Eself,
                E=Ee + Ek + Eself, F_real=Fr, F_recip=Fk, F=Fr + Fk)


def philox4x64_10(counter, key):
    """Philox4x64 with 10 rounds: four 64-bit counter words, two key words."""
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    _load().oracle_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds: four 32-bit counter words, two key words."""
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def theta(seed, step, i, j):
    """Random variable theta_ij of the DPD random force (uniform, unit variance)."""
    return float(_load().oracle_theta(seed, step, i, j))


def _params(p):
    """ctypes parameters; with p["species"] (int per particle) and p["a_table"]
    (nspec x nspec) the conservative amplitude is a_{s_i s_j}.  Returns the
    structure and the species array it points to (keep both alive)."""
    P = _DPDParams(L=p["L"], a=p["a"], gamma=p["gamma"], sigma=p["sigma"], dt=p["dt"],
                   lam=p["lam"], k_bond=p["k_bond"], r0_bond=p["r0_bond"],
                   kappa=p.get("kappa", 0.0), alpha=p.get("alpha", 1.0),
                   r_cut=p.get("r_cut", 1.0), lambda_e=p.get("lambda_e", 0.0),
                   Kc=int(p.get("Kc", 1)), use_elec=int(p.get("use_elec", 0)))
    sp = None
    if p.get("species") is not None:
        sp = np.ascontiguousarray(np.asarray(p["species"], dtype=np.int32))
        tab = np.asarray(p["a_table"], dtype=np.float64)
        ns = tab.shape[0]
        P.nspec = ns
        P.species = sp.ctypes.data
        for a in range(ns):
            for b in range(ns):
                P.atab[4 * a + b] = tab[a, b]
    return P, sp


def dpd_forces(pos, vel, q, bonds, params, seed, step):
    """Total DPD force (conservative, dissipative, random/sqrt(dt), bonds,
    kappa * electrostatics).  Returns (F, E_elec)."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    vel = _f64(vel, (-1, 3))
    q = _f64(q)
    b = np.ascontiguousarray(np.asarray(bonds, dtype=np.int64).reshape(-1, 2))
    F = np.zeros_like(pos)
    E = np.zeros(1)
    P, _sp = _params(params)
    st = lib.oracle_dpd_forces(len(q), _ptr(pos), _ptr(vel), _ptr(q), len(b), _ptr(b),
                               ctypes.byref(P), seed, step, _ptr(F), _ptr(E))
    _check(st, "oracle_dpd_forces")
    return F, float(E[0])


def dpd_step(pos, vel, F, q, bonds, params, seed, step):
    """One modified velocity-Verlet step (Table 2).  Returns new
    (pos, vel, F, E_elec); the inputs are not modified."""
    lib = _load()
    pos = _f64(pos, (-1, 3)).copy()
    vel = _f64(vel, (-1, 3)).copy()
    F = _f64(F, (-1, 3)).copy()
    q = _f64(q)
    b = np.ascontiguousarray(np.asarray(bonds, dtype=np.int64).reshape(-1, 2))
    E = np.zeros(1)
    P, _sp = _params(params)
    st = lib.oracle_dpd_step(len(q), _ptr(pos), _ptr(vel), _ptr(F), _ptr(q), len(b), _ptr(b),
                             ctypes.byref(P), seed, step, _ptr(E))
    _check(st, "oracle_dpd_step")
    return pos, vel, F, float(E[0])


def pair_histogram(pos, sel, cls, ncls, L, r_max, nbins):
    """Counts of unordered selected pairs by (class_lo, class_hi, bin of r);
    returns a (ncls, ncls, nbins) uint64 array (only lo <= hi filled)."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    cls = np.ascontiguousarray(np.asarray(cls, dtype=np.int32))
    h = np.zeros((ncls, ncls, nbins), dtype=np.uint64)
    st = lib.oracle_pair_histogram(len(pos), _ptr(pos), len(sel), _ptr(sel), _ptr(cls), int(ncls), float(L),
                                   float(r_max), int(nbins), _ptr(h))
    _check(st, "oracle_pair_histogram")
    return h


def chain_rg2(pos, beads, L):
    """Squared radius of gyration of each chain; beads is (nchains, len)."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    b = np.ascontiguousarray(np.asarray(beads, dtype=np.int64))
    if b.ndim == 1:
        b = b[None, :]
    out = np.zeros(b.shape[0])
    st = lib.oracle_chain_rg2(len(pos), _ptr(pos), b.shape[0], b.shape[1], _ptr(b), float(L), _ptr(out))
    _check(st, "oracle_chain_rg2")
    return out
