"""Pins of the NumPy NFFT mirror (test infrastructure for GPU intermediates).

The mirror restates the NFFT reciprocal path of Sec. 3.3: window spread
(transposed NFFT, eq. 14), FFT, deconvolution, influence multiply, and the
window-gradient gather.  Its pins: the window transform against numerical
quadrature, the NDFT against numpy's FFT, the direct Ewald oracle within the
NFFT error that decays exponentially with p (Sec. 5), Parseval, and finite
differences of its own energy.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import nfft_mirror as nm


@pytest.mark.parametrize("kind,p", [("kb", 4), ("kb", 2), ("gauss", 4)])
def test_window_transform_by_quadrature(kind, p):
    win = nm.Window(kind, p, 2.0)
    for xi in (0.0, 0.05, 0.125, 0.25):
        val = integrate.quad(lambda t: float(win.phi(t)) * np.cos(2 * np.pi * xi * t), -p, p,
                             limit=400, epsabs=1e-13, epsrel=1e-12)[0]
        ref = float(win.phihat(xi))
        # Both closed-form transforms belong to the untruncated windows; cutting
        # the window at |t| = p costs ~exp(-b p) (KB) or ~exp(-p^2/b) (Gauss).
        tol = 10 * np.exp(-win.b * p) if kind == "kb" else 5e-4
        assert abs(val - ref) < tol * abs(ref)


@pytest.mark.parametrize("kind", ["kb", "gauss"])
def test_window_derivative_by_differences(kind):
    win = nm.Window(kind, 4, 2.0)
    t = np.linspace(-3.9, 3.9, 37)
    h = 1e-6
    fd = (win.phi(t + h) - win.phi(t - h)) / (2 * h)
    assert np.abs(fd - win.dphi(t)).max() < 1e-7


def test_ndft_matches_fft_on_grid_points():
    """eq. 14/19: for charges sitting on mesh points the structure factor is the
    plain DFT of the charge mesh (same sign convention as numpy.fft)."""
    M, L = 16, 4.0
    rs = np.random.default_rng(2)
    idx = rs.integers(0, M, (20, 3))
    q = rs.normal(size=20)
    mesh = np.zeros((M, M, M))
    np.add.at(mesh, (idx[:, 0], idx[:, 1], idx[:, 2]), q)
    G = np.fft.fftn(mesh)
    ks = rs.integers(-M // 2, M // 2, (30, 3))
    S = nm.structure_factor(idx * (L / M), q, L, ks)
    assert np.abs(S - G[ks[:, 0] % M, ks[:, 1] % M, ks[:, 2] % M]).max() < 1e-11


def _small_system(seed=11, nq=120, L=8.0):
    rs = np.random.default_rng(seed)
    pos = rs.uniform(0.0, L, (nq, 3))
    q = np.where(np.arange(nq) % 2 == 0, 1.0, -1.0)
    return pos, q, L


def test_mirror_vs_direct_sum_decays_with_p():
    """Sec. 3.3 / Sec. 5: the NFFT approximates only the reciprocal sum and its
    error falls exponentially with the window half-width p at sigma = 2."""
    pos, q, L = _small_system()
    alpha, Kc, M = 0.4, 8, 32
    Fd, Ed = oracle.recip_direct(pos, q, L, alpha, Kc)
    errs = []
    for p in (2, 3, 4, 5):
        r = nm.recip_nfft(pos, q, L, alpha, Kc, M, nm.Window("kb", p, 2.0))
        ef = np.linalg.norm(r["F"] - Fd) / np.linalg.norm(Fd)
        ee = abs(r["E"] - Ed) / abs(Ed)
        errs.append((ef, ee))
        assert abs(r["E_gather"] - r["E"]) < 1e-11 * abs(r["E"])  # Parseval
    for (f1, _), (f2, _) in zip(errs, errs[1:]):
        assert f2 < 0.3 * f1
    assert errs[2][0] < 3e-5 and errs[2][1] < 1e-6   # p = 4
    assert errs[3][0] < 3e-6


def test_gaussian_window_is_less_accurate_at_p4():
    pos, q, L = _small_system()
    alpha, Kc, M = 0.4, 8, 32
    Fd, _ = oracle.recip_direct(pos, q, L, alpha, Kc)
    e = {}
    for kind in ("kb", "gauss"):
        r = nm.recip_nfft(pos, q, L, alpha, Kc, M, nm.Window(kind, 4, 2.0))
        e[kind] = np.linalg.norm(r["F"] - Fd) / np.linalg.norm(Fd)
    assert e["kb"] < e["gauss"] < 1e-2


def test_mirror_force_is_gradient_of_mirror_energy():
    pos, q, L = _small_system(nq=24, L=6.0)
    alpha, Kc, M = 0.5, 6, 24
    win = nm.Window("kb", 4, 2.0)
    r0 = nm.recip_nfft(pos, q, L, alpha, Kc, M, win)
    h = 1e-5
    for i, a in [(0, 0), (5, 1), (13, 2)]:
        ep = pos.copy(); ep[i, a] += h
        em = pos.copy(); em[i, a] -= h
        fd = -(nm.recip_nfft(ep, q, L, alpha, Kc, M, win)["E"]
               - nm.recip_nfft(em, q, L, alpha, Kc, M, win)["E"]) / (2 * h)
        assert abs(fd - r0["F"][i, a]) < 1e-7 * (1 + abs(fd))
