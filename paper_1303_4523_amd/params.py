"""Choice of the ENUF parameters from a target accuracy (Sec. 5, eq. 29).

Given the accuracy delta of the truncated Ewald sums and a real-space cutoff
r_c (chosen to suit the cell list), eq. 29 fixes the other two:

* real space: erfc(alpha r_c) <= delta, so alpha is the root of
  erfc(alpha r_c) = delta (eq. 29 also writes the Gaussian bound
  exp(-alpha^2 r_c^2); the complementary error function itself is used here);
* reciprocal space: exp(-pi^2 n^2 / (alpha L)^2) <= delta for every wave
  vector left out, so the smallest integer cutoff with
  n_c >= (alpha L / pi) sqrt(-ln delta); with the strict sphere 0 < |k| < Kc
  the first excluded length is Kc itself.

The NFFT adds two parameters (Sec. 5): the oversampling sigma_s (2, after the
paper) and the window half-width p, whose error decays exponentially in p at
fixed sigma_s.  The decay rates are those of the NFFT windows: the
Kaiser-Bessel window's error falls like exp(-b p), b = pi (2 - 1/sigma); the
Gaussian's like exp(-pi p (1 - 1/(2 sigma - 1))).  The prefactors are
calibrated on this implementation (relative force RMS error of the NFFT part,
measured on the paper's second test set, 2000 + 2000 charges at L = 10, for
p = 1..7, sigma = 1.5 and 2, Kc = 7..14): 1000 for Kaiser-Bessel and 4 for the
Gaussian, upper bounds of the measurements for 3 <= p <= 6.  p is the smallest
integer whose modelled NFFT error is below delta, so the forces meet delta
(the paper's p = 2 was chosen on energy errors, which are two orders smaller).
The FFT mesh M is the smallest even 2^a 3^b 5^c with Kc <= M / (2 sigma) and
2p <= M / 2.

Host arithmetic only (no device work); the values feed ``Plan`` / ``DPD``.
"""
import math

from .workloads import mesh_size


def _erfc_root(target, r_cut):
    """alpha with erfc(alpha r_cut) = target (bisection on a monotone function)."""
    lo, hi = 0.0, 1.0
    while math.erfc(hi * r_cut) > target:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if math.erfc(mid * r_cut) > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def window_decay(window, sigma):
    """Exponential decay rate of the NFFT window error in p."""
    if window == "kb":
        return math.pi * (2.0 - 1.0 / sigma)
    if window == "gauss":
        return math.pi * (1.0 - 1.0 / (2.0 * sigma - 1.0))
    raise ValueError(f"unknown window {window!r}")


WINDOW_PREFACTOR = {"kb": 1000.0, "gauss": 4.0}


def nfft_error(window, sigma, p):
    """Modelled relative force error of the NFFT part at half-width p."""
    return WINDOW_PREFACTOR[window] * math.exp(-window_decay(window, sigma) * p)


def choose(L, delta=1e-4, r_cut=3.0, sigma=2.0, window="kb", lam=0.25):
    """ENUF parameters for a box of edge L at accuracy delta: a dict with
    alpha, Kc, M, p, sigma, r_cut, lam, L, window (ready for ``Plan``)."""
    if not (0.0 < delta < 1.0):
        raise ValueError("delta must be in (0, 1)")
    if not (0.0 < r_cut <= 0.5 * L):
        raise ValueError("need 0 < r_cut <= L/2")
    ln = -math.log(delta)
    alpha = _erfc_root(delta, r_cut)
    Kc = int(math.ceil(alpha * L * math.sqrt(ln) / math.pi - 1e-12))
    Kc = max(Kc, 1)
    p = 1
    while nfft_error(window, sigma, p) > delta:
        p += 1
    M = mesh_size(max(2.0 * sigma * Kc, 4.0 * p, 4.0))
    return dict(alpha=alpha, Kc=Kc, M=M, p=p, sigma=sigma, r_cut=r_cut, lam=lam, L=float(L), window=window)
