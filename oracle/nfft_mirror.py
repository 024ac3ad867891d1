"""NumPy statement of the NFFT reciprocal path -- TEST INFRASTRUCTURE.

This is not the parity target (the direct Ewald sum in ``enuf_oracle.c`` is).
It re-states, in plain NumPy and independently of the HIP code, what each
stage of the ENUF reciprocal computation produces, so that tests can check
GPU intermediates and the size of the NFFT approximation error:

* the adjoint NFFT ("transposed" form, eq. 14): charges spread onto the
  oversampled mesh with a window function phi of half-width p mesh cells,
  g[l] = sum_j q_j prod_t phi(M x_{j,t} - l_t), l periodic;
* its FFT G = fftn(g) and the deconvolution S(k) ~ G(k) / prod_t Phi(k_t / M),
  where Phi is the continuous Fourier transform of phi (Sec. 3.3);
* the reciprocal energy of eq. 18/20 restricted to 0 < |k| < Kc;
* the force as the exact gradient of that energy through the window
  (h = unnormalised inverse FFT of c(k) G(k), c = W / prod Phi^2, then
  F_j = -(q_j M / (pi L^2)) sum_l h[l] grad prod_t phi(M x_j - l)).

Windows: the Gaussian named by the paper (Sec. 4) and the Kaiser-Bessel
window of the NFFT literature (Fourmont 2003; Keiner, Kunis & Potts 2009),
both normalised to phi(0) = 1.  Stencil: 2p points per axis starting at
floor(M x) - p + 1.  Every quantity is FP64.  Loops run over particles, so
this is for small inputs only.
"""
import numpy as np
from scipy import special


class Window:
    """A window phi(t) (t in mesh cells, support |t| < p) and its transform."""

    def __init__(self, kind, p, sigma):
        self.kind = kind
        self.p = int(p)
        self.sigma = float(sigma)
        if kind == "kb":
            self.b = np.pi * (2.0 - 1.0 / self.sigma)
            self.phi0 = np.sinh(self.b * self.p) / (np.pi * self.p)
        elif kind == "gauss":
            self.bg = 2.0 * self.sigma * self.p / ((2.0 * self.sigma - 1.0) * np.pi)
            self.phi0 = 1.0 / np.sqrt(np.pi * self.bg)
        else:
            raise ValueError(kind)

    def phi(self, t):
        t = np.asarray(t, dtype=np.float64)
        p = self.p
        if self.kind == "kb":
            s = np.sqrt(np.maximum(p * p - t * t, 0.0))
            safe = np.where(s > 0.0, s, 1.0)
            v = np.where(s > 0.0, np.sinh(self.b * safe) / (np.pi * safe), self.b / np.pi)
        else:
            v = np.exp(-t * t / self.bg) / np.sqrt(np.pi * self.bg)
        return np.where(np.abs(t) <= p, v, 0.0) / self.phi0

    def dphi(self, t):
        t = np.asarray(t, dtype=np.float64)
        p = self.p
        if self.kind == "kb":
            s = np.sqrt(np.maximum(p * p - t * t, 0.0))
            z = self.b * s
            safe = np.where(z > 1e-3, s, 1.0)
            # d/dt sinh(b s)/(pi s) = -(t/pi) (b s cosh(bs) - sinh(bs)) / s^3
            direct = -(t / np.pi) * (self.b * safe * np.cosh(self.b * safe)
                                     - np.sinh(self.b * safe)) / safe ** 3
            series = -(t / np.pi) * self.b ** 3 * (1.0 / 3.0 + z * z / 30.0)
            v = np.where(z > 1e-3, direct, series)
        else:
            v = -2.0 * t / self.bg * np.exp(-t * t / self.bg) / np.sqrt(np.pi * self.bg)
        return np.where(np.abs(t) <= p, v, 0.0) / self.phi0

    def phihat(self, xi):
        """Phi(xi) = integral phi(t) exp(-2 pi i xi t) dt (normalised phi)."""
        xi = np.asarray(xi, dtype=np.float64)
        if self.kind == "kb":
            arg = self.p * np.sqrt(self.b ** 2 - (2.0 * np.pi * xi) ** 2)
            return special.i0(arg) / self.phi0
        return np.exp(-self.bg * (np.pi * xi) ** 2) / self.phi0


def stencil(x, L, M, p):
    """Base index and offsets t - l for the 2p stencil points per axis."""
    t = M * (np.asarray(x, dtype=np.float64) / L)
    base = np.floor(t).astype(np.int64) - p + 1
    offs = t[..., None] - (base[..., None] + np.arange(2 * p))
    return base, offs


def wrap(pos, L):
    pos = np.asarray(pos, dtype=np.float64)
    w = pos - L * np.floor(pos / L)
    return np.where(w >= L, 0.0, w)


def spread(pos, q, L, M, win):
    """Adjoint NFFT: the real M^3 mesh g (index order [x, y, z])."""
    p = win.p
    pos = wrap(pos, L)
    g = np.zeros((M, M, M))
    for j in range(len(q)):
        if q[j] == 0.0:
            continue
        base, offs = stencil(pos[j], L, M, p)
        idx = [(base[a] + np.arange(2 * p)) % M for a in range(3)]
        w = [win.phi(offs[a]) for a in range(3)]
        np.add.at(g, np.ix_(*idx), q[j] * w[0][:, None, None] * w[1][None, :, None]
                  * w[2][None, None, :])
    return g


def influence(L, M, alpha, Kc, win):
    """c(k) = W(k) / prod_t Phi(k_t/M)^2 on the full M^3 FFT grid, zero outside
    0 < |k| < Kc (numpy fftfreq order)."""
    k = np.fft.fftfreq(M, 1.0 / M)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    mask = (K2 > 0) & (K2 < Kc * Kc)
    c = np.zeros((M, M, M))
    W = np.exp(-np.pi ** 2 * K2[mask] / (alpha * L) ** 2) / K2[mask]
    den = (win.phihat(KX[mask] / M) * win.phihat(KY[mask] / M) * win.phihat(KZ[mask] / M)) ** 2
    c[mask] = W / den
    return c


def recip_nfft(pos, q, L, alpha, Kc, M, win):
    """NFFT reciprocal energy and forces.  Returns dict with E (k-space sum),
    E_gather (the same energy through the gathered potential), F, g, G, h."""
    p = win.p
    pos = wrap(pos, L)
    q = np.asarray(q, dtype=np.float64)
    g = spread(pos, q, L, M, win)
    G = np.fft.fftn(g)
    c = influence(L, M, alpha, Kc, win)
    E = float((c * np.abs(G) ** 2).sum() / (2.0 * np.pi * L))
    h = np.real(np.fft.ifftn(c * G)) * M ** 3
    F = np.zeros((len(q), 3))
    A = np.zeros(len(q))
    for j in range(len(q)):
        if q[j] == 0.0:
            continue
        base, offs = stencil(pos[j], L, M, p)
        idx = [(base[a] + np.arange(2 * p)) % M for a in range(3)]
        w = [win.phi(offs[a]) for a in range(3)]
        d = [win.dphi(offs[a]) for a in range(3)]
        hh = h[np.ix_(*idx)]
        A[j] = np.einsum("abc,a,b,c", hh, w[0], w[1], w[2])
        B = np.array([np.einsum("abc,a,b,c", hh, d[0], w[1], w[2]),
                      np.einsum("abc,a,b,c", hh, w[0], d[1], w[2]),
                      np.einsum("abc,a,b,c", hh, w[0], w[1], d[2])])
        F[j] = -(q[j] * M / (np.pi * L ** 2)) * B
    E_gather = float((q * A).sum() / (2.0 * np.pi * L))
    return dict(E=E, E_gather=E_gather, F=F, g=g, G=G, h=h)


def structure_factor(pos, q, L, kvecs):
    """NDFT (eq. 19): S(k) = sum_j q_j exp(-2 pi i k . r_j / L)."""
    pos = np.asarray(pos, dtype=np.float64)
    ph = np.exp(-2j * np.pi * (pos @ np.asarray(kvecs, dtype=np.float64).T) / L)
    return (np.asarray(q)[:, None] * ph).sum(0)
