"""Structure observables sampled on the device (radial distribution
functions, Sec. 5; radius of gyration, Sec. 6).

Thin wrappers over ``enuf_pair_histogram`` and ``enuf_chain_rg2``: the
counting and the unwrapping run in the library's HIP kernels on the current
torch stream, so a trajectory can be sampled between steps without copying
it to the host.  Only the normalisation of the final counts to g(r) is done
here, on the host.
"""
import ctypes
import math

import numpy as np
import torch

from ._lib import check, lib
from .plan import _dev_ptr, _device


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class PairHistogram:
    """Accumulates pair-distance counts by class over samples.

    sel: indices of the particles taken into account; cls: class of each
    selected particle (0 .. ncls-1).  Bins of width r_max / nbins."""

    def __init__(self, n, sel, cls, ncls, L, r_max, nbins, device=None):
        self.device = _device(device)
        self.n = int(n)
        self.L = float(L)
        self.r_max = float(r_max)
        self.nbins = int(nbins)
        self.ncls = int(ncls)
        sel = np.asarray(sel, dtype=np.int64).reshape(-1)
        cls = np.asarray(cls, dtype=np.int32).reshape(-1)
        if sel.shape != cls.shape:
            raise ValueError("one class per selected particle")
        self.class_counts = np.bincount(cls, minlength=self.ncls)[:self.ncls]
        self.sel = torch.as_tensor(sel, device=self.device)
        self.cls = torch.as_tensor(cls, device=self.device)
        # uint64 counters kept in an int64 tensor (counts stay far below 2^63)
        self.hist = torch.zeros(self.ncls * self.ncls * self.nbins, dtype=torch.int64, device=self.device)
        self.samples = 0

    def sample(self, pos):
        """Add the pairs of one configuration (N x 3 FP64 CUDA tensor)."""
        p = _dev_ptr(pos, "pos", (self.n, 3))
        check(lib.enuf_pair_histogram(p, self.n, int(self.sel.shape[0]), ctypes.c_void_p(self.sel.data_ptr()),
                                      ctypes.c_void_p(self.cls.data_ptr()), self.ncls, self.L, self.r_max,
                                      self.nbins, ctypes.c_void_p(self.hist.data_ptr()), _stream(self.device)),
              "enuf_pair_histogram")
        self.samples += 1

    def counts(self):
        """(ncls, ncls, nbins) uint64 counts (entries with class_lo <= class_hi)."""
        return self.hist.cpu().numpy().astype(np.uint64).reshape(self.ncls, self.ncls, self.nbins)

    def rdf(self):
        """(r, g) with g[a, b] the radial distribution function of classes a <= b:
        counts / (pairs * shell volume / V * samples), r the bin centres."""
        h = self.counts().astype(np.float64)
        w = self.r_max / self.nbins
        edges = w * np.arange(self.nbins + 1)
        shell = 4.0 / 3.0 * math.pi * np.diff(edges ** 3)
        V = self.L ** 3
        g = np.zeros_like(h)
        nc = self.class_counts.astype(np.float64)
        for a in range(self.ncls):
            for b in range(a, self.ncls):
                pairs = nc[a] * (nc[a] - 1.0) / 2.0 if a == b else nc[a] * nc[b]
                if pairs > 0 and self.samples > 0:
                    g[a, b] = h[a, b] / (pairs * shell / V * self.samples)
                    g[b, a] = g[a, b]
        return 0.5 * (edges[1:] + edges[:-1]), g


def chain_rg2(pos, beads, L, out=None):
    """Squared radius of gyration of each chain (beads: (nchains, len) int64
    CUDA tensor, bond order) into out (nchains FP64 CUDA tensor, returned)."""
    n = int(pos.shape[0])
    if beads.dim() == 1:
        beads = beads[None, :]
    nch, ln = int(beads.shape[0]), int(beads.shape[1])
    if beads.dtype != torch.int64 or beads.device != pos.device or not beads.is_contiguous():
        raise TypeError("beads must be a contiguous int64 tensor on the positions' device")
    if out is None:
        out = torch.empty(nch, dtype=torch.float64, device=pos.device)
    o = _dev_ptr(out, "out", (nch,))
    check(lib.enuf_chain_rg2(_dev_ptr(pos, "pos", (n, 3)), n, nch, ln, ctypes.c_void_p(beads.data_ptr()),
                             float(L), o, _stream(pos.device)), "enuf_chain_rg2")
    return out
