"""MI355X-native ENUF electrostatics (Ewald summation with the non-uniform FFT).

The computation runs in the HIP library ``libenuf.so`` (C ABI in
``include/enuf.h``).  This package only marshals torch tensors into that ABI.

    >>> import torch, paper_1303_4523_amd as enuf
    >>> plan = enuf.Plan(N, box=10.0, alpha=0.3, p=4, sigma=2.0, M=32, Kc=8,
    ...                  r_cut=3.0, lam=0.25)
    >>> forces, energy = plan.compute(pos, q)     # cuda float64 tensors

``workloads`` (seeded synthetic inputs) is importable without the library.
"""

__all__ = ["Plan", "EnufError"]


def __getattr__(name):
    # The library is loaded lazily so that ``workloads`` stays importable on
    # machines without a GPU build.
    if name in ("Plan", "EnufError"):
        from . import plan as _plan
        return getattr(_plan, name)
    raise AttributeError(name)
