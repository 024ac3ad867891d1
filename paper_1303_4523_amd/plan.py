"""Python face of an ENUF plan: torch tensors in, torch tensors out."""
import ctypes

import torch

from . import _lib
from ._lib import EnufError, check, lib


def _device(device):
    """torch.device for a CUDA index, a torch.device, or None (current device)."""
    if device is None:
        return torch.device("cuda", torch.cuda.current_device())
    if isinstance(device, torch.device):
        return device if device.index is not None else torch.device("cuda", torch.cuda.current_device())
    return torch.device("cuda", int(device))


def _dev_ptr(t, name, shape, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """An ENUF plan for N particles (see include/enuf.h for the parameters)."""

    def __init__(self, N, box, alpha, p, sigma, M, Kc, r_cut, lam, precision="fp64",
                 window="kb", device=None):
        self.N = int(N)
        self.params = dict(box=box, alpha=alpha, p=p, sigma=sigma, M=M, Kc=Kc, r_cut=r_cut, lam=lam)
        self.device = _device(device)
        with torch.cuda.device(self.device):
            h = lib.enuf_plan_create(self.N, float(box), float(alpha), int(p), float(sigma), int(M),
                                     int(Kc), float(r_cut), float(lam))
        if not h:
            raise EnufError(_lib.EINVAL, "enuf_plan_create")
        self._h = ctypes.c_void_p(h)
        self.set_options(precision, window)

    def set_options(self, precision="fp64", window="kb"):
        pr = {"fp64": _lib.FP64, "mixed": _lib.MIXED}[precision]
        wi = {"kb": _lib.WINDOW_KB, "gauss": _lib.WINDOW_GAUSS}[window]
        check(lib.enuf_plan_set_options(self._h, pr, wi), "enuf_plan_set_options")
        self.precision, self.window = precision, window

    def set_force_mode(self, mode="gradient"):
        """'gradient' (exact gradient of the NFFT energy) or 'ik' (eq. 24-25)."""
        m = {"gradient": _lib.FORCE_GRADIENT, "ik": _lib.FORCE_IK}[mode]
        check(lib.enuf_plan_set_force_mode(self._h, m), "enuf_plan_set_force_mode")
        self.force_mode = mode

    def set_parts(self, parts):
        """Work-groups per mesh plane in the spread and gather passes (1 up
        to the creation default min(8, 128 / M)); 1 for systems stepped in a
        batch, which already fills the device."""
        check(lib.enuf_plan_set_parts(self._h, int(parts)), "enuf_plan_set_parts")

    def set_concurrency(self, enable):
        """Real-space term beside the mesh passes (True, the default) or the
        whole evaluation on one stream (False); results are the same."""
        check(lib.enuf_plan_set_concurrency(self._h, int(bool(enable))), "enuf_plan_set_concurrency")

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib.enuf_plan_set_stream(self._h, ctypes.c_void_p(s)), "enuf_plan_set_stream")

    def compute(self, pos, q, forces=None, energy=None):
        """Total energy (1-element tensor) and forces (N x 3), enqueued on the
        current stream."""
        N = self.N
        if forces is None:
            forces = torch.empty((N, 3), dtype=torch.float64, device=self.device)
        if energy is None:
            energy = torch.empty((1,), dtype=torch.float64, device=self.device)
        args = (_dev_ptr(pos, "pos", (N, 3)), _dev_ptr(q, "q", (N,)),
                _dev_ptr(forces, "forces", (N, 3)), _dev_ptr(energy, "energy", (1,)))
        self._bind_stream()
        check(lib.enuf_compute(self._h, *args), "enuf_compute")
        return forces, energy

    def compute_components(self, pos, q, forces=None, energy5=None):
        """Forces and the energy split (E_real, E_slater, E_recip, E_self,
        E_recip via the gathered potential)."""
        N = self.N
        if forces is None:
            forces = torch.empty((N, 3), dtype=torch.float64, device=self.device)
        if energy5 is None:
            energy5 = torch.empty((5,), dtype=torch.float64, device=self.device)
        args = (_dev_ptr(pos, "pos", (N, 3)), _dev_ptr(q, "q", (N,)),
                _dev_ptr(forces, "forces", (N, 3)), _dev_ptr(energy5, "energy5", (5,)))
        self._bind_stream()
        check(lib.enuf_compute_components(self._h, *args), "enuf_compute_components")
        return forces, energy5

    def status(self):
        """Synchronise and return (and clear) the sticky device status code."""
        st = ctypes.c_int(0)
        check(lib.enuf_plan_status(self._h, ctypes.byref(st)), "enuf_plan_status")
        return st.value

    def time_kernel(self, name, max_launches):
        """Start event timing of one kernel of compute() (name as in
        _lib.KERNELS); None stops."""
        k = -1 if name is None else _lib.KERNELS[name]
        check(lib.enuf_plan_time_kernel(self._h, k, int(max_launches)), "enuf_plan_time_kernel")

    def kernel_time(self):
        """(total milliseconds, launches) of the timed kernel."""
        ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
        check(lib.enuf_plan_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)), "enuf_plan_kernel_time")
        return ms.value, n.value

    @property
    def footprint_bytes(self):
        return int(lib.enuf_plan_footprint_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib.enuf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compute_noalloc(pos, q, box, alpha, p, sigma, M, Kc, r_cut, lam, precision="fp64", forces=None,
                    energy5=None, status=None):
    """One evaluation through enuf_compute_noalloc (no plan, no device
    allocation inside the library) on the current stream; forces, energy5 and
    status (1 int32) may be passed preallocated.  Returns (forces, energy5,
    status)."""
    N = int(q.shape[0])
    dev = pos.device
    if forces is None:
        forces = torch.empty((N, 3), dtype=torch.float64, device=dev)
    if energy5 is None:
        energy5 = torch.empty((5,), dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty((1,), dtype=torch.int32, device=dev)
    pr = {"fp64": _lib.FP64, "mixed": _lib.MIXED}[precision]
    args = (_dev_ptr(pos, "pos", (N, 3)), _dev_ptr(q, "q", (N,)), _dev_ptr(forces, "forces", (N, 3)),
            _dev_ptr(energy5, "energy5", (5,)), _dev_ptr(status, "status", (1,), torch.int32))
    s = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        check(lib.enuf_compute_noalloc(N, float(box), float(alpha), int(p), float(sigma), int(M), int(Kc),
                                       float(r_cut), float(lam), pr, *args, ctypes.c_void_p(s)),
              "enuf_compute_noalloc")
    return forces, energy5, status
