"""Batched DPD steps of many independent systems (enuf_batch_* C ABI).

Each member is a DPD integrator (with its own ENUF plan) plus its device
state tensors; one run advances all members with one kernel launch per stage
of the step, replayed from a captured HIP graph.
"""
import ctypes

import torch

from . import _lib
from ._lib import EnufError, check, lib
from .plan import _dev_ptr, _device


class Batch:
    def __init__(self, precision="mixed", device=None, use_graph=True, concurrent=True):
        self.device = _device(device)
        self.precision = precision
        pr = {"fp64": _lib.FP64, "mixed": _lib.MIXED}[precision]
        with torch.cuda.device(self.device):
            h = lib.enuf_batch_create(pr)
        if not h:
            raise EnufError(_lib.EINVAL, "enuf_batch_create")
        self._h = ctypes.c_void_p(h)
        self._members = {}   # id -> (dpd, pos, vel, force): keeps the state tensors alive
        self.set_options(use_graph, concurrent)

    def set_options(self, use_graph=True, concurrent=True):
        """use_graph: True (replay a captured step), False (eager launches) or
        "auto" (capture only for runs of at least GRAPH_AUTO_STEPS steps and
        reuse the graph while the membership is unchanged)."""
        g = _lib.GRAPH_AUTO if use_graph == "auto" else int(bool(use_graph))
        check(lib.enuf_batch_set_options(self._h, g, int(bool(concurrent))), "enuf_batch_set_options")

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib.enuf_batch_set_stream(self._h, ctypes.c_void_p(s)), "enuf_batch_set_stream")

    def add(self, dpd, pos, vel, force, first_step):
        """Add an integrator and its state (force must hold the current force).
        Returns the member id."""
        N = dpd.N
        args = (_dev_ptr(pos, "pos", (N, 3)), _dev_ptr(vel, "vel", (N, 3)), _dev_ptr(force, "force", (N, 3)))
        self._bind_stream()
        mid = lib.enuf_batch_add(self._h, dpd._h, *args, int(first_step))
        if mid < 0:
            raise EnufError(mid, "enuf_batch_add")
        self._members[mid] = (dpd, pos, vel, force)
        return mid

    def remove(self, member_id):
        check(lib.enuf_batch_remove(self._h, int(member_id)), "enuf_batch_remove")
        return self._members.pop(member_id)

    def __len__(self):
        return int(lib.enuf_batch_size(self._h))

    def run(self, nsteps):
        """Advance every member nsteps steps (ordered on the current stream)."""
        self._bind_stream()
        check(lib.enuf_batch_run(self._h, int(nsteps)), "enuf_batch_run")

    def time_kernel(self, name, max_launches):
        """Start event timing of one stage of the batched step (name as in
        _lib.KERNELS); runs are then launched eagerly on one stream.  None
        stops."""
        k = -1 if name is None else _lib.KERNELS[name]
        check(lib.enuf_batch_time_kernel(self._h, k, int(max_launches)), "enuf_batch_time_kernel")

    def kernel_time(self):
        """(total milliseconds, launches) of the timed stage."""
        ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
        check(lib.enuf_batch_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)), "enuf_batch_kernel_time")
        return ms.value, n.value

    @property
    def footprint_bytes(self):
        return int(lib.enuf_batch_footprint_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib.enuf_batch_destroy(self._h)
            self._h = None
        self._members = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
