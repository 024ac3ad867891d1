"""DPD trajectories with ENUF electrostatics on the GPU (Table 2 integrator).

Thin wrapper over the enuf_dpd_* C ABI: state tensors live on the device and
every step runs in the library's HIP kernels.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import EnufError, check, lib
from .plan import Plan, _dev_ptr, _device


class DPD:
    """Integrator for N particles.  `enuf` is a dict of ENUF plan parameters
    (box is taken from L) or None for a system without electrostatics."""

    def __init__(self, L, q, params, bonds=None, enuf=None, precision="fp64", device=None):
        self.device = _device(device)
        qh = np.asarray(q, dtype=np.float64)
        self.nq = int(np.count_nonzero(qh))            # charged particles
        self.enuf = dict(enuf) if enuf is not None else None
        q = torch.as_tensor(qh, device=self.device).contiguous()
        self.N = int(q.shape[0])
        self.L = float(L)
        self.plan = None
        if enuf is not None:
            self.plan = Plan(self.N, L, enuf["alpha"], enuf["p"], enuf["sigma"], enuf["M"], enuf["Kc"],
                             enuf["r_cut"], enuf["lam"], precision=precision, device=self.device)
        b = np.zeros((0, 2), dtype=np.int64) if bonds is None else np.ascontiguousarray(
            np.asarray(bonds, dtype=np.int64).reshape(-1, 2))
        self._bonds = b
        self._q = q
        prm = _lib.DpdParams(a=params["a"], gamma=params["gamma"], sigma=params["sigma"], dt=params["dt"],
                             lam=params["lam"], k_bond=params.get("k_bond", 0.0),
                             r0_bond=params.get("r0_bond", 0.0), kappa=params.get("kappa", 0.0),
                             seed=int(params.get("seed", 0)))
        with torch.cuda.device(self.device):
            h = lib.enuf_dpd_create(self.N, self.L, ctypes.byref(prm),
                                    self.plan._h if self.plan is not None else None,
                                    ctypes.c_void_p(q.data_ptr()), len(b),
                                    b.ctypes.data_as(ctypes.c_void_p) if len(b) else None)
        if not h:
            raise EnufError(_lib.EINVAL, "enuf_dpd_create")
        self._h = ctypes.c_void_p(h)

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib.enuf_dpd_set_stream(self._h, ctypes.c_void_p(s)), "enuf_dpd_set_stream")

    def _state(self, pos, vel, force):
        N = self.N
        return (_dev_ptr(pos, "pos", (N, 3)), _dev_ptr(vel, "vel", (N, 3)), _dev_ptr(force, "force", (N, 3)))

    def forces(self, pos, vel, force, step=0):
        """Total force with vel standing in for the predicted velocities."""
        self._bind_stream()
        check(lib.enuf_dpd_forces(self._h, *self._state(pos, vel, force), int(step)), "enuf_dpd_forces")
        return force

    def run(self, pos, vel, force, first_step, nsteps):
        """Advance nsteps steps in place (force must hold the last force)."""
        self._bind_stream()
        check(lib.enuf_dpd_run(self._h, *self._state(pos, vel, force), int(first_step), int(nsteps)),
              "enuf_dpd_run")

    def prepare_graphs(self, pos, vel, force):
        """Capture the step graphs run() replays for these state tensors (no
        step is taken); later runs on them launch without capturing."""
        self._bind_stream()
        check(lib.enuf_dpd_prepare_graphs(self._h, *self._state(pos, vel, force)), "enuf_dpd_prepare_graphs")

    def set_concurrency(self, enable):
        """Overlap pair forces and real space with the mesh passes (default) or not."""
        check(lib.enuf_dpd_set_concurrency(self._h, int(bool(enable))), "enuf_dpd_set_concurrency")

    def set_graphs(self, enable):
        """Launch the steps of run() as HIP graphs of 8 and 2 steps (default) or eagerly."""
        check(lib.enuf_dpd_set_graphs(self._h, int(bool(enable))), "enuf_dpd_set_graphs")

    def set_species(self, species, a_table):
        """Species-dependent conservative amplitudes a_ij (eq. 3): species is
        an int per particle in [0, nspecies), a_table the symmetric
        nspecies x nspecies amplitudes (nspecies <= 4).  Set before the
        integrator joins a batch."""
        tab = np.ascontiguousarray(np.asarray(a_table, dtype=np.float64))
        ns = int(tab.shape[0])
        if tab.shape != (ns, ns):
            raise ValueError("a_table must be square")
        sp = np.ascontiguousarray(np.asarray(species, dtype=np.int32).reshape(-1))
        if ns > 1 and sp.shape[0] != self.N:
            raise ValueError("one species per particle")
        check(lib.enuf_dpd_set_species(self._h, ns, sp.ctypes.data_as(ctypes.c_void_p),
                                       tab.ctypes.data_as(ctypes.c_void_p)), "enuf_dpd_set_species")

    def energy(self):
        """ENUF energy components of the last evaluation (unscaled by kappa)."""
        e = torch.empty(5, dtype=torch.float64, device=self.device)
        self._bind_stream()
        check(lib.enuf_dpd_energy(self._h, ctypes.c_void_p(e.data_ptr())), "enuf_dpd_energy")
        return e

    def time_kernel(self, name, max_launches):
        """Start event timing of one kernel (name as in _lib.KERNELS); None stops."""
        k = -1 if name is None else _lib.KERNELS[name]
        check(lib.enuf_dpd_time_kernel(self._h, k, int(max_launches)), "enuf_dpd_time_kernel")

    def kernel_time(self):
        """(total milliseconds, launches) of the timed kernel."""
        ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
        check(lib.enuf_dpd_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)), "enuf_dpd_kernel_time")
        return ms.value, n.value

    @property
    def footprint_bytes(self):
        """Device bytes of the integrator and its plan."""
        return int(lib.enuf_dpd_footprint_bytes(self._h))

    def status(self):
        st = ctypes.c_int(0)
        check(lib.enuf_dpd_status(self._h, ctypes.byref(st)), "enuf_dpd_status")
        return st.value

    def close(self):
        if getattr(self, "_h", None):
            lib.enuf_dpd_destroy(self._h)
            self._h = None
        if self.plan is not None:
            self.plan.close()
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
