"""Batched DPD steps of many independent systems (enuf_batch_* C ABI).

Each member is a DPD integrator (with its own ENUF plan) plus its device
state tensors; one run advances all members with one kernel launch per stage
of the step, replayed from a captured HIP graph.
"""
import ctypes
import hashlib
import json
import math
import os

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

    # launch parameters of enuf_batch_set_tuning, with their defaults
    TUNING_DEFAULTS = dict(pass_threads=256, x_threads=128, stage=256, pair_steps=4, x_split_mul=1, pair_seg=26)
    # candidates per stage group: (stages timed, {parameter: values})
    TUNING_SPACE = (
        (("mesh_fwd", "mesh_bwd"), dict(pass_threads=(256, 512), stage=(128, 256, 512))),
        (("mesh_x",), dict(x_threads=(128, 256), x_split_mul=(1, 2, 4))),
        (("dpd_pair",), dict(pair_steps=(4, 8), pair_seg=(10, 20, 26))),
    )

    def set_tuning(self, **params):
        """Launch parameters of the batched step (names as TUNING_DEFAULTS);
        results do not depend on them."""
        bad = set(params) - set(self.TUNING_DEFAULTS)
        if bad:
            raise ValueError(f"unknown tuning parameters {sorted(bad)}")
        p = [int(params.get(k, 0)) for k in self.TUNING_DEFAULTS]
        check(lib.enuf_batch_set_tuning(self._h, *p), "enuf_batch_set_tuning")
        self._tuning = dict(getattr(self, "_tuning", self.TUNING_DEFAULTS), **params)

    def signature(self):
        """Key of the batch's composition for the tuning cache: precision and
        the sorted (M, Kc, p, log2 bucket of N_q, log2 bucket of N) of the
        members."""
        rows = []
        for d, *_ in self._members.values():
            e = d.enuf
            rows.append((int(e["M"]), int(e["Kc"]), int(e["p"]), int(math.log2(max(d.nq, 1))),
                         int(math.log2(max(d.N, 1)))))
        text = json.dumps([self.precision, sorted(rows)])
        return hashlib.sha1(text.encode()).hexdigest()[:16]

    def _stage_us(self, names, steps):
        t = 0.0
        for k in names:
            self.time_kernel(k, steps)
            self.run(steps)
            ms, n = self.kernel_time()
            self.time_kernel(None, 1)
            t += ms / max(n, 1) * 1e3
        return t

    def autotune(self, steps=3, cache=None):
        """Choose the launch parameters by timing each candidate on this
        batch's own steps (eager, one stage group at a time, keeping the
        fastest; the members advance by the steps taken, so tune a batch of
        the same systems built for the purpose, or accept the advance).  With
        `cache` (a JSON file path) a stored choice for the same signature is
        applied without timing, and a new choice is stored.  Returns
        dict(params, default_us, tuned_us, signature, cached) with the timed
        stage groups' microseconds per step under the defaults and the
        choice."""
        key = self.signature()
        store = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                store = json.load(f)
        if key in store:
            self.set_tuning(**store[key]["params"])
            return dict(store[key], signature=key, cached=True)
        best = dict(self.TUNING_DEFAULTS)
        self.set_tuning(**best)
        self.run(1)   # rebuild and warm the kernels
        default_us = {"+".join(n): self._stage_us(n, steps) for n, _ in self.TUNING_SPACE}
        tuned_us = {}
        for names, space in self.TUNING_SPACE:
            tag = "+".join(names)
            choice, t_best = None, None
            keys = list(space)
            combos = [()]
            for k in keys:
                combos = [c + (v,) for c in combos for v in space[k]]
            for combo in combos:
                trial = dict(best, **dict(zip(keys, combo)))
                self.set_tuning(**trial)
                self.run(1)
                t = self._stage_us(names, steps)
                if t_best is None or t < t_best:
                    choice, t_best = dict(zip(keys, combo)), t
            best.update(choice)
            tuned_us[tag] = t_best
        self.set_tuning(**best)
        out = dict(params=best, default_us=default_us, tuned_us=tuned_us)
        if cache:
            store[key] = out
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(store, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(out, signature=key, cached=False)

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
