"""Continuous-batching service for DPD trajectory-segment requests.

A request carries one system (positions, velocities, charges, bonds and its
ENUF / DPD parameters) and a number of DPD steps.  The server keeps every
admitted system resident on the device (its plan, mesh scratch and particle
state) as a member of one batched engine (``enuf_batch_*``): one launch per
stage of the step advances all members together.  Requests that arrive while
others run are admitted at the next step boundary, first come first served,
as long as the HBM footprint of the new system (estimated without allocating)
fits in the budget next to the resident ones; finished members leave at step
boundaries and free their memory.  Members use one work-group per mesh plane
(the batch fills the device), and a member's trajectory is bitwise the one
it gets alone with that setting (each member keeps its own step counter and
random stream).

Reported per request: arrival, admission and completion times (latency =
completion - arrival), the final ENUF energy components and the device
status.  With ``sample_every = k`` every k-th request (by id) also carries an
accuracy sample: after its completion time is taken, its plan evaluates the
electrostatic forces and energies of the final state (same precision and
settings as in the batch) and the host keeps them with the final positions
and charges, for a caller to compare with an independent reference.
Host-side scheduling only: every step of every system runs in the library's
HIP kernels.
"""
import collections
import dataclasses
import time

import numpy as np
import torch

from . import _lib
from ._lib import lib
from .batch import Batch
from .dpd import DPD


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float        # seconds after the start of the stream
    system: object        # workloads.System with meta["enuf"] and meta["dpd"]
    steps: int = 10


@dataclasses.dataclass
class Result:
    rid: int
    N: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    status: int
    energy5: np.ndarray
    footprint: int
    state: tuple = None   # (pos, vel, force) as NumPy arrays when kept
    sample: dict = None   # accuracy sample: pos, q, F (electrostatic), energy5, enuf parameters

    @property
    def latency(self):
        return self.finished - self.arrival


def footprint_estimate(system):
    """Device bytes the request's plan and integrator will hold."""
    e = system.meta["enuf"]
    nb = 0 if system.bonds is None else len(system.bonds)
    a = lib.enuf_plan_footprint_estimate(system.N, float(system.L), int(e["p"]), int(e["M"]), int(e["Kc"]),
                                         float(e["r_cut"]))
    b = lib.enuf_dpd_footprint_estimate(system.N, float(system.L), nb)
    if a == 0 or b == 0:
        raise ValueError(f"invalid system sizes for request: N={system.N} L={system.L} {e}")
    return int(a + b)


class _Member:
    __slots__ = ("req", "dpd", "pos", "vel", "force", "remaining", "admitted", "footprint", "mid")


class Server:
    """Serves a stream of requests on one GPU.

    hbm_budget: bytes of device memory the resident systems may hold.
    max_members: cap on concurrently resident systems.
    keep_state: copy each finished system's final (pos, vel, force) to the host.
    """

    def __init__(self, hbm_budget, max_members=256, precision="mixed", device=0, keep_state=False,
                 sample_every=0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else device
        self.budget = int(hbm_budget)
        self.max_members = int(max_members)
        self.precision = precision
        self.keep_state = keep_state
        self.sample_every = int(sample_every)
        self.stream = torch.cuda.Stream(self.device)   # non-blocking, default priority
        # membership changes every few steps: launch eagerly rather than
        # capture a graph per membership
        self.batch = Batch(precision, device=self.device, use_graph="auto")
        self.used = 0
        self.peak_used = 0
        self.peak_members = 0
        self.host_s = dict(admit=0.0, run=0.0, retire=0.0)   # wall time spent per phase

    def _prepare(self, req, now):
        """Create the system on the device and queue its initial forces (runs
        while the batch is busy; joins the batch at the next step boundary)."""
        s = req.system
        m = _Member()
        m.req = req
        m.dpd = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=s.meta["enuf"], precision=self.precision,
                    device=self.device)
        m.dpd.plan.set_parts(1)   # the batch fills the device
        m.pos = torch.tensor(s.pos, dtype=torch.float64, device=self.device)
        m.vel = torch.tensor(s.vel, dtype=torch.float64, device=self.device)
        m.force = torch.empty_like(m.pos)
        m.dpd.forces(m.pos, m.vel, m.force, step=0)
        m.remaining = req.steps
        m.admitted = now
        m.footprint = m.dpd.footprint_bytes
        m.mid = None
        return m

    def _retire(self, m, now):
        e5 = m.dpd.energy().cpu().numpy()
        st = m.dpd.status()
        state = None
        if self.keep_state:
            state = (m.pos.cpu().numpy(), m.vel.cpu().numpy(), m.force.cpu().numpy())
        self.batch.remove(m.mid)
        sample = None
        if self.sample_every > 0 and m.req.rid % self.sample_every == 0:
            sample = self._accuracy_sample(m)
        m.dpd.close()
        return Result(rid=m.req.rid, N=m.req.system.N, arrival=m.req.arrival, admitted=m.admitted, finished=now,
                      steps=m.req.steps, status=st, energy5=e5, footprint=m.footprint, state=state,
                      sample=sample)

    def _accuracy_sample(self, m):
        """Electrostatic forces and energies of the member's final state from
        its own plan (the completion time is already taken)."""
        F, E5 = m.dpd.plan.compute_components(m.pos, m.dpd._q)
        s = m.req.system
        return dict(pos=m.pos.cpu().numpy(), q=np.asarray(s.q, dtype=np.float64), F=F.cpu().numpy(),
                    energy5=E5.cpu().numpy(), enuf=dict(s.meta["enuf"]), status=m.dpd.plan.status(),
                    precision=self.precision)

    def serve(self, requests, clock=time.perf_counter):
        """Serve the requests (arrival times relative to the call); returns the
        results in completion order.  Requests larger than the whole budget
        are rejected (status EINVAL, no latency).

        Loop: admit what has arrived and fits (creating the systems on the
        device and queueing their initial forces), enqueue the batched steps up
        to the next completion, admit again while the GPU works, then
        synchronise, retire the finished members and let the prepared ones
        join the batch."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active = {}
        ready = []   # prepared, not yet members
        results = []
        t0 = clock()

        def admit():
            while pending and pending[0].arrival <= clock() - t0 and \
                    len(active) + len(ready) < self.max_members:
                req = pending[0]
                need = footprint_estimate(req.system)
                now = clock() - t0
                if need > self.budget:
                    pending.popleft()
                    results.append(Result(rid=req.rid, N=req.system.N, arrival=req.arrival, admitted=now,
                                          finished=now, steps=0, status=_lib.EINVAL, energy5=None,
                                          footprint=need))
                    continue
                if self.used + need > self.budget:
                    break   # first come, first served: wait for memory
                pending.popleft()
                ta = clock()
                m = self._prepare(req, now)
                self.host_s["admit"] += clock() - ta
                ready.append(m)
                self.used += m.footprint
                self.peak_used = max(self.peak_used, self.used)

        with torch.cuda.stream(self.stream):
            while pending or active or ready:
                admit()
                if ready:
                    for m in ready:
                        m.mid = self.batch.add(m.dpd, m.pos, m.vel, m.force, first_step=1)
                        active[m.mid] = m
                    ready.clear()
                self.peak_members = max(self.peak_members, len(active))
                if not active:
                    if pending:
                        wait = pending[0].arrival - (clock() - t0)
                        if wait > 0:
                            time.sleep(min(wait, 0.01))
                    continue
                k = min(m.remaining for m in active.values())
                tr = clock()
                self.batch.run(k)
                for m in active.values():
                    m.remaining -= k
                self.host_s["run"] += clock() - tr
                admit()   # overlaps with the queued steps
                tr = clock()
                self.stream.synchronize()
                self.host_s["run"] += clock() - tr
                now = clock() - t0
                tr = clock()
                for mid in [mid for mid, m in active.items() if m.remaining == 0]:
                    m = active.pop(mid)
                    results.append(self._retire(m, now))
                    self.used -= m.footprint
                self.host_s["retire"] += clock() - tr
        return results

    def close(self):
        if self.batch is not None:
            self.batch.close()
            self.batch = None


def latency_stats(results):
    """p50 / p99 / mean latency (s) and throughput of the served requests."""
    done = [r for r in results if r.steps > 0]
    lat = np.array([r.latency for r in done])
    span = max(r.finished for r in done) - min(r.arrival for r in done)
    psteps = sum(r.N * r.steps for r in done)
    return dict(requests=len(done), rejected=len(results) - len(done),
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), span_s=float(span),
                requests_per_s=len(done) / span, particle_steps_per_s=psteps / span)
