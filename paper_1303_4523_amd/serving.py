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

Creating an admitted system (its plan and integrator, the state upload and
its initial forces) and destroying a finished one take milliseconds of host
time each.  Host threads do that work while the batched steps run: creator
threads build systems on a creation stream (not the server's), and a
closer thread destroys finished ones.  A created system joins the batch, which waits for
its initial forces, at the next step boundary, so the loop itself only joins
prepared systems, launches the steps and reads the finished results.  Memory
is counted from admission until the system is destroyed, so the resident
footprint never exceeds the budget.

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
import queue
import threading
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
    __slots__ = ("req", "dpd", "pos", "vel", "force", "remaining", "admitted", "footprint", "reserved", "mid")


class Server:
    """Serves a stream of requests on one GPU.

    hbm_budget: bytes of device memory the resident systems may hold.
    max_members: cap on concurrently resident systems.
    keep_state: copy each finished system's final (pos, vel, force) to the host.
    creators: host threads that create admitted systems.
    """

    def __init__(self, hbm_budget, max_members=256, precision="mixed", device=0, keep_state=False,
                 sample_every=0, creators=2):
        self.device = torch.device("cuda", device) if isinstance(device, int) else device
        self.budget = int(hbm_budget)
        self.max_members = int(max_members)
        self.precision = precision
        self.keep_state = keep_state
        self.sample_every = int(sample_every)
        self.creators = max(1, int(creators))
        self.stream = torch.cuda.Stream(self.device)   # non-blocking, default priority
        # systems are created (uploads, initial forces) on a stream of their
        # own: a copy on the server's stream would wait for the queued steps
        self.create_stream = torch.cuda.Stream(self.device)
        # membership changes every few steps: launch eagerly rather than
        # capture a graph per membership
        self.batch = Batch(precision, device=self.device, use_graph="auto")
        self.used = 0
        self.peak_used = 0
        self.peak_members = 0
        # wall time per phase: admit (creating systems, on the creator threads),
        # run (launching and waiting for the batched steps), retire (reading
        # results on the loop, destroying systems on the closer thread)
        self.host_s = dict(admit=0.0, run=0.0, retire=0.0)
        self._lock = threading.Lock()

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
        """Read a finished member's results and take it out of the batch (its
        device memory is released later, by _destroy)."""
        e5 = m.dpd.energy().cpu().numpy()
        st = m.dpd.status()
        state = None
        if self.keep_state:
            state = (m.pos.cpu().numpy(), m.vel.cpu().numpy(), m.force.cpu().numpy())
        self.batch.remove(m.mid)
        sample = None
        if self.sample_every > 0 and m.req.rid % self.sample_every == 0:
            sample = self._accuracy_sample(m)
        return Result(rid=m.req.rid, N=m.req.system.N, arrival=m.req.arrival, admitted=m.admitted, finished=now,
                      steps=m.req.steps, status=st, energy5=e5, footprint=m.footprint, state=state,
                      sample=sample)

    @staticmethod
    def _destroy(m):
        """Release a retired member's device memory (waits for the work queued
        on the server's stream)."""
        m.dpd.close()
        m.dpd = m.pos = m.vel = m.force = None

    def _add_time(self, phase, dt):
        with self._lock:
            self.host_s[phase] += dt

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

        Loop: join the systems the creator threads have prepared, launch the
        batched steps up to the next completion (one step while systems are
        being created), admit what has arrived and
        fits (the creator threads build those systems and queue their initial
        forces while the steps run), synchronise, read and retire the finished
        members and hand them to the closer thread."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active = {}
        results = []
        creating = 0   # admitted, not yet joined
        to_create, to_close, made = queue.Queue(), queue.Queue(), queue.Queue()
        freed = queue.Queue()
        t0 = clock()

        def creator():
            with torch.cuda.device(self.device), torch.cuda.stream(self.create_stream):
                while True:
                    job = to_create.get()
                    if job is None:
                        return
                    try:
                        ta = clock()
                        m = self._prepare(job[0], job[1])
                        m.reserved = job[2]
                        self._add_time("admit", clock() - ta)
                        made.put(m)
                    except BaseException as ex:  # handed to the loop, which raises it
                        made.put(ex)
                        return

        def closer():
            with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
                while True:
                    m = to_close.get()
                    if m is None:
                        return
                    try:
                        tc = clock()
                        self._destroy(m)
                        self._add_time("retire", clock() - tc)
                        freed.put(m.reserved)
                    except BaseException as ex:
                        freed.put(ex)
                        return

        def settle_freed():
            while True:
                try:
                    x = freed.get_nowait()
                except queue.Empty:
                    return
                if isinstance(x, BaseException):
                    raise x
                self.used -= x

        def admit():
            nonlocal creating
            settle_freed()
            while pending and pending[0].arrival <= clock() - t0 and \
                    len(active) + creating < self.max_members:
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
                self.used += need   # the estimate is the footprint the system will hold
                self.peak_used = max(self.peak_used, self.used)
                creating += 1
                to_create.put((req, now, need))

        def join(block):
            nonlocal creating
            while creating:
                try:
                    m = made.get(block=block)
                except queue.Empty:
                    return
                block = False
                creating -= 1
                if isinstance(m, BaseException):
                    raise m
                m.mid = self.batch.add(m.dpd, m.pos, m.vel, m.force, first_step=1)
                active[m.mid] = m

        threads = [threading.Thread(target=creator, daemon=True) for _ in range(self.creators)]
        threads.append(threading.Thread(target=closer, daemon=True))
        for th in threads:
            th.start()
        try:
            with torch.cuda.stream(self.stream):
                while pending or active or creating:
                    admit()
                    # with nothing running, wait for a prepared system (or the next arrival)
                    join(block=not active and creating > 0)
                    self.peak_members = max(self.peak_members, len(active))
                    if not active:
                        if pending and not creating:
                            wait = pending[0].arrival - (clock() - t0)
                            if wait > 0:
                                time.sleep(min(wait, 0.01))
                        continue
                    # up to the next completion, or one step while systems are
                    # being created (they join at the next step boundary)
                    k = min(m.remaining for m in active.values())
                    if creating:
                        k = 1
                    tr = clock()
                    self.batch.run(k)
                    for m in active.values():
                        m.remaining -= k
                    self._add_time("run", clock() - tr)
                    admit()   # overlaps with the queued steps
                    tr = clock()
                    self.stream.synchronize()
                    self._add_time("run", clock() - tr)
                    now = clock() - t0
                    tr = clock()
                    for mid in [mid for mid, m in active.items() if m.remaining == 0]:
                        m = active.pop(mid)
                        results.append(self._retire(m, now))
                        to_close.put(m)
                    self._add_time("retire", clock() - tr)
        finally:
            for _ in range(self.creators):
                to_create.put(None)
            to_close.put(None)
            for th in threads:
                th.join()
            while not made.empty():   # prepared but never joined (after an error)
                m = made.get()
                if not isinstance(m, BaseException):
                    self._destroy(m)
                    self.used -= m.reserved
            settle_freed()
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
