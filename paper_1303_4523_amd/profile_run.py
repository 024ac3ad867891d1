"""Short fixed workloads for profiler runs (rocprofv3 counter and trace passes).

    python -m paper_1303_4523_amd.profile_run [--small K] [--single K] [--batch K] [--batch-graph K]

--small K:  K FP64 evaluations (Plan.compute) of the L = 10 system (N = 3000,
            300 charges, M = 32, Kc = 8, p = 4);
--single K: K FP64 evaluations (Plan.compute) of the DPD N = 24000 system
            (M = 64, Kc = 16, p = 4, 1650 charges);
--batch K:  K eager single-stream steps of the 64-replica mixed batch
            (1.01M particles, M = 36-80), after one step that builds it;
--batch-graph K: the same, the K steps replayed from the step graphs (each
            step's combine fused with the next step's pre kernel).
Each prints one line when it ends.  Under a counter pass every dispatch is
serialised, so the runs are kept to a few launches of each kernel.
"""
import argparse

import torch

from . import Plan
from . import workloads as wl
from .batch import Batch
from .dpd import DPD


def small(k, dev):
    s = wl.single_eval_small()
    e = s.meta["enuf"]
    p = Plan(s.N, e["L"], e["alpha"], e["p"], e["sigma"], e["M"], e["Kc"], e["r_cut"], e["lam"],
             precision="fp64", device=dev)
    pos = torch.tensor(s.pos, device=dev)
    q = torch.tensor(s.q, device=dev)
    F, E = p.compute(pos, q)
    for _ in range(k):
        p.compute(pos, q, F, E)
    torch.cuda.synchronize()
    p.close()
    print(f"small: {k} evaluations of N={s.N}", flush=True)


def single(k, dev):
    s = wl.dpd_polyelectrolyte_24k()
    e = s.meta["enuf"]
    p = Plan(s.N, e["L"], e["alpha"], e["p"], e["sigma"], e["M"], e["Kc"], e["r_cut"], e["lam"],
             precision="fp64", device=dev)
    pos = torch.tensor(s.pos, device=dev)
    q = torch.tensor(s.q, device=dev)
    for _ in range(k):
        p.compute(pos, q)
    torch.cuda.synchronize()
    p.close()
    print(f"single: {k} evaluations of N={s.N}", flush=True)


def batch(k, dev, graph=False):
    reps = wl.batched_replicas(64)
    mem = []
    for s in reps:
        d = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=s.meta["enuf"], precision="mixed", device=dev)
        d.plan.set_parts(1)
        pos = torch.tensor(s.pos, device=dev)
        vel = torch.tensor(s.vel, device=dev)
        F = torch.empty_like(pos)
        d.forces(pos, vel, F, step=0)
        mem.append((d, pos, vel, F))
    # eager single-stream steps, or (graph) replayed steps whose combine is
    # fused with the next step's pre kernel
    b = Batch("mixed", device=dev, use_graph=graph, concurrent=False)
    for m in mem:
        b.add(*m, first_step=1)
    b.run(1)
    b.run(k)
    torch.cuda.synchronize()
    b.close()
    for m in mem:
        m[0].close()
    print(f"batch: {k} {'replayed' if graph else 'eager'} steps of {len(reps)} replicas", flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--small", type=int, default=0)
    ap.add_argument("--single", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--batch-graph", type=int, default=0)
    a = ap.parse_args()
    dev = torch.device("cuda", 0)
    if a.small:
        small(a.small, dev)
    if a.single:
        single(a.single, dev)
    if a.batch:
        batch(a.batch, dev)
    if a.batch_graph:
        batch(a.batch_graph, dev, graph=True)


if __name__ == "__main__":
    main()
