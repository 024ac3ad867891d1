"""The paper's structure studies, run on the GPU path.

* ``electrolyte_rdf`` -- set 3 (Sec. 5, Table 3): radial distribution
  functions of neutral beads and ions in a 0.6 M electrolyte.
* ``polyelectrolyte_rg`` -- set 5 (Sec. 6, Table 3): radius of gyration of a
  48-bead chain as its charge fraction f goes from 0 to 1; all fractions
  (and replicas) advance together in one batched engine.

ENUF parameters follow the accuracy rule of eq. 29 at delta = 1e-4 with
r_c = 3 and lambda_e = R_c / 1.125.  Sampling (pair histograms, radii of
gyration) runs in the library's kernels between steps; only the final
normalisation is done on the host.

Usage: python -m paper_1303_4523_amd.studies rdf|rg [--steps K ...]
"""
import argparse
import json
import math
import time

import numpy as np
import torch

from . import workloads as wl
from .batch import Batch
from .dpd import DPD
from .observables import PairHistogram, chain_rg2
from .params import choose

FRACTIONS = (0.0, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 1.0)


def paper_enuf(L):
    return choose(L, delta=1e-4, r_cut=wl.PAPER_R_CUT, sigma=2.0, window="kb", lam=wl.PAPER_LAMBDA_E)


def _state(s, dev):
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    vel = torch.tensor(s.vel, dtype=torch.float64, device=dev)
    return pos, vel, torch.empty_like(pos)


def electrolyte_rdf(steps=200000, equil=10000, every=50, r_max=5.0, nbins=100, precision="fp64", device=0,
                    system=None, progress=None):
    """Set 3: equilibrate, then sample g(r) of the classes neutral (0),
    cation (1), anion (2) every `every` steps.  Returns r, the g's, the mean
    kinetic temperature and the device status."""
    dev = torch.device("cuda", device)
    s = system if system is not None else wl.electrolyte_set3()
    e = paper_enuf(s.L)
    t0 = time.perf_counter()
    with torch.cuda.device(dev):
        d = DPD(s.L, s.q, s.meta["dpd"], enuf=e, precision=precision, device=dev)
        pos, vel, force = _state(s, dev)
        d.forces(pos, vel, force, step=0)
        d.run(pos, vel, force, 1, equil)
        cls = np.where(s.q > 0, 1, np.where(s.q < 0, 2, 0)).astype(np.int32)
        H = PairHistogram(s.N, np.arange(s.N), cls, 3, s.L, r_max, nbins, device=dev)
        nsamp = steps // every
        ke = torch.zeros(nsamp, dtype=torch.float64, device=dev)
        step = 1 + equil
        for k in range(nsamp):
            d.run(pos, vel, force, step, every)
            step += every
            H.sample(pos)
            ke[k] = (vel * vel).sum()
            if progress and (k + 1) % max(1, nsamp // 10) == 0:
                progress(f"rdf: {k + 1}/{nsamp} samples")
        torch.cuda.synchronize(dev)
        st = d.status()
        d.close()
    r, g = H.rdf()
    return dict(r=r, g00=g[0, 0], gpp=g[1, 1], gmm=g[2, 2], gpm=g[1, 2], g0p=g[0, 1], g0m=g[0, 2],
                kT=float(ke.mean().item() / (3.0 * s.N)), status=st, steps=nsamp * every, equil=equil,
                samples=nsamp, seconds=time.perf_counter() - t0, enuf=e, N=s.N, L=s.L)


def polyelectrolyte_rg(fractions=FRACTIONS, L=15.0, replicas=1, steps=50000, equil=10000, every=100,
                       precision="mixed", device=0, progress=None):
    """Set 5 at box L: for every charge fraction (and replica) one system,
    all stepped together in one batch; Rg^2 of the chain sampled every
    `every` steps after `equil` steps.  Returns per fraction the mean Rg,
    its standard error (from replica and block means) and the samples."""
    dev = torch.device("cuda", device)
    t0 = time.perf_counter()
    systems, keys = [], []
    for f in fractions:
        for r in range(replicas):
            systems.append(wl.polyelectrolyte_set5(f, L=L, seed=wl.BASE_SEED + 8 + 100000 * r))
            keys.append((f, r))
    e = paper_enuf(L)
    nsamp = steps // every
    with torch.cuda.device(dev):
        stream = torch.cuda.Stream(dev)
        with torch.cuda.stream(stream):
            batch = Batch(precision, device=dev)
            members = []
            for s in systems:
                d = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=e, precision=precision, device=dev)
                d.plan.set_parts(1)   # the batch fills the device
                d.set_species(s.meta["species"], s.meta["a_table"])
                pos, vel, force = _state(s, dev)
                d.forces(pos, vel, force, step=0)
                batch.add(d, pos, vel, force, first_step=1)
                beads = torch.as_tensor(s.meta["chain"], device=dev)
                members.append((d, pos, vel, beads))
            batch.run(equil)
            rg2 = torch.zeros((nsamp, len(members)), dtype=torch.float64, device=dev)
            for k in range(nsamp):
                batch.run(every)
                for m, (d, pos, vel, beads) in enumerate(members):
                    chain_rg2(pos, beads, L, out=rg2[k, m:m + 1])
                if progress and (k + 1) % max(1, nsamp // 10) == 0:
                    progress(f"rg: {k + 1}/{nsamp} samples")
            stream.synchronize()
            status = [d.status() for (d, _, _, _) in members]
            kT = [float((vel * vel).sum().item()) / (3.0 * s.N) for (_, _, vel, _), s in zip(members, systems)]
            batch.close()
            for (d, _, _, _) in members:
                d.close()
    rg2 = rg2.cpu().numpy()
    out = {}
    for f in fractions:
        cols = [i for i, (ff, _) in enumerate(keys) if ff == f]
        rg = np.sqrt(rg2[:, cols])
        # standard error from 10 blocks of every replica's time series
        nb = 10
        blocks = np.array([b.mean(0) for b in np.array_split(rg, nb)]).reshape(-1)
        out[f] = dict(rg=float(rg.mean()), err=float(blocks.std(ddof=1) / math.sqrt(len(blocks))),
                      rg2=float(rg2[:, cols].mean()))
    return dict(fractions=out, status=status, kT=kT, steps=nsamp * every, equil=equil, samples=nsamp,
                replicas=replicas, L=L, N=systems[0].N, enuf=e, seconds=time.perf_counter() - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["rdf", "rg"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--equil", type=int, default=None)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--L", type=float, default=15.0)
    ap.add_argument("--replicas", type=int, default=1)
    ap.add_argument("--precision", default=None)
    a = ap.parse_args()

    def say(msg):
        print(msg, flush=True)

    kw = {k: v for k, v in dict(steps=a.steps, equil=a.equil, every=a.every).items() if v is not None}
    if a.study == "rdf":
        res = electrolyte_rdf(precision=a.precision or "fp64", progress=say, **kw)
        rows = {k: [round(float(x), 4) for x in res[k]] for k in ("r", "g00", "gpp", "gmm", "gpm")}
        res = {k: v for k, v in res.items() if not isinstance(v, np.ndarray)}
        res.update(rows)
    else:
        res = polyelectrolyte_rg(L=a.L, replicas=a.replicas, precision=a.precision or "mixed", progress=say,
                                 **kw)
        res["fractions"] = {str(k): v for k, v in res["fractions"].items()}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
