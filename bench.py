#!/usr/bin/env python3
"""Benchmark: ENUF-DPD particle-steps/s on one MI355X.

Workload: the DPD trajectory with ENUF electrostatics in FP64 -- box 20^3 at
density 3 (N = 24000), one 50-bead polyelectrolyte chain with charge fraction
0.5, 25 counterions, 800 + 800 salt ions (1650 charged beads), a = 25,
gamma = 4.5, sigma = 3, dt = 0.03, bonds k = 4 / r0 = 0.7, velocity-Verlet
lambda = 0.65; ENUF alpha = 0.3, r_cut = 3, lambda_e = 0.25, M = 64, Kc = 16,
p = 4, sigma_s = 2, Kaiser-Bessel window.  Synthetic seeded input.

One step = the whole path: predictor/drift, DPD pair forces + bonds, the ENUF
electrostatics (compaction, real space, three mesh passes, combine) and the
closing half kick.  `value` = N * steps / wall time of the timed steps, with
all state resident on the GPU and the stream synchronised on both sides.

Prints one JSON line (rank 0).  --gpus above 1 is not supported: this build
runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=10,
                    help="oracle DPD steps timed on the host for cpu_baseline (0 = skip)")
    ap.add_argument("--time-kernel", default="mesh_bwd",
                    help="kernel whose launches are event-timed for the roofline entry")
    ap.add_argument("--serial", action="store_true",
                    help="run each step on one stream (no overlap of pair, real-space and mesh kernels)")
    return ap.parse_args()


def kernel_model(name, s, e):
    """Algorithmic work of one launch of the timed kernel: (bound, amount, unit).

    mesh_fwd / mesh_bwd are ALU/LDS bound (the mesh never leaves LDS); their
    algorithmic flops count the window stencil (2p)^3 per charge (1 multiply-add
    each, 2 flops) and the FFT butterflies 5 n log2 n per complex line of the
    z and y transforms of every plane.  dpd_pair counts 2 x (pairs within R_c)
    x 60 flops (distance, weights and the three forces); the Philox rounds are
    integer work and are not counted.
    """
    M, Kc, p = e["M"], e["Kc"], e["p"]
    nq = int((s.q != 0).sum())
    fft_line = 5.0 * M * math.log2(M)
    if name in ("mesh_fwd", "mesh_bwd"):
        spread = nq * (2 * p) ** 3 * (2.0 if name == "mesh_fwd" else 6.0)
        ffts = M * (M / 2 + Kc) * fft_line      # per plane: M/2 packed z lines + Kc y lines
        return "alu", spread + ffts, "flop"
    if name == "mesh_x":
        return "alu", (2 * Kc - 1) * Kc * 2 * fft_line, "flop"
    if name == "dpd_pair":
        pairs = 0.5 * s.N * 3.0 * 4.0 / 3.0 * math.pi   # density 3, R_c = 1
        return "alu", 2 * pairs * 60.0, "flop"
    return "alu", float("nan"), "flop"


def cpu_baseline(s, prm, e, nsteps):
    import numpy as np
    import oracle
    P = dict(prm, alpha=e["alpha"], r_cut=e["r_cut"], lambda_e=e["lam"], Kc=e["Kc"], use_elec=1)
    F, _ = oracle.dpd_forces(s.pos, s.vel, s.q, s.bonds, P, seed=prm["seed"], step=0)
    pos, vel = s.pos.copy(), s.vel.copy()
    t0 = time.perf_counter()
    for k in range(1, nsteps + 1):
        pos, vel, F, _ = oracle.dpd_step(pos, vel, F, s.q, s.bonds, P, seed=prm["seed"], step=k)
    dt = time.perf_counter() - t0
    return {"value": s.N * nsteps / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{nsteps} DPD steps of the same N=24000 system (O(N^2) pair loops, direct "
                      f"Ewald over all |k|<{e['Kc']}), {dt:.2f} s on the host"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} is not supported; this build runs on a single GPU "
              "(independent systems shard trivially, see DESIGN.md)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_1303_4523_amd import workloads as wl
    from paper_1303_4523_amd.dpd import DPD

    s = wl.dpd_polyelectrolyte_24k()
    e = s.meta["enuf"]
    prm = dict(s.meta["dpd"], seed=20240613)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    d = DPD(s.L, s.q, prm, bonds=s.bonds, enuf=e, precision="fp64", device=0)
    if a.serial:
        d.set_concurrency(False)
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    vel = torch.tensor(s.vel, dtype=torch.float64, device=dev)
    F = torch.empty_like(pos)
    d.forces(pos, vel, F, step=0)
    if a.warmup:
        d.run(pos, vel, F, 1, a.warmup)
    torch.cuda.synchronize()
    st = d.status()
    if st != 0:
        raise RuntimeError(f"device status {st} after warm-up")

    K = a.steps
    d.time_kernel(a.time_kernel, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.run(pos, vel, F, 1 + a.warmup, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, kn = d.kernel_time()
    d.time_kernel(None, 1)
    st = d.status()
    if st != 0:
        raise RuntimeError(f"device status {st} after the timed steps")
    if not bool(torch.isfinite(pos).all()):
        raise RuntimeError("non-finite positions after the timed steps")
    elapsed = t1 - t0
    value = s.N * K / elapsed

    bound, amount, unit = kernel_model(a.time_kernel, s, e)
    avg_s = (kms / max(kn, 1)) * 1e-3
    achieved = amount / avg_s / 1e12 if unit == "flop" else amount / avg_s / 1e9
    peak = PEAK_FP64_TFLOPS if unit == "flop" else PEAK_HBM_GBS
    roofline = {"bound": bound, "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s" if unit == "flop" else "GB/s", "frac": achieved / peak,
                "traffic": None, "kernel": a.time_kernel, "avg_launch_us": avg_s * 1e6,
                "launches": kn}

    out = {
        "metric": "ENUF particle-steps/s at N=24k (DPD with ENUF electrostatics, FP64)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": a.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "DPD polyelectrolyte + salt, L=20, N=24000, Nq=1650, ENUF M=64 Kc=16 p=4",
                   "N": s.N, "Nq": s.Nq, "box": s.L, "M": e["M"], "Kc": e["Kc"], "p": e["p"],
                   "precision": "fp64", "window": "kaiser-bessel",
                   "schedule": "serial" if a.serial else "forked streams"},
        "roofline": roofline,
    }
    if a.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(s, prm, e, a.cpu_steps)
    d.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
