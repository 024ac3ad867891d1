#!/usr/bin/env python3
"""Benchmark: ENUF-DPD particle-steps/s on one MI355X.

Headline workload (`value`): the DPD trajectory with ENUF electrostatics in
FP64 -- box 20^3 at density 3 (N = 24000), one 50-bead polyelectrolyte chain
with charge fraction 0.5, 25 counterions, 800 + 800 salt ions (1650 charged
beads), a = 25, gamma = 4.5, sigma = 3, dt = 0.03, bonds k = 4 / r0 = 0.7,
velocity-Verlet lambda = 0.65; ENUF alpha = 0.3, r_cut = 3, lambda_e = 0.25,
M = 64, Kc = 16, p = 4, sigma_s = 2, Kaiser-Bessel window.  Synthetic seeded
input.  One step = the whole path: predictor/drift, DPD pair forces + bonds,
the ENUF electrostatics (real space, three mesh passes, combine) and the
closing half kick.  `value` = N * steps / wall time of the timed steps, with
all state resident on the GPU and the stream synchronised on both sides.

Also reported in the same JSON line:
  roofline      the dominant kernel of the headline step, event-timed here;
  cpu_baseline  the FP64 oracle's DPD steps on the host cores;
  batched       64 uneven replicas stepped together in the mixed mode (one
                launch per stage, graph replay) vs the same systems stepped
                one at a time by the plain FP64 path;
  serving       a stream of 10-step requests (N 3000-200000, charge fraction
                0.05-1, valency 1-3) with continuous batching: capacity, then
                Poisson arrivals at 70 % of it with p50 / p99 latency.

Prints one JSON line (rank 0).  --gpus above 1 is not supported: this build
runs on one GPU.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector

# Flops of one pair evaluation of the pair kernel, counted once per unordered
# pair within R_c: minimum image (3 x 4), r^2 (5), r and 1/r (2), unit
# vector (3), weight (1), relative velocity projection (6), force magnitude
# (9), force components (3), theta from the Philox word (3); the Philox
# rounds are integer work and are not counted.
PAIR_FLOPS = 44.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=200,
                    help="at most this many oracle DPD steps timed on the host for cpu_baseline (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="stop the cpu_baseline sample after the step that passes this many seconds")
    ap.add_argument("--time-kernel", default="dpd_pair",
                    help="kernel whose launches are event-timed for the roofline entry")
    ap.add_argument("--serial", action="store_true",
                    help="run each step on one stream (no overlap of pair, real-space and mesh kernels)")
    ap.add_argument("--batched-steps", type=int, default=200, help="steps of the 64-replica batch (0 = skip)")
    ap.add_argument("--serving-requests", type=int, default=150, help="requests of the serving stream (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 512 MiB device-to-device five times (scale of the HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE
    counters: 512 MiB read and 512 MiB written per launch."""
    import torch
    torch.cuda.set_device(0)
    n = 64 << 20
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": n * 8, "copy_bytes_written_per_launch": n * 8}), flush=True)


def kernel_model(name, s, e):
    """Algorithmic work of one launch of the timed kernel: (bound, amount, unit)."""
    M, Kc, p = e["M"], e["Kc"], e["p"]
    nq = int((s.q != 0).sum())
    fft_line = 5.0 * M * math.log2(M)
    if name == "dpd_pair":
        pairs = 0.5 * s.N * 3.0 * 4.0 / 3.0 * math.pi   # density 3, R_c = 1
        return "alu", pairs * PAIR_FLOPS, "flop"
    if name in ("mesh_fwd", "mesh_bwd"):
        spread = nq * (2 * p) ** 3 * (2.0 if name == "mesh_fwd" else 6.0)
        ffts = M * (M / 2 + Kc) * fft_line      # per plane: M/2 packed z lines + Kc y lines
        return "alu", spread + ffts, "flop"
    if name == "mesh_x":
        return "alu", (2 * Kc - 1) * Kc * 2 * fft_line, "flop"
    return "alu", float("nan"), "flop"


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    it was taken on the kernel source as it is now (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_dpd24k_fp64.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    mb = re.search(r"traffic_bytes_per_launch\s*=\s*([0-9.eE+]+)", text)
    ms = re.search(r"source_sha256\s*=\s*([0-9a-f]{64})", text)
    if not (mb and ms):
        return None
    src = os.path.join(ROOT, "paper_1303_4523_amd", "csrc", "enuf_dpd.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != ms.group(1):
        return None
    return float(mb.group(1))


def cpu_baseline(s, prm, e, max_steps, seconds):
    import oracle
    P = dict(prm, alpha=e["alpha"], r_cut=e["r_cut"], lambda_e=e["lam"], Kc=e["Kc"], use_elec=1)
    F, _ = oracle.dpd_forces(s.pos, s.vel, s.q, s.bonds, P, seed=prm["seed"], step=0)
    pos, vel = s.pos.copy(), s.vel.copy()
    t0 = time.perf_counter()
    nsteps = 0
    while nsteps < max_steps and (nsteps == 0 or time.perf_counter() - t0 < seconds):
        nsteps += 1
        pos, vel, F, _ = oracle.dpd_step(pos, vel, F, s.q, s.bonds, P, seed=prm["seed"], step=nsteps)
    dt = time.perf_counter() - t0
    return {"value": s.N * nsteps / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{nsteps} DPD steps of the same N=24000 system (O(N^2) pair loops, direct "
                      f"Ewald over all |k|<{e['Kc']}), {dt:.2f} s on the host"}


def _state(s, dev):
    import torch
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    vel = torch.tensor(s.vel, dtype=torch.float64, device=dev)
    return pos, vel, torch.empty_like(pos)


def batched(nsteps, dev):
    """64 replicas in one batch (mixed) vs one at a time (plain FP64)."""
    import torch
    from paper_1303_4523_amd import workloads as wl
    from paper_1303_4523_amd.batch import Batch
    from paper_1303_4523_amd.dpd import DPD
    reps = wl.batched_replicas(64)
    N = sum(r.N for r in reps)
    mem = []
    for s in reps:
        d = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=s.meta["enuf"], precision="mixed", device=dev)
        d.plan.set_parts(1)   # the batch fills the device
        pos, vel, F = _state(s, dev)
        d.forces(pos, vel, F, step=0)
        mem.append((d, pos, vel, F))
    b = Batch("mixed", device=dev)
    for m in mem:
        b.add(*m, first_step=1)
    b.run(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(nsteps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    status = max(abs(m[0].status()) for m in mem)
    b.close()
    for m in mem:
        m[0].close()
    # the plain path: each system alone in FP64, a bounded number of steps
    plain_steps = 20
    tot = 0.0
    for s in reps:
        d = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=s.meta["enuf"], precision="fp64", device=dev)
        pos, vel, F = _state(s, dev)
        d.forces(pos, vel, F, step=0)
        torch.cuda.synchronize()
        a = time.perf_counter()
        d.run(pos, vel, F, 1, plain_steps)
        torch.cuda.synchronize()
        tot += time.perf_counter() - a
        d.close()
    value = N * nsteps / dt
    plain = N * plain_steps / tot
    return {"workload": "64 replicas, N log-uniform 3000-48000 (sum %d), f 0.1-1, valency 1-3, own M/Kc" % N,
            "precision": "mixed", "steps": nsteps, "ms_per_step": dt / nsteps * 1e3,
            "particle_steps_per_s": value, "plain_fp64_particle_steps_per_s": plain,
            "speedup_vs_plain_fp64": value / plain, "status": status}


def serving(nreq, dev):
    """Capacity (all requests at t = 0), then Poisson arrivals at 70 % of it."""
    import torch
    from paper_1303_4523_amd import workloads as wl
    from paper_1303_4523_amd.dpd import DPD
    from paper_1303_4523_amd.serving import Request, Server, latency_stats
    systems = [wl.serving_request(r) for r in range(nreq)]
    budget = 64 << 30
    srv = Server(hbm_budget=budget, device=dev.index)
    srv.serve([Request(rid=i, arrival=0.0, system=systems[i]) for i in range(min(4, nreq))])   # warm-up
    srv.close()
    srv = Server(hbm_budget=budget, device=dev.index)
    cap = latency_stats(srv.serve([Request(rid=i, arrival=0.0, system=s) for i, s in enumerate(systems)]))
    srv.close()
    rate = 0.7 * cap["requests_per_s"]
    arr = wl.poisson_arrivals(nreq, rate)
    srv = Server(hbm_budget=budget, device=dev.index)
    res = srv.serve([Request(rid=i, arrival=float(arr[i]), system=s) for i, s in enumerate(systems)])
    st = latency_stats(res)
    peak = srv.peak_members
    srv.close()
    status = max(abs(r.status) for r in res)
    # the plain path: one request at a time, FP64 (creation excluded)
    tot, ps = 0.0, 0
    for s in systems[:min(nreq, 40)]:
        d = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=s.meta["enuf"], precision="fp64", device=dev)
        pos, vel, F = _state(s, dev)
        torch.cuda.synchronize()
        a = time.perf_counter()
        d.forces(pos, vel, F, 0)
        d.run(pos, vel, F, 1, 10)
        torch.cuda.synchronize()
        tot += time.perf_counter() - a
        ps += s.N * 10
        d.close()
    return {"workload": f"{nreq} requests x 10 DPD steps, N log-uniform 3000-200000, charge fraction 0.05-1, "
                        "valency 1-3, mixed precision, HBM budget 64 GiB",
            "capacity_requests_per_s": cap["requests_per_s"],
            "capacity_particle_steps_per_s": cap["particle_steps_per_s"],
            "rate_requests_per_s": rate, "p50_latency_ms": st["p50_s"] * 1e3, "p99_latency_ms": st["p99_s"] * 1e3,
            "mean_latency_ms": st["mean_s"] * 1e3, "throughput_requests_per_s": st["requests_per_s"],
            "throughput_particle_steps_per_s": st["particle_steps_per_s"], "peak_resident_requests": peak,
            "plain_fp64_particle_steps_per_s": ps / tot, "status": status}


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration()
        return 0
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} is not supported; this build runs on a single GPU "
              "(independent systems would run one process per GPU)", file=sys.stderr)
        return 2
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
    pos, vel, F = _state(s, dev)
    d.forces(pos, vel, F, step=0)
    if a.warmup:
        d.run(pos, vel, F, 1, a.warmup)
    torch.cuda.synchronize()
    st = d.status()
    if st != 0:
        raise RuntimeError(f"device status {st} after warm-up")

    K = a.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.run(pos, vel, F, 1 + a.warmup, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = d.status()
    if st != 0:
        raise RuntimeError(f"device status {st} after the timed steps")
    if not bool(torch.isfinite(pos).all()):
        raise RuntimeError("non-finite positions after the timed steps")
    elapsed = t1 - t0
    value = s.N * K / elapsed

    # event timing of the roofline kernel on separate steps (the events sit on
    # the stream that kernel is launched on)
    d.time_kernel(a.time_kernel, K)
    d.run(pos, vel, F, 1 + a.warmup + K, K)
    kms, kn = d.kernel_time()
    d.time_kernel(None, 1)
    bound, amount, unit = kernel_model(a.time_kernel, s, e)
    avg_s = (kms / max(kn, 1)) * 1e-3
    achieved = amount / avg_s / 1e12
    traffic = measured_traffic(a.time_kernel)
    roofline = {"bound": bound, "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic, "kernel": a.time_kernel,
                "avg_launch_us": avg_s * 1e6, "launches": kn}
    d.close()

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
                   "schedule": "serial" if a.serial else "forked stream"},
        "roofline": roofline,
    }
    if a.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(s, prm, e, a.cpu_steps, a.cpu_seconds)
    if a.batched_steps > 0:
        out["batched"] = batched(a.batched_steps, dev)
    if a.serving_requests > 0:
        out["serving"] = serving(a.serving_requests, dev)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
