#!/usr/bin/env python3
"""Benchmark: ENUF-DPD particle-steps/s on one MI355X.

Headline workload (`value`): the DPD trajectory with ENUF electrostatics in
FP64 -- box 20^3 at density 3 (N = 24000), one 50-bead polyelectrolyte chain
with charge fraction 0.5, 25 counterions, 800 + 800 salt ions (1650 charged
beads), a = 25, gamma = 4.5, sigma = 3, dt = 0.03, bonds k = 4 / r0 = 0.7,
velocity-Verlet lambda = 0.65; ENUF alpha = 0.3, r_cut = 3, lambda_e = 0.25,
M = 64, Kc = 16, p = 4, sigma_s = 2, Kaiser-Bessel window.  Synthetic seeded
input.  One step = the whole path: predictor/drift, DPD pair forces + bonds,
the ENUF electrostatics (real space, mesh passes, combine) and the closing
half kick.  The step graphs are captured before the warm-up (reported as
graph_capture_ms); `value` = N * steps / GPU event time of the timed steps,
with all state resident on the GPU and the stream synchronised on both sides.

Also reported in the same JSON line:
  roofline       the dominant kernel of the headline step (event-timed here);
  step_kernels   every kernel class of the headline step, event-timed;
  roofline_mesh  spread and gather (and the other mesh passes) against the HBM
                 roofline from their algorithmic bytes: the headline step, the
                 N-sweep system at L = 40 in the mixed mode, and the 64-replica
                 batch (aggregate over its members);
  single_eval    enuf_compute timed alone: the L = 10 system (1000 evaluations,
                 FP64) and the N sweep L = 10 ... 40 (100 evaluations each,
                 FP64 and mixed);
  cpu_baseline   the FP64 oracle's DPD steps on the host cores (all threads,
                 and one thread), with the CPU model;
  batched        64 uneven replicas stepped together in the mixed mode vs the
                 same systems stepped one at a time by the plain FP64 path
                 (graphs captured before timing on both sides), with each
                 path's measured force error;
  serving        the 2000-request stream (N 3000-200000, charge fraction
                 0.05-1, valency 1-3) with continuous batching: capacity, then
                 Poisson arrivals at 70 % of it with p50 / p99 latency, against
                 the plain FP64 path serving the same stream one request at a
                 time; 1 % of the requests carry an accuracy sample checked
                 against the oracle after the stream.

Prints one JSON line.  --gpus above 1 is not supported: the library and this
benchmark run on one GPU.
"""
import argparse
import json
import math
import os
import platform
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

# kernel classes of a DPD step ("dpd_post": the closing kernel, which in a run
# is step k's combine fused with step k+1's predictor and binning)
STEP_KERNELS = ["dpd_pair", "real", "mesh_fwd", "mesh_x", "mesh_bwd", "dpd_post"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=200,
                    help="at most this many oracle DPD steps timed on the host for cpu_baseline (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="stop the cpu_baseline sample after the step that passes this many seconds")
    ap.add_argument("--serial", action="store_true",
                    help="run each step on one stream (no overlap of pair, real-space and mesh kernels)")
    ap.add_argument("--single-evals", type=int, default=1, help="time enuf_compute (configs 1 and 3); 0 = skip")
    ap.add_argument("--batched-steps", type=int, default=200, help="steps of the 64-replica batch (0 = skip)")
    ap.add_argument("--serving-requests", type=int, default=2000, help="requests of the serving stream (0 = skip)")
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


# ---------------------------------------------------------------------------
# Algorithmic work models (minimum bytes the method must move, per launch)
# ---------------------------------------------------------------------------
def mesh_bytes(M, Kc, nq, s):
    """Algorithmic HBM bytes of the mesh stages of one evaluation with s-byte
    reals (spread: charges in, mesh out; FFT per direction: real mesh in,
    half spectrum out; gather: mesh and charges in, forces out)."""
    half = M * M * (M // 2 + 1) * 2 * s
    return {"spread": nq * 4 * s + M ** 3 * s,
            "fft": M ** 3 * s + half,
            "gather": M ** 3 * s + nq * 4 * s + nq * 24}


def kernel_work(name, systems, s):
    """(bound, amount, unit) of one launch of a step kernel over `systems`
    (list of (N, nq, M, Kc, density)); s is the mesh real size in bytes."""
    if name == "dpd_pair":
        pairs = sum(0.5 * N * rho * 4.0 / 3.0 * math.pi for (N, nq, M, Kc, rho) in systems)
        return "alu", pairs * PAIR_FLOPS, "flop"
    tot = {"spread": 0.0, "fft": 0.0, "gather": 0.0}
    for (N, nq, M, Kc, rho) in systems:
        for k, v in mesh_bytes(M, Kc, nq, s).items():
            tot[k] += v
    # the fused passes: spread + the z/y transforms of each plane; x transforms
    # + influence + inverse x; inverse y/z transforms + gather.  Each is
    # credited with the stage it is named for (the transforms are extra work)
    if name == "mesh_fwd":
        return "hbm", tot["spread"], "byte"
    if name == "mesh_bwd":
        return "hbm", tot["gather"], "byte"
    if name == "mesh_x":
        return "hbm", tot["fft"], "byte"
    return None, float("nan"), ""


def roofline_entry(name, systems, s, avg_s, workload):
    bound, amount, unit = kernel_work(name, systems, s)
    if bound is None:
        return None
    if unit == "flop":
        ach = amount / avg_s / 1e12
        return {"kernel": name, "workload": workload, "bound": bound, "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS, "algorithmic_flops": amount,
                "avg_launch_us": avg_s * 1e6}
    ach = amount / avg_s / 1e9
    return {"kernel": name, "workload": workload, "bound": bound, "achieved": ach, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "algorithmic_bytes": amount, "avg_launch_us": avg_s * 1e6}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the kernel source as it is now (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_dpd24k_fp64.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    mb = re.search(r"traffic_bytes_per_launch\s*=\s*([0-9.eE+]+)", text)
    ms = re.search(r"source_sha256\s*=\s*([0-9a-f]{64})", text)
    mf = re.search(r"source_file\s*=\s*(\S+)", text)
    if not (mb and ms):
        return None
    src = os.path.join(ROOT, "paper_1303_4523_amd", "csrc", mf.group(1) if mf else "enuf_dpd.hip")
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != ms.group(1):
        return None
    return float(mb.group(1))


def progress(msg):
    """One line per finished section on stderr (a long run shows its steps)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _state(s, dev):
    import torch
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    vel = torch.tensor(s.vel, dtype=torch.float64, device=dev)
    return pos, vel, torch.empty_like(pos)


# ---------------------------------------------------------------------------
# Headline: the N = 24000 FP64 DPD step
# ---------------------------------------------------------------------------
def headline(a, dev):
    import torch
    from paper_1303_4523_amd import workloads as wl
    from paper_1303_4523_amd.dpd import DPD

    s = wl.dpd_polyelectrolyte_24k()
    e = s.meta["enuf"]
    prm = dict(s.meta["dpd"], seed=20240613)
    d = DPD(s.L, s.q, prm, bonds=s.bonds, enuf=e, precision="fp64", device=0)
    if a.serial:
        d.set_concurrency(False)
    pos, vel, F = _state(s, dev)
    d.forces(pos, vel, F, step=0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    d.prepare_graphs(pos, vel, F)
    capture_ms = (time.perf_counter() - t) * 1e3
    if a.warmup:
        d.run(pos, vel, F, 1, a.warmup)
    torch.cuda.synchronize()
    st = d.status()
    if st != 0:
        raise RuntimeError(f"device status {st} after warm-up")

    K = a.steps
    e0, e1 = _events()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    d.run(pos, vel, F, 1 + a.warmup, K)
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gpu_s = e0.elapsed_time(e1) * 1e-3
    st = d.status()
    if st != 0:
        raise RuntimeError(f"device status {st} after the timed steps")
    if not bool(torch.isfinite(pos).all()):
        raise RuntimeError("non-finite positions after the timed steps")

    # every kernel class of the step, event-timed on its stream in eager
    # single-stream steps (separate from the timed ones), so that each pair of
    # events brackets the kernel alone and not its wait for CUs held by the
    # kernels of the other chain; the events add the dispatch of each launch
    # (about 2-3 us) to the execution time a kernel trace reports
    first = 1 + a.warmup + K
    nk = max(10, min(K, 200))
    kern = {}
    d.set_concurrency(False)
    for name in STEP_KERNELS:
        d.time_kernel(name, nk)
        d.run(pos, vel, F, first, nk)
        first += nk
        ms, n = d.kernel_time()
        d.time_kernel(None, 1)
        kern[name] = (ms / max(n, 1)) * 1e-3
    d.close()
    nq = s.Nq
    systems = [(s.N, nq, e["M"], e["Kc"], 3.0)]
    dom = max(kern, key=kern.get)
    roof = roofline_entry(dom, systems, 8, kern[dom], "DPD N=24000 FP64 step")
    traffic = measured_traffic(dom)
    roofline = {"bound": roof["bound"], "achieved": roof["achieved"], "peak": roof["peak"], "unit": roof["unit"],
                "frac": roof["frac"], "traffic": traffic, "kernel": dom, "avg_launch_us": roof["avg_launch_us"],
                "launches": nk}
    mesh = [roofline_entry(k, systems, 8, kern[k], "DPD N=24000 FP64 step (M=64, Nq=1650)")
            for k in ("mesh_fwd", "mesh_x", "mesh_bwd")]
    out = {
        "value": s.N * K / gpu_s,
        "ms_per_step": gpu_s / K * 1e3,
        "host_ms_per_step": (t1 - t0) / K * 1e3,
        "graph_capture_ms": capture_ms,
        "roofline": roofline,
        "step_kernels_us": {k: v * 1e6 for k, v in kern.items()},
        "mesh": mesh,
        "config": {"workload": "DPD polyelectrolyte + salt, L=20, N=24000, Nq=1650, ENUF M=64 Kc=16 p=4",
                   "N": s.N, "Nq": nq, "box": s.L, "M": e["M"], "Kc": e["Kc"], "p": e["p"],
                   "precision": "fp64", "window": "kaiser-bessel",
                   "schedule": "serial" if a.serial else "forked stream",
                   "launch": "HIP graphs of 8 and 2 steps captured before the warm-up"},
    }
    return out, (s, prm, e)


# ---------------------------------------------------------------------------
# Single evaluations (enuf_compute): config 1 and the config 3 N sweep
# ---------------------------------------------------------------------------
def _time_compute(plan, tp, tq, n):
    import torch
    F, E = plan.compute(tp, tq)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for _ in range(n):
        plan.compute(tp, tq, F, E)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / n


def single_evals(dev):
    import torch
    from paper_1303_4523_amd import Plan
    from paper_1303_4523_amd import workloads as wl

    def plan_for(s, precision):
        e = s.meta["enuf"]
        return Plan(s.N, e["L"], e["alpha"], e["p"], e["sigma"], e["M"], e["Kc"], e["r_cut"], e["lam"],
                    precision=precision)

    out = {}
    s = wl.single_eval_small()
    tp = torch.tensor(s.pos, device=dev)
    tq = torch.tensor(s.q, device=dev)
    p = plan_for(s, "fp64")
    dt = _time_compute(p, tp, tq, 1000)
    if p.status() != 0:
        raise RuntimeError("device status after the L=10 evaluations")
    p.close()
    out["L10_fp64"] = {"workload": "L=10, N=3000, Nq=300, M=32, Kc=8, p=4, FP64", "evaluations": 1000,
                       "us_per_eval": dt * 1e6, "evaluations_per_s": 1.0 / dt, "particle_evals_per_s": s.N / dt}
    sweep = []
    mesh40 = []
    for L in (10, 15, 20, 30, 40):
        s = wl.n_sweep(L)
        e = s.meta["enuf"]
        tp = torch.tensor(s.pos, device=dev)
        tq = torch.tensor(s.q, device=dev)
        row = {"L": L, "N": s.N, "Nq": s.Nq, "M": e["M"], "Kc": e["Kc"]}
        for prec in ("fp64", "mixed"):
            p = plan_for(s, prec)
            dt = _time_compute(p, tp, tq, 100)
            if L == 40 and prec == "mixed":
                systems = [(s.N, s.Nq, e["M"], e["Kc"], 3.0)]
                for k in ("mesh_fwd", "mesh_x", "mesh_bwd"):
                    p.time_kernel(k, 100)
                    for _ in range(100):
                        p.compute(tp, tq)
                    ms, n = p.kernel_time()
                    p.time_kernel(None, 1)
                    mesh40.append(roofline_entry(k, systems, 4, ms / max(n, 1) * 1e-3,
                                                 f"N sweep L=40 (N={s.N}, Nq={s.Nq}, M={e['M']}) mixed"))
            if p.status() != 0:
                raise RuntimeError(f"device status after the L={L} {prec} evaluations")
            p.close()
            row[f"{prec}_us_per_eval"] = dt * 1e6
            row[f"{prec}_particle_evals_per_s"] = s.N / dt
        sweep.append(row)
    out["n_sweep"] = sweep
    return out, mesh40


# ---------------------------------------------------------------------------
# CPU legs: the oracle on the host cores
# ---------------------------------------------------------------------------
def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(s, prm, e, max_steps, seconds):
    import oracle
    P = dict(prm, alpha=e["alpha"], r_cut=e["r_cut"], lambda_e=e["lam"], Kc=e["Kc"], use_elec=1)
    F, _ = oracle.dpd_forces(s.pos, s.vel, s.q, s.bonds, P, seed=prm["seed"], step=0)

    def steps(limit, secs):
        pos, vel, FF = s.pos.copy(), s.vel.copy(), F.copy()
        t0 = time.perf_counter()
        n = 0
        while n < limit and (n == 0 or time.perf_counter() - t0 < secs):
            n += 1
            pos, vel, FF, _ = oracle.dpd_step(pos, vel, FF, s.q, s.bonds, P, seed=prm["seed"], step=n)
        return n, time.perf_counter() - t0

    cores = oracle.num_threads()
    n, dt = steps(max_steps, seconds)
    oracle.set_threads(1)
    n1, dt1 = steps(max(1, max_steps // 10), seconds / 3)
    oracle.set_threads(cores)
    return {"value": s.N * n / dt, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} DPD steps of the same N=24000 system (O(N^2) pair loops, direct "
                      f"Ewald over all |k|<{e['Kc']}), {dt:.2f} s on {cores} host threads",
            "single_thread_value": s.N * n1 / dt1,
            "single_thread_sample": f"{n1} steps, {dt1:.2f} s on 1 thread",
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def oracle_errors(samples, nbeads=1000):
    """Force and energy errors of GPU accuracy samples against the oracle:
    S(k) over every charge, forces at up to nbeads seeded charged beads."""
    import numpy as np
    import oracle
    errs = []
    for smp in samples:
        e = smp["enuf"]
        q = smp["q"]
        qi = np.nonzero(q)[0]
        sel = np.sort(np.random.default_rng(7).choice(qi, min(nbeads, len(qi)), replace=False))
        ref = oracle.ewald(smp["pos"], q, e["L"], e["alpha"], e["Kc"], e["r_cut"], e["lam"], sel=sel)
        Fs, Fr = smp["F"][sel], ref["F"]
        ef = float(np.linalg.norm(Fs - Fr) / np.linalg.norm(Fr))
        rms = np.sqrt(np.mean(np.sum(Fr ** 2, axis=1)))
        wp = float(np.max(np.linalg.norm(Fs - Fr, axis=1)) / rms)
        E5 = smp["energy5"]
        er = float(abs(E5[2] + E5[3] - ref["E_recip"] - ref["E_self"]) / abs(ref["E_recip"] + ref["E_self"]))
        errs.append({"N": len(q), "Nq": int(len(qi)), "M": e["M"], "precision": smp.get("precision"),
                     "force_rel_rms": ef, "worst_particle": wp, "energy_recip_self_rel": er,
                     "status": int(smp.get("status", 0))})
    return errs


def _summary(errs, key):
    import numpy as np
    v = [x[key] for x in errs]
    return {"median": float(np.median(v)), "max": float(np.max(v)), "n": len(v)} if v else None


# ---------------------------------------------------------------------------
# Batched replicas (config 4)
# ---------------------------------------------------------------------------
def _accuracy_sample(plan, pos, q, precision, enuf):
    F, E5 = plan.compute_components(pos, q)
    return dict(pos=pos.cpu().numpy(), q=q.cpu().numpy(), F=F.cpu().numpy(), energy5=E5.cpu().numpy(),
                enuf=dict(enuf), status=plan.status(), precision=precision)


def batched(nsteps, dev):
    """64 replicas in one batch (mixed) vs one at a time (plain FP64)."""
    import torch
    from paper_1303_4523_amd import Plan
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
    # launch parameters: each stage group's candidates timed on the batch's own
    # steps (the states advance; the timed run below uses the choice)
    tune = b.autotune(steps=3)
    progress(f"batched tuning {tune['params']}")
    torch.cuda.synchronize()
    t = time.perf_counter()
    b.run(1)   # rebuilds the member table and captures the last-step graph (the warm-up run below
               # captures the step graphs with the fused combine + pre kernel)
    torch.cuda.synchronize()
    capture_ms = (time.perf_counter() - t) * 1e3
    b.run(10)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    b.run(nsteps)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3
    # per-stage times (eager single-stream steps) for the aggregate roofline
    systems = [(r.N, r.Nq, r.meta["enuf"]["M"], r.meta["enuf"]["Kc"], 3.0) for r in reps]
    stages, mesh = {}, []
    for k in ("dpd_pre", "dpd_pair", "real", "mesh_fwd", "mesh_x", "mesh_bwd", "combine"):
        b.time_kernel(k, 10)
        b.run(10)
        ms, n = b.kernel_time()
        b.time_kernel(None, 1)
        stages[k] = ms / max(n, 1) * 1e3
        if k.startswith("mesh"):
            mesh.append(roofline_entry(k, systems, 4, ms / max(n, 1) * 1e-3,
                                       f"64-replica batch aggregate (N={N}, sum Nq={sum(x[1] for x in systems)}) mixed"))
    status = max(abs(m[0].status()) for m in mem)
    # accuracy of the mixed members: the largest two by mesh
    big = sorted(range(len(reps)), key=lambda i: -reps[i].meta["enuf"]["M"])[:2]
    samples_mixed = [_accuracy_sample(mem[i][0].plan, mem[i][1], mem[i][0]._q, "mixed", reps[i].meta["enuf"])
                     for i in big]
    b.close()
    # the plain path: each system alone in FP64 (graphs captured first), the
    # same members' final states evaluated in FP64 for its accuracy
    plain_steps = 20
    tot = 0.0
    samples_fp64 = []
    for i, s in enumerate(reps):
        d = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=s.meta["enuf"], precision="fp64", device=dev)
        pos, vel, F = _state(s, dev)
        d.forces(pos, vel, F, step=0)
        d.prepare_graphs(pos, vel, F)
        d.run(pos, vel, F, 1, 2)
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        d.run(pos, vel, F, 3, plain_steps)
        e1.record()
        torch.cuda.synchronize()
        tot += e0.elapsed_time(e1) * 1e-3
        if i in big:
            pm = mem[i]
            samples_fp64.append(_accuracy_sample(d.plan, pm[1], pm[0]._q, "fp64", s.meta["enuf"]))
        d.close()
    for m in mem:
        m[0].close()
    value = N * nsteps / dt
    plain = N * plain_steps / tot
    out = {"workload": "64 replicas, N log-uniform 3000-48000 (sum %d), f 0.1-1, valency 1-3, own M/Kc" % N,
           "precision": "mixed", "steps": nsteps, "ms_per_step": dt / nsteps * 1e3,
           "graph_capture_ms": capture_ms, "particle_steps_per_s": value,
           "plain_fp64_particle_steps_per_s": plain, "speedup_vs_plain_fp64": value / plain,
           "stage_us": stages, "status": status,
           "tuning": {"params": tune["params"], "default_us": tune["default_us"], "tuned_us": tune["tuned_us"],
                      "note": "eager single-stream microseconds per step of each tuned stage group"}}
    return out, mesh, samples_mixed + samples_fp64


# ---------------------------------------------------------------------------
# Serving stream (config 5)
# ---------------------------------------------------------------------------
def serving(nreq, dev):
    """Capacity (all requests at t = 0), then Poisson arrivals at 70 % of it;
    the plain FP64 path serves the same stream one request at a time."""
    import numpy as np
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
    cap_host = dict(srv.host_s)
    srv.close()
    progress(f"serving capacity {cap['requests_per_s']:.1f} requests/s")
    rate = 0.7 * cap["requests_per_s"]
    arr = wl.poisson_arrivals(nreq, rate)
    srv = Server(hbm_budget=budget, device=dev.index, sample_every=100)
    res = srv.serve([Request(rid=i, arrival=float(arr[i]), system=s) for i, s in enumerate(systems)])
    st = latency_stats(res)
    peak = srv.peak_members
    srv.close()
    status = max(abs(r.status) for r in res)
    samples = [r.sample for r in res if r.sample is not None]
    # the plain path: the same stream served one request at a time in FP64
    # (creation, initial forces and 10 steps per request; FIFO queue on the
    # same arrival times)
    service = np.zeros(nreq)
    gpu = 0.0
    ps = 0
    plain_samples = []
    for i, s in enumerate(systems):
        torch.cuda.synchronize()
        a = time.perf_counter()
        d = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=s.meta["enuf"], precision="fp64", device=dev)
        d.set_graphs(False)   # a 10-step request does not amortise a capture
        pos, vel, F = _state(s, dev)
        e0, e1 = _events()
        e0.record()
        d.forces(pos, vel, F, 0)
        d.run(pos, vel, F, 1, 10)
        e1.record()
        torch.cuda.synchronize()
        service[i] = time.perf_counter() - a
        gpu += e0.elapsed_time(e1) * 1e-3
        ps += s.N * 10
        if i % 100 == 0:
            plain_samples.append(_accuracy_sample(d.plan, pos, d._q, "fp64", s.meta["enuf"]))
        if i % 500 == 499:
            progress(f"plain serving {i + 1} requests")
        d.close()
    done = np.zeros(nreq)
    tfree = 0.0
    for i in range(nreq):
        start = max(tfree, arr[i])
        done[i] = start + service[i]
        tfree = done[i]
    lat = done - arr
    return {"workload": f"{nreq} requests x 10 DPD steps, N log-uniform 3000-200000, charge fraction 0.05-1, "
                        "valency 1-3, mixed precision, HBM budget 64 GiB",
            "capacity_requests_per_s": cap["requests_per_s"],
            "capacity_particle_steps_per_s": cap["particle_steps_per_s"],
            "capacity_host_s": cap_host,
            "rate_requests_per_s": rate, "p50_latency_ms": st["p50_s"] * 1e3, "p99_latency_ms": st["p99_s"] * 1e3,
            "mean_latency_ms": st["mean_s"] * 1e3, "throughput_requests_per_s": st["requests_per_s"],
            "throughput_particle_steps_per_s": st["particle_steps_per_s"], "peak_resident_requests": peak,
            "plain_fp64_particle_steps_per_s": ps / service.sum(),
            "plain_fp64_gpu_particle_steps_per_s": ps / gpu,
            "plain_fp64_p50_latency_ms": float(np.percentile(lat, 50)) * 1e3,
            "plain_fp64_p99_latency_ms": float(np.percentile(lat, 99)) * 1e3,
            "status": status}, samples, plain_samples


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration()
        return 0
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} is not supported; the library runs on a single GPU "
              "(independent systems would run one process per GPU)", file=sys.stderr)
        return 2
    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    h, (s, prm, e) = headline(a, dev)
    progress(f"headline {h['ms_per_step'] * 1e3:.1f} us/step")
    out = {
        "metric": "ENUF particle-steps/s at N=24k (DPD with ENUF electrostatics, FP64)",
        "value": h["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": h["ms_per_step"],
        "host_ms_per_step": h["host_ms_per_step"],
        "graph_capture_ms": h["graph_capture_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": h["config"],
        "roofline": h["roofline"],
        "step_kernels_us": h["step_kernels_us"],
    }
    roof_mesh = list(h["mesh"])
    samples = {}
    if a.single_evals:
        se, mesh40 = single_evals(dev)
        out["single_eval"] = se
        progress("single evaluations")
        roof_mesh += mesh40
    if a.batched_steps > 0:
        bt, mesh, smp = batched(a.batched_steps, dev)
        out["batched"] = bt
        progress(f"batched {bt['ms_per_step']:.3f} ms/step")
        roof_mesh += mesh
        samples["batched"] = smp
    if a.serving_requests > 0:
        sv, smp, psmp = serving(a.serving_requests, dev)
        out["serving"] = sv
        progress("serving")
        samples["serving"] = smp
        samples["serving_plain"] = psmp
    out["roofline_mesh"] = roof_mesh
    if a.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(s, prm, e, a.cpu_steps, a.cpu_seconds)
        progress("cpu baseline")
        # accuracy of the GPU paths against the oracle (after all GPU timing)
        if "batched" in samples:
            errs = oracle_errors(samples["batched"])
            out["batched"]["accuracy"] = {
                "mixed_force_rel_rms": _summary([x for x in errs if x["precision"] == "mixed"], "force_rel_rms"),
                "fp64_force_rel_rms": _summary([x for x in errs if x["precision"] == "fp64"], "force_rel_rms"),
                "members": errs}
        if "serving" in samples:
            errs = oracle_errors(samples["serving"])
            perrs = oracle_errors(samples["serving_plain"])
            out["serving"]["accuracy"] = {
                "sample": "every 100th request: oracle S(k) over all charges, forces at <= 1000 charged beads",
                "mixed_force_rel_rms": _summary(errs, "force_rel_rms"),
                "mixed_worst_particle": _summary(errs, "worst_particle"),
                "mixed_energy_rel": _summary(errs, "energy_recip_self_rel"),
                "plain_fp64_force_rel_rms": _summary(perrs, "force_rel_rms"),
                "plain_fp64_worst_particle": _summary(perrs, "worst_particle")}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
