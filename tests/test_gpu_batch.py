"""Batched DPD steps (one launch per stage for many systems) against the
single-system path and the oracle."""
import numpy as np
import pytest

import oracle
from paper_1303_4523_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV).contiguous()


def _replicas(ids, n_max=9000):
    return [wl.replica(s, n_max=n_max) for s in ids]


def _member(s, precision="mixed", first_step=1, parts=None):
    """Integrator, state tensors and initial forces of one replica; parts:
    work-groups per mesh plane (None: the plan's default; 1: as the serving
    loop sets)."""
    from paper_1303_4523_amd.dpd import DPD
    d = DPD(s.L, s.q, s.meta["dpd"], bonds=s.bonds, enuf=s.meta["enuf"], precision=precision, device=0)
    if parts is not None:
        d.plan.set_parts(parts)
    pos, vel = _t(s.pos), _t(s.vel)
    F = torch.empty_like(pos)
    d.forces(pos, vel, F, step=first_step - 1)
    return d, pos, vel, F


def _alone(s, nsteps, precision="mixed", first_step=1, parts=None):
    d, pos, vel, F = _member(s, precision, first_step, parts)
    d.run(pos, vel, F, first_step, nsteps)
    st = d.status()
    e5 = d.energy().cpu().numpy()
    out = (pos.cpu().numpy(), vel.cpu().numpy(), F.cpu().numpy(), e5)
    d.close()
    assert st == 0
    return out


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("use_graph,concurrent", [(True, True), (False, True), (True, False), ("auto", True)])
def test_batch_equals_each_system_alone(use_graph, concurrent):
    """Six uneven replicas (valency 1-3, charge fraction 0.1-1, different M
    and Kc) stepped together: every member's state is bitwise the one it gets
    when stepped alone."""
    from paper_1303_4523_amd.batch import Batch
    reps = _replicas([0, 1, 2, 3, 5, 10])
    print("case: batch of", [r.meta["name"] for r in reps], f"graph={use_graph} concurrent={concurrent}",
          flush=True)
    b = Batch("mixed", device=0, use_graph=use_graph, concurrent=concurrent)
    members = []
    for s in reps:
        d, pos, vel, F = _member(s)
        b.add(d, pos, vel, F, first_step=1)
        members.append((d, pos, vel, F))
    assert len(b) == len(reps)
    b.run(4)
    torch.cuda.synchronize()
    for s, (d, pos, vel, F) in zip(reps, members):
        got = (pos.cpu().numpy(), vel.cpu().numpy(), F.cpu().numpy(), d.energy().cpu().numpy())
        assert d.status() == 0
        ref = _alone(s, 4)
        assert _same(got, ref), s.meta["name"]
    b.close()
    for d, *_ in members:
        d.close()


def test_chunked_pair_segments_equal_alone():
    """A member with 22-25 DPD cells per side: in the batch its whole columns
    (one segment each) stage more particles than the batched pair kernel's
    stage holds, so every segment is taken in chunks, with velocities read
    from their cell slots; alone it runs 10-cell segments with staged
    velocities and no chunks.  After three replayed steps the states and
    energies are bitwise equal."""
    from paper_1303_4523_amd.batch import Batch
    big = wl.replica(2, n_min=36000, n_max=48000)
    small = wl.replica(5, n_max=6000)
    reps = [big, small]
    print("case: chunked segments", [r.meta["name"] for r in reps], flush=True)
    b = Batch("mixed", device=0, use_graph=True, concurrent=False)
    mem = [_member(r) for r in reps]
    for m in mem:
        b.add(*m, first_step=1)
    b.run(3)
    torch.cuda.synchronize()
    for r, (d, pos, vel, F) in zip(reps, mem):
        assert d.status() == 0
        got = (pos.cpu().numpy(), vel.cpu().numpy(), F.cpu().numpy(), d.energy().cpu().numpy())
        assert _same(got, _alone(r, 3)), r.meta["name"]
    b.close()
    for m in mem:
        m[0].close()


@pytest.mark.parametrize("L,density", [(2.5, 3.0), (6.0, 12.0), (4.0, 40.0)])
def test_batched_pair_regimes_equal_alone(L, density):
    """The batched pair kernel's other routes: a grid of 2 cells per side,
    dense cells whose segments are taken in chunks, and cells so dense that a
    z-cell's neighbourhood exceeds the stage (candidates and velocities from
    global memory).  Three replayed batched steps give bitwise the state the
    system gets stepped alone (whose kernel stages its velocities and takes
    10-cell segments)."""
    from paper_1303_4523_amd.batch import Batch
    from paper_1303_4523_amd.dpd import DPD
    rs = np.random.default_rng(11)
    n = int(round(density * L ** 3))
    pos0 = rs.uniform(0.0, L, (n, 3))
    vel0 = rs.normal(size=(n, 3))
    vel0 -= vel0.mean(0)
    q = np.zeros(n)
    nq = min(40, 2 * (n // 4))
    q[:nq // 2] = 1.0
    q[nq // 2:nq] = -1.0
    prm = dict(a=25.0, gamma=4.5, sigma=3.0, dt=0.01, lam=0.65, k_bond=4.0, r0_bond=0.7, kappa=1.1, seed=17)
    M = wl.mesh_size(max(3.2 * L, 16.0))  # the plan needs 2p <= M/2
    enuf = wl.enuf_params(L, M=M, Kc=max(1, min(int(0.8 * L), M // 4)), r_cut=min(3.0, 0.45 * L))
    print(f"case: batched pair regime L={L} density={density} N={n} M={M}", flush=True)

    def member():
        d = DPD(L, q, prm, enuf=enuf, precision="mixed", device=0)
        pos, vel = _t(pos0), _t(vel0)
        F = torch.empty_like(pos)
        d.forces(pos, vel, F, step=0)
        return d, pos, vel, F

    d, pos, vel, F = member()
    d.run(pos, vel, F, 1, 3)
    torch.cuda.synchronize()
    ref = (pos.cpu().numpy(), vel.cpu().numpy(), F.cpu().numpy(), d.energy().cpu().numpy())
    assert d.status() == 0
    d.close()
    b = Batch("mixed", device=0, use_graph=True, concurrent=False)
    d, pos, vel, F = member()
    b.add(d, pos, vel, F, first_step=1)
    b.run(3)
    torch.cuda.synchronize()
    got = (pos.cpu().numpy(), vel.cpu().numpy(), F.cpu().numpy(), d.energy().cpu().numpy())
    assert d.status() == 0
    b.close()
    d.close()
    assert _same(got, ref)


def test_replayed_runs_of_any_length_equal_eager():
    """Replayed runs fuse each step's combine with the next step's pre kernel
    and alternate the two bin-count sets, the last step of a run using the
    set of its parity.  Runs of 1, 2, 3, 1 and 5 steps (both parities of the
    last step, runs starting after either) give bitwise the states and
    energies of the same runs launched eagerly, after every run."""
    from paper_1303_4523_amd.batch import Batch
    reps = _replicas([1, 4, 7])
    lengths = (1, 2, 3, 1, 5)
    print("case: run lengths", lengths, [r.meta["name"] for r in reps], flush=True)
    got = {}
    for use_graph in (True, False):
        b = Batch("mixed", device=0, use_graph=use_graph, concurrent=False)
        mem = [_member(s) for s in reps]
        for m in mem:
            b.add(*m, first_step=1)
        got[use_graph] = []
        for n in lengths:
            b.run(n)
            torch.cuda.synchronize()
            assert all(m[0].status() == 0 for m in mem)
            got[use_graph].append([tuple(t.cpu().numpy() for t in m[1:]) + (m[0].energy().cpu().numpy(),)
                                   for m in mem])
        b.close()
        for m in mem:
            m[0].close()
    for k, n in enumerate(lengths):
        for a, c in zip(got[True][k], got[False][k]):
            assert _same(a, c), f"after run {k} ({n} steps)"


def _dense_member_system():
    """A densely charged DPD system: one fully charged chain, its counterions
    and 1:1 salt at 1.2 cations per unit volume (about 2.5 charges per unit
    volume, some 280 real-space pairs per charge within r_cut = 3)."""
    import math
    L = 10.5
    seed = wl.BASE_SEED + 77
    s = wl.polyelectrolyte(L, 3.0, 50, 1.0, 1.2, 1, seed)
    M = wl.mesh_size(3.2 * L)
    s.meta["enuf"] = wl.enuf_params(L, M=M, Kc=min(int(math.floor(0.8 * L)), M // 4))
    s.meta["dpd"] = dict(wl.DPD_DEFAULTS, L=L, seed=seed)
    s.meta["name"] = f"dense salt L={L} N={s.N}"
    return s


def test_dense_member_equals_alone():
    """With a densely charged member the real-space kernels flush their pair
    queues within a charge's scan (the batched kernel tests four candidates
    per lane and pass, the single-system one two): every member of the batch
    is still bitwise the state it gets alone."""
    from paper_1303_4523_amd.batch import Batch
    reps = [_dense_member_system()] + _replicas([3])
    print("case: dense batch", [r.meta["name"] for r in reps], flush=True)
    b = Batch("mixed", device=0)
    members = []
    for s in reps:
        d, pos, vel, F = _member(s)
        b.add(d, pos, vel, F, first_step=1)
        members.append((d, pos, vel, F))
    b.run(3)
    torch.cuda.synchronize()
    for s, (d, pos, vel, F) in zip(reps, members):
        got = (pos.cpu().numpy(), vel.cpu().numpy(), F.cpu().numpy(), d.energy().cpu().numpy())
        assert d.status() == 0
        assert _same(got, _alone(s, 3)), s.meta["name"]
    b.close()
    for d, *_ in members:
        d.close()


def test_graph_replays_match_eager_steps():
    """Each replay of the captured step, with host reads and synchronisation
    between replays, equals the eager launch sequence."""
    from paper_1303_4523_amd.batch import Batch
    reps = _replicas([4, 7, 9])
    runs = {}
    for use_graph in (True, False):
        b = Batch("mixed", device=0, use_graph=use_graph)
        mem = [_member(s) for s in reps]
        for d, pos, vel, F in mem:
            b.add(d, pos, vel, F, first_step=1)
        snaps = []
        for step in range(5):
            b.run(1)
            torch.cuda.synchronize()
            snaps.append([p.cpu().numpy() for _, p, _, _ in mem] + [F.cpu().numpy() for *_, F in mem])
            _ = torch.zeros(1000, device=DEV).sum().item()   # unrelated eager work between replays
        runs[use_graph] = snaps
        b.close()
        for d, *_ in mem:
            d.close()
    for a, c in zip(runs[True], runs[False]):
        assert all(np.array_equal(x, y) for x, y in zip(a, c))


def test_membership_changes_between_runs():
    """Members join with their own step index and leave; the others continue
    as if alone."""
    from paper_1303_4523_amd.batch import Batch
    r0, r1, r2 = _replicas([0, 6, 8])
    b = Batch("mixed", device=0)
    m0 = _member(r0)
    m1 = _member(r1)
    i0 = b.add(*m0, first_step=1)
    i1 = b.add(*m1, first_step=1)
    b.run(2)
    m2 = _member(r2, first_step=5)
    b.add(*m2, first_step=5)
    b.run(1)
    b.remove(i0)
    b.run(2)
    torch.cuda.synchronize()
    got0 = tuple(t.cpu().numpy() for t in m0[1:])
    got1 = tuple(t.cpu().numpy() for t in m1[1:])
    got2 = tuple(t.cpu().numpy() for t in m2[1:])
    assert _same(got0, _alone(r0, 3)[:3])
    assert _same(got1, _alone(r1, 5)[:3])
    assert _same(got2, _alone(r2, 3, first_step=5)[:3])
    b.close()
    for m in (m0, m1, m2):
        m[0].close()
    assert i1 != i0


def test_auto_graph_policy_matches_eager():
    """use_graph="auto": a long run captures and replays the step graph, a
    shorter run of the same membership replays it again, and after a member
    leaves a short run launches eagerly; the states equal those of an eager
    batch taken through the same runs."""
    from paper_1303_4523_amd import _lib
    from paper_1303_4523_amd.batch import Batch
    reps = _replicas([4, 7, 9])
    print("case: auto graph policy", [r.meta["name"] for r in reps], flush=True)
    out = {}
    for mode in ("auto", False):
        b = Batch("mixed", device=0, use_graph=mode)
        mem = [_member(s) for s in reps]
        ids = [b.add(*m, first_step=1) for m in mem]
        b.run(_lib.GRAPH_AUTO_STEPS)
        b.run(3)
        b.remove(ids[0])
        b.run(2)
        torch.cuda.synchronize()
        out[mode] = [tuple(t.cpu().numpy() for t in m[1:]) for m in mem]
        b.close()
        for m in mem:
            m[0].close()
    for a, c in zip(out["auto"], out[False]):
        assert _same(a, c)


_TUNED = [dict(pass_threads=512, x_threads=256, stage=128, pair_steps=8, x_split_mul=4, pair_seg=3),
          dict(pass_threads=256, x_threads=512, stage=32, pair_steps=4, x_split_mul=8, pair_seg=1)]


@pytest.mark.parametrize("tuning", _TUNED, ids=["mid", "extremes"])
def test_tuning_does_not_change_results(tuning):
    """Launch parameters other than the defaults (512-thread mesh passes,
    256-thread x pass, stage 128, 8 pair steps, 4x x-split, 3-cell pair
    segments; or the extremes: stage 32, 8x x-split, 1-cell pair segments)
    give bitwise the states and energies of the defaults."""
    from paper_1303_4523_amd.batch import Batch
    reps = _replicas([0, 3, 5, 10])
    print("case: tuning", tuning, [r.meta["name"] for r in reps], flush=True)
    out = {}
    for tuned in (False, True):
        b = Batch("mixed", device=0)
        if tuned:
            b.set_tuning(**tuning)
        mem = [_member(s) for s in reps]
        for m in mem:
            b.add(*m, first_step=1)
        b.run(3)
        torch.cuda.synchronize()
        out[tuned] = [tuple(t.cpu().numpy() for t in m[1:]) + (m[0].energy().cpu().numpy(),) for m in mem]
        b.close()
        for m in mem:
            m[0].close()
    for a, c in zip(out[False], out[True]):
        assert _same(a, c)


def test_autotune_caches_its_choice(tmp_path):
    """autotune times the candidates once, stores the choice under the
    batch's signature, and a batch of the same systems reuses it."""
    from paper_1303_4523_amd.batch import Batch
    reps = _replicas([4, 7])
    cache = str(tmp_path / "tune.json")
    got = []
    for _ in range(2):
        b = Batch("mixed", device=0)
        mem = [_member(s) for s in reps]
        for m in mem:
            b.add(*m, first_step=1)
        got.append(b.autotune(steps=1, cache=cache))
        b.run(1)
        torch.cuda.synchronize()
        assert all(m[0].status() == 0 for m in mem)
        b.close()
        for m in mem:
            m[0].close()
    assert not got[0]["cached"] and got[1]["cached"]
    assert got[0]["params"] == got[1]["params"] and got[0]["signature"] == got[1]["signature"]
    with pytest.raises(Exception):
        Batch("mixed", device=0).set_tuning(pass_threads=128)
    with pytest.raises(Exception):
        Batch("mixed", device=0).set_tuning(pair_seg=27)


def test_mixed_member_against_oracle():
    """A replica with z = 3 salt in the mixed mode: forces at step 0 and the
    state after three steps against the FP64 oracle (mixed bar 5e-4)."""
    s = wl.replica(8, n_max=6000)
    e, dp = s.meta["enuf"], s.meta["dpd"]
    print("case:", s.meta["name"], flush=True)
    d, pos, vel, F = _member(s, "mixed", first_step=1)
    F0 = F.cpu().numpy()
    from paper_1303_4523_amd.batch import Batch
    b = Batch("mixed", device=0)
    b.add(d, pos, vel, F, first_step=1)
    b.run(3)
    torch.cuda.synchronize()
    gp, gF = pos.cpu().numpy(), F.cpu().numpy()
    assert d.status() == 0
    b.close()
    d.close()
    P = dict(dp, alpha=e["alpha"], r_cut=e["r_cut"], lambda_e=e["lam"], Kc=e["Kc"], use_elec=1)
    Fo, _ = oracle.dpd_forces(s.pos, s.vel, s.q, s.bonds, P, seed=dp["seed"], step=0)
    err0 = np.linalg.norm(F0 - Fo) / np.linalg.norm(Fo)
    op, ov = s.pos.copy(), s.vel.copy()
    for k in range(1, 4):
        op, ov, Fo, _ = oracle.dpd_step(op, ov, Fo, s.q, s.bonds, P, seed=dp["seed"], step=k)
    ddp = gp - op
    ddp -= s.L * np.round(ddp / s.L)
    err3 = np.linalg.norm(gF - Fo) / np.linalg.norm(Fo)
    print(f"mixed member: step-0 force rel {err0:.3e}, after 3 steps force rel {err3:.3e}, "
          f"max |dr| {np.abs(ddp).max():.3e}")
    assert err0 < 5e-4 and err3 < 5e-4
    assert np.abs(ddp).max() < 1e-5


def _requests(ids, n_max=12000, steps=10, rate=None):
    from paper_1303_4523_amd.serving import Request
    t = wl.poisson_arrivals(len(ids), rate) if rate else np.zeros(len(ids))
    return [Request(rid=r, arrival=float(a), system=wl.serving_request(r, n_max=n_max), steps=steps)
            for r, a in zip(ids, t)]


def test_serving_results_equal_alone_and_in_the_mix():
    """Requests of different N, charge fraction and valency arriving over time
    are served with continuous batching; each result is bitwise the one the
    request gets when its system is stepped alone."""
    from paper_1303_4523_amd.serving import Server, latency_stats
    reqs = _requests(range(8), rate=400.0)
    print("case: serving", [r.system.meta["name"] for r in reqs], flush=True)
    srv = Server(hbm_budget=8 << 30, precision="mixed", device=0, keep_state=True)
    res = srv.serve(reqs)
    srv.close()
    assert len(res) == len(reqs) and all(r.status == 0 for r in res)
    st = latency_stats(res)
    print(f"serving: {st}, peak members {srv.peak_members}")
    for r in res:
        s = reqs[r.rid].system
        alone = _alone(s, 10, parts=1)
        assert _same(r.state, alone[:3]), s.meta["name"]
        assert np.array_equal(r.energy5, alone[3])


def test_serving_admission_respects_the_budget():
    """With a budget that holds only a few systems, admission waits for memory
    (first come, first served) and the resident footprint never exceeds it;
    the estimate equals the footprint the created system holds."""
    from paper_1303_4523_amd.serving import Server, footprint_estimate
    reqs = _requests(range(6), n_max=9000, steps=4)
    est = [footprint_estimate(r.system) for r in reqs]
    budget = int(2.5 * max(est))
    srv = Server(hbm_budget=budget, precision="mixed", device=0)
    res = srv.serve(reqs)
    srv.close()
    print(f"case: budget {budget} B, peak used {srv.peak_used} B, peak members {srv.peak_members}", flush=True)
    assert all(r.status == 0 for r in res) and len(res) == len(reqs)
    assert srv.peak_used <= budget
    assert srv.peak_members < len(reqs)
    by_id = {r.rid: r for r in res}
    assert all(by_id[i].footprint == est[i] for i in range(len(reqs)))
    # a request larger than the whole budget is rejected, not queued forever
    srv2 = Server(hbm_budget=min(est) // 2, precision="mixed", device=0)
    res2 = srv2.serve(reqs[:1])
    srv2.close()
    assert res2[0].status == -1 and res2[0].steps == 0


def test_serving_reports_a_failed_creation():
    """A request whose system cannot be created (its charges are not neutral,
    which the footprint estimate does not check) makes serve raise the
    library's error from the creator thread; the server's threads end and the
    server can be closed."""
    import threading

    from paper_1303_4523_amd._lib import EnufError
    from paper_1303_4523_amd.serving import Server
    reqs = _requests(range(3), n_max=6000, steps=2)
    bad = reqs[1].system
    bad.q = np.array(bad.q, dtype=np.float64)
    bad.q[np.flatnonzero(bad.q)[0]] += 1.0
    print("case: serving with a non-neutral request", [r.system.meta["name"] for r in reqs], flush=True)
    before = threading.active_count()
    srv = Server(hbm_budget=8 << 30, precision="mixed", device=0)
    with pytest.raises(EnufError):
        srv.serve(reqs)
    srv.close()
    assert threading.active_count() == before
