"""GPU parity of enuf_compute against the FP64 CPU oracle (direct Ewald).

Bars: relative force RMS <= 1e-5 and relative energy
<= 1e-6 for the FP64 path; <= 5e-4 and <= 1e-4 for the mixed path.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1303_4523_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": (1e-5, 1e-6), "mixed": (5e-4, 1e-4)}


def _plan(N, e, precision="fp64", window="kb"):
    from paper_1303_4523_amd import Plan
    return Plan(N, e["L"], e["alpha"], e["p"], e["sigma"], e["M"], e["Kc"], e["r_cut"], e["lam"],
                precision=precision, window=window)


def _run(plan, pos, q, components=True):
    dev = torch.device("cuda", 0)
    tp = torch.tensor(pos, dtype=torch.float64, device=dev).contiguous()
    tq = torch.tensor(q, dtype=torch.float64, device=dev).contiguous()
    if components:
        F, E = plan.compute_components(tp, tq)
    else:
        F, E = plan.compute(tp, tq)
    torch.cuda.synchronize()
    return F.cpu().numpy(), E.cpu().numpy(), plan.status()


# Per-particle bar beside the RMS one: no single force may be off by more than
# this fraction of the RMS force (one wrong particle among many would pass an
# RMS bar).
PER_PARTICLE = {"fp64": 1e-3, "mixed": 5e-2}


def _errors(F, E5, ref):
    ef = np.linalg.norm(F - ref["F"]) / np.linalg.norm(ref["F"])
    Et = E5[0] + E5[2] + E5[3]
    ee = abs(Et - ref["E"]) / abs(ref["E"])
    return ef, ee, Et


def _worst_particle(F, Fref):
    """max_i |F_i - Fref_i| / RMS_i |Fref_i| (over the rows given)."""
    rms = np.sqrt(np.mean(np.sum(Fref ** 2, axis=1)))
    return float(np.max(np.linalg.norm(F - Fref, axis=1)) / rms)


def _case(sys_, precision="fp64", window="kb", **over):
    e = dict(sys_.meta["enuf"], **over)
    print(f"case: {sys_.meta.get('name')} precision={precision} window={window} {e}", flush=True)
    plan = _plan(sys_.N, e, precision, window)
    F, E5, st = _run(plan, sys_.pos, sys_.q)
    ref = oracle.ewald(sys_.pos, sys_.q, e["L"], e["alpha"], e["Kc"], e["r_cut"], e["lam"])
    plan.close()
    return F, E5, st, ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_eval_small_parity(precision):
    """L = 10, N = 3000, 300 charges, M = 32, Kc = 8, p = 4 (Kaiser-Bessel)."""
    s = wl.single_eval_small()
    F, E5, st, ref = _case(s, precision)
    assert st == 0
    ef, ee, Et = _errors(F, E5, ref)
    wp = _worst_particle(F, ref["F"])
    print(f"force rel rms {ef:.3e}  energy rel {ee:.3e}  worst particle {wp:.3e}  E={Et:.10f} ref={ref['E']:.10f}")
    tf, te = TOL[precision]
    assert ef <= tf and ee <= te
    assert wp <= PER_PARTICLE[precision]
    # components: the real-space and self terms are exact sums
    assert abs(E5[0] - ref["E_real"]) < 1e-9 * abs(ref["E_real"]) + 1e-9
    assert abs(E5[1] - ref["E_slater"]) < 1e-9 * abs(ref["E_slater"]) + 1e-9
    assert abs(E5[3] - ref["E_self"]) < 1e-12 * abs(ref["E_self"])
    # Parseval: the gathered potential reproduces the k-space energy
    assert abs(E5[4] - E5[2]) < (1e-9 if precision == "fp64" else 1e-4) * abs(E5[2])
    # neutral particles get exactly zero force
    assert np.all(F[s.q == 0.0] == 0.0)


def test_real_space_forces_exact():
    """The real-space forces are exact sums (fixed-point rounding 2^-36 only)."""
    s = wl.single_eval_small()
    e = s.meta["enuf"]
    # a Kc = 1 plan has no wave vectors: the output is real space only
    from paper_1303_4523_amd import Plan
    p0 = Plan(s.N, e["L"], e["alpha"], e["p"], e["sigma"], e["M"], 1, e["r_cut"], e["lam"])
    F, E5, st = _run(p0, s.pos, s.q)
    p0.close()
    Fr, Ee, Es = oracle.real_space(s.pos, s.q, e["L"], e["alpha"], e["r_cut"], e["lam"])
    assert st == 0
    assert E5[2] == 0.0
    assert np.abs(F - Fr).max() < 1e-9
    assert abs(E5[0] - Ee) < 1e-8


def test_real_space_pairs_at_the_cutoff():
    """Pairs 1e-9 inside and outside r_cut, at coordinates near 100 in a box
    of 120 (where FP32 positions are off by up to 4e-6) and across the
    periodic boundary: the FP32 pre-test of the scan keeps every pair the
    exact FP64 test takes, so the forces and energy are the oracle's exact
    real-space sums, the pair outside contributing nothing."""
    from paper_1303_4523_amd import Plan
    L, rc = 120.0, 3.0
    pos = np.array([[100.123456789, 60.5, 60.5], [100.123456789 + rc * (1 - 1e-9), 60.5, 60.5],
                    [10.5, 100.0987654321, 20.25], [10.5, 100.0987654321 + rc * (1 + 1e-9), 20.25],
                    [50.25, 30.5, 0.0004], [50.25, 30.5, L - rc + 0.0004 + 3e-9]])
    q = np.array([1.0, -1.0, 2.0, -2.0, 1.0, -1.0])
    print("case: two pairs inside r_cut (one across the boundary), one just outside", flush=True)
    p0 = Plan(len(q), L, 0.3, 4, 2.0, 32, 1, rc, 0.25)   # Kc = 1: real space only
    F, E5, st = _run(p0, pos, q)
    p0.close()
    Fr, Ee, Es = oracle.real_space(pos, q, L, 0.3, rc, 0.25)
    _, Eb, _ = oracle.real_space(pos[2:4], q[2:4], L, 0.3, rc, 0.25)
    assert st == 0
    assert Eb == 0.0 and Ee != 0.0
    assert np.abs(F[2:4]).max() == 0.0
    assert np.abs(F - Fr).max() < 1e-9
    assert abs(E5[0] - Ee) < 1e-8


@pytest.mark.parametrize("M,Kc,p,N,L", [(24, 6, 3, 257, 6.0), (30, 7, 3, 500, 7.5), (40, 10, 4, 1000, 8.0),
                                         (48, 12, 5, 1100, 12.0)])
def test_mixed_radix_meshes(M, Kc, p, N, L):
    """Meshes with radix 2, 3, 4 and 5 passes, ragged particle counts."""
    s = wl.electrolyte(L, N, N // 10, N // 10, 4242 + M)
    e = dict(alpha=0.35, p=p, sigma=2.0, M=M, Kc=Kc, r_cut=min(3.0, L / 2), lam=0.25, L=L)
    s.meta["enuf"] = e
    s.meta["name"] = f"mesh M={M}"
    F, E5, st, ref = _case(s)
    ef, ee, _ = _errors(F, E5, ref)
    print(f"M={M} p={p}: force {ef:.3e} energy {ee:.3e}")
    assert st == 0
    # p = 3 windows are less accurate; the bar scales with the NFFT error
    tf = 1e-5 if p >= 4 else 1e-4
    assert ef <= tf and ee <= 1e-6


def test_gaussian_window_p6():
    s = wl.single_eval_small()
    F, E5, st, ref = _case(s, "fp64", "gauss", p=6)
    ef, ee, _ = _errors(F, E5, ref)
    print(f"gauss p=6: force {ef:.3e} energy {ee:.3e}")
    assert st == 0 and ef <= 1e-5 and ee <= 1e-6


def test_deterministic_bitwise():
    s = wl.single_eval_small()
    plan = _plan(s.N, s.meta["enuf"])
    a = _run(plan, s.pos, s.q)
    b = _run(plan, s.pos, s.q)
    plan.close()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_overlapped_and_serial_evaluations_are_identical(precision):
    """The real-space term beside the mesh passes (two streams) gives bitwise
    the forces and energies of one stream, also for back-to-back evaluations
    of different inputs enqueued without a synchronisation between them."""
    dev = torch.device("cuda", 0)
    systems = [wl.single_eval_small(), wl.n_sweep(15)]
    print("case: overlapped vs serial", precision, [s.N for s in systems], flush=True)
    out = {}
    for conc in (True, False):
        res = []
        for s in systems:
            plan = _plan(s.N, s.meta["enuf"], precision)
            plan.set_concurrency(conc)
            tp = torch.tensor(s.pos, device=dev)
            tq = torch.tensor(s.q, device=dev)
            shifted = tp + 0.37
            runs = [plan.compute_components(x, tq) for x in (tp, shifted, tp)]
            torch.cuda.synchronize()
            res.append([(F.cpu().numpy(), E.cpu().numpy()) for F, E in runs] + [plan.status()])
            plan.close()
        out[conc] = res
    for a, b in zip(out[True], out[False]):
        assert a[-1] == 0 and b[-1] == 0
        for (Fa, Ea), (Fb, Eb) in zip(a[:-1], b[:-1]):
            assert np.array_equal(Fa, Fb) and np.array_equal(Ea, Eb)
        assert np.array_equal(a[0][0], a[2][0])          # same input, same result
        assert not np.array_equal(a[0][0], a[1][0])      # the shifted input was evaluated


def test_evaluation_captured_in_a_graph_matches_eager():
    """A graph captured around Plan.compute (the plan then keeps the whole
    evaluation on the capturing stream) replays the eager result bitwise,
    with eager evaluations of other inputs between the replays."""
    dev = torch.device("cuda", 0)
    s = wl.single_eval_small()
    print("case: graph capture of Plan.compute", s.N, flush=True)
    plan = _plan(s.N, s.meta["enuf"])
    tp = torch.tensor(s.pos, device=dev)
    tq = torch.tensor(s.q, device=dev)
    F, E = plan.compute(tp, tq)
    torch.cuda.synchronize()
    Fe, Ee = F.clone(), E.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.compute(tp, tq, F, E)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.compute(tp, tq, F, E)
    other = tp + 0.5
    for _ in range(3):
        F.zero_()
        E.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(F, Fe) and torch.equal(E, Ee)
        Fo, _ = plan.compute(other, tq)
        torch.cuda.synchronize()
        assert not torch.equal(Fo, Fe)
    assert plan.status() == 0
    del g
    plan.close()


def test_edge_cases():
    e = dict(L=10.0, alpha=0.3, p=4, sigma=2.0, M=32, Kc=8, r_cut=3.0, lam=0.25)
    rs = np.random.default_rng(0)
    # no charges at all
    pos = rs.uniform(0, 10, (50, 3))
    plan = _plan(50, e)
    F, E5, st = _run(plan, pos, np.zeros(50))
    assert st == 0 and np.all(F == 0.0) and np.all(E5 == 0.0)
    # one neutral particle
    plan1 = _plan(1, e)
    F, E5, st = _run(plan1, pos[:1], np.zeros(1))
    assert st == 0 and np.all(F == 0.0)
    plan1.close()
    # coincident Slater pair: E = -1/lambda, no force
    pos2 = np.array([[3.0, 3.0, 3.0], [3.0, 3.0, 3.0]] + [[1.0, 1.0, 1.0]] * 48)
    q2 = np.zeros(50)
    q2[0], q2[1] = 1.0, -1.0
    F, E5, st = _run(plan, pos2, q2)
    ref = oracle.ewald(pos2, q2, 10.0, 0.3, 8, 3.0, 0.25)
    assert st == 0
    assert abs(E5[0] + E5[2] + E5[3] - ref["E"]) < 1e-6 * abs(ref["E"])
    assert np.abs(F).max() < 1e-9
    # non-neutral input is flagged
    q3 = np.zeros(50)
    q3[:3] = 1.0
    _, _, st = _run(plan, pos, q3)
    assert st == -4
    # non-finite input is flagged and the call still completes
    pos4 = pos.copy()
    pos4[7, 1] = np.nan
    q4 = np.zeros(50)
    q4[7], q4[8] = 1.0, -1.0
    _, _, st = _run(plan, pos4, q4)
    assert st == -5
    # positions far outside the box are wrapped
    q5 = np.zeros(50)
    q5[:10] = 1.0
    q5[10:20] = -1.0
    a = _run(plan, pos, q5)
    b = _run(plan, pos + 10.0 * rs.integers(-5, 6, (50, 3)), q5)
    assert np.abs(a[0] - b[0]).max() < 1e-9
    plan.close()
    # coincident point charges are an error
    e0 = dict(e, lam=0.0)
    plan0 = _plan(50, e0)
    _, _, st = _run(plan0, pos2, q2)
    plan0.close()
    assert st == -7


def test_force_is_gradient_of_gpu_energy():
    """The window-gradient force is the exact derivative of the NFFT energy."""
    s = wl.electrolyte(8.0, 400, 40, 40, 99)
    e = dict(L=8.0, alpha=0.4, p=4, sigma=2.0, M=32, Kc=8, r_cut=3.0, lam=0.25)
    plan = _plan(s.N, e)
    F0, _, _ = _run(plan, s.pos, s.q)
    h = 1e-4
    qi = np.nonzero(s.q)[0]
    for i in qi[:4]:
        for a in range(3):
            pp = s.pos.copy(); pp[i, a] += h
            pm = s.pos.copy(); pm[i, a] -= h
            _, Ep, _ = _run(plan, pp, s.q)
            _, Em, _ = _run(plan, pm, s.q)
            fd = -((Ep[0] + Ep[2]) - (Em[0] + Em[2])) / (2 * h)
            assert abs(fd - F0[i, a]) < 1e-5 * (1 + abs(fd))
    plan.close()


# LDS budgets (bytes) that force 2 and 4 row chunks at M = 32 (FP64) and 2 (mixed),
# with the charge stage shrunk to what fits beside the rows
CHUNK_CAPS = {"fp64": (13000, 11000), "mixed": (11000, 9400)}


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_row_chunked_planes_match(monkeypatch, precision, which):
    """A lowered LDS budget makes the plane passes work in chunks of mesh rows
    (two partial slots per charge) and stage the plane's charges in smaller
    batches; the result equals the one-chunk plane to rounding and still
    meets the oracle bar."""
    cap = CHUNK_CAPS[precision][which]
    s = wl.single_eval_small()
    e = s.meta["enuf"]
    whole = _plan(s.N, e, precision)
    Fw, Ew, stw = _run(whole, s.pos, s.q)
    fp_whole = whole.footprint_bytes
    whole.close()
    monkeypatch.setenv("ENUF_MAX_LDS_BYTES", str(cap))
    print(f"case: chunked planes, precision={precision}, LDS cap {cap}", flush=True)
    chunked = _plan(s.N, e, precision)
    Fc, Ec, stc = _run(chunked, s.pos, s.q)
    fp_chunked = chunked.footprint_bytes
    chunked.close()
    assert stw == 0 and stc == 0
    # the second slot of the gather partials is allocated only for chunked planes
    assert fp_chunked - fp_whole == s.N * 2 * e["p"] * 32
    d = np.linalg.norm(Fc - Fw) / np.linalg.norm(Fw)
    print(f"chunked vs whole plane: force rel {d:.3e}, E_recip {Ec[2]:.15e} vs {Ew[2]:.15e}")
    assert d < (1e-12 if precision == "fp64" else 1e-6)
    assert Ec[2] == Ew[2]   # the spread is an exact fixed-point sum; same FFT lines
    ref = oracle.ewald(s.pos, s.q, e["L"], e["alpha"], e["Kc"], e["r_cut"], e["lam"])
    ef, ee, _ = _errors(Fc, Ec, ref)
    tf, te = TOL[precision]
    assert ef <= tf and ee <= te


_SWEEP_REF = {}


def _sweep_ref(L):
    if L not in _SWEEP_REF:
        s = wl.n_sweep(L)
        e = s.meta["enuf"]
        _SWEEP_REF[L] = (s, oracle.ewald(s.pos, s.q, e["L"], e["alpha"], e["Kc"], e["r_cut"], e["lam"]))
    return _SWEEP_REF[L]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("L", [15, 20, 30, 40])
def test_n_sweep_parity(L, precision):
    """The N sweep at density 3 with 10 % charges: L = 15 ... 40, N = 10125 ...
    192000, M = 3.2 L, Kc = 0.8 L (L = 40 in FP64 runs the row-chunked planes),
    every force and the energy against the full direct-Ewald oracle."""
    s, ref = _sweep_ref(L)
    e = s.meta["enuf"]
    print(f"case: n_sweep L={L} N={s.N} Nq={s.Nq} M={e['M']} Kc={e['Kc']} {precision}", flush=True)
    plan = _plan(s.N, e, precision)
    F, E5, st = _run(plan, s.pos, s.q)
    plan.close()
    ef, ee, Et = _errors(F, E5, ref)
    wp = _worst_particle(F, ref["F"])
    scale = abs(ref["E_real"]) + abs(ref["E_recip"]) + abs(ref["E_self"])
    print(f"L={L} {precision}: force rel rms {ef:.3e}  energy rel {ee:.3e} "
          f"(vs sum of |components| {abs(Et - ref['E']) / scale:.3e})  worst particle {wp:.3e}")
    assert st == 0
    tf, te = TOL[precision]
    assert ef <= tf and ee <= te
    assert wp <= PER_PARTICLE[precision]
    assert np.all(F[s.q == 0.0] == 0.0)


# The largest systems the batched and serving workloads run, against the
# oracle: every force and the energy where the direct sums are affordable,
# otherwise S(k) over all charges with the forces of a seeded sample of 1000
# charged beads (the reciprocal energy and the self term are still exact
# sums over every charge).
_BIG_REF = {}


def _big_system(which):
    if which == "replica_largest":
        # the largest member (by mesh) of the 64-replica batched workload: M = 80
        reps = [wl.replica(s) for s in range(64)]
        return max(reps, key=lambda r: (r.meta["enuf"]["M"], r.N))
    if which == "replica_m90":
        # the recipe of the batched workload at its largest N (48000) with the
        # densest charges (f = 1, z = 3): M = 90 = 2 3^2 5, Kc = 20
        L = (48000 / 3.0) ** (1.0 / 3.0)
        s = wl.polyelectrolyte(L, 3.0, 50, 1.0, 0.1, 3, wl.BASE_SEED + 900)
        M = wl.mesh_size(3.2 * L)
        s.meta["enuf"] = wl.enuf_params(L, M=M, Kc=min(int(np.floor(0.8 * L + 1e-9)), M // 4))
        s.meta["name"] = f"replica recipe N={s.N} f=1 z=3 M={M}"
        return s
    if which == "request_m144":
        # the most densely charged M = 144 request of the 2000-request serving
        # stream (N = 199627, 185421 charged, Kc = 32)
        return wl.serving_request(986)
    raise ValueError(which)


def _big_ref(which):
    if which not in _BIG_REF:
        s = _big_system(which)
        e = s.meta["enuf"]
        sel = None
        if s.Nq > 20000:
            qi = np.nonzero(s.q)[0]
            sel = np.sort(np.random.default_rng(20240613).choice(qi, 1000, replace=False))
        ref = oracle.ewald(s.pos, s.q, e["L"], e["alpha"], e["Kc"], e["r_cut"], e["lam"], sel=sel)
        _BIG_REF[which] = (s, sel, ref)
    return _BIG_REF[which]


@pytest.mark.parametrize("which,precision", [("replica_largest", "mixed"), ("replica_m90", "mixed"),
                                             ("replica_m90", "fp64"), ("request_m144", "mixed"),
                                             ("request_m144", "fp64")])
def test_largest_workload_meshes(which, precision):
    """Meshes of the batched (M = 80, 90) and serving (M = 144, row-chunked in
    FP64) workloads, with the member settings (one work-group per plane)."""
    s, sel, ref = _big_ref(which)
    e = s.meta["enuf"]
    print(f"case: {s.meta['name']} N={s.N} Nq={s.Nq} M={e['M']} Kc={e['Kc']} {precision} "
          f"sample={'all' if sel is None else len(sel)}", flush=True)
    plan = _plan(s.N, e, precision)
    plan.set_parts(1)
    F, E5, st = _run(plan, s.pos, s.q)
    plan.close()
    assert st == 0
    tf, te = TOL[precision]
    if sel is None:
        ef, ee, _ = _errors(F, E5, ref)
        Fs, Fr = F, ref["F"]
    else:
        Fs, Fr = F[sel], ref["F"]
        ef = np.linalg.norm(Fs - Fr) / np.linalg.norm(Fr)
        # E_recip and E_self are complete sums in the sampled reference too
        ee = abs(E5[2] + E5[3] - ref["E_recip"] - ref["E_self"]) / abs(ref["E_recip"] + ref["E_self"])
    wp = _worst_particle(Fs, Fr)
    print(f"{which} {precision}: force rel rms {ef:.3e} energy rel {ee:.3e} worst particle {wp:.3e}")
    assert ef <= tf and ee <= te
    assert wp <= PER_PARTICLE[precision]
    assert np.all(F[s.q == 0.0] == 0.0)


def _plan_ik(N, e, precision="fp64"):
    plan = _plan(N, e, precision)
    plan.set_force_mode("ik")
    return plan


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ik_differentiation_parity(precision):
    """Forces by ik-differentiation (eq. 24-25): three fields i k_t h gathered
    with the window.  Same oracle bars; the k-space energy is the same sum."""
    for s in (wl.single_eval_small(), wl.n_sweep(20)):
        e = s.meta["enuf"]
        print(f"case: ik {s.meta['name']} {precision}", flush=True)
        plan = _plan_ik(s.N, e, precision)
        F, E5, st = _run(plan, s.pos, s.q)
        plan.close()
        g = _plan(s.N, e, precision)
        Fg, Eg, _ = _run(g, s.pos, s.q)
        g.close()
        ref = oracle.ewald(s.pos, s.q, e["L"], e["alpha"], e["Kc"], e["r_cut"], e["lam"])
        ef, ee, _ = _errors(F, E5, ref)
        efg, _, _ = _errors(Fg, Eg, ref)
        print(f"ik: force rel rms {ef:.3e} energy rel {ee:.3e} (gradient forces {efg:.3e})")
        assert st == 0
        tf, te = TOL[precision]
        assert ef <= tf and ee <= te
        assert E5[2] == Eg[2] and E5[4] == 0.0


def test_ik_forces_conserve_momentum():
    """ik-differentiation: sum_j F_j = -(2/L^2) sum_l h_t[l] g[l] =
    i sum_k k_t c(k) |G(k)|^2 = 0 by the k -> -k symmetry, so the total
    reciprocal force vanishes to rounding; the window-gradient force (the
    exact gradient of the approximate energy) does not have this property."""
    s = wl.n_sweep(20)
    e = s.meta["enuf"]
    # reciprocal part only: a Kc-only comparison needs the real-space forces
    # removed; they cancel pairwise exactly in fixed point
    out = {}
    for mode in ("gradient", "ik"):
        plan = _plan(s.N, e)
        plan.set_force_mode(mode)
        F, E5, st = _run(plan, s.pos, s.q)
        plan.close()
        assert st == 0
        out[mode] = np.abs(F.sum(0)).max() / np.abs(F).sum(1).mean()
        print(f"case: {mode}: |sum F| / mean |F| = {out[mode]:.3e}", flush=True)
    assert out["ik"] < 1e-9
    assert out["gradient"] > 100 * out["ik"]
