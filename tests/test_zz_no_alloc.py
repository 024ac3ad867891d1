"""enuf_compute_noalloc (no plan, buffers in a fixed device array) against
enuf_compute_components on a plan of the same parameters: two calls in a
row, the second smaller, in FP64 and in the mixed mode, bitwise and within the
oracle bars."""
import numpy as np
import pytest

import oracle
from paper_1303_4523_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"fp64": (1e-5, 1e-6), "mixed": (5e-4, 1e-4)}


def _plan_eval(s, e, precision):
    from paper_1303_4523_amd import Plan
    plan = Plan(s.N, e["L"], e["alpha"], e["p"], e["sigma"], e["M"], e["Kc"], e["r_cut"], e["lam"],
                precision=precision)
    F, E5 = plan.compute_components(torch.tensor(s.pos, device="cuda:0"), torch.tensor(s.q, device="cuda:0"))
    st = plan.status()
    plan.close()
    return F.cpu().numpy(), E5.cpu().numpy(), st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_plan_two_calls(precision):
    from paper_1303_4523_amd.plan import compute_noalloc
    big = wl.n_sweep(20)                  # N = 24000, M = 64, Kc = 16
    small = wl.single_eval_small()        # N = 3000, M = 32, Kc = 8
    out = []
    for s in (big, small):
        e = s.meta["enuf"]
        print(f"case: noalloc {s.meta['name']} {precision}", flush=True)
        F, E5, st = compute_noalloc(torch.tensor(s.pos, device="cuda:0"), torch.tensor(s.q, device="cuda:0"),
                                    e["L"], e["alpha"], e["p"], e["sigma"], e["M"], e["Kc"], e["r_cut"], e["lam"],
                                    precision=precision)
        torch.cuda.synchronize()
        out.append((s, e, F.cpu().numpy(), E5.cpu().numpy(), int(st.cpu().item())))
    for s, e, F, E5, st in out:
        Fp, Ep, stp = _plan_eval(s, e, precision)
        assert st == 0 and stp == 0
        # same kernels, configuration and tables: the same bits
        assert np.array_equal(F, Fp), s.meta["name"]
        assert np.array_equal(E5, Ep), s.meta["name"]
        ref = oracle.ewald(s.pos, s.q, e["L"], e["alpha"], e["Kc"], e["r_cut"], e["lam"])
        ef = np.linalg.norm(F - ref["F"]) / np.linalg.norm(ref["F"])
        ee = abs(E5[0] + E5[2] + E5[3] - ref["E"]) / abs(ref["E"])
        print(f"{s.meta['name']} {precision}: force {ef:.3e} energy {ee:.3e}")
        tf, te = TOL[precision]
        assert ef <= tf and ee <= te


def test_noalloc_reports_status_and_limits():
    from paper_1303_4523_amd._lib import EnufError
    from paper_1303_4523_amd.plan import compute_noalloc
    e = dict(L=10.0, alpha=0.3, p=4, sigma=2.0, M=32, Kc=8, r_cut=3.0, lam=0.25)
    rs = np.random.default_rng(3)
    pos = torch.tensor(rs.uniform(0, 10, (50, 3)), device="cuda:0")
    q = np.zeros(50)
    q[:3] = 1.0   # not neutral
    print("case: noalloc status of a non-neutral input", flush=True)
    _, _, st = compute_noalloc(pos, torch.tensor(q, device="cuda:0"), e["L"], e["alpha"], e["p"], e["sigma"],
                               e["M"], e["Kc"], e["r_cut"], e["lam"])
    assert int(st.cpu().item()) == -4
    # too large for the static array (checked on the host before any launch)
    n = 2_000_000
    with pytest.raises(EnufError, match="scratch"):
        compute_noalloc(torch.zeros((n, 3), dtype=torch.float64, device="cuda:0"),
                        torch.zeros(n, dtype=torch.float64, device="cuda:0"), 100.0, 0.3, 4, 2.0, 128, 32, 3.0,
                        0.25)
    with pytest.raises(EnufError, match="M must be"):
        compute_noalloc(pos, torch.tensor(q, device="cuda:0"), 10.0, 0.3, 4, 2.0, 288, 8, 3.0, 0.25)
