"""Structure regressions of the paper's physics studies on the GPU path:
electrolyte radial distribution functions (set 3, Sec. 5) and the radius of
gyration of a polyelectrolyte against its charge fraction (set 5, Sec. 6).
Shortened runs; the full-length figures are produced by
``python -m paper_1303_4523_amd.studies``."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _band(r, g, lo, hi):
    m = (r >= lo) & (r < hi)
    return float(g[m].mean())


def test_electrolyte_set3_structure():
    """Set 3 (4000 beads, 132 + 132 ions, density 4): the thermostat holds
    kT = 1; every g(r) tends to 1 beyond r = 3; in the first shell unlike ions
    are enriched and like ions depleted relative to the solvent; no ion
    pairs collapse (g_+- ~ 0 below r = 0.3); and the product relation
    g_+- g_++/-- = g_00^2 holds across 0.5 <= r < 3."""
    from paper_1303_4523_amd.studies import electrolyte_rdf
    print("case: electrolyte set 3, 60000 steps", flush=True)
    res = electrolyte_rdf(steps=60000, equil=5000, every=50)
    r, g00, gpm = res["r"], res["g00"], res["gpm"]
    glike = 0.5 * (res["gpp"] + res["gmm"])
    print(f"kT {res['kT']:.4f}  {res['seconds']:.1f} s", flush=True)
    assert res["status"] == 0
    assert abs(res["kT"] - 1.0) < 0.03
    for g in (g00, gpm, glike):
        assert abs(_band(r, g, 3.0, 5.0) - 1.0) < 0.03
    s00, spm, slk = (_band(r, g, 0.6, 1.1) for g in (g00, gpm, glike))
    print(f"first shell: g00 {s00:.3f} g+- {spm:.3f} g++/-- {slk:.3f}")
    assert spm > s00 + 0.1 and slk < s00 - 0.05
    assert _band(r, gpm, 0.0, 0.3) < 0.05
    m = (r >= 0.5) & (r < 3.0)
    prod, sq = gpm[m] * glike[m], g00[m] ** 2
    rel = prod.sum() / sq.sum() - 1.0
    print(f"sum g+- g++/-- / sum g00^2 - 1 = {rel:.4f}; max bin deviation "
          f"{np.max(np.abs(prod / sq - 1.0)):.3f}")
    assert abs(rel) < 0.03
    assert np.all(np.abs(prod / sq - 1.0) < 0.2)


def test_polyelectrolyte_rg_grows_with_charge():
    """Set 5 in a 12^3 box: a fully charged chain (f = 1, with its
    counterions) is clearly larger than the neutral one (f = 0), and the
    neutral chain has the size of a 48-bead coil of bond length ~0.75."""
    from paper_1303_4523_amd.studies import polyelectrolyte_rg
    print("case: polyelectrolyte set 5, L=12, f in {0, 1}, 2 replicas", flush=True)
    res = polyelectrolyte_rg(fractions=(0.0, 1.0), L=12.0, replicas=2, steps=30000, equil=10000, every=100)
    rg0, rg1 = res["fractions"][0.0]["rg"], res["fractions"][1.0]["rg"]
    print(f"Rg(f=0) {rg0:.3f}  Rg(f=1) {rg1:.3f}  ratio {rg1 / rg0:.3f}  kT {np.mean(res['kT']):.4f}  "
          f"{res['seconds']:.1f} s", flush=True)
    assert all(st == 0 for st in res["status"])
    assert 1.5 < rg0 < 3.0
    assert rg1 > 1.2 * rg0
    assert all(abs(t - 1.0) < 0.05 for t in res["kT"])
