"""The C-ABI library loads, exports every symbol include/enuf.h declares, and
rejects invalid plans on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "enuf.h")
LIB = os.path.join(ROOT, "paper_1303_4523_amd", "libenuf.so")

needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libenuf.so not built")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(enuf_[a-z0-9_]+)\s*\(", src)))


def _defines():
    src = open(HEADER).read()
    return {k: int(v) for k, v in re.findall(r"#define\s+(ENUF_[A-Z0-9_]+)\s+(-?\d+)", src)}


@needs_lib
def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


@needs_lib
def test_binding_lists_every_declared_symbol_and_code():
    from paper_1303_4523_amd import _lib
    assert sorted(_lib.EXPORTED) == _declared()
    d = _defines()
    assert d["ENUF_OK"] == _lib.OK and d["ENUF_EINVAL"] == _lib.EINVAL
    assert d["ENUF_ENONNEUTRAL"] == _lib.ENONNEUTRAL and d["ENUF_EOVERFLOW"] == _lib.EOVERFLOW
    assert d["ENUF_MIXED"] == _lib.MIXED and d["ENUF_WINDOW_GAUSS"] == _lib.WINDOW_GAUSS
    assert d["ENUF_GRAPH_AUTO"] == _lib.GRAPH_AUTO and d["ENUF_GRAPH_AUTO_STEPS"] == _lib.GRAPH_AUTO_STEPS


GOOD = dict(N=100, box=10.0, alpha=0.3, p=4, sigma=2.0, M=32, Kc=8, r_cut=3.0, lam=0.25)
BAD = [
    dict(N=0), dict(box=-1.0), dict(box=float("nan")), dict(alpha=0.0), dict(p=0), dict(p=16),
    dict(sigma=0.5), dict(M=31), dict(M=28), dict(M=14, p=4), dict(Kc=0), dict(Kc=9),
    dict(r_cut=5.1), dict(r_cut=0.0), dict(lam=-0.1), dict(M=2),
    dict(M=1250),  # 2 x 5^4: a radix-2 pass of 625 butterflies per line, more than a work-group holds
]


@needs_lib
@pytest.mark.parametrize("over", BAD)
def test_invalid_plans_fail_on_host(over):
    """Validation happens before any HIP call, so it runs without a GPU."""
    from paper_1303_4523_amd import _lib
    a = dict(GOOD, **over)
    h = _lib.lib.enuf_plan_create(a["N"], a["box"], a["alpha"], a["p"], a["sigma"], a["M"], a["Kc"],
                                  a["r_cut"], a["lam"])
    assert not h
    assert _lib.last_error() != ""


@needs_lib
def test_null_plan_calls_are_rejected():
    from paper_1303_4523_amd import _lib
    L = _lib.lib
    assert L.enuf_compute(None, None, None, None, None) == _lib.EINVAL
    assert L.enuf_plan_set_options(None, 0, 0) == _lib.EINVAL
    assert L.enuf_plan_set_stream(None, None) == _lib.EINVAL
    assert L.enuf_plan_footprint_bytes(None) == 0
    L.enuf_destroy(None)
