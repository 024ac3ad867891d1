"""ctypes binding of libenuf.so (the C ABI declared in include/enuf.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.
There is no CPU fallback: importing this module raises if the library has not
been built.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libenuf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_1303_4523_amd/build.py` (hipcc, gfx950)")

lib = ctypes.CDLL(LIB_PATH)

_i64, _int, _dbl, _vp, _sz = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t

lib.enuf_plan_create.argtypes = [_i64, _dbl, _dbl, _int, _dbl, _int, _int, _dbl, _dbl]
lib.enuf_plan_create.restype = _vp
lib.enuf_destroy.argtypes = [_vp]
lib.enuf_destroy.restype = None
lib.enuf_last_error.argtypes = []
lib.enuf_last_error.restype = ctypes.c_char_p
lib.enuf_plan_set_stream.argtypes = [_vp, _vp]
lib.enuf_plan_set_stream.restype = _int
lib.enuf_plan_set_options.argtypes = [_vp, _int, _int]
lib.enuf_plan_set_options.restype = _int
lib.enuf_compute.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.enuf_compute.restype = _int
lib.enuf_compute_components.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.enuf_compute_components.restype = _int
lib.enuf_plan_status.argtypes = [_vp, ctypes.POINTER(_int)]
lib.enuf_plan_status.restype = _int
lib.enuf_plan_footprint_bytes.argtypes = [_vp]
lib.enuf_plan_footprint_bytes.restype = _sz
lib.enuf_plan_set_force_mode.argtypes = [_vp, _int]
lib.enuf_plan_set_force_mode.restype = _int
lib.enuf_compute_noalloc.argtypes = [_i64, _dbl, _dbl, _int, _dbl, _int, _int, _dbl, _dbl, _int,
                                     _vp, _vp, _vp, _vp, _vp, _vp]
lib.enuf_compute_noalloc.restype = _int



class DpdParams(ctypes.Structure):
    """enuf_dpd_params of include/enuf.h."""
    _fields_ = [("a", _dbl), ("gamma", _dbl), ("sigma", _dbl), ("dt", _dbl), ("lam", _dbl),
                ("k_bond", _dbl), ("r0_bond", _dbl), ("kappa", _dbl), ("seed", ctypes.c_uint64)]


lib.enuf_dpd_create.argtypes = [_i64, _dbl, ctypes.POINTER(DpdParams), _vp, _vp, _i64, _vp]
lib.enuf_dpd_create.restype = _vp
lib.enuf_dpd_set_stream.argtypes = [_vp, _vp]
lib.enuf_dpd_set_stream.restype = _int
lib.enuf_dpd_forces.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_uint64]
lib.enuf_dpd_forces.restype = _int
lib.enuf_dpd_run.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_uint64, _int]
lib.enuf_dpd_run.restype = _int
lib.enuf_dpd_prepare_graphs.argtypes = [_vp, _vp, _vp, _vp]
lib.enuf_dpd_prepare_graphs.restype = _int
lib.enuf_dpd_set_concurrency.argtypes = [_vp, _int]
lib.enuf_dpd_set_concurrency.restype = _int
lib.enuf_dpd_set_graphs.argtypes = [_vp, _int]
lib.enuf_dpd_set_graphs.restype = _int
lib.enuf_dpd_energy.argtypes = [_vp, _vp]
lib.enuf_dpd_energy.restype = _int
lib.enuf_dpd_status.argtypes = [_vp, ctypes.POINTER(_int)]
lib.enuf_dpd_status.restype = _int
lib.enuf_dpd_destroy.argtypes = [_vp]
lib.enuf_dpd_destroy.restype = None
lib.enuf_dpd_time_kernel.argtypes = [_vp, _int, _int]
lib.enuf_dpd_time_kernel.restype = _int
lib.enuf_dpd_kernel_time.argtypes = [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_int)]
lib.enuf_dpd_kernel_time.restype = _int
lib.enuf_plan_time_kernel.argtypes = [_vp, _int, _int]
lib.enuf_plan_time_kernel.restype = _int
lib.enuf_plan_kernel_time.argtypes = [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_int)]
lib.enuf_plan_kernel_time.restype = _int
lib.enuf_batch_time_kernel.argtypes = [_vp, _int, _int]
lib.enuf_batch_time_kernel.restype = _int
lib.enuf_batch_kernel_time.argtypes = [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_int)]
lib.enuf_batch_kernel_time.restype = _int
lib.enuf_dpd_footprint_bytes.argtypes = [_vp]
lib.enuf_dpd_footprint_bytes.restype = _sz
lib.enuf_plan_footprint_estimate.argtypes = [_i64, _dbl, _int, _int, _int, _dbl]
lib.enuf_plan_footprint_estimate.restype = _sz
lib.enuf_dpd_footprint_estimate.argtypes = [_i64, _dbl, _i64]
lib.enuf_dpd_footprint_estimate.restype = _sz

lib.enuf_batch_create.argtypes = [_int]
lib.enuf_batch_create.restype = _vp
lib.enuf_batch_destroy.argtypes = [_vp]
lib.enuf_batch_destroy.restype = None
lib.enuf_batch_set_stream.argtypes = [_vp, _vp]
lib.enuf_batch_set_stream.restype = _int
lib.enuf_batch_set_options.argtypes = [_vp, _int, _int]
lib.enuf_batch_set_options.restype = _int
lib.enuf_batch_set_tuning.argtypes = [_vp, _int, _int, _int, _int, _int, _int]
lib.enuf_batch_set_tuning.restype = _int
lib.enuf_batch_add.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_uint64]
lib.enuf_batch_add.restype = _int
lib.enuf_batch_remove.argtypes = [_vp, _int]
lib.enuf_batch_remove.restype = _int
lib.enuf_batch_size.argtypes = [_vp]
lib.enuf_batch_size.restype = _int
lib.enuf_batch_run.argtypes = [_vp, _int]
lib.enuf_batch_run.restype = _int
lib.enuf_batch_footprint_bytes.argtypes = [_vp]
lib.enuf_batch_footprint_bytes.restype = _sz
lib.enuf_plan_set_parts.argtypes = [_vp, _int]
lib.enuf_plan_set_parts.restype = _int
lib.enuf_plan_set_concurrency.argtypes = [_vp, _int]
lib.enuf_plan_set_concurrency.restype = _int
lib.enuf_dpd_set_species.argtypes = [_vp, _int, _vp, _vp]
lib.enuf_dpd_set_species.restype = _int
lib.enuf_pair_histogram.argtypes = [_vp, _i64, _i64, _vp, _vp, _int, _dbl, _dbl, _int, _vp, _vp]
lib.enuf_pair_histogram.restype = _int
lib.enuf_chain_rg2.argtypes = [_vp, _i64, _int, _int, _vp, _dbl, _vp, _vp]
lib.enuf_chain_rg2.restype = _int

# Kernel ids of the timing hook (ENUF_K_* in include/enuf.h).
KERNELS = {"dpd_pre": 0, "dpd_pair": 1, "prep_count": 2, "prep_compact": 3, "real": 4,
           "mesh_fwd": 5, "mesh_x": 6, "mesh_bwd": 7, "combine": 8, "dpd_post": 9}

# Every function the header declares (checked by the CPU test suite).
EXPORTED = [
    "enuf_plan_create", "enuf_destroy", "enuf_last_error", "enuf_plan_set_stream",
    "enuf_plan_set_options", "enuf_compute", "enuf_compute_components", "enuf_plan_status",
    "enuf_plan_footprint_bytes",
    "enuf_dpd_create", "enuf_dpd_set_stream", "enuf_dpd_set_concurrency", "enuf_dpd_set_graphs",
    "enuf_dpd_forces", "enuf_dpd_run", "enuf_dpd_prepare_graphs",
    "enuf_dpd_energy", "enuf_dpd_status", "enuf_dpd_destroy",
    "enuf_dpd_time_kernel", "enuf_dpd_kernel_time", "enuf_dpd_footprint_bytes",
    "enuf_batch_create", "enuf_batch_destroy", "enuf_batch_set_stream", "enuf_batch_set_options",
    "enuf_batch_set_tuning",
    "enuf_batch_add", "enuf_batch_remove", "enuf_batch_size", "enuf_batch_run", "enuf_batch_footprint_bytes",
    "enuf_plan_footprint_estimate", "enuf_dpd_footprint_estimate", "enuf_plan_set_force_mode",
    "enuf_dpd_set_species", "enuf_pair_histogram", "enuf_chain_rg2", "enuf_plan_set_parts",
    "enuf_plan_set_concurrency",
    "enuf_plan_time_kernel", "enuf_plan_kernel_time", "enuf_batch_time_kernel", "enuf_batch_kernel_time",
    "enuf_compute_noalloc",
]

# Status codes (include/enuf.h).
OK, EINVAL, ENOMEM, EDEVICE, ENONNEUTRAL, ENONFINITE, EBUSY, ECOINCIDENT, EOVERFLOW = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
                ENONNEUTRAL: "ENONNEUTRAL", ENONFINITE: "ENONFINITE", EBUSY: "EBUSY",
                ECOINCIDENT: "ECOINCIDENT", EOVERFLOW: "EOVERFLOW"}
FP64, MIXED = 0, 1
WINDOW_KB, WINDOW_GAUSS = 0, 1
GRAPH_AUTO, GRAPH_AUTO_STEPS = 2, 16
FORCE_GRADIENT, FORCE_IK = 0, 1


class EnufError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib.enuf_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({msg})")


def last_error() -> str:
    return lib.enuf_last_error().decode(errors="replace")


def check(code, where):
    if code != OK:
        raise EnufError(code, where)
