"""ctypes binding of the C ABI in include/sog.h (argument marshalling only).

Every entry point of the library has a Python function of the same name here.  The
library is loaded from this package directory (libsog_hip.so, built by
``paper_2412_04595_amd.build``); if it is missing, loading raises -- there is no
fallback of any kind.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsog_hip.so")

SOG_OK = 0
(SOG_ERR_INVALID_ARG, SOG_ERR_NOT_NEUTRAL, SOG_ERR_OUT_OF_BOX, SOG_ERR_TOL_UNREACHABLE, SOG_ERR_OUT_OF_MEMORY,
 SOG_ERR_DEVICE) = range(1, 7)
STATUS = {
    0: "SOG_OK",
    1: "SOG_ERR_INVALID_ARG",
    2: "SOG_ERR_NOT_NEUTRAL",
    3: "SOG_ERR_OUT_OF_BOX",
    4: "SOG_ERR_TOL_UNREACHABLE",
    5: "SOG_ERR_OUT_OF_MEMORY",
    6: "SOG_ERR_DEVICE",
}
SOG_PREC_FP64, SOG_PREC_FP32_BULK = 0, 1
SOG_LONG_AUTO, SOG_LONG_DIRECT, SOG_LONG_FFT = 0, 1, 2
SOG_WINDOW_AUTO, SOG_WINDOW_GAUSSIAN, SOG_WINDOW_ES, SOG_WINDOW_KB = 0, 1, 2, 3

EXPORTS = (
    "sog_options_default",
    "sog_plan",
    "sog_plan_ex",
    "sog_energy_potential_force",
    "sog_energy_potential_force_static",
    "sog_energy_potential_gradient",
    "sog_potential_parts",
    "sog_plan_resolve",
    "sog_plan_info",
    "sog_plan_tuning",
    "sog_plan_sizes_get",
    "sog_kernel_times",
    "sog_kernel_times_reset",
    "sog_destroy",
    "sog_batch_plan",
    "sog_batch_energy_potential_force",
    "sog_batch_plan_info",
    "sog_batch_graph_info",
    "sog_batch_destroy",
    "sog_status_string",
    "sog_last_error",
)


class sog_params(C.Structure):
    _fields_ = [
        ("b", C.c_double), ("r0", C.c_double), ("omega", C.c_double),
        ("rc", C.c_double),
        ("M", C.c_int32), ("m", C.c_int32), ("set_m", C.c_int32),
        ("mid_I", C.c_int32 * 3), ("mid_Izs", C.c_int32), ("mid_Pw", C.c_int32 * 3), ("mid_S", C.c_double),
        ("long_form", C.c_int32), ("long_P", C.c_int32), ("long_nk", C.c_int32 * 2),
        ("long_I", C.c_int32 * 2), ("long_Pw", C.c_int32 * 2), ("long_S", C.c_double),
        ("mid_window", C.c_int32), ("mid_beta", C.c_double), ("long_Q", C.c_int32),
        ("mid_nu", C.c_int32), ("eta", C.c_double),
    ]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        return d


class sog_options(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p),
        ("pointers_on_device", C.c_int32), ("check_inputs", C.c_int32), ("timing", C.c_int32),
        ("params", sog_params), ("static_workspace", C.c_int32), ("deterministic", C.c_int32),
        ("eager", C.c_int32), ("autotune", C.c_int32),
    ]


class sog_plan_sizes(C.Structure):
    _fields_ = [
        ("mid_grid_points", C.c_int64), ("long_points", C.c_int64), ("device_bytes", C.c_int64),
        ("near_cells", C.c_int32 * 3), ("tile", C.c_int32 * 3),
        ("near_degree", C.c_int32), ("mid_zband", C.c_int32 * 2),
    ]


class sog_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char_p), ("total_ms", C.c_double), ("launches", C.c_int64)]


_lib = None


def lib():
    """The loaded library (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_04595_amd.build`")
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7 (same soname
        # as the system one this library links), and whichever loads first serves both.
        # Load torch's first when torch is installed, so that torch device tensors and
        # streams keep working after the library is loaded.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.sog_options_default.argtypes = [C.POINTER(sog_options)]
        L.sog_options_default.restype = None
        L.sog_plan.argtypes = [dp, C.c_int64, C.c_double, C.POINTER(P)]
        L.sog_plan.restype = C.c_int
        L.sog_plan_ex.argtypes = [dp, C.c_int64, C.c_double, C.POINTER(sog_options), C.POINTER(P)]
        L.sog_plan_ex.restype = C.c_int
        L.sog_energy_potential_force.argtypes = [P, P, P, P, P, P]
        L.sog_energy_potential_force.restype = C.c_int
        L.sog_energy_potential_force_static.argtypes = [P, P, P, P, P, P]
        L.sog_energy_potential_force_static.restype = C.c_int
        L.sog_energy_potential_gradient.argtypes = [P, P, P, P, P, P]
        L.sog_energy_potential_gradient.restype = C.c_int
        L.sog_potential_parts.argtypes = [P, P, P, P, P]
        L.sog_potential_parts.restype = C.c_int
        L.sog_plan_resolve.argtypes = [dp, C.c_int64, C.c_double, C.POINTER(sog_options), C.POINTER(sog_params)]
        L.sog_plan_resolve.restype = C.c_int
        L.sog_plan_info.argtypes = [P, C.POINTER(sog_params)]
        L.sog_plan_info.restype = C.c_int
        L.sog_plan_sizes_get.argtypes = [P, C.POINTER(sog_plan_sizes)]
        L.sog_plan_sizes_get.restype = C.c_int
        L.sog_kernel_times.argtypes = [P, C.POINTER(sog_kernel_time), C.c_int32, C.POINTER(C.c_int32)]
        L.sog_kernel_times.restype = C.c_int
        L.sog_kernel_times_reset.argtypes = [P]
        L.sog_kernel_times_reset.restype = C.c_int
        L.sog_destroy.argtypes = [P]
        L.sog_destroy.restype = None
        L.sog_batch_plan.argtypes = [C.c_int32, dp, C.POINTER(C.c_int64), C.c_double, C.POINTER(sog_options),
                                     C.POINTER(P)]
        L.sog_batch_plan.restype = C.c_int
        L.sog_batch_energy_potential_force.argtypes = [P, P, P, P, P, P]
        L.sog_batch_energy_potential_force.restype = C.c_int
        L.sog_batch_graph_info.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.sog_batch_graph_info.restype = C.c_int
        L.sog_batch_plan_info.argtypes = [P, C.c_int32, C.POINTER(sog_params)]
        L.sog_batch_plan_info.restype = C.c_int
        L.sog_batch_destroy.argtypes = [P]
        L.sog_batch_destroy.restype = None
        L.sog_status_string.argtypes = [C.c_int]
        L.sog_status_string.restype = C.c_char_p
        L.sog_last_error.argtypes = []
        L.sog_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class SogError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status):
    if status != SOG_OK:
        raise SogError(status, sog_last_error())


def sog_last_error():
    return lib().sog_last_error().decode()


def sog_status_string(s):
    return lib().sog_status_string(s).decode()


def sog_options_default():
    o = sog_options()
    lib().sog_options_default(C.byref(o))
    return o


def sog_plan(box, n, tol):
    h = C.c_void_p()
    b = (C.c_double * 3)(*box)
    _check(lib().sog_plan(b, int(n), float(tol), C.byref(h)))
    return h


def sog_plan_ex(box, n, tol, options):
    h = C.c_void_p()
    b = (C.c_double * 3)(*box)
    _check(lib().sog_plan_ex(b, int(n), float(tol), C.byref(options) if options is not None else None, C.byref(h)))
    return h


def sog_energy_potential_force(plan, x_ptr, q_ptr, energy_ptr, phi_ptr, force_ptr):
    """Pointers are integers (host or device addresses, as the plan was made for) or None."""
    st = lib().sog_energy_potential_force(plan, x_ptr, q_ptr, energy_ptr, phi_ptr, force_ptr)
    _check(st)


def sog_energy_potential_force_static(plan, x_ptr, q_ptr, energy_ptr, phi_ptr, force_ptr):
    _check(lib().sog_energy_potential_force_static(plan, x_ptr, q_ptr, energy_ptr, phi_ptr, force_ptr))


def sog_energy_potential_gradient(plan, x_ptr, q_ptr, energy_ptr, phi_ptr, grad_ptr):
    _check(lib().sog_energy_potential_gradient(plan, x_ptr, q_ptr, energy_ptr, phi_ptr, grad_ptr))


def sog_potential_parts(plan, x_ptr, q_ptr, phi_parts_ptr, grad_parts_ptr):
    _check(lib().sog_potential_parts(plan, x_ptr, q_ptr, phi_parts_ptr, grad_parts_ptr))


def sog_plan_resolve(box, n, tol, options=None):
    p = sog_params()
    b = (C.c_double * 3)(*box)
    _check(lib().sog_plan_resolve(b, int(n), float(tol), C.byref(options) if options is not None else None,
                                  C.byref(p)))
    return p


def sog_plan_info(plan):
    p = sog_params()
    _check(lib().sog_plan_info(plan, C.byref(p)))
    return p


def sog_plan_tuning(plan, max_count=16):
    """[(rc, m, ms), ...] of the discretisations an autotuned plan timed ([] otherwise)."""
    cnt = C.c_int32(0)
    rc = (C.c_double * max_count)()
    m = (C.c_int32 * max_count)()
    ms = (C.c_double * max_count)()
    _check(lib().sog_plan_tuning(plan, int(max_count), C.byref(cnt), rc, m, ms))
    return [(rc[i], m[i], ms[i]) for i in range(min(cnt.value, max_count))]


def sog_plan_sizes_get(plan):
    s = sog_plan_sizes()
    _check(lib().sog_plan_sizes_get(plan, C.byref(s)))
    return s


def sog_kernel_times(plan):
    cnt = C.c_int32(0)
    _check(lib().sog_kernel_times(plan, None, 0, C.byref(cnt)))
    arr = (sog_kernel_time * max(cnt.value, 1))()
    _check(lib().sog_kernel_times(plan, arr, cnt.value, C.byref(cnt)))
    return {arr[i].name.decode(): (arr[i].total_ms, arr[i].launches) for i in range(cnt.value)}


def sog_kernel_times_reset(plan):
    _check(lib().sog_kernel_times_reset(plan))


def sog_destroy(plan):
    if plan:
        lib().sog_destroy(plan)


def sog_batch_plan(boxes, ns, tol, options):
    """boxes: sequence of (Lx, Ly, Lz); ns: particle counts, one per system."""
    h = C.c_void_p()
    k = len(ns)
    b = (C.c_double * (3 * k))(*[float(v) for box in boxes for v in box])
    n = (C.c_int64 * k)(*[int(v) for v in ns])
    _check(lib().sog_batch_plan(k, b, n, float(tol), C.byref(options) if options is not None else None, C.byref(h)))
    return h


def sog_batch_energy_potential_force(batch, x_ptr, q_ptr, energy_ptr, phi_ptr, force_ptr):
    _check(lib().sog_batch_energy_potential_force(batch, x_ptr, q_ptr, energy_ptr, phi_ptr, force_ptr))


def sog_batch_graph_info(batch):
    g, k = C.c_int32(0), C.c_int32(0)
    _check(lib().sog_batch_graph_info(batch, C.byref(g), C.byref(k)))
    return g.value, k.value


def sog_batch_plan_info(batch, s):
    p = sog_params()
    _check(lib().sog_batch_plan_info(batch, int(s), C.byref(p)))
    return p


def sog_batch_destroy(batch):
    if batch:
        lib().sog_batch_destroy(batch)
