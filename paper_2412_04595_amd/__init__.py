"""MI355X (gfx950) fast spectral sum-of-Gaussians solver for quasi-2D electrostatics.

The work happens in the HIP library libsog_hip.so behind the C ABI of include/sog.h;
``_lib`` binds each entry point under its C name.  ``Solver`` is a convenience wrapper
that marshals NumPy arrays (host pointers) or torch device tensors (device pointers,
torch's current stream) into those calls; it computes nothing itself.
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import (SOG_LONG_AUTO, SOG_LONG_DIRECT, SOG_LONG_FFT, SOG_PREC_FP32_BULK, SOG_PREC_FP64, SogError,
                   sog_batch_destroy, sog_batch_energy_potential_force, sog_batch_graph_info, sog_batch_plan,
                   sog_batch_plan_info,
                   sog_destroy, sog_energy_potential_force, sog_energy_potential_force_static,
                   sog_energy_potential_gradient, sog_kernel_times,
                   sog_kernel_times_reset,
                   sog_last_error, sog_options_default, sog_plan, sog_plan_ex, sog_plan_info, sog_plan_resolve,
                   sog_plan_tuning,
                   sog_plan_sizes_get,
                   sog_potential_parts, sog_status_string)

PRECISION = {"fp64": SOG_PREC_FP64, "fp32": SOG_PREC_FP32_BULK}
LONG_FORM = {"auto": SOG_LONG_AUTO, "direct": SOG_LONG_DIRECT, "fft": SOG_LONG_FFT}


def make_options(precision="fp64", device=0, stream=None, on_device=False, check_inputs=True, timing=False,
                 params=None, static_workspace=False, deterministic=False, autotune=False, eager=False):
    """sog_options from keyword arguments; ``params`` is a dict of sog_params fields."""
    o = sog_options_default()
    o.eager = int(bool(eager))
    o.static_workspace = int(bool(static_workspace))
    o.deterministic = int(bool(deterministic))
    o.autotune = int(bool(autotune))
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.device = int(device)
    o.stream = stream
    o.pointers_on_device = int(bool(on_device))
    o.check_inputs = int(bool(check_inputs))
    o.timing = int(bool(timing))
    for k, v in (params or {}).items():
        if k == "long_form" and isinstance(v, str):
            v = LONG_FORM[v]
        cur = getattr(o.params, k)
        if hasattr(cur, "__len__"):
            for i, vi in enumerate(v):
                cur[i] = vi
        else:
            setattr(o.params, k, v)
    return o


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


class Solver:
    """One plan: N particles in box (Lx, Ly, Lz) at relative tolerance tol.

    Host mode (on_device=False): call with float64 NumPy arrays x (N,3) and q (N,).
    Device mode (on_device=True): call with float64 torch tensors on the plan's device;
    the work is queued on torch's current stream."""

    def __init__(self, box, n, tol, precision="fp64", device=0, on_device=False, check_inputs=True,
                 timing=False, params=None, stream=None, static_workspace=False, deterministic=False,
                 autotune=False, eager=False):
        self.box = tuple(float(v) for v in box)
        self.n = int(n)
        self.on_device = bool(on_device)
        self.device = int(device)
        if self.on_device and stream is None:
            import torch
            stream = torch.cuda.current_stream(self.device).cuda_stream
        self.options = make_options(precision, device, stream, on_device, check_inputs, timing, params,
                                    static_workspace, deterministic, autotune, eager)
        self.plan = sog_plan_ex(self.box, self.n, float(tol), self.options)

    def close(self):
        if getattr(self, "plan", None):
            sog_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _inputs(self, x, q):
        if self.on_device:
            import torch
            assert x.dtype == torch.float64 and q.dtype == torch.float64 and x.is_cuda and q.is_cuda
            x = x.contiguous()
            q = q.contiguous()
            assert tuple(x.shape) == (self.n, 3) and tuple(q.shape) == (self.n,)
            return x, q
        x = np.ascontiguousarray(x, dtype=np.float64)
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert x.shape == (self.n, 3) and q.shape == (self.n,)
        return x, q

    def _alloc(self, *shape):
        if self.on_device:
            import torch
            return torch.empty(*shape, dtype=torch.float64, device=f"cuda:{self.device}")
        return np.empty(shape, dtype=np.float64)

    def __call__(self, x, q, energy=True, potential=True, forces=True, static=False, energy_on_device=False):
        """Returns (U, phi, force); entries not requested are None.  static: through
        sog_energy_potential_force_static (the library's static scratch).  U is a float,
        read back from the device (which waits for the call to finish), or with
        energy_on_device a one-element tensor where the call leaves it (device plans)."""
        x, q = self._inputs(x, q)
        U = self._alloc(1) if energy else None
        phi = self._alloc(self.n) if potential else None
        F = self._alloc(self.n, 3) if forces else None
        call = sog_energy_potential_force_static if static else sog_energy_potential_force
        call(self.plan, _ptr(x), _ptr(q), _ptr(U), _ptr(phi), _ptr(F))
        if U is not None and not energy_on_device:
            U = float(U[0])
        return U, phi, F

    def potential_gradient(self, x, q, energy=True):
        """Returns (U, phi, grad phi at the particles) from one call."""
        x, q = self._inputs(x, q)
        U = self._alloc(1) if energy else None
        phi = self._alloc(self.n)
        g = self._alloc(self.n, 3)
        sog_energy_potential_gradient(self.plan, _ptr(x), _ptr(q), _ptr(U), _ptr(phi), _ptr(g))
        if U is not None:
            U = float(U[0])
        return U, phi, g

    def parts(self, x, q):
        """(phi_parts (3,N), grad_parts (3,N,3)) for the near, mid and long parts."""
        x, q = self._inputs(x, q)
        pp = self._alloc(3, self.n)
        gp = self._alloc(3, self.n, 3)
        sog_potential_parts(self.plan, _ptr(x), _ptr(q), _ptr(pp), _ptr(gp))
        return pp, gp

    def info(self):
        return sog_plan_info(self.plan).as_dict()

    def tuning(self):
        """[(rc, m, ms), ...] timed by an autotuned plan ([] otherwise)."""
        return sog_plan_tuning(self.plan)

    def sizes(self):
        s = sog_plan_sizes_get(self.plan)
        return dict(mid_grid_points=s.mid_grid_points, long_points=s.long_points, device_bytes=s.device_bytes,
                    near_cells=list(s.near_cells), tile=list(s.tile), near_degree=s.near_degree,
                    mid_zband=list(s.mid_zband))

    def kernel_times(self):
        return sog_kernel_times(self.plan)

    def reset_kernel_times(self):
        sog_kernel_times_reset(self.plan)


class BatchSolver:
    """Independent systems solved by one call (sog_batch_plan): boxes[s] and ns[s] give
    system s; inputs and outputs hold the systems one after another.  Same host/device
    modes as Solver; __call__ returns (energies (nsys,), phi, force)."""

    def __init__(self, boxes, ns, tol, precision="fp64", device=0, on_device=False, check_inputs=True,
                 params=None, stream=None, deterministic=False):
        self.boxes = [tuple(float(v) for v in b) for b in boxes]
        self.ns = [int(v) for v in ns]
        self.n = sum(self.ns)
        self.offsets = np.concatenate([[0], np.cumsum(self.ns)]).astype(np.int64)
        self.on_device = bool(on_device)
        self.device = int(device)
        if self.on_device and stream is None:
            import torch
            stream = torch.cuda.current_stream(self.device).cuda_stream
        self.options = make_options(precision, device, stream, on_device, check_inputs, False, params,
                                    deterministic=deterministic)
        self.batch = sog_batch_plan(self.boxes, self.ns, float(tol), self.options)

    def close(self):
        if getattr(self, "batch", None):
            sog_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, s):
        return sog_batch_plan_info(self.batch, s).as_dict()

    def graph_info(self):
        """(groups of systems sharing kernels, kernel launches per call)"""
        return sog_batch_graph_info(self.batch)

    def __call__(self, x, q):
        x, q = Solver._inputs(self, x, q)
        U = Solver._alloc(self, len(self.ns))
        phi = Solver._alloc(self, self.n)
        F = Solver._alloc(self, self.n, 3)
        sog_batch_energy_potential_force(self.batch, _ptr(x), _ptr(q), _ptr(U), _ptr(phi), _ptr(F))
        return U, phi, F


def plan_parameters(box, n, tol, precision="fp64", params=None, deterministic=False):
    """The parameters the planner picks (host only, no GPU needed)."""
    return sog_plan_resolve(box, n, tol, make_options(precision, params=params,
                                                      deterministic=deterministic)).as_dict()


def device_count():
    """Number of HIP devices the library sees (0 on a machine without a GPU)."""
    n = C.c_int(0)
    try:
        hip = C.CDLL("libamdhip64.so")
    except OSError:
        return 0
    if hip.hipGetDeviceCount(C.byref(n)) != 0:
        return 0
    return n.value
