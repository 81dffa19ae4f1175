"""Error behaviour of the C ABI on the GPU: every bad input returns a status (and a
message), never a crash, and the plan stays usable afterwards."""
import ctypes as C
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _plan(n=1000, box=(20.0, 20.0, 20.0), tol=1e-4, precision="fp64"):
    import paper_2412_04595_amd as sog
    return sog.Solver(box, n, tol, precision=precision)


def _status(fn):
    import paper_2412_04595_amd as sog
    try:
        fn()
        return 0
    except sog.SogError as e:
        assert sog.sog_last_error()
        return e.status


def test_input_errors_and_recovery():
    from paper_2412_04595_amd import _lib
    x, q = workloads.uniform(1000, (20.0, 20.0, 20.0), 11)
    print("[gpu] error statuses", flush=True)
    s = _plan()
    U0, p0, F0 = s(x, q)
    bad_q = q.copy()
    bad_q[0] += 1.0
    assert _status(lambda: s(x, bad_q)) == _lib.SOG_ERR_NOT_NEUTRAL
    bad_z = x.copy()
    bad_z[3, 2] = 20.5
    assert _status(lambda: s(bad_z, q)) == _lib.SOG_ERR_OUT_OF_BOX
    bad_z[3, 2] = -0.25
    assert _status(lambda: s(bad_z, q)) == _lib.SOG_ERR_OUT_OF_BOX
    nan_x = x.copy()
    nan_x[7, 0] = np.nan
    assert _status(lambda: s(nan_x, q)) == _lib.SOG_ERR_INVALID_ARG
    inf_q = q.copy()
    inf_q[9] = np.inf
    assert _status(lambda: s(x, inf_q)) == _lib.SOG_ERR_INVALID_ARG
    # NULL inputs
    assert _status(lambda: _lib.sog_energy_potential_force(s.plan, None, q.ctypes.data, None, None, None)) \
        == _lib.SOG_ERR_INVALID_ARG
    # the plan still works and gives the same answer
    U1, p1, F1 = s(x, q)
    s.close()
    assert abs(U1 - U0) <= 1e-13 * abs(U0)
    assert np.max(np.abs(p1 - p0)) <= 1e-13 * np.max(np.abs(p0))


def test_outputs_may_be_omitted():
    x, q = workloads.uniform(1000, (20.0, 20.0, 20.0), 12)
    s = _plan()
    U, phi, F = s(x, q)
    U2, _, _ = s(x, q, potential=False, forces=False)
    _, phi2, _ = s(x, q, energy=False, forces=False)
    s.close()
    assert abs(U2 - U) <= 1e-13 * abs(U)
    assert np.max(np.abs(phi2 - phi)) <= 1e-13 * np.max(np.abs(phi))


def test_plan_errors():
    import paper_2412_04595_amd as sog
    from paper_2412_04595_amd import _lib
    assert _status(lambda: sog.Solver((20, 20, 20), 1000, 1e-4, device=99)) == _lib.SOG_ERR_INVALID_ARG
    assert _status(lambda: sog.Solver((20, 20, 20), 1000, 1e-20)) == _lib.SOG_ERR_TOL_UNREACHABLE
    assert _lib.lib().sog_energy_potential_force(None, None, None, None, None, None) == _lib.SOG_ERR_INVALID_ARG
    _lib.lib().sog_destroy(None)  # NULL is ignored


def test_workspace_cap_gives_out_of_memory():
    """SOG_MAX_DEVICE_BYTES caps the plan's workspace; a plan above it fails cleanly."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2412_04595_amd as sog\n"
            "from paper_2412_04595_amd import _lib\n"
            "try:\n"
            "    sog.Solver((100, 100, 100), 1000000, 1e-4, precision='fp32')\n"
            "    print('no error')\n"
            "except sog.SogError as e:\n"
            "    print('status', e.status)\n") % ROOT
    env = dict(os.environ, SOG_MAX_DEVICE_BYTES="1000000")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert "status 5" in r.stdout, r.stdout + r.stderr
