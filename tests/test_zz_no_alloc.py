"""sog_energy_potential_force_static (the entry point that allocates nothing: every
per-call buffer in the library's static device scratch) against sog_energy_potential_force
on the same inputs, through the C ABI.

Two calls in a row through the static entry point, the second with a smaller system, so
that the second runs on the scratch the first left behind; each result is compared with
the ordinary entry point's on an ordinary plan, element by element, at the parity
tolerances (float64: 1e-12 of the largest value; float32 bulk: 3e-5 potentials, 1e-4
forces).  Plans made with static_workspace hold no per-call buffers; the ordinary entry
points refuse them, and a plan whose per-call buffers exceed the scratch is refused with
the sizes in the message."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12, 1e-12), "fp32": (3e-5, 3e-5, 1e-4)}  # energy, potentials, forces
BOX = (24.0, 24.0, 18.0)
SIZES = ((3000, 71), (1200, 72))  # the second call is the smaller input


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _ordinary(n, x, q, precision, on_device):
    import torch
    import paper_2412_04595_amd as sog
    s = sog.Solver(BOX, n, 1e-6 if precision == "fp64" else 1e-4, precision=precision, on_device=on_device)
    if on_device:
        U, phi, F = s(torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
        torch.cuda.synchronize()
        phi, F = phi.cpu().numpy(), F.cpu().numpy()
    else:
        U, phi, F = s(x, q)
    s.close()
    return U, phi, F


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("on_device", [True, False])
def test_static_entry_point_matches_ordinary_calls(precision, on_device):
    import torch
    import paper_2412_04595_amd as sog
    tol = 1e-6 if precision == "fp64" else 1e-4
    inputs = [(n,) + workloads.uniform(n, BOX, seed) for n, seed in SIZES]
    refs = [_ordinary(n, x, q, precision, on_device) for n, x, q in inputs]
    plans = [sog.Solver(BOX, n, tol, precision=precision, on_device=on_device, static_workspace=True)
             for n, _, _ in inputs]
    for (n, x, q), s, (U0, p0, F0) in zip(inputs, plans, refs):
        print(f"[gpu] static entry point {precision} device={on_device} N={n}", flush=True)
        if on_device:
            U, phi, F = s(torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda(), static=True)
            torch.cuda.synchronize()
            phi, F = phi.cpu().numpy(), F.cpu().numpy()
        else:
            U, phi, F = s(x, q, static=True)
        eU, ep, eF = abs(U - U0) / abs(U0), _rel(phi, p0), _rel(F, F0)
        print(f"    U {eU:.2e} phi {ep:.2e} F {eF:.2e}", flush=True)
        tU, tp, tF = TOL[precision]
        assert eU < tU and ep < tp and eF < tF
    for s in plans:
        s.close()


def test_static_plans_and_limits():
    import paper_2412_04595_amd as sog
    from paper_2412_04595_amd import _lib
    n, x, q = (1200,) + workloads.uniform(1200, BOX, 73)
    print("[gpu] static plans: refusals and limits", flush=True)
    s = sog.Solver(BOX, n, 1e-6, static_workspace=True)
    with pytest.raises(sog.SogError) as e:
        s(x, q)  # the ordinary entry point refuses a plan without per-call buffers
    assert e.value.status == _lib.SOG_ERR_INVALID_ARG and "static_workspace" in str(e.value)
    U1, p1, F1 = s(x, q, static=True)
    s.close()
    # an ordinary plan runs through the static entry point too, and gives its own result
    o = sog.Solver(BOX, n, 1e-6)
    U2, p2, F2 = o(x, q, static=True)
    U3, p3, F3 = o(x, q)
    o.close()
    assert abs(U1 - U3) < 1e-12 * abs(U3) and abs(U2 - U3) < 1e-12 * abs(U3)
    assert _rel(p1, p3) < 1e-12 and _rel(p2, p3) < 1e-12 and _rel(F2, F3) < 1e-12
    # a plan whose per-call buffers exceed the scratch: refused at plan time with the sizes
    with pytest.raises(sog.SogError) as e:
        sog.Solver((100.0, 100.0, 100.0), 1_000_000, 1e-4, precision="fp32", on_device=True, static_workspace=True)
    assert e.value.status == _lib.SOG_ERR_OUT_OF_MEMORY and "static scratch" in str(e.value)
    # ... and at call time when an ordinary plan of that size calls the static entry point
    import torch
    big = sog.Solver((100.0, 100.0, 100.0), 1_000_000, 1e-4, precision="fp32", on_device=True, check_inputs=False)
    xb, qb = workloads.uniform(1_000_000, (100.0, 100.0, 100.0), 2)
    with pytest.raises(sog.SogError) as e:
        big(torch.from_numpy(xb).cuda(), torch.from_numpy(qb).cuda(), static=True)
    assert e.value.status == _lib.SOG_ERR_OUT_OF_MEMORY
    big.close()
