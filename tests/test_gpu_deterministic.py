"""The deterministic mode (sog_options.deterministic): bitwise identical results for the
same inputs, call after call and plan after plan, and the same operator as the atomic
mode and the oracle.

Cases: the Sec. 5.1 box (mid range and the direct long range), a slab with the
long range's FFT form, clustered input (cells of hundreds of particles), the widest
window in float64 (small tiles: 4 tile colours per direction), a strongly confined box
(every Gaussian long range, App. C's Taylor form), and the 10^6 cube at full size.

Tolerances against the oracle are the parity tests' (1e-12 of each part's max in
float64; 3e-5 / 1e-4 in float32-bulk); against the atomic mode 1e-13 (float64) and 3e-6
(float32) of the largest magnitude, the rounding of a different summation order."""
import numpy as np
import pytest

import workloads
from tests._cases import CASES, gpu_params, oracle_params

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12), "fp32": (3e-5, 1e-4)}
ORDER_TOL = {"fp64": 1e-13, "fp32": 3e-6}


def _inputs(name):
    c = CASES[name]
    x, q = getattr(workloads, c.get("gen", "uniform"))(c["N"], c["box"], c["seed"], **c.get("gen_args", {}))
    return c, x, q


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _parts(c, x, q, precision, deterministic):
    import paper_2412_04595_amd as sog
    tol = 1e-6 if precision == "fp64" else 1e-4
    s = sog.Solver(c["box"], c["N"], tol, precision=precision, params=gpu_params(c), deterministic=deterministic)
    out = [s.parts(x, q) for _ in range(2)]
    U = s(x, q)[0]
    s.close()
    return out, U


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cube_small", "slab_mid_fft", "clustered", "pw15", "confined_taylor"])
def test_deterministic_mode(name, precision):
    from oracle import fast
    c, x, q = _inputs(name)
    print(f"[gpu] deterministic {name} {precision} N={c['N']}", flush=True)
    (d1, d2), Ud = _parts(c, x, q, precision, True)
    (d3, _), Ud2 = _parts(c, x, q, precision, True)  # a second plan
    for a, b in ((d1, d2), (d1, d3)):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), "deterministic results differ"
    assert Ud == Ud2
    (a1, a2), Ua = _parts(c, x, q, precision, False)
    same = np.array_equal(a1[0], a2[0]) and np.array_equal(a1[1], a2[1])
    ref = fast.solve(x, q, c["box"], oracle_params(c), parts=True)
    tphi, tgrad = TOL[precision]
    for k, part in enumerate(("near", "mid", "long")):
        rp, rg = ref["phi_" + part], ref["grad_" + part]
        if np.max(np.abs(rp)) == 0:
            continue
        ep, eg = _rel(d1[0][k], rp), _rel(d1[1][k], rg)
        op, og = _rel(d1[0][k], a1[0][k]), _rel(d1[1][k], a1[1][k])
        print(f"    {part}: vs oracle phi {ep:.2e} grad {eg:.2e}; vs atomic phi {op:.2e} grad {og:.2e}", flush=True)
        assert ep < tphi and eg < tgrad
        assert op < ORDER_TOL[precision] and og < ORDER_TOL[precision]
    print(f"    atomic mode repeated {'bitwise' if same else 'with last-bit differences'}", flush=True)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_deterministic_mode_at_full_size(precision):
    """The 10^6 cube at the planner's parameters: two calls bitwise equal, sampled targets
    within the tolerance, as in the atomic mode."""
    import os
    import torch
    import paper_2412_04595_amd as sog
    name = "cube_1e6"
    print(f"[gpu] deterministic full size {name} {precision}", flush=True)
    x, q, box = workloads.named(name)
    xt = torch.from_numpy(x).cuda()
    qt = torch.from_numpy(q).cuda()
    s = sog.Solver(box, len(q), 1e-4, precision=precision, on_device=True, deterministic=True)
    U1, phi1, F1 = s(xt, qt)
    U2, phi2, F2 = s(xt, qt)
    torch.cuda.synchronize()
    s.close()
    assert U1 == U2 and torch.equal(phi1, phi2) and torch.equal(F1, F2)
    d = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", f"{name}_targets.txt"), comments="#")
    idx, rphi, rgrad = d[:, 0].astype(np.int64), d[:, 1], d[:, 2:5]
    phi, F = phi1.cpu().numpy(), F1.cpu().numpy()
    rF = -q[idx, None] * rgrad
    ephi = np.max(np.abs(phi[idx] - rphi)) / np.max(np.abs(rphi))
    eF = np.max(np.abs(F[idx] - rF)) / np.max(np.abs(rF))
    print(f"    phi {ephi:.2e} F {eF:.2e}", flush=True)
    assert ephi < 1e-4 and eF < 1e-4


def test_deterministic_batch():
    """A batch of 12 systems of the 256-system mix (every height ratio, sizes 500 to 20000)
    in the deterministic mode: two calls bitwise equal, and within float32 order rounding
    of the atomic mode's batch."""
    import paper_2412_04595_amd as sog
    specs = [workloads.batch_specs()[i] for i in workloads.BATCH_CHECKED]
    x, q, boxes, ns = workloads.batch(specs)
    print(f"[gpu] deterministic batch of {len(ns)} systems, {len(q)} particles", flush=True)
    b = sog.BatchSolver(boxes, ns, 1e-4, precision="fp32", deterministic=True)
    E1, p1, F1 = b(x, q)
    E2, p2, F2 = b(x, q)
    b.close()
    assert np.array_equal(E1, E2) and np.array_equal(p1, p2) and np.array_equal(F1, F2)
    a = sog.BatchSolver(boxes, ns, 1e-4, precision="fp32")
    Ea, pa, Fa = a(x, q)
    a.close()
    ep, eF = _rel(p1, pa), _rel(F1, Fa)
    print(f"    vs atomic batch: phi {ep:.2e} F {eF:.2e}", flush=True)
    assert ep < 3e-6 and eF < 3e-5
