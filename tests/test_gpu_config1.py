"""The Sec. 5.1 accuracy box (N = 1000 uniform +/-1 in 20^3, seed 1) solved at the
library's own plan for each tolerance, against Ewald2D on every particle
(tests/golden/cube_small_ewald2d.txt, written by the oracle): the energy, every
potential and every force within tol (relative; L-infinity over particles for phi and F,
as the paper measures)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube_small_ewald2d.txt")


def _ewald():
    d = np.loadtxt(GOLDEN, comments="#")
    U = next(float(l.split()[2]) for l in open(GOLDEN) if l.startswith("# U "))
    return U, d[:, 1], d[:, 2:5]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp64", 1e-8), ("fp64", 1e-4), ("fp32", 1e-4)])
def test_own_plan_meets_tol_against_ewald2d(precision, tol):
    import paper_2412_04595_amd as sog
    import workloads
    x, q, box = workloads.named("cube_small")
    Uref, phiref, gref = _ewald()
    Fref = -q[:, None] * gref
    s = sog.Solver(box, len(q), tol, precision=precision)
    U, phi, F = s(x, q)
    s.close()
    eU = abs(U - Uref) / abs(Uref)
    ephi = float(np.max(np.abs(phi - phiref)) / np.max(np.abs(phiref)))
    eF = float(np.max(np.abs(F - Fref)) / np.max(np.abs(Fref)))
    print(f"[gpu] cube_small {precision} tol {tol:g}: |dU|/|U| {eU:.2e} phi {ephi:.2e} F {eF:.2e}", flush=True)
    assert eU <= tol and ephi <= tol and eF <= tol
