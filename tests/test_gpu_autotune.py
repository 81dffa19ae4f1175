"""Autotuned plans (sog_options.autotune): the planner's cheapest few discretisations are
timed on the device and the fastest kept.

* the tuning record lists distinct r_c with positive times, and the plan's own parameters
  are those of the fastest;
* the autotuned plan meets the tolerance: the layered 2e5 workload (whose float64 plan the
  cost model ranks wrongly) against its golden sampled targets, and the Sec. 5.1 box at
  tol 1e-6 against the oracle's fast method at the plan's parameters, part by part;
* autotune with static_workspace is refused."""
import os

import numpy as np
import pytest

import workloads
from tests._cases import oracle_params_from_info

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _check_tuning(s):
    t = s.tuning()
    info = s.info()
    print("    tuning:", [(round(rc, 3), m, round(ms, 3)) for rc, m, ms in t], flush=True)
    assert 1 <= len(t) <= 3
    assert len({rc for rc, _, _ in t}) == len(t)
    assert all(ms > 0 for _, _, ms in t)
    rc, m, _ = min(t, key=lambda e: e[2])
    assert info["rc"] == rc and info["m"] == m
    return info


def test_autotuned_layered_meets_tolerance():
    import torch
    import paper_2412_04595_amd as sog
    name = "layered_2e5"
    print(f"[gpu] autotune {name} fp64", flush=True)
    x, q, box = workloads.named(name)
    xt = torch.from_numpy(x).cuda()
    qt = torch.from_numpy(q).cuda()
    s = sog.Solver(box, len(q), 1e-4, precision="fp64", on_device=True, autotune=True)
    info = _check_tuning(s)
    U, phi, F = s(xt, qt)
    s.close()
    d = np.loadtxt(os.path.join(HERE, "golden", f"{name}_targets.txt"), comments="#")
    idx, rphi, rgrad = d[:, 0].astype(np.int64), d[:, 1], d[:, 2:5]
    phi, F = phi.cpu().numpy(), F.cpu().numpy()
    rF = -q[idx, None] * rgrad
    ephi = np.max(np.abs(phi[idx] - rphi)) / np.max(np.abs(rphi))
    eF = np.max(np.abs(F[idx] - rF)) / np.max(np.abs(rF))
    print(f"    rc {info['rc']:.3f} m {info['m']}: phi {ephi:.2e} F {eF:.2e}", flush=True)
    assert ephi < 1e-4 and eF < 1e-4


def test_autotuned_plan_matches_oracle():
    import paper_2412_04595_amd as sog
    from oracle import fast
    x, q = workloads.uniform(1000, (20.0, 20.0, 20.0), 1)
    box = (20.0, 20.0, 20.0)
    print("[gpu] autotune Sec. 5.1 box fp64 tol 1e-6", flush=True)
    s = sog.Solver(box, 1000, 1e-6, precision="fp64", autotune=True)
    info = _check_tuning(s)
    pp, gp = s.parts(x, q)
    s.close()
    ref = fast.solve(x, q, box, oracle_params_from_info(info), parts=True)
    for k, part in enumerate(("near", "mid", "long")):
        rp, rg = ref["phi_" + part], ref["grad_" + part]
        if np.max(np.abs(rp)) == 0:
            continue
        ep = np.max(np.abs(pp[k] - rp)) / np.max(np.abs(rp))
        eg = np.max(np.abs(gp[k] - rg)) / np.max(np.abs(rg))
        print(f"    {part}: phi {ep:.2e} grad {eg:.2e}", flush=True)
        assert ep < 1e-12 and eg < 1e-12


def test_autotune_refuses_static_workspace():
    import paper_2412_04595_amd as sog
    import paper_2412_04595_amd._lib as L
    with pytest.raises(sog.SogError) as e:
        sog.Solver((20.0, 20.0, 20.0), 1000, 1e-6, autotune=True, static_workspace=True)
    assert e.value.status == L.SOG_ERR_INVALID_ARG
