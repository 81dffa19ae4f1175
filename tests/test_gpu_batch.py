"""Batched independent systems (sog_batch_plan / sog_batch_energy_potential_force) on the
GPU: one call launches one captured HIP graph whose kernels each run for every system of
a group of systems that share kernels.

* the 256-system batch (N log-uniform in [500, 20000], Lz/Lx in {1/8, 1, 8}) in float32:
  sampled targets of twelve systems against tests/golden/batch_256_targets.txt (the
  oracle's exact SOG sum per system, written by tests/golden/make_golden.py), and per
  system U_s = 1/2 sum q phi over that system's particles;
* a small batch in float64 against one plan per system (the same kernels; only the order
  of the gridding's atomic additions differs), over several graph replays with new
  inputs and eager device work in between, in device and host pointer modes;
* the input check names the failing system (non-neutral, z out of the box, non-finite).
"""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-4


def _golden():
    d = np.loadtxt(os.path.join(HERE, "golden", "batch_256_targets.txt"), comments="#")
    return d[:, 0].astype(np.int64), d[:, 1].astype(np.int64), d[:, 2], d[:, 3:6]


def test_batch_256_sampled_targets():
    import torch
    import paper_2412_04595_amd as sog
    print("[gpu] batch of 256 systems, fp32", flush=True)
    x, q, boxes, ns = workloads.batch()
    b = sog.BatchSolver(boxes, ns, TOL, precision="fp32", on_device=True, check_inputs=True)
    groups, launches = b.graph_info()
    print(f"    {groups} groups of systems, {launches} kernel launches per call", flush=True)
    assert launches <= 40 * groups and groups <= 16
    U, phi, F = b(torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    U, phi, F = U.cpu().numpy(), phi.cpu().numpy(), F.cpu().numpy()
    off = b.offsets
    sysi, idx, rphi, rgrad = _golden()
    worst = 0.0
    for s in sorted(set(sysi.tolist())):
        m = sysi == s
        g = off[s] + idx[m]
        rF = -q[g, None] * rgrad[m]
        ephi = np.max(np.abs(phi[g] - rphi[m])) / np.max(np.abs(rphi[m]))
        eF = np.max(np.abs(F[g] - rF)) / np.max(np.abs(rF))
        info = b.info(int(s))
        print(f"    system {s}: N={ns[s]} box={tuple(round(v, 2) for v in boxes[s])} m={info['m']} "
              f"long={info['long_form']}: phi {ephi:.2e} F {eF:.2e}", flush=True)
        worst = max(worst, ephi, eF)
        assert ephi < TOL and eF < TOL, s
    for s in range(len(ns)):
        qs, ps = q[off[s]:off[s + 1]], phi[off[s]:off[s + 1]]
        assert abs(U[s] - 0.5 * float(qs @ ps)) <= 1e-10 * float(np.sum(np.abs(qs * ps))), s
    assert np.all(np.isfinite(F))
    b.close()
    print(f"    worst sampled error {worst:.2e}", flush=True)


def _small_batch():
    specs = [workloads.batch_specs()[s] for s in (136, 82, 144, 93, 32, 86)]
    x, q, boxes, ns = workloads.batch(specs)
    return x, q, boxes, ns


def _single(sog, boxes, ns, x, q, precision, off):
    phis, Fs, Us = [], [], []
    for s in range(len(ns)):
        p = sog.Solver(boxes[s], ns[s], TOL, precision=precision)
        U, phi, F = p(x[off[s]:off[s + 1]], q[off[s]:off[s + 1]])
        p.close()
        phis.append(phi)
        Fs.append(F)
        Us.append(U)
    return np.array(Us), np.concatenate(phis), np.concatenate(Fs)


def test_batch_equals_one_plan_per_system_over_replays():
    import torch
    import paper_2412_04595_amd as sog
    print("[gpu] small batch fp64 vs single plans, 3 replays", flush=True)
    x, q, boxes, ns = _small_batch()
    b = sog.BatchSolver(boxes, ns, TOL, precision="fp64", on_device=True, check_inputs=True)
    off = b.offsets
    rng = np.random.default_rng(7)
    for rep in range(3):
        # new positions each replay: a random shift of each system in x, y (wrapped by the
        # solver) and a fresh permutation of the charges within each system
        xr, qr = x.copy(), q.copy()
        for s in range(len(ns)):
            sl = slice(off[s], off[s + 1])
            xr[sl, :2] += rng.random(2) * np.asarray(boxes[s][:2])
            qr[sl] = rng.permutation(qr[sl])
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        U, phi, F = b(torch.from_numpy(xr).cuda(), torch.from_numpy(qr).cuda())
        torch.cuda.synchronize()
        U, phi, F = U.cpu().numpy(), phi.cpu().numpy(), F.cpu().numpy()
        rU, rphi, rF = _single(sog, boxes, ns, xr, qr, "fp64", off)
        for s in range(len(ns)):
            sl = slice(off[s], off[s + 1])
            ephi = np.max(np.abs(phi[sl] - rphi[sl])) / np.max(np.abs(rphi[sl]))
            eF = np.max(np.abs(F[sl] - rF[sl])) / np.max(np.abs(rF[sl]))
            assert ephi < 1e-11 and eF < 1e-11, (rep, s, ephi, eF)
            assert abs(U[s] - rU[s]) <= 1e-11 * abs(rU[s]), (rep, s)
        print(f"    replay {rep}: ok ({float(junk):.1f})", flush=True)
    b.close()


def test_batch_host_pointers_match_device_pointers():
    import torch
    import paper_2412_04595_amd as sog
    print("[gpu] small batch fp32, host vs device pointers", flush=True)
    x, q, boxes, ns = _small_batch()
    bd = sog.BatchSolver(boxes, ns, TOL, precision="fp32", on_device=True)
    Ud, pd, Fd = bd(torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    bh = sog.BatchSolver(boxes, ns, TOL, precision="fp32", on_device=False)
    Uh, ph, Fh = bh(x, q)
    # float atomics in the gridding make the two runs differ by float32 rounding only
    assert np.max(np.abs(ph - pd.cpu().numpy())) <= 1e-5 * np.max(np.abs(ph))
    assert np.max(np.abs(Fh - Fd.cpu().numpy())) <= 1e-5 * np.max(np.abs(Fh))
    assert np.allclose(Uh, Ud.cpu().numpy(), rtol=1e-5, atol=0)
    bd.close()
    bh.close()


@pytest.mark.parametrize("case, status", [("charge", 2), ("z", 3), ("nan", 1)])
def test_batch_input_check_names_the_system(case, status):
    import paper_2412_04595_amd as sog
    print(f"[gpu] batch input check: {case}", flush=True)
    x, q, boxes, ns = _small_batch()
    b = sog.BatchSolver(boxes, ns, TOL, precision="fp32", on_device=False, check_inputs=True)
    off = b.offsets
    s = 3
    if case == "charge":
        q[off[s]] += 0.5
    elif case == "z":
        x[off[s] + 1, 2] = boxes[s][2] + 0.25
    else:
        x[off[s] + 2, 0] = np.nan
    with pytest.raises(sog.SogError) as ei:
        b(x, q)
    assert ei.value.status == status
    assert f"system {s}" in str(ei.value)
    b.close()
