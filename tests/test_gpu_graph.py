"""The graph-replayed call (the default; sog_options.eager = 0): the first
sog_energy_potential_force of a plan captures its kernels into a HIP graph, later calls
replay it.  Each case replays the graph several times on new inputs, with eager work of
the program (torch kernels, an eager plan's call, synchronisations) between the replays,
and checks every replay against the eager plan's result on the same inputs: float64
within 1e-12 of the largest value, float32 within 3e-6 (the atomics' summation order).
Also: host pointers, omitted outputs, and input errors reported after the capture."""
import numpy as np
import pytest

import workloads
from tests._cases import CASES, gpu_params

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 3e-6}


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cube_small", "slab_mid_fft", "confined_taylor", "clustered"])
def test_graph_replays_match_eager_calls(name, precision):
    import torch
    import paper_2412_04595_amd as sog
    c = CASES[name]
    x, q = getattr(workloads, c.get("gen", "uniform"))(c["N"], c["box"], c["seed"], **c.get("gen_args", {}))
    print(f"[gpu] graph replays {name} {precision}", flush=True)
    tol = 1e-6 if precision == "fp64" else 1e-4
    g = sog.Solver(c["box"], c["N"], tol, precision=precision, params=gpu_params(c), on_device=True)
    e = sog.Solver(c["box"], c["N"], tol, precision=precision, params=gpu_params(c), on_device=True, eager=True)
    rng = np.random.default_rng(5)
    for rep in range(4):
        xs = x.copy()
        xs[:, :2] += rng.uniform(-0.3, 0.3, size=(len(q), 2))  # x, y wrap; z stays in the box
        qs = q * (1.0 if rep % 2 == 0 else -1.0)
        xt = torch.from_numpy(xs).cuda()
        qt = torch.from_numpy(qs).cuda()
        junk = torch.randn(1 << 20, device="cuda").cumsum(0)  # the program's own eager work
        Ue, pe, Fe = e(xt, qt)
        torch.cuda.synchronize()
        Ug, pg, Fg = g(xt, qt)
        junk = junk * 2
        torch.cuda.synchronize()
        ep, eF = _rel(pg.cpu(), pe.cpu()), _rel(Fg.cpu(), Fe.cpu())
        eU = abs(Ug - Ue) / abs(Ue)
        print(f"    replay {rep}: phi {ep:.1e} F {eF:.1e} U {eU:.1e}", flush=True)
        assert ep < TOL[precision] and eF < TOL[precision] and eU < TOL[precision]
    g.close()
    e.close()


def test_graph_host_pointers_and_partial_outputs():
    import paper_2412_04595_amd as sog
    import paper_2412_04595_amd._lib as L
    c = CASES["cube_small"]
    x, q = workloads.uniform(c["N"], c["box"], c["seed"])
    print("[gpu] graph host pointers", flush=True)
    g = sog.Solver(c["box"], c["N"], 1e-6, params=gpu_params(c))
    e = sog.Solver(c["box"], c["N"], 1e-6, params=gpu_params(c), eager=True)
    Ue, pe, Fe = e(x, q)
    for _ in range(3):
        Ug, pg, Fg = g(x, q)
        assert _rel(pg, pe) < 1e-12 and _rel(Fg, Fe) < 1e-12 and abs(Ug - Ue) < 1e-12 * abs(Ue)
    U1, p1, F1 = g(x, q, energy=True, potential=False, forces=False)
    assert p1 is None and F1 is None and abs(U1 - Ue) < 1e-12 * abs(Ue)
    _, p2, F2 = g(x, q, energy=False, potential=True, forces=False)
    assert _rel(p2, pe) < 1e-12
    # an input error after the capture is reported, and the plan keeps working
    bad = x.copy()
    bad[3, 2] = c["box"][2] + 1.0
    with pytest.raises(sog.SogError) as err:
        g(bad, q)
    assert err.value.status == L.SOG_ERR_OUT_OF_BOX
    Ug, pg, Fg = g(x, q)
    assert _rel(pg, pe) < 1e-12
    g.close()
    e.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_calls_queued_without_host_reads(precision):
    """Calls queued back to back with every output left on the device (the energy as a
    one-element tensor: no host read between calls, as the benchmark times them), on
    different inputs, each checked afterwards against an eager plan's call on its inputs."""
    import torch
    import paper_2412_04595_amd as sog
    c = CASES["cube_small"]
    x, q = workloads.uniform(c["N"], c["box"], c["seed"])
    print(f"[gpu] graph calls queued {precision}", flush=True)
    tol = 1e-6 if precision == "fp64" else 1e-4
    g = sog.Solver(c["box"], c["N"], tol, precision=precision, params=gpu_params(c), on_device=True)
    e = sog.Solver(c["box"], c["N"], tol, precision=precision, params=gpu_params(c), on_device=True, eager=True)
    rng = np.random.default_rng(9)
    ins, outs = [], []
    for rep in range(5):
        xs = x.copy()
        xs[:, :2] += rng.uniform(-0.3, 0.3, size=(len(q), 2))
        qs = q * (1.0 if rep % 2 == 0 else -1.0)
        xt, qt = torch.from_numpy(xs).cuda(), torch.from_numpy(qs).cuda()
        ins.append((xt, qt))
        outs.append(g(xt, qt, energy_on_device=True))
    torch.cuda.synchronize()
    for rep, ((xt, qt), (Ug, pg, Fg)) in enumerate(zip(ins, outs)):
        assert isinstance(Ug, torch.Tensor) and Ug.is_cuda and Ug.numel() == 1
        Ue, pe, Fe = e(xt, qt)
        ep, eF = _rel(pg.cpu(), pe.cpu()), _rel(Fg.cpu(), Fe.cpu())
        eU = abs(float(Ug[0]) - Ue) / abs(Ue)
        print(f"    call {rep}: phi {ep:.1e} F {eF:.1e} U {eU:.1e}", flush=True)
        assert ep < TOL[precision] and eF < TOL[precision] and eU < TOL[precision]
    g.close()
    e.close()
