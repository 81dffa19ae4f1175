"""The differentiable binding (paper_2412_04595_amd.autograd) against central finite
differences of the library's own operator (FP64), on a small two-layer system: gradients
in x and q of L = U + c.phi for a random cotangent c (one extra solve with c as charges),
and dU/dx = -F of sog_energy_potential_force."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BOX = (24.0, 24.0, 12.0)
N = 400


def _system(seed=11):
    rng = np.random.default_rng(seed)
    x = np.empty((N, 3))
    x[:, :2] = rng.random((N, 2)) * BOX[0]
    z = np.concatenate([rng.normal(2.5, 1.0, N // 2), rng.normal(9.5, 1.0, N - N // 2)])
    x[:, 2] = np.clip(z, 0.0, BOX[2])
    q = np.ones(N)
    q[N // 2:] = -1.0
    rng.shuffle(q)
    return x, q


def test_gradients_match_finite_differences():
    import torch
    from paper_2412_04595_amd.autograd import Differentiable
    print("[gpu] autograd FD check", flush=True)
    xn, qn = _system()
    D = Differentiable(BOX, N, 1e-8, precision="fp64")
    x = torch.from_numpy(xn).cuda().requires_grad_()
    q = torch.from_numpy(qn).cuda().requires_grad_()
    c = torch.from_numpy(np.random.default_rng(12).normal(size=N)).cuda()
    U, phi, _ = D(x, q)
    dx, dq = torch.autograd.grad(U + (c * phi).sum(), (x, q))
    dx, dq = dx.cpu().numpy(), dq.cpu().numpy()

    def loss(xv, qv):
        U1, phi1, _ = D.adjoint.potential_gradient(torch.from_numpy(xv).cuda(), torch.from_numpy(qv).cuda())
        return U1 + float((c * phi1).sum())

    rng = np.random.default_rng(13)
    h = 1e-4
    err_x = 0.0
    for i in rng.choice(N, 32, replace=False):
        for d in range(3):
            xp, xm = xn.copy(), xn.copy()
            xp[i, d] += h
            xm[i, d] -= h
            fd = (loss(xp, qn) - loss(xm, qn)) / (2 * h)
            err_x = max(err_x, abs(fd - dx[i, d]))
    err_q = 0.0
    for j in rng.choice(N, 32, replace=False):
        qp, qm = qn.copy(), qn.copy()
        qp[j] += h
        qm[j] -= h
        fd = (loss(xn, qp) - loss(xn, qm)) / (2 * h)
        err_q = max(err_q, abs(fd - dq[j]))
    sx, sq = np.max(np.abs(dx)), np.max(np.abs(dq))
    print(f"    dL/dx: max |FD - autograd| / max |dL/dx| = {err_x / sx:.2e};  dL/dq: {err_q / sq:.2e}", flush=True)
    assert err_x <= 1e-4 * sx
    assert err_q <= 1e-7 * sq  # L is quadratic in q: central differences are exact up to rounding
    D.close()


def test_energy_gradient_is_minus_force():
    import torch
    import paper_2412_04595_amd as sog
    from paper_2412_04595_amd.autograd import Differentiable
    print("[gpu] autograd dU/dx = -F", flush=True)
    xn, qn = _system(21)
    D = Differentiable(BOX, N, 1e-6, precision="fp64")
    x = torch.from_numpy(xn).cuda().requires_grad_()
    q = torch.from_numpy(qn).cuda()
    U, phi, _ = D(x, q)
    (dx,) = torch.autograd.grad(U, (x,))
    s = sog.Solver(BOX, N, 1e-6, precision="fp64", on_device=True)
    U2, phi2, F = s(x.detach(), q)
    torch.cuda.synchronize()
    assert abs(float(U.detach()) - U2) <= 1e-12 * abs(U2)
    assert torch.allclose(dx, -F, rtol=0, atol=1e-12 * float(F.abs().max()))
    s.close()
    D.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cube_small", "slab_mid_fft", "confined_taylor"])
def test_cotangent_solve_matches_oracle(name, precision):
    """The adjoint solve (charges = a cotangent of the potentials, not neutral: a plan
    without input checks) against the oracle's fast method run with the same charges and
    parameters, element by element: A g and grad (A g) for random normal g.  The oracle
    needs no neutrality either (every k = 0 constant is left out on both sides), so this
    pins the operator the backward pass applies.  Tolerances as the parity tests."""
    import torch
    import paper_2412_04595_amd as sog
    import workloads
    from oracle import fast
    from tests._cases import CASES, gpu_params, oracle_params
    c = CASES[name]
    x, _q = workloads.uniform(c["N"], c["box"], c["seed"])
    g = np.random.default_rng(99).normal(size=c["N"])
    print(f"[gpu] cotangent solve {name} {precision}: sum g = {g.sum():.3f}", flush=True)
    ref = fast.solve(x, g, c["box"], oracle_params(c))
    s = sog.Solver(c["box"], c["N"], 1e-6 if precision == "fp64" else 1e-4, precision=precision, on_device=True,
                   check_inputs=False, params=gpu_params(c))
    _U, phi, grad = s.potential_gradient(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    s.close()
    phi, grad = phi.cpu().numpy(), grad.cpu().numpy()
    ep = np.max(np.abs(phi - ref["phi"])) / np.max(np.abs(ref["phi"]))
    eg = np.max(np.abs(grad - ref["grad"])) / np.max(np.abs(ref["grad"]))
    print(f"    phi {ep:.2e} grad {eg:.2e}", flush=True)
    tp, tg = (1e-12, 1e-12) if precision == "fp64" else (3e-5, 1e-4)
    assert ep < tp and eg < tg


def test_layered_2e5_autograd():
    """The differentiation workload: N = 2e5 in 150 x 150 x 60, two Gaussian layers with
    enriched charges (a large z dipole), tolerance 1e-4.
    * FP32-bulk autograd forces dU/dx against the oracle's forces -q grad phi at the sampled
      targets of tests/golden/layered_2e5_targets.txt (SOG-direct): relative L-inf <= 1e-4;
    * FP64 autograd dL/dx for L = U + c.phi against central differences (h = 1e-4) of the
      FP64 operator at 3 x 32 random coordinates (float32 energies are too noisy for
      differences at h = 1e-4), and FP32-bulk autograd against the same differences: 1e-4
      of max |dL/dx|."""
    import os
    import torch
    import workloads
    from paper_2412_04595_amd.autograd import Differentiable
    name = "layered_2e5"
    xn, qn, box = workloads.named(name)
    N = len(qn)
    print(f"[gpu] autograd {name}", flush=True)
    d = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", f"{name}_targets.txt"), comments="#")
    idx, rgrad = d[:, 0].astype(np.int64), d[:, 2:5]
    rF = -qn[idx, None] * rgrad
    c = torch.from_numpy(np.random.default_rng(77).normal(size=N) / np.sqrt(N)).cuda()
    grads = {}
    for prec in ("fp32", "fp64"):
        D = Differentiable(box, N, 1e-4, precision=prec)
        x = torch.from_numpy(xn).cuda().requires_grad_()
        q = torch.from_numpy(qn).cuda()
        U, phi, _ = D(x, q)
        (dU,) = torch.autograd.grad(U, (x,), retain_graph=True)
        (dL,) = torch.autograd.grad(U + (c * phi).sum(), (x,))
        grads[prec] = dL.cpu().numpy()
        eF = np.max(np.abs(-dU.cpu().numpy()[idx] - rF)) / np.max(np.abs(rF))
        print(f"    {prec}: forces -dU/dx vs the oracle's at {idx.size} targets: {eF:.2e}", flush=True)
        assert eF < 1e-4
        if prec == "fp64":
            def loss(xv):
                U1, phi1, _ = D.adjoint.potential_gradient(torch.from_numpy(xv).cuda(), q)
                return U1 + float((c * phi1).sum())
            rng = np.random.default_rng(78)
            pick = rng.choice(N, 32, replace=False)
            fd = np.zeros((32, 3))
            h = 1e-4
            for a, i in enumerate(pick):
                for k in range(3):
                    xp, xm = xn.copy(), xn.copy()
                    xp[i, k] += h
                    xm[i, k] -= h
                    fd[a, k] = (loss(xp) - loss(xm)) / (2 * h)
        D.close()
    s = np.max(np.abs(grads["fp64"]))
    e64 = np.max(np.abs(grads["fp64"][pick] - fd)) / s
    e32 = np.max(np.abs(grads["fp32"][pick] - fd)) / s
    print(f"    dL/dx vs central differences of the FP64 operator: fp64 {e64:.2e} fp32 {e32:.2e}", flush=True)
    assert e64 < 1e-4 and e32 < 1e-4
