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
