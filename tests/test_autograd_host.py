"""The adjoint algebra of paper_2412_04595_amd.autograd, on the CPU: the autograd function
driven by a dense stand-in solver with the same contract (phi = A(x) q, A symmetric, and
grad phi at the particles) must pass torch.autograd.gradcheck for U and phi in x and q.
The library's own operator is checked against finite differences by the GPU test."""
import torch

from paper_2412_04595_amd.autograd import _SogFunction


class DenseSolver:
    """phi_i = sum_j K(|x_i - x_j|) q_j + c q_i with a smooth symmetric K (the self term c
    like the SOG self term); grad_i = sum_{j != i} K'(r) (x_i - x_j)/r q_j."""

    c = -0.7

    def potential_gradient(self, x, q, energy=True):
        d = x[:, None, :] - x[None, :, :]
        r2 = (d * d).sum(-1)
        K = torch.exp(-r2 / 2) + 0.3 * torch.exp(-r2 / 5)
        dK = -torch.exp(-r2 / 2) - 0.3 * 2 / 5 * torch.exp(-r2 / 5)  # (dK/dr)/r
        eye = torch.eye(len(q), dtype=x.dtype)
        K = K * (1 - eye)
        dK = dK * (1 - eye)
        phi = K @ q + self.c * q
        grad = (dK[:, :, None] * d * q[None, :, None]).sum(1)
        U = float(0.5 * (q * phi).sum()) if energy else None
        return U, phi, grad


def test_adjoint_matches_finite_differences():
    g = torch.Generator().manual_seed(7)
    n = 9
    x = (torch.rand(n, 3, generator=g, dtype=torch.float64) * 3).requires_grad_()
    q = torch.randn(n, generator=g, dtype=torch.float64).requires_grad_()
    s = DenseSolver()
    f = lambda x, q: _SogFunction.apply(x, q, s, s)[:2]  # U and phi
    assert torch.autograd.gradcheck(f, (x, q), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_energy_gradient_is_minus_force_and_potential():
    g = torch.Generator().manual_seed(8)
    n = 7
    x = (torch.rand(n, 3, generator=g, dtype=torch.float64) * 3).requires_grad_()
    q = torch.randn(n, generator=g, dtype=torch.float64).requires_grad_()
    s = DenseSolver()
    U, phi, grad = _SogFunction.apply(x, q, s, s)
    dx, dq = torch.autograd.grad(U, (x, q))
    assert torch.allclose(dx, q.detach()[:, None] * grad, rtol=1e-12, atol=1e-12)  # dU/dx_i = -F_i
    assert torch.allclose(dq, phi.detach(), rtol=1e-12, atol=1e-12)               # dU/dq = phi
