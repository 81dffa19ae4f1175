"""Differentiable energy and potentials for PyTorch (torch.autograd) on the library's solves.

The method computes phi = A(x) q with A(x) symmetric (the SOG operator of eqs. splitting
and phisplit as discretised: the gathers use the same window and Chebyshev basis as the
gridding and anterpolation, and the multipliers are real and even), U = q.phi / 2, and the
gradient of the potential at the particles, grad phi(x_i) (Sec. 2.1: F_i = -q_i grad phi(x_i)).
For a loss L(U, phi) with cotangents gU and gphi:

    dL/dq   = gU phi + A(x) gphi
    dL/dx_i = (gU q_i + gphi_i) grad phi_q(x_i) + q_i grad phi_g(x_i),   phi_g = A(x) gphi,

so the adjoint of every step (gridding, FFTs, scaling, gathering, anterpolation and
interpolation, near-field pairs) is one more library call with the cotangent of the
potentials as charges.  Those charges need not be neutral; that call runs on a plan made
without the input checks (the sum of the charges then multiplies only the k = 0 constant,
which every call leaves out, so the operator stays symmetric).  All solves run in the HIP
library; the backward combines their outputs with elementwise device ops.
"""
import torch

from . import Solver


class _SogFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, q, solver, adjoint):
        U, phi, grad = solver.potential_gradient(x.detach(), q.detach())
        ctx.adjoint = adjoint
        ctx.mark_non_differentiable(grad)
        ctx.save_for_backward(x, q, phi, grad)
        return torch.tensor(U, dtype=torch.float64, device=x.device), phi, grad

    @staticmethod
    def backward(ctx, gU, gphi, _ggrad):
        x, q, phi, grad = ctx.saved_tensors
        gu = gU if gU is not None else torch.zeros((), dtype=torch.float64, device=x.device)
        w = gu * q                 # weight of grad phi_q(x_i) from the energy
        dq = gu * phi
        dx_extra = None
        if gphi is not None and bool(torch.any(gphi != 0)):
            g = gphi.detach().contiguous()
            _, phi_g, grad_g = ctx.adjoint.potential_gradient(x.detach(), g, energy=False)
            dq = dq + phi_g
            w = w + g
            dx_extra = q[:, None] * grad_g
        dx = w[:, None] * grad
        if dx_extra is not None:
            dx = dx + dx_extra
        return dx, dq, None, None


class Differentiable:
    """U, phi and grad phi for N particles in a box at tolerance tol, differentiable in x and q.

    Inputs are float64 torch tensors on the GPU; the forward solve checks the inputs
    (neutral charges, z in [0, Lz]) like any call, the adjoint solve does not."""

    def __init__(self, box, n, tol, precision="fp64", device=0, params=None):
        self.solver = Solver(box, n, tol, precision=precision, device=device, on_device=True, check_inputs=True,
                             params=params)
        self.adjoint = Solver(box, n, tol, precision=precision, device=device, on_device=True, check_inputs=False,
                              params=params)

    def __call__(self, x, q):
        """(U, phi, grad): U and phi carry gradients to x and q; grad (= grad phi at x_i) does not."""
        return _SogFunction.apply(x, q, self.solver, self.adjoint)

    def close(self):
        self.solver.close()
        self.adjoint.close()
