"""torch.autograd wrapper of the canonical density matrix and its adjoint.

forward:  P0 = canonical Fermi-operator expansion of H0 (Algorithm 1, order 0),
          computed by dmpt_mu_newton;
backward: dL/dH0 = dmpt_backward(H0, ..., Abar = dL/dP0), the hand-written
          reverse sweep of the recursion with mu0 following H0 through
          Tr P0 = Ne.

Only the H0 input is differentiable; the gradient is symmetric, so it is
exact for symmetric perturbations of H0.
"""
import torch


class DMPTFermi(torch.autograd.Function):
    """P0 = DMPTFermi.apply(H0, beta, Ne, n, context)."""

    @staticmethod
    def forward(ctx, H0, beta, Ne, n, lib_ctx):
        H0 = H0.contiguous()
        P0, _, _, mu, _ = lib_ctx.mu_newton(H0, beta=beta, Ne=Ne, n=n, order=0)
        ctx.save_for_backward(H0)
        ctx.args = (float(beta), float(Ne), int(n), lib_ctx, float(mu[0]))
        return P0

    @staticmethod
    def backward(ctx, grad_out):
        (H0,) = ctx.saved_tensors
        beta, Ne, n, lib_ctx, mu0 = ctx.args
        G, _ = lib_ctx.backward(H0, beta, Ne, n, grad_out.contiguous().to(torch.float64), mu0=mu0)
        return G, None, None, None, None


def fermi_canonical(H0, beta, Ne, n, lib_ctx):
    """Differentiable canonical density matrix of H0 (see DMPTFermi)."""
    return DMPTFermi.apply(H0, beta, Ne, n, lib_ctx)
