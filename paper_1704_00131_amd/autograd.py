"""log det(1 + B(beta,0)) of a continuous HS field as a differentiable torch
function.  Forward: the stabilised log-determinant of the UDV chain.
Backward: the adjoint pass of the library (d log det / d phi_{i,tau} =
coupling (1 - G(tau)_ii), recomputed from the stored checkpoints), scaled by
the incoming gradient.  Both run in the HIP library; this module only moves
the field into the chain's buffer."""
import torch


class LogDet(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, chain):
        chain.load_field(phi).init()
        ctx.chain = chain
        ctx.save_for_backward(phi.detach().clone())
        return torch.tensor(chain.logdet(), dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, grad_out):
        (phi,) = ctx.saved_tensors
        chain = ctx.chain
        chain.load_field(phi).init()
        g, _ = chain.grad_logdet()
        return grad_out * g, None


def logdet(phi, chain):
    """Differentiable log|det(1 + B(beta,0))| of the field phi ([L, N], float64,
    on the chain's device) for the chain's model (one colour)."""
    return LogDet.apply(phi, chain)
