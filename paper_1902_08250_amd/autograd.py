"""torch.autograd.Function around the GPU apply.

Forward: u = G q (lmfmm_apply).  Backward for a real loss with upstream
gradient grad_u (torch's convention for complex tensors, dL/dRe + i dL/dIm):
  * grad_q = conj(G^T conj(grad_u))   (lmfmm_apply_adjoint)
  * grad_src, grad_tgt = coordinate gradients of L = Re sum conj(grad_u) u
    (lmfmm_grad_coords).
Nothing from the forward pass is stored beyond the inputs: the tree and the
expansions are rebuilt by the backward calls.
"""
import torch


class LMFMMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, src, q, tgt):
        ctx.plan = plan
        ctx.save_for_backward(src, q, tgt)
        return plan.apply(src.contiguous(), q.contiguous(), tgt.contiguous())

    @staticmethod
    def backward(ctx, grad_u):
        src, q, tgt = ctx.saved_tensors
        plan = ctx.plan
        w = grad_u.conj().resolve_conj().contiguous()
        grad_src = grad_q = grad_tgt = None
        if ctx.needs_input_grad[2]:
            grad_q = plan.apply_adjoint(src, tgt, w).conj().resolve_conj()
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[3]:
            ds, dt = plan.grad_coords(src, q.contiguous(), tgt, w)
            grad_src = ds if ctx.needs_input_grad[1] else None
            grad_tgt = dt if ctx.needs_input_grad[3] else None
        return None, grad_src, grad_q, grad_tgt


def lmfmm_apply(plan, src, q, tgt):
    """Differentiable u = G q (see LMFMMFunction)."""
    return LMFMMFunction.apply(plan, src, q, tgt)
