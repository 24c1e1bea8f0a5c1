"""torch.autograd.Function around the FMM energy and its adjoint.

    plan = Plan(p=8, precision="mixed")
    E = FMMEnergy.apply(pos, q, plan)          # (n_inst,) energies, E_k = 1/2 q^T A q
    E.sum().backward()                         # pos.grad, q.grad from fmm_backward

The forward runs fmm_build_tree, fmm_upward and fmm_evaluate on the plan; the
backward calls fmm_backward, the exact adjoint of the matrix A the FMM
applied.  The plan holds the forward state, so it must not be rebuilt
between the forward and the backward of one graph.
"""
import torch

from .fmm import Plan


class FMMEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, plan, offsets=None):
        if not isinstance(plan, Plan):
            raise TypeError("plan must be a paper_1203_0889_amd.fmm.Plan")
        plan.build_tree(pos.detach().contiguous(), q.detach().contiguous(), offsets)
        plan.upward()
        out = plan.evaluate(phi=False, field=False, force=False, energy=True)
        ctx.plan = plan
        return out["energy"]

    @staticmethod
    def backward(ctx, grad_energy):
        want_pos, want_q = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gp, gq = ctx.plan.backward(grad_energy.detach().to(torch.float64).contiguous(), want_pos, want_q)
        return gp, gq, None, None


def fmm_energy(pos, q, plan, offsets=None):
    """Energies of the instances (differentiable in pos and q)."""
    return FMMEnergy.apply(pos, q, plan, offsets)
