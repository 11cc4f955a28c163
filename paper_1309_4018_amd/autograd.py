"""Differentiable solvation energy (torch.autograd.Function).

Forward: the treecode BEM solve of libpbtc for the given charge values.
Backward: libpbtc's adjoint solve (GMRES on the transposed operator), which
returns dE/dq for every charge together with dE/dkappa and dE/deps per
region; the latter two are kept on the plan (``plan.last_param_grads``).

The adjoint needs the forward solution of the same charges.  Each forward
records the charge values it solved for and the plan's solve counter; when
the plan has solved for other charges since (two energies of one plan in one
graph, or a solve in between), backward solves for the recorded charges
again before the adjoint step.
"""

from __future__ import annotations

import numpy as np
import torch


class SolvationEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, plan):
        qh = q.detach().to("cpu", torch.float64).numpy().copy()
        plan.set_charge_values(qh)
        res = plan.solve()
        ctx.plan = plan
        ctx.q_host = qh
        ctx.solve_id = plan.solve_count
        ctx.q_device = q.device
        return torch.tensor(res["energy_kJmol"], dtype=torch.float64, device=q.device)

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        if plan.solve_count != ctx.solve_id:
            plan.set_charge_values(ctx.q_host)
            plan.solve()
        dq, dk, de = plan.backward(float(g))
        plan.last_param_grads = {"dE_dkappa": dk, "dE_deps": de}
        return torch.from_numpy(np.asarray(dq)).to(ctx.q_device), None


def solvation_energy(q, plan):
    """Energy [kJ/mol] of charge values ``q`` (tensor, requires_grad allowed)."""
    return SolvationEnergy.apply(q, plan)
