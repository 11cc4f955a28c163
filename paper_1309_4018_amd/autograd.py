"""Differentiable solvation energy (torch.autograd.Function).

Forward: the treecode BEM solve of libpbtc for the given charge values.
Backward: libpbtc's adjoint solve (GMRES on the transposed operator), which
returns dE/dq for every charge together with dE/dkappa and dE/deps per
region; the latter two are kept on the plan (``plan.last_param_grads``).
"""

from __future__ import annotations

import numpy as np
import torch


class SolvationEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, plan):
        plan.set_charge_values(q.detach().to("cpu", torch.float64).numpy())
        res = plan.solve()
        ctx.plan = plan
        ctx.q_device = q.device
        return torch.tensor(res["energy_kJmol"], dtype=torch.float64, device=q.device)

    @staticmethod
    def backward(ctx, g):
        dq, dk, de = ctx.plan.backward(float(g))
        ctx.plan.last_param_grads = {"dE_dkappa": dk, "dE_deps": de}
        return torch.from_numpy(np.asarray(dq)).to(ctx.q_device), None


def solvation_energy(q, plan):
    """Energy [kJ/mol] of charge values ``q`` (tensor, requires_grad allowed)."""
    return SolvationEnergy.apply(q, plan)
