"""Field synthesis by gradient descent through the full 3PCF (forward + hand-written adjoint).

Given target sums Z* (the raw full-3PCF sums of Alg. 5 for some field), adjust a density
field delta so that its sums match: minimise L = sum (Z(delta) - Z*)^2 / sum Z*^2 with Adam.
Z(delta) and dL/d delta run in the library (sb_forward / sb_backward through ZetaFn); the
optimiser update is a plain torch elementwise step on the device.
"""
from __future__ import annotations

import torch

from .api import Plan, ZetaFn


def synthesize(plan: Plan, target, init, steps: int = 200, lr: float = 0.05, history_every: int = 1):
    """Run `steps` Adam steps from `init` (a float32 device tensor of the plan's one field
    shape) towards the float64 target sums `target` (shape (lmax+1, nb, nb)).

    Returns (delta, losses): the final field and the loss before each recorded step
    (every `history_every` steps, plus the loss of the final field)."""
    if plan.ndim != 3 or plan.npcf != 3 or len(plan.shapes) != 1:
        raise ValueError("synthesis needs a one-field full-3PCF plan")
    target = target.to(device=plan.device, dtype=torch.float64)
    den = torch.sum(target * target)
    delta = init.detach().to(device=plan.device, dtype=torch.float32).clone().requires_grad_(True)
    opt = torch.optim.Adam([delta], lr=lr)
    losses = []
    for it in range(steps):
        opt.zero_grad(set_to_none=True)
        z = ZetaFn.apply(delta, plan)
        loss = torch.sum((z - target) ** 2) / den
        loss.backward()
        if it % history_every == 0:
            losses.append(float(loss.detach()))
        opt.step()
    with torch.no_grad():
        z = plan.forward([delta.detach()])[0]
        losses.append(float(torch.sum((z - target) ** 2) / den))
    return delta.detach(), losses
