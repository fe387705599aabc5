"""torch.autograd wrapper of n LB steps: the wetting objective as a differentiable function of the
per-wall-node wettability G_w, with the library's hand-written adjoint as the backward pass."""
from __future__ import annotations

import torch


class LBMRun(torch.autograd.Function):
    """L = w_centroid * y_c + w_wet * l_w of the state after `nsteps` steps from `state0` (a
    blob of Sim.save_state), as a function of gw, a (2, nx) float64 tensor. Forward runs the
    checkpointed forward (every K steps); backward runs the adjoint with per-segment
    recomputation and returns dL/dG_w."""

    @staticmethod
    def forward(ctx, gw, sim, state0, nsteps, K, w_centroid, w_wet):
        sim.load_state(state0)
        sim.set_gw(gw.detach().cpu().numpy())
        ws = sim.adjoint_workspace(nsteps, K)
        sim.forward_ckpt(nsteps, K, ws)
        L = sim.loss(w_centroid, w_wet)
        ctx.sim, ctx.ws, ctx.args = sim, ws, (nsteps, K, w_centroid, w_wet)
        return torch.tensor(L, dtype=torch.float64, device=gw.device)

    @staticmethod
    def backward(ctx, gL):
        nsteps, K, wc, ww = ctx.args
        g = ctx.sim.backward(nsteps, K, ctx.ws, wc, ww)
        return g.to(gL.device) * gL, None, None, None, None, None, None


def lbm_run(gw, sim, state0, nsteps, K, w_centroid=1.0, w_wet=1.0):
    """Differentiable wetting objective (see LBMRun)."""
    return LBMRun.apply(gw, sim, state0, nsteps, K, w_centroid, w_wet)
