"""Differentiable MPS rollouts: torch.autograd.Function over the HIP
library's forward steps and hand-written adjoint kernels.

MPSRollout.apply(u0, nu, g, params, pos0, ptype, nsteps, K) runs nsteps
steps from (pos0, u0) with viscosity nu and body acceleration g, and returns
(pos_T, vel_T, flags_T, type_T).  The backward pass walks the steps in
reverse with checkpointing every K steps: the forward saves the state every K
steps; for each segment, in reverse, the checkpoint is restored, the segment
re-run saving each step's input state, and the steps are walked back with
mps_step_adjoint.  Gradients flow to u0, nu and g; neighbour lists,
free-surface flags, p-hat argmins and clamp masks of every step are frozen
at their forward values.  Device memory: (ceil(nsteps/K) + K) state slots.

Two-phase model (rho_i, nu_i given): the per-particle laminar viscosities
are nu_i + nu, so the gradient with respect to nu is that of a common shift
of all of them (pass nu = 0 for the derivative at nu_i).
"""
from __future__ import annotations

import math

import torch

from . import mps as _mps
from .workloads import FLUID

# device memory of the last rollout's library context (state, work arrays
# and tape), bytes
last_device_bytes = 0


class MPSRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, nu, g, params, pos0, ptype, nsteps, K, rho_i=None, nu_i=None):
        global last_device_bytes
        dim = int(params["dim"])
        gl = [float(x) for x in g.detach().cpu().tolist()] + [0.0] * (3 - dim)
        if nu_i is not None:
            prm = dict(params, g=gl)
            sim = _mps.MPS(prm, pos0, u0.detach(), ptype, rho_i=rho_i, nu_i=nu_i + float(nu))
        else:
            prm = dict(params, nu=float(nu), g=gl)
            sim = _mps.MPS(prm, pos0, u0.detach(), ptype, rho_i=rho_i)
        nseg = math.ceil(nsteps / K)
        sim.tape_alloc(nseg + K)
        last_device_bytes = sim.device_bytes()
        for s in range(nsteps):
            if s % K == 0:
                sim.tape_save(s // K)
            st = sim.step_raw(1)
            if st not in (_mps.OK, _mps.E_CG_NOCONV):
                sim._check(st, "mps_step")
        out = sim.state()
        ctx.sim, ctx.nsteps, ctx.K, ctx.nseg, ctx.dim = sim, nsteps, K, nseg, dim
        ctx.mark_non_differentiable(out["flags"], out["type"])
        return out["pos"], out["vel"], out["flags"], out["type"]

    @staticmethod
    def backward(ctx, gpos, gvel, gflags, gtype):
        sim = ctx.sim
        n, dim = sim.n, ctx.dim
        z = torch.zeros((n, dim), dtype=torch.float64, device="cuda")
        rb = z if gpos is None else gpos.to(torch.float64).contiguous()
        ub = z if gvel is None else gvel.to(torch.float64).contiguous()
        nub = 0.0
        gb = [0.0] * dim
        nseg, K, T = ctx.nseg, ctx.K, ctx.nsteps
        for seg in reversed(range(nseg)):
            s0, s1 = seg * K, min(seg * K + K, T)
            sim.tape_load(seg)
            for s in range(s0, s1):
                sim.tape_save(nseg + s - s0)
                if s < s1 - 1:
                    sim.step_raw(1)
            for s in reversed(range(s0, s1)):
                sim.tape_load(nseg + s - s0)
                rb, ub, dn, dg = sim.step_adjoint(rb, ub)
                nub += dn
                gb = [gb[a] + dg[a] for a in range(dim)]
        sim.close()
        ctx.sim = None
        g_nu = torch.tensor(nub, dtype=torch.float64)
        g_g = torch.tensor(gb, dtype=torch.float64)
        return ub, g_nu, g_g, None, None, None, None, None, None, None


def final_loss(pos, vel, flags, ptype, w_ke: float = 1.0, w_var: float = 9.81):
    """w_ke * mean fluid kinetic energy |u|^2/2 + w_var * variance of the
    vertical coordinate of the fluid particles flagged free surface in the
    last step (that set is taken as given)."""
    f = ptype == FLUID
    ke = 0.5 * (vel[f] ** 2).sum(dim=1).mean()
    s = f & (flags == 1)
    if int(s.sum()) == 0:
        return w_ke * ke
    y = pos[s, pos.shape[1] - 1]
    var = ((y - y.mean()) ** 2).mean()
    return w_ke * ke + w_var * var


def rollout(u0, nu, g, params, pos0, ptype, nsteps, K=50, rho_i=None, nu_i=None):
    return MPSRollout.apply(u0, nu, g, params, pos0, ptype, nsteps, K, rho_i, nu_i)
