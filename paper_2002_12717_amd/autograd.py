"""torch.autograd.Function around the library's discrete adjoint.

``DrivenHubbardLoss.apply(c, U, prop, system_args)`` runs the checkpointed
forward propagation on the GPU (g1g2_forward_checkpointed) and returns the
loss L = sum_i a_i d_i(T) + sum_i b_i (n^up_ii + n^dn_ii)(T); backward runs the
reverse sweep (g1g2_adjoint) and returns dL/dc and dL/dU.  Only marshalling
happens here; every numerical step runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch


class DrivenHubbardLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, U, prop, drive, a, b, dt, nsteps, interval=0):
        """c: drive coefficients (float64 CPU tensor), U: 0-d tensor, prop: a
        binding.Propagator (Hubbard SOA) holding the initial state, drive:
        (x, t_center, tau), a/b: site weights (numpy)."""
        x, tc, tau = drive
        cc = c.detach().cpu().numpy().astype(np.float64)
        prop.set_U(float(U))
        prop.set_drive(x, cc, tc, tau)
        prop.forward_checkpointed(dt, nsteps, interval)
        nu, nd, docc = prop.site_observables()
        loss = float(np.dot(a, docc) + np.dot(b, nu + nd))
        ctx.prop, ctx.a, ctx.b, ctx.m = prop, np.asarray(a, np.float64), np.asarray(b, np.float64), len(cc)
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        _, gc, gU = ctx.prop.adjoint(ctx.a, ctx.b, ctx.m)
        g = grad_out.item()
        return (torch.as_tensor(gc * g, dtype=torch.float64),
                torch.tensor(gU * g, dtype=torch.float64), None, None, None, None, None, None, None)
