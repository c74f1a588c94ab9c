"""Gradient oracle for the driven Hubbard propagation.

The loss is a weighted sum of final-time site observables,
    L = sum_i a_i d_i(T) + sum_i b_i (n^up_ii(T) + n^dn_ii(T)),
with n_ii = Im G^<_ii (n = -i G^<, eq:g-glsymm) and the double occupation
d_i = n^up_ii n^dn_ii - Re A_iiii (energy expression of the Hubbard model).
The gradient with respect to the drive coefficients c_m and U is the exact
derivative of the discrete RK4 map, obtained by reverse-mode automatic
differentiation of ``integrate.propagate_hubbard`` (torch autograd on the CPU,
float64/complex128).  It is pinned against central finite differences in the
tests.
"""
from __future__ import annotations

import numpy as np
import torch

from . import integrate


def loss_from_state(y, a, b):
    X, Y, A = y[0], y[1], y[2]
    ns = X.shape[0]
    r = torch.arange(ns)
    nu = torch.imag(torch.diagonal(X))
    nd = torch.imag(torch.diagonal(Y))
    d = nu * nd - torch.real(A[r, r, r, r])
    return (torch.as_tensor(a) * d).sum() + (torch.as_tensor(b) * (nu + nd)).sum()


def loss_and_gradient(system, a, b, nsteps=None, selfenergy="soa"):
    """Returns (L, dL/dc [M], dL/dU) for a ``workloads.HubbardSystem`` with a drive."""
    c = torch.tensor(np.asarray(system.drive.c, dtype=np.float64), requires_grad=True)
    U = torch.tensor(float(system.U), dtype=torch.float64, requires_grad=True)
    y, _ = integrate.propagate_hubbard(system, nsteps=nsteps, selfenergy=selfenergy, U=U, c=c)
    L = loss_from_state(y, np.asarray(a, np.float64), np.asarray(b, np.float64))
    L.backward()
    return float(L.detach()), c.grad.numpy().copy(), float(U.grad)


def loss_only(system, a, b, nsteps=None, c=None, U=None, selfenergy="soa"):
    cc = None if c is None else torch.as_tensor(np.asarray(c, np.float64))
    UU = system.U if U is None else float(U)
    with torch.no_grad():
        y, _ = integrate.propagate_hubbard(system, nsteps=nsteps, selfenergy=selfenergy, U=UU, c=cc)
        return float(loss_from_state(y, np.asarray(a, np.float64), np.asarray(b, np.float64)))
