"""Time stepping of the time-local G1-G2 system.

The paper names no integrator; the G1-G2 equations form a closed system of
ordinary differential equations (end of Sec. III.C).  The oracle uses the
classical fourth-order Runge-Kutta method in its textbook form, with the
time-dependent one-particle Hamiltonian evaluated at the stage times
t, t+dt/2, t+dt/2, t+dt.
"""
from __future__ import annotations

import math
from typing import Callable, Sequence, Tuple

import numpy as np
import torch

from . import general, hubbard


def rk4_step(f: Callable, t: float, y: Sequence[torch.Tensor], dt: float) -> Tuple[torch.Tensor, ...]:
    """One classical RK4 step for a tuple of tensors: y_{n+1} = y_n + dt/6 (k1 + 2k2 + 2k3 + k4)."""
    k1 = f(t, y)
    k2 = f(t + 0.5 * dt, [a + 0.5 * dt * b for a, b in zip(y, k1)])
    k3 = f(t + 0.5 * dt, [a + 0.5 * dt * b for a, b in zip(y, k2)])
    k4 = f(t + dt, [a + dt * b for a, b in zip(y, k3)])
    return tuple(a + (dt / 6.0) * (b1 + 2.0 * b2 + 2.0 * b3 + b4)
                 for a, b1, b2, b3, b4 in zip(y, k1, k2, k3, k4))


def _t(x):
    return torch.as_tensor(np.asarray(x), dtype=torch.complex128)


# --------------------------------------------------------------------------- general basis
def general_rhs_fn(h0, w, selfenergy="soa", kick=None, kick_until=None, switch=None):
    """f(t, (G1, G2)) for a general-basis system; ``kick`` is added to h0 for t < kick_until;
    ``switch`` = (t_on, tau) ramps the interaction, w(t) = w phi(t) (see switch_factor)."""
    h0 = _t(h0)
    w = _t(w)
    hk = None if kick is None else h0 + _t(kick)

    def f(t, y):
        h = hk if (hk is not None and t < kick_until) else h0
        wt = w if switch is None else w * switch_factor(t, switch)
        return general.rhs(h, wt, y[0], y[1], selfenergy)

    return f


def propagate_general(system, nsteps=None, selfenergy="soa", g2_0=None, record=None,
                      observables_every=0):
    """Propagate a ``workloads.GeneralSystem``.  The optional kick acts during the
    whole first step (all four stages): h0 + kick for t < dt/2 ... evaluated at
    stage times t < dt (strictly: stages of step 0 are at 0, dt/2, dt/2, dt and
    the kick is applied to all four), then h0."""
    dt = system.dt
    nsteps = system.nsteps if nsteps is None else nsteps
    h0 = _t(system.h0)
    w = _t(system.w)
    hk = None if system.kick is None else h0 + _t(system.kick)
    g1 = _t(system.g1)
    nb = g1.shape[0]
    g2 = torch.zeros((nb,) * 4, dtype=torch.complex128) if g2_0 is None else _t(g2_0)
    rec = []
    t = 0.0
    for n in range(nsteps):
        h = hk if (hk is not None and n == 0) else h0
        f = (lambda tt, y, h=h: general.rhs(h, w, y[0], y[1], selfenergy))
        if observables_every and n % observables_every == 0:
            from .observables import general_observables
            rec.append(general_observables(h0, w, g1, g2, t))
        g1, g2 = rk4_step(f, t, (g1, g2), dt)
        t = (n + 1) * dt
    if observables_every:
        from .observables import general_observables
        rec.append(general_observables(h0, w, g1, g2, t))
    return g1, g2, rec


# --------------------------------------------------------------------------- Hubbard
def switch_factor(t, switch=None):
    """Adiabatic switching of the interaction, one way to prepare a correlated
    initial state (Sec. III.F, Sec. VIII): the interaction is turned on slowly
    from an uncorrelated start.  switch = (t_on, tau): U(t) = U phi(t) with
    phi = 0 before t_on, sin^2(pi x / 2), x = (t - t_on) / tau, during the
    ramp and 1 after it; None: phi = 1."""
    if switch is None:
        return 1.0
    t_on, tau = switch
    x = (t - t_on) / tau
    if x <= 0.0:
        return 0.0
    if x >= 1.0:
        return 1.0
    return math.sin(0.5 * math.pi * x) ** 2


def hubbard_h0(system, t, c=None):
    """Spin-resolved h0(t): static part plus the optional drive on the diagonal.
    ``c`` overrides the drive coefficients (a real tensor, for gradients)."""
    h0u = _t(system.h0[0])
    h0d = _t(system.h0[1])
    d = system.drive
    if d is None:
        return h0u, h0d
    cc = torch.as_tensor(d.c, dtype=torch.float64) if c is None else c
    phi = torch.exp(-torch.as_tensor((t - d.t_center) ** 2, dtype=torch.float64) / (2.0 * d.tau ** 2))
    v = (cc * phi).sum() * torch.as_tensor(d.x, dtype=torch.float64)
    dv = torch.diag_embed(v.to(torch.complex128))
    return h0u + dv, h0d + dv


def hubbard_rhs_fn(system, selfenergy="soa", U=None, c=None, direct=False, switch=None):
    UU = system.U if U is None else U

    def f(t, y):
        h0u, h0d = hubbard_h0(system, t, c)
        Ut = UU * switch_factor(t, switch) if switch is not None else UU
        if selfenergy in ("gw", "dsl"):
            return hubbard.rhs(h0u, h0d, Ut, y[0], y[1], y[2], selfenergy, B=y[3], C=y[4], direct=direct)
        return hubbard.rhs(h0u, h0d, Ut, y[0], y[1], y[2], selfenergy, direct=direct)

    return f


def hubbard_initial(system, selfenergy="soa", g2_0=None):
    X = _t(system.g1[0])
    Y = _t(system.g1[1])
    ns = X.shape[0]
    A = torch.zeros((ns,) * 4, dtype=torch.complex128) if g2_0 is None else _t(g2_0)
    if selfenergy in ("gw", "dsl"):
        return [X, Y, A, torch.zeros_like(A), torch.zeros_like(A)]
    return [X, Y, A]


def propagate_hubbard(system, nsteps=None, selfenergy="soa", U=None, c=None, g2_0=None,
                      observables_every=0, direct=False, state=None, t0=0.0, switch=None):
    """Propagate a ``workloads.HubbardSystem`` with RK4; returns (state, records).
    Observables use the interaction at their time (U phi(t) when switching)."""
    from .observables import hubbard_observables
    dt = system.dt
    nsteps = system.nsteps if nsteps is None else nsteps
    f = hubbard_rhs_fn(system, selfenergy, U, c, direct, switch)
    y = hubbard_initial(system, selfenergy, g2_0) if state is None else list(state)
    UU = system.U if U is None else U
    rec = []
    t = t0
    for n in range(nsteps):
        if observables_every and n % observables_every == 0:
            h0u, h0d = hubbard_h0(system, t, c)
            rec.append(hubbard_observables(h0u, h0d, UU * switch_factor(t, switch), y[0], y[1], y[2], t))
        y = list(rk4_step(f, t, y, dt))
        t = t0 + (n + 1) * dt
    if observables_every:
        h0u, h0d = hubbard_h0(system, t, c)
        rec.append(hubbard_observables(h0u, h0d, UU * switch_factor(t, switch), y[0], y[1], y[2], t))
    return y, rec


# --------------------------------------------------------------------------- jellium
def propagate_jellium(system, nsteps=None, selfenergy="soa", state=None, t0=0.0, observables_every=0):
    """RK4 propagation of a ``workloads.JelliumSystem`` (uncorrelated start
    unless ``state`` = (G1 [2][Nb], G2 [2][2][Nb]^3) is given); returns the
    final (G1, G2) and the observables every ``observables_every`` steps."""
    from . import jellium
    nsteps = system.nsteps if nsteps is None else nsteps
    nb = system.nb
    if state is None:
        g1 = _t(system.g1)
        g2 = torch.zeros((2, 2, nb, nb, nb), dtype=torch.complex128)
    else:
        g1, g2 = state
    f = lambda t, y: jellium.rhs(system.eps, system.v, y[0], y[1], system.dims, selfenergy)  # noqa: E731
    rec = []
    t = t0
    for n in range(nsteps):
        if observables_every and n % observables_every == 0:
            rec.append(jellium.observables(system.eps, system.v, g1, g2, system.dims, t))
        g1, g2 = rk4_step(f, t, (g1, g2), system.dt)
        t = t0 + (n + 1) * system.dt
    if observables_every:
        rec.append(jellium.observables(system.eps, system.v, g1, g2, system.dims, t))
    return (g1, g2), rec
