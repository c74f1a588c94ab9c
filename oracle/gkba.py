"""Brute-force (non-Markovian) HF-GKBA collision integrals for the second-Born
and the GW selfenergies, used to pin the central claim of the paper: the G1-G2
equations reproduce the ordinary HF-GKBA result exactly (end of Sec. III.C for
second Born, Sec. IV.A-B for GW).

Given a history G^<(t_m), h^HF(t_m) on a uniform grid t_m = m*dt:
  * Hartree-Fock propagator U(t_n, t_m), built from one-step exponentials
    exp(-i h^HF(t_{n-1/2}) dt) with h^HF(t_{n-1/2}) = (h^HF(t_{n-1}) + h^HF(t_n))/2;
    the paper's modified propagator is curly-U(t, t') = -i U(t, t') for t >= t'
    (eq:prop_b with eq:unity_prop and App. A).
  * GKBA reconstruction (eq:GKBA_propa, eq:GKBA_propb):
        G^><(t, t') = U(t, t') G^><(t'),   G^><(t', t) = G^><(t') U(t, t')^dagger   (t >= t').
  * Second-Born selfenergy (eq:sigma-soa, fermions):
        Sigma^><_ij(t,t') = (i)^2 sum w_iklp(t) w^-_qrsj(t') G^><_lq(t,t') G^><_pr(t,t') G^<>_sk(t',t).
  * Collision integral (eq:definition_D, first line):
        I_ij(t) = sum_k int_{t0}^t dt' [Sigma^>_ik(t,t') G^<_kj(t',t) - Sigma^<_ik(t,t') G^>_kj(t',t)],
    evaluated with the trapezoidal rule on the grid.
GW (Sec. IV.A) replaces the selfenergy by Sigma^><_ij(t,t') = i sum_kl
W^><_ilkj(t,t') G^><_kl(t,t') (eq:sigma-gw), with the screened interaction
(singular part removed) given by the two-time integral equation eq:W-def; the
GKBA propagators reconstruct every two-time G that it contains.
All tensors are torch complex128 (CPU).
"""
from __future__ import annotations

import torch

from .general import w_minus

EIN = torch.einsum


def _expm_h(h: torch.Tensor, dt: float) -> torch.Tensor:
    hh = 0.5 * (h + h.conj().T)
    e, v = torch.linalg.eigh(hh)
    return (v * torch.exp(-1j * e * dt)) @ v.conj().T


def propagators(hhfs, dt: float, n: int):
    """U(t_n, t_m) for m = 0..n (list indexed by m)."""
    steps = [_expm_h(0.5 * (hhfs[m] + hhfs[m + 1]), dt) for m in range(n)]
    out = [None] * (n + 1)
    u = torch.eye(hhfs[0].shape[0], dtype=torch.complex128)
    out[n] = u
    for m in range(n - 1, -1, -1):
        u = u @ steps[m]           # U(t_n, t_m) = U(t_n, t_{m+1}) U(t_{m+1}, t_m)
        out[m] = u
    return out


def sigma_soa(w, wm, g_a_ttp, g_b_ttp, g_c_tpt):
    """(i)^2 sum_{k' l p q r s} w_{i k' l p} w^-_{q r s k} G^a_lq(t,t') G^b_pr(t,t') G^c_{s k'}(t',t)."""
    t = EIN("qrsk,pr->qpsk", wm, g_b_ttp)
    t = EIN("qpsk,lq->lpsk", t, g_a_ttp)
    t = EIN("lpsk,sm->lpmk", t, g_c_tpt)
    return -EIN("imlp,lpmk->ik", w, t)


def collision_integral(w: torch.Tensor, gls, hhfs, dt: float, n: int) -> torch.Tensor:
    """I(t_n) from the history gls[0..n], hhfs[0..n] (trapezoidal rule)."""
    nb = w.shape[0]
    one = torch.eye(nb, dtype=torch.complex128)
    wm = w_minus(w)
    us = propagators(hhfs, dt, n)
    total = torch.zeros((nb, nb), dtype=torch.complex128)
    for m in range(n + 1):
        u = us[m]
        gl_m = gls[m]
        gg_m = gl_m - 1j * one
        gl_ttp = u @ gl_m                     # G^<(t_n, t_m)
        gg_ttp = u @ gg_m                     # G^>(t_n, t_m)
        gl_tpt = gl_m @ u.conj().T            # G^<(t_m, t_n)
        gg_tpt = gg_m @ u.conj().T            # G^>(t_m, t_n)
        sg = sigma_soa(w, wm, gg_ttp, gg_ttp, gl_tpt)
        sl = sigma_soa(w, wm, gl_ttp, gl_ttp, gg_tpt)
        integrand = sg @ gl_tpt - sl @ gg_tpt
        weight = 0.5 if (m == 0 or m == n) else 1.0
        total = total + weight * dt * integrand
    return total


# --------------------------------------------------------------------------- GW
def _pair(x: torch.Tensor) -> torch.Tensor:
    """4-index tensor x_abcd as the matrix over index pairs [(a,c),(b,d)]."""
    nb = x.shape[0]
    return x.permute(0, 2, 1, 3).reshape(nb * nb, nb * nb)


def _fock_pair(ga: torch.Tensor, gb: torch.Tensor) -> torch.Tensor:
    """G^{F}_{qspr}(t,t') = G^a_qr(t,t') G^b_sp(t',t) (eq:g2f-def) as the pair
    matrix [(p,q),(r,s)], the layout in which eq:W-def is a matrix product."""
    nb = ga.shape[0]
    return EIN("qr,sp->pqrs", ga, gb).reshape(nb * nb, nb * nb)


def _trapezoid(m: int, dt: float) -> torch.Tensor:
    """Weights of the trapezoidal rule on the grid points 0..m of [0, m dt]."""
    c = torch.full((m + 1,), dt, dtype=torch.complex128)
    c[0] = c[m] = 0.5 * dt
    return c if m > 0 else torch.zeros(1, dtype=torch.complex128)


def screened_interaction(w: torch.Tensor, gls, hhfs, dt: float, n: int):
    """W^>(t_m, t_m') and W^<(t_m, t_m') on the whole grid, 0 <= m, m' <= n, as
    pair matrices W[(i,k),(j,l)] = W_ijkl, from eq:W-def (fermions, hbar = 1):

      W^><(t,t') = -i A [ P^><(t,t') A + int_0^t  P^R(t,tb) W^><(tb,t') dtb
                                        + int_0^t' P^><(t,tb) W^A(tb,t') dtb ]

    with A[(i,k),(p,q)] = w_ipkq, P^><[(p,q),(r,s)] = G^{F,><}_qspr (eq:g2f-def,
    with the GKBA reconstruction of eq:GKBA_propa/b), P^R = P^> - P^< and
    W^A = W^< - W^> (the Langreth structure of the two integrals).  Only
    t >= t' is solved; t < t' follows from eq:Wsymm, W^><(t,t') = W^<>(t',t)^T
    in pair form.  Both integrals use the trapezoidal rule; its end point at
    tb = t makes each time step a small linear solve (and, on the diagonal
    t = t', couples W^> and W^<).  Cost O(n^3 Nb^6): tiny systems only."""
    nb = w.shape[0]
    d = nb * nb
    one = torch.eye(nb, dtype=torch.complex128)
    eye_d = torch.eye(d, dtype=torch.complex128)
    A = _pair(w)
    u0 = propagators_from_start(hhfs, dt, n)

    def U(m, mb):                      # U(t_m, t_mb) = U(t_m, 0) U(t_mb, 0)^dagger
        return u0[m] @ u0[mb].conj().T

    gl = list(gls)
    gg = [g - 1j * one for g in gls]
    Wg = torch.zeros((n + 1, n + 1, d, d), dtype=torch.complex128)
    Wl = torch.zeros_like(Wg)
    for m in range(n + 1):
        us = [U(m, mb) for mb in range(m + 1)]
        Pg = torch.stack([_fock_pair(us[mb] @ gg[mb], gl[mb] @ us[mb].conj().T) for mb in range(m + 1)])
        Pl = torch.stack([_fock_pair(us[mb] @ gl[mb], gg[mb] @ us[mb].conj().T) for mb in range(m + 1)])
        PR = Pg - Pl
        if m == 0:
            Wg[0, 0] = -1j * A @ Pg[0] @ A
            Wl[0, 0] = -1j * A @ Pl[0] @ A
            continue
        c = _trapezoid(m, dt)
        half = 0.5 * dt
        # columns m' < m: every term but the end point tb = t is known
        tau = torch.zeros((m, m), dtype=torch.complex128)      # tau[mb, m'] on [0, t_m']
        for q in range(1, m):
            tau[:q + 1, q] = _trapezoid(q, dt)
        WA = Wl[:m, :m] - Wg[:m, :m]
        rg = Pg[:m] @ A + EIN("a,aij,abjk->bik", c[:m], PR[:m], Wg[:m, :m]) \
            + EIN("ab,aij,abjk->bik", tau, Pg[:m], WA)
        rl = Pl[:m] @ A + EIN("a,aij,abjk->bik", c[:m], PR[:m], Wl[:m, :m]) \
            + EIN("ab,aij,abjk->bik", tau, Pl[:m], WA)
        lhs = eye_d + 1j * half * (A @ PR[m])
        Wg[m, :m] = torch.linalg.solve(lhs, -1j * (A @ rg))
        Wl[m, :m] = torch.linalg.solve(lhs, -1j * (A @ rl))
        Wg[:m, m] = Wl[m, :m].transpose(-1, -2)                 # eq:Wsymm
        Wl[:m, m] = Wg[m, :m].transpose(-1, -2)
        # diagonal m' = m: end points of both integrals hold W^>(t,t), W^<(t,t)
        WAc = Wl[:m, m] - Wg[:m, m]
        rg = Pg[m] @ A + EIN("a,aij,ajk->ik", c[:m], PR[:m], Wg[:m, m]) \
            + EIN("a,aij,ajk->ik", c[:m], Pg[:m], WAc)
        rl = Pl[m] @ A + EIN("a,aij,ajk->ik", c[:m], PR[:m], Wl[:m, m]) \
            + EIN("a,aij,ajk->ik", c[:m], Pl[:m], WAc)
        # W> = -iA(rg + half[PR W> + Pg (W< - W>)]), W< = -iA(rl + half[PR W< + Pl (W< - W>)])
        big = torch.zeros((2 * d, 2 * d), dtype=torch.complex128)
        big[:d, :d] = eye_d + 1j * half * (A @ (PR[m] - Pg[m]))
        big[:d, d:] = 1j * half * (A @ Pg[m])
        big[d:, :d] = -1j * half * (A @ Pl[m])
        big[d:, d:] = eye_d + 1j * half * (A @ (PR[m] + Pl[m]))
        sol = torch.linalg.solve(big, torch.cat([-1j * (A @ rg), -1j * (A @ rl)], 0))
        Wg[m, m], Wl[m, m] = sol[:d], sol[d:]
    return Wg, Wl


def propagators_from_start(hhfs, dt: float, n: int):
    """U(t_m, t_0) for m = 0..n from the same one-step exponentials as ``propagators``."""
    u = [torch.eye(hhfs[0].shape[0], dtype=torch.complex128)]
    for m in range(n):
        u.append(_expm_h(0.5 * (hhfs[m] + hhfs[m + 1]), dt) @ u[-1])
    return u


def gw_collision_integral(w: torch.Tensor, gls, hhfs, dt: float, n: int) -> torch.Tensor:
    """I(t_n) of GW-HF-GKBA: eq:definition_D (first line) with the selfenergy
    eq:sigma-gw, Sigma^><_ik(t,tb) = i sum_ab W^><_ibak(t,tb) G^><_ab(t,tb),
    the screened interaction from ``screened_interaction`` and the trapezoidal
    rule over tb."""
    nb = w.shape[0]
    one = torch.eye(nb, dtype=torch.complex128)
    Wg, Wl = screened_interaction(w, gls, hhfs, dt, n)
    u0 = propagators_from_start(hhfs, dt, n)
    c = _trapezoid(n, dt)
    total = torch.zeros((nb, nb), dtype=torch.complex128)
    for mb in range(n + 1):
        u = u0[n] @ u0[mb].conj().T
        gl_m = gls[mb]
        gg_m = gl_m - 1j * one
        sg = 1j * EIN("iabk,ab->ik", Wg[n, mb].reshape(nb, nb, nb, nb), u @ gg_m)
        sl = 1j * EIN("iabk,ab->ik", Wl[n, mb].reshape(nb, nb, nb, nb), u @ gl_m)
        total = total + c[mb] * (sg @ (gl_m @ u.conj().T) - sl @ (gg_m @ u.conj().T))
    return total
