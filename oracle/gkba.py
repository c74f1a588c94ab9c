"""Brute-force (non-Markovian) HF-GKBA collision integral for the second-Born
selfenergy, used to pin the central claim of the paper: the G1-G2 equations
reproduce the ordinary HF-GKBA result exactly (end of Sec. III.C).

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
