"""Observables of the G1-G2 state.

n = -i G^< (eq:g-glsymm, fermions).  The total energy is the expectation value
of the Hamiltonian eq:h, with the two-particle density matrix split into its
Hartree, Fock and correlated parts; the correlated part c2 = (i hbar)^2 G2
(eq:ini-g2), so with <c+_i c+_j c_l c_k> = n_ki n_lj - n_kj n_li - G2_klij:
    E = Tr(h0 n) + 1/2 sum w_ijkl (n_ki n_lj - n_kj n_li) - 1/2 Re sum w_ijkl G2_klij.
The paper does not print this formula; it asserts conservation of the total
energy by the scheme (Sec. VIII).  For the Hubbard model the same expression
with the interaction of eq:wmatrix-hubbard reads
    E = sum_s Tr(h0^s n^s) + U sum_i (n^up_ii n^dn_ii - Re A_iiii).
"""
from __future__ import annotations

import torch

EIN = torch.einsum


def general_observables(h0, w, gl, g2, t=0.0):
    n = -1j * gl
    e_kin = torch.real(torch.trace(h0 @ n))
    e_mf = 0.5 * torch.real(EIN("ijkl,ki,lj->", w, n, n) - EIN("ijkl,kj,li->", w, n, n))
    e_corr = -0.5 * torch.real(EIN("ijkl,klij->", w, g2))
    nb = gl.shape[0]
    m = g2.reshape(nb * nb, nb * nb)
    herm = (m - m.conj().T).abs().max() / max(m.abs().max(), 1e-300)
    exch = (g2 - g2.permute(1, 0, 3, 2)).abs().max() / max(g2.abs().max(), 1e-300)
    return dict(t=float(t), N=float(torch.real(torch.trace(n))), E_kin=float(e_kin),
                E_mf=float(e_mf), E_corr=float(e_corr), E_tot=float(e_kin + e_mf + e_corr),
                herm_resid=float(herm), exch_resid=float(exch))


def hubbard_observables(h0u, h0d, U, X, Y, A, t=0.0):
    nu = -1j * X
    nd = -1j * Y
    ns = X.shape[0]
    r = torch.arange(ns)
    e_kin = torch.real(torch.trace(h0u @ nu) + torch.trace(h0d @ nd))
    duu = torch.real(torch.diagonal(nu))
    ddd = torch.real(torch.diagonal(nd))
    aiiii = torch.real(A[r, r, r, r])
    docc = duu * ddd - aiiii
    e_mf = U * (duu * ddd).sum()
    e_corr = -U * aiiii.sum()
    m = A.reshape(ns * ns, ns * ns)
    herm = (m - m.conj().T).abs().max() / max(float(m.abs().max()), 1e-300)
    return dict(t=float(t), N_up=float(torch.real(torch.trace(nu))),
                N_dn=float(torch.real(torch.trace(nd))), E_kin=float(e_kin),
                E_mf=float(e_mf), E_corr=float(e_corr), E_tot=float(e_kin + e_mf + e_corr),
                docc=docc.detach(), herm_resid=float(herm))


def hubbard_imbalance(X, Y, x):
    """Density imbalance (N_left - N_right) / N, left/right being the sites with
    negative/positive profile x_i (for the 8x8 drive x_i = i_x - 3.5 this is the
    difference of the two halves of the cluster)."""
    n = torch.real(torch.diagonal(-1j * X)) + torch.real(torch.diagonal(-1j * Y))
    x = torch.as_tensor(x, dtype=torch.float64)
    s = (x < 0).to(torch.float64) - (x > 0).to(torch.float64)
    return float((s * n).sum() / n.sum())
