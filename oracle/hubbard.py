"""G1-G2 equations for the Fermi-Hubbard model (Secs. III.D, IV.D, V.A-B, VII).

Spin-resolved variables: X = G^{<,up}, Y = G^{<,down} (Ns x Ns), and the pair
function A = G2^{up down up down}_ijkl ([Ns]^4).  For GW two more channels are
needed: B = G2^{up up up up} and C = G2^{down down down down}.  The channel
G2^{down up down up}_ijkl equals A_jilk by the exchange symmetry eq:Gsymm_a.

The on-site interaction U may be a float or a real 0-d tensor (autograd).
"""
from __future__ import annotations

import torch

EIN = torch.einsum


def _eye(n):
    return torch.eye(n, dtype=torch.complex128)


def _diag(v):
    return torch.diag_embed(v)


def hf_hamiltonians(h0u, h0d, X, Y, U):
    """Sec. III.D: h^{HF,up}_ij = h0_ij - i U delta_ij G^{<,down}_ii, and up <-> down."""
    hu = h0u - 1j * U * _diag(torch.diagonal(Y))
    hd = h0d - 1j * U * _diag(torch.diagonal(X))
    return hu, hd


def collision_integrals(A, U):
    """eq:colint_hubbard: I^up_ij = -i U A_iiji.  For spin down the same formula
    with up <-> down reads I^down_ij = -i U G2^{du du}_iiji = -i U A_iiij
    (exchange symmetry eq:Gsymm_a)."""
    ns = A.shape[0]
    r = torch.arange(ns)
    # A[i, i, j, i] -> matrix over (i, j); A[i, i, i, j] -> matrix over (i, j)
    Iu = -1j * U * A[r, r, :, r]
    Id = -1j * U * A[r, r, r, :]
    return Iu, Id


def commutator(hu, hd, A):
    """[h^(2),HF_{up down}, A] with h^(2)_ijkl = delta_jl h^up_ik + delta_ik h^down_jl
    (eq:twopart_hamiltonian_hubbard), dense sums over one index each."""
    return (EIN("ip,pjkl->ijkl", hu, A) + EIN("jp,ipkl->ijkl", hd, A)
            - EIN("ijpl,pk->ijkl", A, hu) - EIN("ijkp,pl->ijkl", A, hd))


def commutator_same_spin(h, B):
    """[h^(2),HF_{ss}, B] for an equal-spin channel (both particles see h^{HF,s})."""
    return (EIN("ip,pjkl->ijkl", h, B) + EIN("jp,ipkl->ijkl", h, B)
            - EIN("ijpl,pk->ijkl", B, h) - EIN("ijkp,pl->ijkl", B, h))


def phi_direct(X, Y):
    """Occupation factor of eq:phi-hubbard (the 'direct' Ns^5 form):
    (i hbar)^4 sum_p [X>_ip Y>_jp X<_pk Y<_pl - X<_ip Y<_jp X>_pk Y>_pl]."""
    n = X.shape[0]
    Xg = X - 1j * _eye(n)
    Yg = Y - 1j * _eye(n)
    return (EIN("ip,jp,pk,pl->ijkl", Xg, Yg, X, Y) - EIN("ip,jp,pk,pl->ijkl", X, Y, Xg, Yg))


def phi_cubic(X, Y):
    """Occupation factor after eliminating G^<G^<G^<G^< (eq:soa-cubic-scheme):
    (i)^2 (d_ij - d_kl) X_ik Y_jl + (i)^3 [X_ij X_jk - X_lk X_il] Y_jl
                                  + (i)^3 [Y_ji Y_il - Y_kl Y_jk] X_ik."""
    n = X.shape[0]
    d = _eye(n)
    t1 = -(EIN("ij,ik,jl->ijkl", d, X, Y) - EIN("kl,ik,jl->ijkl", d, X, Y))
    t2 = -1j * (EIN("ij,jk,jl->ijkl", X, X, Y) - EIN("lk,il,jl->ijkl", X, X, Y))
    t3 = -1j * (EIN("ji,il,ik->ijkl", Y, Y, X) - EIN("kl,jk,ik->ijkl", Y, Y, X))
    return t1 + t2 + t3


def source(X, Y, U, direct: bool = False):
    """eq:g2-hubbard: Psi = U Phi / (i hbar)^2."""
    phi = phi_direct(X, Y) if direct else phi_cubic(X, Y)
    return -U * phi


def ladder_pp_direct(X, Y, U, A):
    """eq:lambdapp_hubb: (i hbar)^2 U sum_p [X>_ip Y>_jp - X<_ip Y<_jp] A_ppkl."""
    n = X.shape[0]
    r = torch.arange(n)
    Xg = X - 1j * _eye(n)
    Yg = Y - 1j * _eye(n)
    D = A[r, r, :, :]                       # D[p, k, l] = A_ppkl
    f = Xg.unsqueeze(1) * Yg.unsqueeze(0) - X.unsqueeze(1) * Y.unsqueeze(0)   # f[i, j, p]
    return -U * EIN("ijp,pkl->ijkl", f, D)


def ladder_pp(X, Y, U, A):
    """Reformulated particle-particle ladder (Sec. VII.C):
    delta_ij U A_iikl + i U (Y_ji A_iikl + X_ij A_jjkl)."""
    n = X.shape[0]
    r = torch.arange(n)
    D = A[r, r, :, :]                       # D[p, k, l] = A_ppkl
    d = _eye(n)
    return (U * EIN("ij,ikl->ijkl", d, D)
            + 1j * U * (EIN("ji,ikl->ijkl", Y, D) + EIN("ij,jkl->ijkl", X, D)))


def ladder_ph_direct(X, Y, U, A):
    """eq:lambdaph_hubb: (i hbar)^2 U sum_p [X>_ip Y<_pl - X<_ip Y>_pl] A_pjkp."""
    n = X.shape[0]
    Xg = X - 1j * _eye(n)
    Yg = Y - 1j * _eye(n)
    return -U * (EIN("ip,pl,pjkp->ijkl", Xg, Y, A) - EIN("ip,pl,pjkp->ijkl", X, Yg, A))


def ladder_ph(X, Y, U, A):
    """Reformulated particle-hole ladder (Sec. VII.C):
    i U [Y_il A_ijki - X_il A_ljkl]."""
    n = X.shape[0]
    r = torch.arange(n)
    Ai = A[r, :, :, r]                                  # Ai[i, j, k] = A_ijki
    Al = torch.stack([A[l, :, :, l] for l in range(n)])  # Al[l, j, k] = A_ljkl
    return 1j * U * (EIN("il,ijk->ijkl", Y, Ai) - EIN("il,ljk->ijkl", X, Al))


def polarization(Xs, A, U, swap_pair: bool = False):
    """Reformulated Hubbard polarization (Sec. VII.B): for the channel whose
    second/fourth spin is s, Pi_ijkl = -i U G^{<,s}_jl [P_ijkj - P_ilkl],
    where P is the channel with opposite spin on those slots.
    ``swap_pair`` reads P_abcd = A_badc (channel down-up-down-up from A)."""
    P = A.permute(1, 0, 3, 2) if swap_pair else A
    n = A.shape[0]
    Pj = torch.stack([P[:, j, :, j] for j in range(n)], dim=1)   # Pj[i, j, k] = P_ijkj
    return -1j * U * (EIN("jl,ijk->ijkl", Xs, Pj) - EIN("jl,ilk->ijkl", Xs, Pj))


def polarization_direct(Xs, P, U):
    """eq:pihubbardtrans / eq:pihubbardcis: -(i hbar)^2 U sum_p
    [G>_jp G<_pl - G<_jp G>_pl] P_ipkp (G = G^{<,s} of the spin on slots j,l)."""
    n = Xs.shape[0]
    Xg = Xs - 1j * _eye(n)
    return U * (EIN("jp,pl,ipkp->ijkl", Xg, Xs, P) - EIN("jp,pl,ipkp->ijkl", Xs, Xg, P))


def _pk(x):
    return x.permute(2, 3, 0, 1).conj()


def _pl(x):
    return x.permute(3, 2, 1, 0).conj()


SELFENERGIES = ("soa", "tpp", "tph", "gw", "dsl")


def rhs(h0u, h0d, U, X, Y, A, selfenergy: str = "soa", B=None, C=None, direct: bool = False):
    """Time derivatives of the spin-resolved Hubbard G1-G2 system.

    G1 (eq:eom_g1_hubbard): dX/dt = -i([h^up, X] + I^up + I^up^dagger), same for Y.
    G2 (eq:g2-hubbard and its TPP/TPH/GW analogues):
      dA/dt = -i([h2_{ud}, A] + Psi + extra), with extra per selfenergy:
        tpp: L^pp - [L^pp_klij]^*      (Sec. V.A Hubbard EOM)
        tph: L^ph - [L^ph_klij]^*      (Sec. V.B Hubbard EOM)
        gw : Pi^{udud}_ijkl - [Pi^{dudu}_lkji]^*   (eq:g2-gw-hubbard1 with each
             spin attached to its index; Pi^{dudu} built from Y... see below)
    For gw the equal-spin channels B (up) and C (down) obey eq:g2-gw-hubbard2:
      dB/dt = -i([h2_uu, B] + Pi^{uuuu} - [Pi^{uuuu}_lkji]^*), same for C.
    dsl (Sec. VI: polarization and both ladders on top of the source): the gw
    equations with, on A, the tpp and tph ladder terms added as well.  The
    ladders vanish on B and C (their quasi-Hamiltonians need a pair of
    opposite spins), and the exchange form of the source that DSL takes equals
    Psi on A, because the exchanged on-site interaction pairs equal spins.
    Returns (dX, dY, dA) or (dX, dY, dA, dB, dC) for gw and dsl.
    """
    if selfenergy not in SELFENERGIES:
        raise ValueError(selfenergy)
    hu, hd = hf_hamiltonians(h0u, h0d, X, Y, U)
    Iu, Id = collision_integrals(A, U)
    dX = -1j * (hu @ X - X @ hu + Iu + Iu.conj().T)
    dY = -1j * (hd @ Y - Y @ hd + Id + Id.conj().T)
    S = commutator(hu, hd, A) + source(X, Y, U, direct=direct)
    if selfenergy == "tpp":
        lam = ladder_pp_direct(X, Y, U, A) if direct else ladder_pp(X, Y, U, A)
        S = S + lam - _pk(lam)
    elif selfenergy == "tph":
        lam = ladder_ph_direct(X, Y, U, A) if direct else ladder_ph(X, Y, U, A)
        S = S + lam - _pk(lam)
    if selfenergy == "dsl":
        for lam in ((ladder_pp_direct(X, Y, U, A) if direct else ladder_pp(X, Y, U, A)),
                    (ladder_ph_direct(X, Y, U, A) if direct else ladder_ph(X, Y, U, A))):
            S = S + lam - _pk(lam)
    if selfenergy in ("gw", "dsl"):
        # Pi^{up dn up dn}_ijkl: spin down on slots j, l; partner channel B (up up).
        pi_udud = polarization(Y, B, U) if not direct else polarization_direct(Y, B, U)
        # Pi^{dn up dn up}_ijkl: spin up on slots j, l; partner channel C (down down).
        pi_dudu = polarization(X, C, U) if not direct else polarization_direct(X, C, U)
        S = S + pi_udud - _pl(pi_dudu)
        # equal-spin channels: Pi^{ss ss} built from the opposite-spin channel
        # with spin s' on slots p: for uuuu that is A (up dn up dn),
        # for dddd it is G2^{dn up dn up} = A_badc.
        pi_uuuu = (polarization(X, A, U) if not direct else polarization_direct(X, A, U))
        Ad = A.permute(1, 0, 3, 2)
        pi_dddd = (polarization(Y, Ad, U) if not direct else polarization_direct(Y, Ad, U))
        dA = -1j * S
        dB = -1j * (commutator_same_spin(hu, B) + pi_uuuu - _pl(pi_uuuu))
        dC = -1j * (commutator_same_spin(hd, C) + pi_dddd - _pl(pi_dddd))
        return dX, dY, dA, dB, dC
    return dX, dY, -1j * S
