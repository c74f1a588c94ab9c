"""G1-G2 equations in a general single-particle basis (Secs. II-VI).

All tensors are torch complex128 on the CPU.  Index order of every 4-index
tensor is [i][j][k][l] as written in the paper.
"""
from __future__ import annotations

import torch

EIN = torch.einsum


def eye(n: int) -> torch.Tensor:
    return torch.eye(n, dtype=torch.complex128)


def greater(gl: torch.Tensor) -> torch.Tensor:
    """G^> = G^< + delta/(i hbar) = G^< - i 1 on the time diagonal (eq:g-glsymm)."""
    return gl - 1j * eye(gl.shape[-1])


def w_minus(w: torch.Tensor) -> torch.Tensor:
    """Antisymmetrized interaction w^-_ijkl = w_ijkl - w_ijlk (Sec. II.B, fermions)."""
    return w - w.permute(0, 1, 3, 2)


def hf_hamiltonian(h0: torch.Tensor, w: torch.Tensor, gl: torch.Tensor) -> torch.Tensor:
    """Hartree-Fock Hamiltonian, eq:h_HF with the fermion sign:
    h^HF_ij = h0_ij - i sum_kl w^-_ikjl G^<_lk."""
    return h0 - 1j * EIN("ikjl,lk->ij", w_minus(w), gl)


def collision_integral(w: torch.Tensor, g2: torch.Tensor) -> torch.Tensor:
    """Time-local collision integral, eq:definition_D / eq:eom_gone-I (fermions):
    I_ij = -i sum_klp w_iklp G2_lpjk."""
    return -1j * EIN("iklp,lpjk->ij", w, g2)


def g1_rhs(hhf: torch.Tensor, gl: torch.Tensor, coll: torch.Tensor) -> torch.Tensor:
    """eq:eom_gone-2: i dG^</dt = [h^HF, G^<] + I + I^dagger."""
    return -1j * (hhf @ gl - gl @ hhf + coll + coll.conj().transpose(0, 1))


def two_particle_commutator(hhf: torch.Tensor, g2: torch.Tensor) -> torch.Tensor:
    """[h^(2),HF, G2] with h^(2),HF_ijkl = delta_jl h_ik + delta_ik h_jl
    (eq:twopart_hamiltonian), written out as sums over one index each."""
    left = EIN("ip,pjkl->ijkl", hhf, g2) + EIN("jq,iqkl->ijkl", hhf, g2)
    right = EIN("ijpl,pk->ijkl", g2, hhf) + EIN("ijkq,ql->ijkl", g2, hhf)
    return left - right


def source(wx: torch.Tensor, gg: torch.Tensor, gl: torch.Tensor) -> torch.Tensor:
    """Two-particle source Psi (eq:psi-pm-def) evaluated as in eq:soa-skalierung:
    (i hbar)^2 [sum_p G>_ip sum_q G>_jq sum_r G<_rk sum_s wx_pqrs G<_sl - (> <-> <)].
    Pass wx = w^- for Psi^- (SOA, TPP, TPH, DSL) or wx = w for GW without exchange."""

    def chain(a, b):
        t = EIN("pqrs,sl->pqrl", wx, b)
        t = EIN("rk,pqrl->pqkl", b, t)
        t = EIN("jq,pqkl->pjkl", a, t)
        return EIN("ip,pjkl->ijkl", a, t)

    return -(chain(gg, gl) - chain(gl, gg))


# --------------------------------------------------------------------------- GW
def gw_hcorr(w: torch.Tensor, gg: torch.Tensor, gl: torch.Tensor) -> torch.Tensor:
    """Effective quasi-Hamiltonian of GW, eq:gwhcorr with the fermion sign
    (-(i hbar)^2 = +1) and the Fock products of eq:g2f-def at equal times
    (G^{F,>}_jplq = G>_jq G<_pl):
    h^eps_ijkl = sum_pq w_qipk (G>_jq G<_pl - G<_jq G>_pl)."""
    return EIN("qipk,jq,pl->ijkl", w, gg, gl) - EIN("qipk,jq,pl->ijkl", w, gl, gg)


def gw_polarization(heps: torch.Tensor, g2: torch.Tensor) -> torch.Tensor:
    """Polarization term, eq:gwpi: Pi_ijkl = sum_pq h^eps_qjpl G2_ipkq."""
    return EIN("qjpl,ipkq->ijkl", heps, g2)


# ---------------------------------------------------------------- T matrix (pp)
def tpp_hcorr(w: torch.Tensor, gg: torch.Tensor, gl: torch.Tensor) -> torch.Tensor:
    """eq:HTPPcorr with G^{H,>}_ijpq = G>_ip G>_jq (eq:g2h-def):
    h^pp_ijkl = (i hbar)^2 sum_pq (G>_ip G>_jq - G<_ip G<_jq) w_pqkl."""
    return -(EIN("ip,jq,pqkl->ijkl", gg, gg, w) - EIN("ip,jq,pqkl->ijkl", gl, gl, w))


def tpp_ladder(hpp: torch.Tensor, g2: torch.Tensor) -> torch.Tensor:
    """eq:lambdapp: Lambda^pp_ijkl = sum_pq h^pp_ijpq G2_pqkl."""
    return EIN("ijpq,pqkl->ijkl", hpp, g2)


# ---------------------------------------------------------------- T matrix (ph)
def tph_hcorr(w: torch.Tensor, gg: torch.Tensor, gl: torch.Tensor) -> torch.Tensor:
    """eq:HTPHcorr with G^{F,>}_iqlp = G>_ip G<_ql (eq:g2f-def):
    h^ph_ijkl = (i hbar)^2 sum_pq (G>_ip G<_ql - G<_ip G>_ql) w_pjkq."""
    return -(EIN("ip,ql,pjkq->ijkl", gg, gl, w) - EIN("ip,ql,pjkq->ijkl", gl, gg, w))


def tph_ladder(hph: torch.Tensor, g2: torch.Tensor) -> torch.Tensor:
    """eq:lambdaph: Lambda^ph_ijkl = sum_pq h^ph_ipql G2_qjkp."""
    return EIN("ipql,qjkp->ijkl", hph, g2)


def partner_lkji(x: torch.Tensor) -> torch.Tensor:
    """[x_lkji]^* as an [i][j][k][l] tensor (partner of Pi in eq:g2-eq-gw-pi)."""
    return x.permute(3, 2, 1, 0).conj()


def partner_klij(x: torch.Tensor) -> torch.Tensor:
    """[x_klij]^* as an [i][j][k][l] tensor (partner of Lambda, eq:g2-eq-tpp-lambda)."""
    return x.permute(2, 3, 0, 1).conj()


SELFENERGIES = ("soa", "gw", "gw_x", "tpp", "tph", "dsl", "dsl_x")


def correlation_terms(selfenergy: str, w: torch.Tensor, gg: torch.Tensor, gl: torch.Tensor,
                      g2: torch.Tensor) -> torch.Tensor:
    """Right-hand side S of  i dG2/dt - [h^(2),HF, G2] = S  for each selfenergy:
      soa : Psi^-                                   (eq:result_eom_soa)
      gw  : Psi(w) + Pi - [Pi_lkji]^*               (eq:g2-eq-gw-pi)
      gw_x: Psi^- + Pi - [Pi_lkji]^*                (GW with exchange, Sec. IV.B end)
      tpp : Psi^- + L^pp - [L^pp_klij]^*            (eq:g2-eq-tpp-lambda)
      tph : Psi^- + L^ph - [L^ph_klij]^*            (eq:g2-eq-tph-lambda)
      dsl : Psi^- + Pi - [Pi_lkji]^* + L - [L_klij]^*, L = L^pp + L^ph
                                                    (eq:g2-dsl-equation-pi-lambda)
      dsl_x: dsl with w^- in place of w in h^eps and h^ph, the exchange
             terms of the polarization and particle-hole channels; Sec. VI
             equates DSL with neglecting three-particle correlations, and
             in a general basis only this form reaches that order (with the
             on-site Hubbard w both do; they differ there only in the
             equal-spin and spin-flip channels)
    """
    if selfenergy not in SELFENERGIES:
        raise ValueError(selfenergy)
    wm = w_minus(w)
    wx = wm if selfenergy == "dsl_x" else w     # interaction of h^eps and h^ph
    s = source(w if selfenergy == "gw" else wm, gg, gl)
    if selfenergy in ("gw", "gw_x", "dsl", "dsl_x"):
        pi = gw_polarization(gw_hcorr(wx, gg, gl), g2)
        s = s + pi - partner_lkji(pi)
    lam = None
    if selfenergy in ("tpp", "dsl", "dsl_x"):
        lam = tpp_ladder(tpp_hcorr(w, gg, gl), g2)
    if selfenergy in ("tph", "dsl", "dsl_x"):
        lph = tph_ladder(tph_hcorr(wx, gg, gl), g2)
        lam = lph if lam is None else lam + lph
    if lam is not None:
        s = s + lam - partner_klij(lam)
    return s


def rhs(h0: torch.Tensor, w: torch.Tensor, gl: torch.Tensor, g2: torch.Tensor,
        selfenergy: str = "soa"):
    """Time derivatives (dG^</dt, dG2/dt) of the closed time-local system
    eq:eom_gone-2 + eq:eom_gone-I + the G2 equation of ``selfenergy``."""
    hhf = hf_hamiltonian(h0, w, gl)
    gg = greater(gl)
    dg1 = g1_rhs(hhf, gl, collision_integral(w, g2))
    dg2 = -1j * (two_particle_commutator(hhf, g2) + correlation_terms(selfenergy, w, gg, gl, g2))
    return dg1, dg2
