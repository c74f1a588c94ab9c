"""Selected elements of the general-basis G2 right-hand side (test infrastructure).

For a system too large for the full-tensor oracle (Nb = 64: every Nb^6 term
of ``general.rhs`` is ~7e10 complex multiply-adds), the same equations are
evaluated for a list of elements (i, j, k, l) only, each at O(Nb^4) cost:

  dG2_ijkl/dt = -i ( [h^(2),HF, G2]_ijkl + S_ijkl )          (eq:result_eom_soa)

  [h2, G2]_ijkl = sum_p h_ip G2_pjkl + h_jp G2_ipkl - G2_ijpl h_pk - G2_ijkp h_pl
                                                             (eq:twopart_hamiltonian)
  Psi^(x)_ijkl  = -sum_pqrs x_pqrs (G>_ip G>_jq G<_rk G<_sl - G<_ip G<_jq G>_rk G>_sl)
                                                             (eq:psi-pm-def)
  GW:  Pi_ijkl  = sum_pq h^eps_qjpl G2_ipkq,
       h^eps_abcd = sum_pq w_qapc (G>_bq G<_pd - G<_bq G>_pd)  (eq:gwpi, eq:gwhcorr)
  TPP: L_ijkl   = sum_pq h^pp_ijpq G2_pqkl,
       h^pp_ijkl  = -sum_pq (G>_ip G>_jq - G<_ip G<_jq) w_pqkl  (eq:lambdapp, eq:HTPPcorr)
  TPH: L_ijkl   = sum_pq h^ph_ipql G2_qjkp,
       h^ph_ijkl  = -sum_pq (G>_ip G<_ql - G<_ip G>_ql) w_pjkq  (eq:lambdaph, eq:HTPHcorr)

with S as in ``general.correlation_terms`` (partners [Pi_lkji]^* and
[L_klij]^*).  Only the quasi-Hamiltonian slices an element needs are formed.
It shares no code with the HIP library; the tests pin it against
``general.rhs`` on small systems.
"""
from __future__ import annotations

import torch

from . import general as G

EIN = torch.einsum


def _psi(wx, gg, gl, i, j, k, l):
    a = EIN("pqrs,p,q,r,s->", wx, gg[i], gg[j], gl[:, k], gl[:, l])
    b = EIN("pqrs,p,q,r,s->", wx, gl[i], gl[j], gg[:, k], gg[:, l])
    return -(a - b)


def _heps_slice(w, gg, gl, b, d):
    """H[a][c] = h^eps_abcd for fixed (b, d)."""
    return EIN("qapc,q,p->ac", w, gg[b], gl[:, d]) - EIN("qapc,q,p->ac", w, gl[b], gg[:, d])


def _pi(w, gg, gl, g2, i, j, k, l):
    H = _heps_slice(w, gg, gl, j, l)           # H[q][p] = h^eps_qjpl
    return EIN("qp,pq->", H, g2[i, :, k, :])   # sum_pq h^eps_qjpl G2_ipkq


def _hpp_slice(w, gg, gl, i, j):
    """H[p][q] = h^pp_ijpq."""
    return -(EIN("rspq,r,s->pq", w, gg[i], gg[j]) - EIN("rspq,r,s->pq", w, gl[i], gl[j]))


def _lpp(w, gg, gl, g2, i, j, k, l):
    return EIN("pq,pq->", _hpp_slice(w, gg, gl, i, j), g2[:, :, k, l])


def _hph_slice(w, gg, gl, i, l):
    """H[p][q] = h^ph_ipql."""
    return -(EIN("xpqy,x,y->pq", w, gg[i], gl[:, l]) - EIN("xpqy,x,y->pq", w, gl[i], gg[:, l]))


def _lph(w, gg, gl, g2, i, j, k, l):
    return EIN("pq,qp->", _hph_slice(w, gg, gl, i, l), g2[:, j, k, :])   # sum_pq h^ph_ipql G2_qjkp


def g2_rhs_elements(h0, w, gl, g2, selfenergy, elements):
    """dG2/dt at the listed (i, j, k, l); returns a complex128 tensor of len(elements)."""
    if selfenergy not in G.SELFENERGIES:
        raise ValueError(selfenergy)
    hhf = G.hf_hamiltonian(h0, w, gl)
    gg = G.greater(gl)
    wm = G.w_minus(w)
    wx = w if selfenergy == "gw" else wm
    out = []
    for (i, j, k, l) in elements:
        comm = (hhf[i] @ g2[:, j, k, l] + hhf[j] @ g2[i, :, k, l]
                - g2[i, j, :, l] @ hhf[:, k] - g2[i, j, k, :] @ hhf[:, l])
        s = _psi(wx, gg, gl, i, j, k, l)
        if selfenergy in ("gw", "gw_x", "dsl"):
            s = s + _pi(w, gg, gl, g2, i, j, k, l) - torch.conj(_pi(w, gg, gl, g2, l, k, j, i))
        if selfenergy in ("tpp", "dsl"):
            s = s + _lpp(w, gg, gl, g2, i, j, k, l) - torch.conj(_lpp(w, gg, gl, g2, k, l, i, j))
        if selfenergy in ("tph", "dsl"):
            s = s + _lph(w, gg, gl, g2, i, j, k, l) - torch.conj(_lph(w, gg, gl, g2, k, l, i, j))
        out.append(-1j * (comm + s))
    return torch.stack(out)
