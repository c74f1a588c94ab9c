"""G1-G2 equations for jellium (the uniform electron gas) in a plane-wave basis.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Basis: plane waves on a periodic momentum grid with dims (Lx, Ly, Lz), momentum
index n = x + Lx (y + Ly z) and components added modulo the grid, so the finite
basis is closed under momentum addition and momentum conservation is exact.
The pair interaction is eq:jellium-w-matrix in the convention of eq:h,
    w_{k1 k2 k3 k4}^{a b c d} = delta_ac delta_bd delta(k1 + k2 - k3 - k4) v[k1 - k3],
with v[0] = 0 (the neutralizing background removes the q = 0 term, so the
Hartree part of h^HF vanishes).  G1 is diagonal in momentum and spin,
G^{<,s}_p; G2 is stored in the momentum-transfer form of eq:g2-def-jellium,
    G2[a][b][P][Pb][Q] = G2^{a b a b}_{(P-Q, a), (Pb+Q, b), (P, a), (Pb, b)},
for all four spin pairs (a, b) (the library keeps up-up, up-down and
down-down; down-up follows from eq:Gsymm_a).

The equations are those of Sec. III.E (eq:jellium-g1, eq:jellium-g2), Sec. IV.D
(eq:jellium-gwpi), Sec. V.A (eq:jellium-lambdapp) and Sec. V.B
(eq:jellium-lambdaph), with the fermion signs; the G1 equation is eq:eom_gone
with h^HF and G^< diagonal, so the commutator vanishes and
i dG^<_p/dt = I_p + conj(I_p) (eq:jellium-g1 writes the I term only).
``tests/test_oracle_pins.py`` pins every right-hand side against the
general-basis equations (oracle/general.py) with the plane-wave w above.
All tensors are torch complex128 (CPU); plain gathers and sums, no blocking.
"""
from __future__ import annotations

import numpy as np
import torch

EIN = torch.einsum


# --------------------------------------------------------------------------- momentum grid
def grid_components(dims):
    """Integer components (x, y, z) of every momentum index, shape [Nb, 3]."""
    lx, ly, lz = (list(dims) + [1, 1])[:3]
    n = np.arange(lx * ly * lz)
    return np.stack([n % lx, (n // lx) % ly, n // (lx * ly)], 1)


def grid_index(comp, dims):
    lx, ly, lz = (list(dims) + [1, 1])[:3]
    c = np.asarray(comp)
    return (c[..., 0] % lx) + lx * ((c[..., 1] % ly) + ly * (c[..., 2] % lz))


def add_table(dims):
    """add[a][b] = index of momentum a + b; sub[a][b] = index of a - b."""
    c = grid_components(dims)
    add = grid_index(c[:, None, :] + c[None, :, :], dims)
    sub = grid_index(c[:, None, :] - c[None, :, :], dims)
    return torch.as_tensor(add), torch.as_tensor(sub)


# --------------------------------------------------------------------------- equations
def hf_energies(eps, v, gl, sub):
    """h^{HF,s}_p = eps^s_p + i sum_pb v[p - pb] G^{<,s}_pb (Sec. III.E; the
    Hartree term is v[0] sum G^< = 0)."""
    vm = v[sub]                                   # vm[p][pb] = v[p - pb]
    return eps.to(torch.complex128) + 1j * EIN("pq,sq->sp", vm.to(torch.complex128), gl)


def collision_integral(v, g2):
    """I^a_P = -i sum_{b, Pb, Q} v[Q] G2[a][b][P][Pb][Q] (eq:jellium-g1)."""
    return -1j * EIN("q,abpkq->ap", v.to(torch.complex128), g2)


def g1_rhs(v, g2):
    """dG^{<,a}_P/dt = -i (I^a_P + conj(I^a_P)) (eq:eom_gone, diagonal h and G^<)."""
    i1 = collision_integral(v, g2)
    return -1j * (i1 + i1.conj())


def _gathers(dims, nb):
    add, sub = add_table(dims)
    P = torch.arange(nb)[:, None, None]
    Pb = torch.arange(nb)[None, :, None]
    Q = torch.arange(nb)[None, None, :]
    return add, sub, P, Pb, Q


def commutator(h, g2, dims):
    """G2 (h^a_{P-Q} + h^b_{Pb+Q} - h^a_P - h^b_Pb) (the commutator of eq:jellium-g2)."""
    nb = h.shape[1]
    add, sub, P, Pb, Q = _gathers(dims, nb)
    out = torch.zeros_like(g2)
    for a in range(2):
        for b in range(2):
            e = h[a][sub[P, Q]] + h[b][add[Pb, Q]] - h[a][P] - h[b][Pb]
            out[a, b] = g2[a, b] * e
    return out


def source(v, gg, gl, dims, exchange):
    """Psi^{(+-)}: (1/(i)^2) [v[Q] - delta_ab v[P - Q - Pb]] Phi (eq:jellium-g2), with
    Phi = G>_{P-Q} G>_{Pb+Q} G<_P G<_Pb - G<_{P-Q} G<_{Pb+Q} G>_P G>_Pb ((i)^4 = 1);
    exchange=False keeps v[Q] only (GW without exchange, Sec. IV.D)."""
    nb = gl.shape[1]
    add, sub, P, Pb, Q = _gathers(dims, nb)
    out = torch.zeros((2, 2, nb, nb, nb), dtype=torch.complex128)
    vc = v.to(torch.complex128)
    for a in range(2):
        for b in range(2):
            w = vc[Q].expand(nb, nb, nb).clone()
            if exchange and a == b:
                w = w - vc[sub[sub[P, Q], Pb]]
            phi = (gg[a][sub[P, Q]] * gg[b][add[Pb, Q]] * gl[a][P] * gl[b][Pb]
                   - gl[a][sub[P, Q]] * gl[b][add[Pb, Q]] * gg[a][P] * gg[b][Pb])
            out[a, b] = -w * phi
    return out


def polarization(v, gg, gl, g2, dims):
    """Pi^{ab}_{P,Pb,Q} = (G>^b_{Pb+Q} G<^b_Pb - G<^b_{Pb+Q} G>^b_Pb) v[Q]
    sum_{K,s} G2[a][s][P][K][Q] (eq:jellium-gwpi, fermions: -(i)^2 = +1)."""
    nb = gl.shape[1]
    add, sub, P, Pb, Q = _gathers(dims, nb)
    S = g2.sum(dim=(1, 3))                        # S[a][P][Q] = sum_{s,K} G2[a][s][P][K][Q]
    out = torch.zeros_like(g2)
    vc = v.to(torch.complex128)
    for a in range(2):
        for b in range(2):
            f = gg[b][add[Pb, Q]] * gl[b][Pb] - gl[b][add[Pb, Q]] * gg[b][Pb]
            out[a, b] = f * vc[Q] * S[a][P, Q]
    return out


def pp_ladder(v, gg, gl, g2, dims):
    """Lambda^{pp,ab}_{P,Pb,Q} = (i)^2 (G>^a_{P-Q} G>^b_{Pb+Q} - G<^a_{P-Q} G<^b_{Pb+Q})
    sum_K v[K - Q] G2[a][b][P][Pb][K] (eq:jellium-lambdapp)."""
    nb = gl.shape[1]
    add, sub, P, Pb, Q = _gathers(dims, nb)
    vkq = v.to(torch.complex128)[sub]             # vkq[K][Q] = v[K - Q]
    out = torch.zeros_like(g2)
    for a in range(2):
        for b in range(2):
            f = gg[a][sub[P, Q]] * gg[b][add[Pb, Q]] - gl[a][sub[P, Q]] * gl[b][add[Pb, Q]]
            out[a, b] = -f * EIN("pbk,kq->pbq", g2[a, b], vkq)
    return out


def ph_ladder(v, gg, gl, g2, dims):
    """Lambda^{ph,ab}_{P,Pb,Q} = (i)^2 (G>^a_{P-Q} G<^b_Pb - G<^a_{P-Q} G>^b_Pb)
    sum_K v[K] G2[a][b][P][Pb-K][Q+K] (eq:jellium-lambdaph)."""
    nb = gl.shape[1]
    add, sub, P, Pb, Q = _gathers(dims, nb)
    vc = v.to(torch.complex128)
    out = torch.zeros_like(g2)
    for a in range(2):
        for b in range(2):
            f = gg[a][sub[P, Q]] * gl[b][Pb] - gl[a][sub[P, Q]] * gg[b][Pb]
            acc = torch.zeros((nb, nb, nb), dtype=torch.complex128)
            for K in range(nb):
                acc = acc + vc[K] * g2[a, b][P, sub[Pb, K], add[Q, K]]
            out[a, b] = -f * acc
    return out


def partner_pi(x, dims):
    """[x^{ba}_{Pb+Q, P-Q, Q}]^* as an [a][b][P][Pb][Q] tensor (partner of Pi)."""
    nb = x.shape[2]
    add, sub, P, Pb, Q = _gathers(dims, nb)
    out = torch.zeros_like(x)
    for a in range(2):
        for b in range(2):
            out[a, b] = x[b, a][add[Pb, Q], sub[P, Q], Q.expand(nb, nb, nb)].conj()
    return out


def partner_ladder(x, dims):
    """[x^{ab}_{P-Q, Pb+Q, -Q}]^* (partner of the ladders, Sec. V.A-B)."""
    nb = x.shape[2]
    add, sub, P, Pb, Q = _gathers(dims, nb)
    zero = torch.zeros_like(Q)
    out = torch.zeros_like(x)
    for a in range(2):
        for b in range(2):
            out[a, b] = x[a, b][sub[P, Q], add[Pb, Q], sub[zero, Q]].conj()
    return out


SELFENERGIES = ("soa", "gw", "gw_x", "tpp", "tph")


def rhs(eps, v, gl, g2, dims, selfenergy="soa"):
    """(dG1/dt [2][Nb], dG2/dt [2][2][Nb]^3) of the jellium G1-G2 system:
      soa : Psi^- (eq:jellium-g2)
      gw  : Psi (v[Q] only) + Pi - partner (Sec. IV.D)
      gw_x: Psi^- + Pi - partner
      tpp : Psi^- + Lambda^pp - partner (Sec. V.A)
      tph : Psi^- + Lambda^ph - partner (Sec. V.B)"""
    if selfenergy not in SELFENERGIES:
        raise ValueError(selfenergy)
    eps = torch.as_tensor(eps, dtype=torch.float64)
    v = torch.as_tensor(v, dtype=torch.float64)
    _, sub = add_table(dims)
    h = hf_energies(eps, v, gl, sub)
    gg = gl - 1j
    s = source(v, gg, gl, dims, exchange=selfenergy != "gw")
    if selfenergy in ("gw", "gw_x"):
        pi = polarization(v, gg, gl, g2, dims)
        s = s + pi - partner_pi(pi, dims)
    elif selfenergy == "tpp":
        lam = pp_ladder(v, gg, gl, g2, dims)
        s = s + lam - partner_ladder(lam, dims)
    elif selfenergy == "tph":
        lam = ph_ladder(v, gg, gl, g2, dims)
        s = s + lam - partner_ladder(lam, dims)
    dg2 = -1j * (commutator(h, g2, dims) + s)
    return g1_rhs(v, g2), dg2


def observables(eps, v, gl, g2, dims, t=0.0):
    """N^s = sum_p n^s_p; E = sum eps n - 1/2 sum_s sum_{p,pb} v[p - pb] n^s_p n^s_pb
    - 1/2 Re sum_{ab} sum v[Q] G2[a][b][P][Pb][Q] (the energy of eq:h, as for the
    general basis, with the plane-wave w)."""
    eps = torch.as_tensor(eps, dtype=torch.float64)
    v = torch.as_tensor(v, dtype=torch.float64)
    _, sub = add_table(dims)
    n = torch.real(-1j * gl)
    e_kin = float((eps * n).sum())
    e_mf = float(-0.5 * EIN("pq,sp,sq->", v[sub], n, n))
    e_corr = float(-0.5 * torch.real(EIN("q,abpkq->", v.to(torch.complex128), g2)))
    return dict(t=float(t), N_up=float(n[0].sum()), N_dn=float(n[1].sum()), E_kin=e_kin, E_mf=e_mf,
                E_corr=e_corr, E_tot=e_kin + e_mf + e_corr)


# --------------------------------------------------------------------------- general-basis view
def plane_wave_w(v, dims):
    """eq:jellium-w-matrix as a general-basis w over spin orbitals o = s Nb + p."""
    v = np.asarray(v, dtype=np.float64)
    nb = len(v)
    add, sub = (t.numpy() for t in add_table(dims))
    w = np.zeros((2 * nb,) * 4, dtype=np.complex128)
    for a in range(2):
        for b in range(2):
            for k1 in range(nb):
                for k2 in range(nb):
                    for k3 in range(nb):
                        k4 = sub[add[k1, k2], k3]
                        w[a * nb + k1, b * nb + k2, a * nb + k3, b * nb + k4] = v[sub[k1, k3]]
    return w


def to_general(g2, dims):
    """Embed the jellium channels into a general-basis [2Nb]^4 tensor."""
    nb = g2.shape[2]
    add, sub = add_table(dims)
    out = torch.zeros((2 * nb,) * 4, dtype=torch.complex128)
    for a in range(2):
        for b in range(2):
            for P in range(nb):
                for Pb in range(nb):
                    for Q in range(nb):
                        out[a * nb + int(sub[P, Q]), b * nb + int(add[Pb, Q]), a * nb + P, b * nb + Pb] = \
                            g2[a, b, P, Pb, Q]
    return out


def from_general(x, nb, dims):
    """The jellium channels of a general-basis [2Nb]^4 tensor."""
    add, sub = add_table(dims)
    out = torch.zeros((2, 2, nb, nb, nb), dtype=torch.complex128)
    for a in range(2):
        for b in range(2):
            for P in range(nb):
                for Pb in range(nb):
                    for Q in range(nb):
                        out[a, b, P, Pb, Q] = x[a * nb + int(sub[P, Q]), b * nb + int(add[Pb, Q]),
                                                a * nb + P, b * nb + Pb]
    return out
