"""Seeded synthetic workloads shaped like the paper's systems.

Conventions (fixed here once and used by every caller):
  * hbar = 1, fermions.
  * One-particle state variable is G^<(t0) = i * n, n the one-particle density
    matrix (Sec. II.B, relation between G^< and n); it is anti-Hermitian.
  * Hubbard inputs are spin resolved: h0[sigma] and G1[sigma] with sigma=0 (up)
    and 1 (down), each Ns x Ns.
  * Pair interaction w_ijkl is the coefficient of 1/2 c+_i c+_j c_l c_k in the
    Hamiltonian (Sec. II.A); generated tensors satisfy w_ijkl = w_jilk and
    w_ijkl = conj(w_klij) exactly.
  * All random draws go through ``rng(*keys)`` = numpy default_rng seeded with
    [12717, *keys]; the draw order of every builder is fixed and documented.

Nothing here evaluates the G1-G2 equations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED = 12717

__all__ = [
    "rng", "chain_hopping", "square_hopping", "gue", "factorized_w",
    "aufbau_gless", "random_gless", "random_g2", "hubbard_spin_orbital_w",
    "HubbardSystem", "GeneralSystem", "Drive",
    "hubbard_chain_system", "general_system", "gw_system",
    "batched_clusters", "adjoint_system",
    "JelliumSystem", "momentum_components", "jellium_system", "random_jellium_state",
]


def rng(*keys: int) -> np.random.Generator:
    return np.random.default_rng([SEED, *[int(k) for k in keys]])


# ----------------------------------------------------------------------------
# lattices and random matrices
# ----------------------------------------------------------------------------

def chain_hopping(ns: int, J: float = 1.0, periodic: bool = False) -> np.ndarray:
    """Nearest-neighbour hopping -J on a 1D chain (Hubbard model, Sec. III.D)."""
    h = np.zeros((ns, ns), dtype=np.complex128)
    for i in range(ns - 1):
        h[i, i + 1] = h[i + 1, i] = -J
    if periodic and ns > 2:
        h[0, ns - 1] = h[ns - 1, 0] = -J
    return h


def square_hopping(lx: int, ly: int, J: float = 1.0, periodic: bool = True) -> np.ndarray:
    """Nearest-neighbour hopping on an lx x ly square cluster; site s = x + lx*y."""
    ns = lx * ly
    h = np.zeros((ns, ns), dtype=np.complex128)

    def site(x, y):
        return x + lx * y

    for y in range(ly):
        for x in range(lx):
            s = site(x, y)
            for dx, dy in ((1, 0), (0, 1)):
                xx, yy = x + dx, y + dy
                if xx >= lx or yy >= ly:
                    if not periodic:
                        continue
                    xx %= lx
                    yy %= ly
                t = site(xx, yy)
                if t == s:
                    continue
                h[s, t] = -J
                h[t, s] = -J
    return h


def gue(n: int, r: np.random.Generator, sigma: float = 1.0) -> np.ndarray:
    """Random Hermitian matrix, off-diagonal E|h_ij|^2 = sigma^2, diagonal N(0, sigma^2).

    Draw order: real parts (n x n), then imaginary parts (n x n).
    """
    a = (r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))) / math.sqrt(2.0)
    return sigma * (a + a.conj().T) / math.sqrt(2.0)


def factorized_w(nb: int, rank: int, r: np.random.Generator) -> np.ndarray:
    """w_ijkl = sum_Q B^Q_ik B^Q_jl with Hermitian B^Q = (L^Q + L^Q^H)/sqrt(2).

    L^Q has i.i.d. CN(0, 1/rank) entries (draw order: real parts [rank,nb,nb],
    then imaginary parts).  The tensor satisfies both Coulomb symmetries of the
    pair interaction exactly (w_ijkl = w_jilk, w_ijkl = conj(w_klij)).
    """
    lq = (r.standard_normal((rank, nb, nb)) + 1j * r.standard_normal((rank, nb, nb))) \
        / math.sqrt(2.0 * rank)
    b = (lq + np.conj(np.swapaxes(lq, 1, 2))) / math.sqrt(2.0)
    # contraction over the auxiliary index Q only (input construction)
    w = np.einsum("qik,qjl->ijkl", b, b, optimize=True)
    return np.ascontiguousarray(w)


def aufbau_gless(h: np.ndarray, nocc: int) -> np.ndarray:
    """G^< = i * P, P the projector on the nocc lowest eigenvectors of h."""
    e, v = np.linalg.eigh(h)
    if 0 < nocc < len(e) and e[nocc] - e[nocc - 1] < 1e-8:
        raise ValueError("degenerate Fermi level: Aufbau occupation is ambiguous")
    vo = v[:, :nocc]
    return 1j * (vo @ vo.conj().T)


def random_gless(nb: int, r: np.random.Generator) -> np.ndarray:
    """Random admissible G^< = i n: n Hermitian with eigenvalues in [0, 1]."""
    a = r.standard_normal((nb, nb)) + 1j * r.standard_normal((nb, nb))
    q, _ = np.linalg.qr(a)
    ev = r.uniform(0.0, 1.0, nb)
    n = (q * ev) @ q.conj().T
    n = 0.5 * (n + n.conj().T)
    return 1j * n


def random_g2(nb: int, r: np.random.Generator, scale: float = 0.05,
              exchange: bool = True) -> np.ndarray:
    """Random correlated pair function: Hermitian as an (ij),(kl) pair matrix and,
    if ``exchange``, symmetric under (ij)(kl) -> (ji)(lk).  Both symmetries hold
    bit-exactly."""
    a = scale * (r.standard_normal((nb,) * 4) + 1j * r.standard_normal((nb,) * 4))
    m = a.reshape(nb * nb, nb * nb)
    m = 0.5 * (m + m.conj().T)
    g = m.reshape((nb,) * 4)
    if exchange:
        g = 0.5 * (g + g.transpose(1, 0, 3, 2))
    return np.ascontiguousarray(g)


def hubbard_spin_orbital_w(ns: int, U: float) -> np.ndarray:
    """Hubbard pair interaction in the spin-orbital basis o = s + ns*sigma
    (Sec. III.D): w = U delta(all four sites equal) delta(s1=s3) delta(s2=s4) (1-delta(s1=s2))."""
    nb = 2 * ns
    w = np.zeros((nb,) * 4, dtype=np.complex128)
    for s in range(ns):
        for a in range(2):
            b = 1 - a
            w[s + ns * a, s + ns * b, s + ns * a, s + ns * b] = U
    return w


# ----------------------------------------------------------------------------
# systems
# ----------------------------------------------------------------------------

@dataclass
class Drive:
    """On-site drive v_i(t) = sum_m c_m exp(-(t - t_m)^2 / (2 tau^2)) x_i, added
    to the diagonal of h0 for both spins."""
    x: np.ndarray            # [Ns]
    c: np.ndarray            # [M]
    t_center: np.ndarray     # [M]
    tau: float

    def potential(self, t: float) -> np.ndarray:
        phi = np.exp(-((t - self.t_center) ** 2) / (2.0 * self.tau ** 2))
        return float(np.dot(self.c, phi)) * self.x


@dataclass
class HubbardSystem:
    name: str
    ns: int
    U: float
    h0: np.ndarray               # [2, Ns, Ns] complex128 (t >= 0)
    g1: np.ndarray               # [2, Ns, Ns] complex128, G^<(t0)
    dt: float
    nsteps: int
    drive: Optional[Drive] = None
    meta: dict = field(default_factory=dict)


@dataclass
class GeneralSystem:
    name: str
    nb: int
    h0: np.ndarray               # [Nb, Nb]
    w: np.ndarray                # [Nb]^4
    g1: np.ndarray               # [Nb, Nb]
    dt: float
    nsteps: int
    kick: Optional[np.ndarray] = None   # added to h0 during step 0 only
    meta: dict = field(default_factory=dict)


def _neel_init(h: np.ndarray, nocc: tuple, stagger: np.ndarray, amp: float,
               jitter: Optional[np.ndarray] = None) -> np.ndarray:
    g = []
    for sig, s_sigma in ((0, 1.0), (1, -1.0)):
        v = amp * s_sigma * stagger
        if jitter is not None:
            v = v + jitter
        g.append(aufbau_gless(h + np.diag(v), nocc[sig]))
    return np.stack(g)


def hubbard_chain_system(ns: int = 8, U: float = 1.0, J: float = 1.0,
                         nup: Optional[int] = None, ndn: Optional[int] = None,
                         confinement: float = 0.5, dt: float = 0.02,
                         nsteps: int = 1000, periodic: bool = False) -> HubbardSystem:
    """1D Hubbard chain, uncorrelated Neel-like initial state (configuration of
    8 sites, U=1, half filling).  The staggered confinement +-0.5 (sign flipped
    between spins) only prepares G^<(t0); it is switched off at t = 0."""
    nup = ns // 2 if nup is None else nup
    ndn = ns // 2 if ndn is None else ndn
    hop = chain_hopping(ns, J, periodic)
    stagger = np.array([(-1.0) ** i for i in range(ns)])
    g1 = _neel_init(hop, (nup, ndn), stagger, confinement)
    return HubbardSystem("hubbard_chain", ns, U, np.stack([hop, hop]), g1, dt, nsteps,
                         meta=dict(J=J, nup=nup, ndn=ndn, periodic=periodic))


def general_system(nb: int = 32, rank: int = 64, nocc: int = 8, dt: float = 0.01,
                   nsteps: int = 2000, key: int = 2) -> GeneralSystem:
    """General-basis molecule-like system.  Draw order from rng(key): h (GUE),
    then the factor L of w.  G^<(t0) is the Aufbau projector of h."""
    r = rng(key, nb, rank)
    h = gue(nb, r)
    w = factorized_w(nb, rank, r)
    g1 = aufbau_gless(h, nocc)
    return GeneralSystem("general_soa", nb, h, w, g1, dt, nsteps,
                         meta=dict(rank=rank, nocc=nocc))


def gw_system(nb: int = 64, rank: int = 128, nocc: int = 16, dt: float = 0.01,
              nsteps: int = 500, kick_scale: float = 0.1, key: int = 3) -> GeneralSystem:
    """General-basis GW workload: as ``general_system`` plus a one-step kick
    dh = kick_scale * GUE drawn after w."""
    r = rng(key, nb, rank)
    h = gue(nb, r)
    w = factorized_w(nb, rank, r)
    kick = kick_scale * gue(nb, r)
    g1 = aufbau_gless(h, nocc)
    return GeneralSystem("general_gw", nb, h, w, g1, dt, nsteps, kick=kick,
                         meta=dict(rank=rank, nocc=nocc))


def batched_clusters(n: int = 512, lmin: int = 3, lmax: int = 6, umin: float = 0.5,
                     umax: float = 4.0, fmin: float = 0.3, fmax: float = 0.7,
                     dt: float = 0.02, nsteps: int = 1000) -> List[HubbardSystem]:
    """Ragged batch of periodic 2D Hubbard clusters.  Per cluster c, rng(4, c)
    draws, in order: Lx, Ly (uniform integers in [lmin, lmax]), U ~ U[umin, umax],
    filling f ~ U[fmin, fmax], then an on-site jitter 0.01*U(-1,1) per site that
    (with the Neel confinement 0.5) lifts degeneracies of the initial state only."""
    out = []
    for c in range(n):
        r = rng(4, c)
        lx = int(r.integers(lmin, lmax + 1))
        ly = int(r.integers(lmin, lmax + 1))
        U = float(r.uniform(umin, umax))
        f = float(r.uniform(fmin, fmax))
        ns = lx * ly
        nocc = max(1, int(round(f * ns)))
        jitter = 0.01 * r.uniform(-1.0, 1.0, ns)
        hop = square_hopping(lx, ly, 1.0, periodic=True)
        stagger = np.array([(-1.0) ** (s % lx + s // lx) for s in range(ns)])
        g1 = _neel_init(hop, (nocc, nocc), stagger, 0.5, jitter)
        out.append(HubbardSystem(f"cluster{c}", ns, U, np.stack([hop, hop]), g1, dt, nsteps,
                                 meta=dict(lx=lx, ly=ly, filling=f, nocc=nocc)))
    return out


def adjoint_system(lx: int = 8, ly: int = 8, U: float = 2.0, nmodes: int = 64,
                   T: float = 40.0, dt: float = 0.01, nsteps: Optional[int] = None,
                   key: int = 5) -> HubbardSystem:
    """Open 2D Hubbard cluster at half filling, Neel initial state, driven by a
    uniform field x_i = ix - (lx-1)/2 with nmodes Gaussian pulses centred at
    t_m = (m + 1/2) T / nmodes, width tau = T / nmodes; c_m ~ N(0, 0.1^2)
    drawn from rng(key, lx, ly)."""
    ns = lx * ly
    hop = square_hopping(lx, ly, 1.0, periodic=False)
    stagger = np.array([(-1.0) ** (s % lx + s // lx) for s in range(ns)])
    g1 = _neel_init(hop, (ns // 2, ns // 2), stagger, 0.5)
    r = rng(key, lx, ly)
    c = 0.1 * r.standard_normal(nmodes)
    tc = (np.arange(nmodes) + 0.5) * T / nmodes
    x = np.array([(s % lx) - 0.5 * (lx - 1) for s in range(ns)], dtype=np.float64)
    drive = Drive(x=x, c=c, t_center=tc, tau=T / nmodes)
    if nsteps is None:
        nsteps = int(round(T / dt))
    return HubbardSystem("hubbard_adjoint", ns, U, np.stack([hop, hop]), g1, dt, nsteps,
                         drive=drive, meta=dict(lx=lx, ly=ly))


# ----------------------------------------------------------------------------
# jellium (plane waves on a periodic momentum grid)
# ----------------------------------------------------------------------------

@dataclass
class JelliumSystem:
    """Uniform electron gas in a plane-wave basis: momenta on a periodic grid
    ``dims`` (index n = x + Lx (y + Ly z), components added modulo the grid),
    one-particle energies eps[spin][n], pair interaction v[q] (v[0] = 0),
    diagonal G^{<,s}_n = i n^s_n."""
    name: str
    dims: tuple
    nb: int
    eps: np.ndarray           # [2, Nb] float64
    v: np.ndarray             # [Nb] float64
    g1: np.ndarray            # [2, Nb] complex128
    dt: float
    nsteps: int
    meta: dict = field(default_factory=dict)


def momentum_components(dims) -> np.ndarray:
    """Minimum-image integer components m(n) of every grid index, [Nb, 3]
    (each component in [-L/2, L/2) for even L)."""
    d = (list(dims) + [1, 1])[:3]
    n = np.arange(d[0] * d[1] * d[2])
    c = np.stack([n % d[0], (n // d[0]) % d[1], n // (d[0] * d[1])], 1)
    L = np.asarray(d)
    return np.where(c >= (L + 1) // 2, c - L, c)


def jellium_system(dims=(6, 6, 6), lbox: float = 2.0 * math.pi, coupling: float = 10.0,
                   temperature: float = 1.0, mu=(2.0, 1.5), dt: float = 0.02,
                   nsteps: int = 500) -> JelliumSystem:
    """Jellium after an interaction quench: momenta k = 2 pi m / lbox on the
    grid, eps = |k|^2 / 2 for both spins, Coulomb v[q] = coupling 4 pi / (Omega
    |k(q)|^2) with Omega = lbox^3 (v[0] = 0), and an uncorrelated spin-polarized
    Fermi-Dirac start n^s = 1 / (exp((eps - mu_s) / T) + 1).  No random draws."""
    m = momentum_components(dims)
    k = 2.0 * math.pi / lbox * m
    k2 = (k * k).sum(1)
    eps1 = 0.5 * k2
    omega = lbox ** 3
    v = np.zeros_like(k2)
    v[k2 > 0] = coupling * 4.0 * math.pi / (omega * k2[k2 > 0])
    occ = np.stack([1.0 / (np.exp((eps1 - mu[s]) / temperature) + 1.0) for s in range(2)])
    g1 = (1j * occ).astype(np.complex128)
    nb = len(eps1)
    return JelliumSystem("jellium", tuple(dims), nb, np.stack([eps1, eps1]), v, g1, dt, nsteps,
                         meta=dict(lbox=lbox, coupling=coupling, temperature=temperature, mu=tuple(mu)))


def random_jellium_state(dims, r: np.random.Generator, scale: float = 0.05):
    """Random diagonal G^< (occupations in (0, 1)) and a random G2 in the
    momentum-transfer layout g2[a][b][P][Pb][Q] with the pair symmetries of
    eq:Gsymm_a/b in that layout: g2[a][b][P][Pb][Q] = g2[b][a][Pb][P][-Q] and
    g2[a][b][P][Pb][Q] = conj(g2[a][b][P-Q][Pb+Q][-Q]).  Draw order: 2 nb
    uniform occupations, then the real and imaginary parts of the 4 nb^3 G2
    entries."""
    d = (list(dims) + [1, 1])[:3]
    nb = d[0] * d[1] * d[2]
    gl = (1j * r.uniform(0.05, 0.95, (2, nb))).astype(np.complex128)
    x = scale * (r.standard_normal((2, 2, nb, nb, nb)) + 1j * r.standard_normal((2, 2, nb, nb, nb)))
    c = np.stack([np.arange(nb) % d[0], (np.arange(nb) // d[0]) % d[1], np.arange(nb) // (d[0] * d[1])], 1)

    def idx(comp):
        return (comp[..., 0] % d[0]) + d[0] * ((comp[..., 1] % d[1]) + d[1] * (comp[..., 2] % d[2]))

    add = idx(c[:, None] + c[None, :])
    sub = idx(c[:, None] - c[None, :])
    neg = idx(-c)
    P = np.arange(nb)[:, None, None]
    Pb = np.arange(nb)[None, :, None]
    Q = np.arange(nb)[None, None, :]
    ex = np.empty_like(x)
    for a in range(2):
        for b in range(2):
            ex[a, b] = x[b, a][Pb, P, neg[Q]]
    x = 0.5 * (x + ex)
    he = np.empty_like(x)
    for a in range(2):
        for b in range(2):
            he[a, b] = np.conj(x[a, b][sub[P, Q], add[Pb, Q], neg[Q]])
    return gl, 0.5 * (x + he)
