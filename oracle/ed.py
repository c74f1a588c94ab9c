"""Exact diagonalization in Fock space (textbook; used as an independent pin).

Jordan-Wigner encoding of n <= 10 spin orbitals: basis state b = sum_o occ_o 2^o,
c_o |...1_o...> = (-1)^{sum_{o'<o} occ_o'} |...0_o...>.  The Hamiltonian is
eq:h with exactly its operator order:
    H = sum_ij h_ij c+_i c_j + 1/2 sum_ijkl w_ijkl c+_i c+_j c_l c_k.
The initial state is the Slater determinant of the occupied eigenvectors of a
given one-particle density matrix (an uncorrelated state, G2(t0) = 0).
Outputs n_ij(t) = <c+_j c_i> (the paper's n, eq:g-glsymm) and <H>.
"""
from __future__ import annotations

import numpy as np


def annihilators(n: int):
    dim = 1 << n
    cs = []
    for o in range(n):
        c = np.zeros((dim, dim))
        for b in range(dim):
            if (b >> o) & 1:
                sign = (-1) ** bin(b & ((1 << o) - 1)).count("1")
                c[b ^ (1 << o), b] = sign
        cs.append(c)
    return cs


class FockSystem:
    def __init__(self, h: np.ndarray, w: np.ndarray):
        n = h.shape[0]
        self.n = n
        self.c = annihilators(n)
        cd = [c.T for c in self.c]
        self.cd = cd
        dim = 1 << n
        H = np.zeros((dim, dim), dtype=np.complex128)
        for i in range(n):
            for j in range(n):
                if h[i, j] != 0:
                    H += h[i, j] * (cd[i] @ self.c[j])
        nz = np.argwhere(np.abs(w) > 0)
        for i, j, k, l in nz:
            H += 0.5 * w[i, j, k, l] * (cd[i] @ cd[j] @ self.c[l] @ self.c[k])
        self.H = H
        self.evals, self.evecs = np.linalg.eigh(H)

    def slater(self, n0: np.ndarray) -> np.ndarray:
        """|Phi> = prod_a c+_{phi_a} |0> for the eigenvectors phi_a of n0 with eigenvalue 1."""
        ev, v = np.linalg.eigh(n0)
        occ = v[:, ev > 0.5]
        dim = 1 << self.n
        psi = np.zeros(dim, dtype=np.complex128)
        psi[0] = 1.0
        for a in range(occ.shape[1]):
            op = sum(occ[o, a] * self.cd[o] for o in range(self.n))
            psi = op @ psi
        return psi / np.linalg.norm(psi)

    def evolve(self, psi0: np.ndarray, t: float) -> np.ndarray:
        coef = self.evecs.conj().T @ psi0
        return self.evecs @ (np.exp(-1j * self.evals * t) * coef)

    def density_matrix(self, psi: np.ndarray) -> np.ndarray:
        n = self.n
        out = np.zeros((n, n), dtype=np.complex128)
        for i in range(n):
            for j in range(n):
                out[i, j] = np.vdot(psi, self.cd[j] @ (self.c[i] @ psi))
        return out

    def energy(self, psi: np.ndarray) -> float:
        return float(np.real(np.vdot(psi, self.H @ psi)))
