"""Write the stored expected values under tests/golden/ from the CPU oracle.

Test infrastructure: this script imports only ``oracle`` (the FP64 reference
implementation) and ``workloads`` (the seeded input generators); no value in
these files comes from the GPU library.  Each file holds the oracle's
trajectory of one workload, or the oracle's right-hand-side elements of a
seeded state, sampled so that the GPU tests can compare full-length runs
without re-running the oracle (which takes minutes to hours at these sizes).

    python tests/golden/make_golden.py general_soa_nb32       # ~10 min, 8 threads
    python tests/golden/make_golden.py general_gw_nb64_rhs    # ~2 min
    python tests/golden/make_golden.py general_gw_nb64        # ~2 h, 8 threads

Files (numpy .npz, no pickled objects):
  general_soa_nb32.npz      Nb = 32 SOA molecule, rank-64 w, 8 particles,
                            dt = 0.01, the full 2000 RK4 steps: G1 every 250
                            steps, E and N every 50, 256 G2 elements every 250.
  general_gw_nb64.npz       Nb = 64 GW molecule, rank-128 w, 16 particles,
                            one-step kick 0.1*GUE, dt = 0.01, the full 500
                            steps: G1 in full at steps 1, 5, 100, 500 and at
                            256 entries every 25 steps, E every 25 steps, 320
                            G2 elements at steps 5 and 500.
  general_gw_nb64_rhs.npz   dG2/dt of the Nb = 64 GW closure (with and without
                            exchange) at 320 elements of a seeded random
                            state; the elements cover every 64-row and
                            64-column block of the polarization product and
                            of its partner.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import elements as OE, general as OG, integrate as OI, observables as OO  # noqa: E402
from workloads import general_system, gw_system, random_g2, random_gless, rng  # noqa: E402


def T(x):
    return torch.as_tensor(np.asarray(x), dtype=torch.complex128)


def element_list(nb: int, n: int):
    """n index quadruples in which each of i, j, k, l takes every value 0..nb-1
    (n a multiple of nb), spread by co-prime strides; they hit every row block
    (i) and column block (j) of the pair product, and through the partner
    conj(Pi_lkji) every l and k block as well."""
    q = np.arange(n)
    b = q // nb
    return np.stack([q % nb, (7 * q + 3 + 17 * b) % nb, (13 * q + 5 + 31 * b) % nb,
                     (29 * q + 11 + 47 * b) % nb], 1)


def g1_entry_list(nb: int, n: int):
    """The diagonal plus n - nb off-diagonal entries (i, j) of G1."""
    q = np.arange(n - nb)
    off = np.stack([q % nb, (q * 5 + 1 + q // nb) % nb], 1)
    off = off[off[:, 0] != off[:, 1]]
    return np.concatenate([np.stack([np.arange(nb)] * 2, 1), off], 0)


def _trajectory(s, selfenergy, nsteps, full_at, sample_every, obs_every, g2_at, g2_idx, g1_idx):
    h0, w = T(s.h0), T(s.w)
    hk = None if s.kick is None else h0 + T(s.kick)
    g1 = T(s.g1)
    g2 = torch.zeros((s.nb,) * 4, dtype=torch.complex128)
    out = dict(full_steps=[], full_g1=[], samp_steps=[], samp_g1=[], samp_scale=[], obs_steps=[],
               E_tot=[], E_corr=[], N=[], g2_steps=[], g2_vals=[])
    t = 0.0
    t0 = time.time()
    for n in range(nsteps + 1):
        if n in full_at:
            out["full_steps"].append(n)
            out["full_g1"].append(g1.numpy().copy())
        if n % sample_every == 0:
            out["samp_steps"].append(n)
            out["samp_g1"].append(g1.numpy()[g1_idx[:, 0], g1_idx[:, 1]])
            out["samp_scale"].append(float(g1.abs().max()))
        if n % obs_every == 0:
            o = OO.general_observables(h0, w, g1, g2, t)
            out["obs_steps"].append(n)
            out["E_tot"].append(o["E_tot"])
            out["E_corr"].append(o["E_corr"])
            out["N"].append(o["N"])
        if n in g2_at:
            out["g2_steps"].append(n)
            out["g2_vals"].append(g2.numpy()[tuple(g2_idx.T)])
        if n == nsteps:
            break
        h = hk if (hk is not None and n == 0) else h0
        f = (lambda tt, y, h=h: OG.rhs(h, w, y[0], y[1], selfenergy))
        g1, g2 = OI.rk4_step(f, t, (g1, g2), s.dt)
        t = (n + 1) * s.dt
        if n % 10 == 9:
            print(f"step {n + 1}/{nsteps}  {time.time() - t0:.0f} s", flush=True)
    return {k: np.asarray(v) for k, v in out.items()}


def general_soa_nb32():
    s = general_system()
    g2_idx = element_list(32, 256)
    res = _trajectory(s, "soa", 2000, full_at=set(range(0, 2001, 250)), sample_every=250,
                      obs_every=50, g2_at=set(range(0, 2001, 250)), g2_idx=g2_idx,
                      g1_idx=g1_entry_list(32, 64))
    np.savez(os.path.join(HERE, "general_soa_nb32.npz"), g2_idx=g2_idx, dt=s.dt, **res)


def general_gw_nb64():
    s = gw_system()
    g2_idx = element_list(64, 320)
    res = _trajectory(s, "gw", 500, full_at={1, 5, 100, 500}, sample_every=25, obs_every=25,
                      g2_at={5, 500}, g2_idx=g2_idx, g1_idx=g1_entry_list(64, 256))
    np.savez(os.path.join(HERE, "general_gw_nb64.npz"), g2_idx=g2_idx,
             g1_idx=g1_entry_list(64, 256), dt=s.dt, **res)


def rhs_state(nb: int = 64):
    """The seeded random state of the element test (also drawn by the GPU test)."""
    s = gw_system()
    r = rng(371, nb)
    return s, random_gless(nb, r), random_g2(nb, r, scale=0.02)


def general_gw_nb64_rhs():
    s, gl, g2 = rhs_state()
    idx = element_list(64, 320)
    vals = {}
    for se in ("gw", "gw_x"):
        t0 = time.time()
        vals[se] = OE.g2_rhs_elements(T(s.h0), T(s.w), T(gl), T(g2), se, [tuple(e) for e in idx]).numpy()
        print(f"{se}: {len(idx)} elements in {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "general_gw_nb64_rhs.npz"), idx=idx, gw=vals["gw"], gw_x=vals["gw_x"])


if __name__ == "__main__":
    {"general_soa_nb32": general_soa_nb32, "general_gw_nb64": general_gw_nb64,
     "general_gw_nb64_rhs": general_gw_nb64_rhs}[sys.argv[1]]()
