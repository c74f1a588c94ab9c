"""Jellium (Sec. III.E, Sec. IV.D) on the GPU against the FP64 oracle.

The library keeps the up-up, up-down and down-down blocks of G2 in the
momentum-transfer layout; the oracle keeps all four spin pairs (its down-up
block follows from the others by eq:Gsymm_a).  Tolerances as elsewhere:
binary64 1e-12 for one right-hand side and 1e-10 over trajectories, mixed
precision 1e-5, all relative to the largest element.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import integrate as OI
from oracle import jellium as OJ
from workloads import jellium_system, random_jellium_state, rng

pytestmark = pytest.mark.gpu

BLOCKS = ((0, 0), (0, 1), (1, 1))


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def three(g2):
    """The library's three blocks of a [2][2][nb]^3 oracle tensor."""
    g2 = g2.numpy() if hasattr(g2, "numpy") else g2
    return np.stack([g2[a, b] for a, b in BLOCKS])


def _se(B, se):
    return (B.GW, B.GW_EXCHANGE) if se == "gw_x" else ({"soa": B.SOA, "gw": B.GW, "tpp": B.TPP, "tph": B.TPH}[se], 0)


@pytest.mark.parametrize("dims", [(5,), (3, 3), (2, 3, 2), (4, 4, 4), (10,)])
@pytest.mark.parametrize("se", ["soa", "gw", "gw_x", "tpp", "tph"])
def test_jellium_rhs_parity(lib, dims, se):
    """One right-hand side at a random momentum-conserving state with the pair
    symmetries, every element of dG1 and of the three G2 blocks, on one-, two-
    and three-dimensional grids (the stage's 64-momentum tiles are ragged on
    all of them; the 10-point grid has a dimension longer than the others)."""
    from paper_2002_12717_amd import binding as B
    nb = int(np.prod(dims))
    r = rng(611, nb, len(se))
    gl, g2 = random_jellium_state(dims, r)
    s = jellium_system(dims=dims, lbox=5.0, coupling=3.0)
    code, fl = _se(B, se)
    say(f"[jellium rhs] dims={dims} {se}")
    p = B.Jellium(code, dims, s.eps, s.v, gl, flags=fl)
    G1 = torch.as_tensor(gl, dtype=torch.complex128).cuda()
    G2 = torch.as_tensor(three(g2), dtype=torch.complex128).cuda()
    d1, d2 = torch.zeros_like(G1), torch.zeros_like(G2)
    p.rhs(0.0, G1, G2, d1, d2)
    p.close()
    r1, r2 = OJ.rhs(s.eps, s.v, torch.as_tensor(gl), torch.as_tensor(g2), dims, se)
    e1, e2 = rel(d1.cpu().numpy(), r1.numpy()), rel(d2.cpu().numpy(), three(r2))
    say(f"   err dG1 {e1:.2e}  dG2 {e2:.2e}")
    assert e1 < 1e-12 and e2 < 1e-12


@pytest.mark.parametrize("dims,se,prec", [((3, 3), "soa", "fp64"), ((3, 3), "gw", "fp64"),
                                          ((4, 4, 2), "gw", "fp64"), ((4, 4, 2), "soa", "mixed"),
                                          ((3, 3), "gw_x", "mixed"), ((4, 4, 4), "gw", "fp64"),
                                          ((3, 3), "tpp", "fp64"), ((2, 3, 2), "tph", "fp64"),
                                          ((4, 4, 2), "tpp", "mixed"), ((3, 3), "tph", "mixed")])
def test_jellium_trajectory_parity(lib, dims, se, prec):
    """An interaction quench from the spin-polarized Fermi-Dirac state: G1, the
    three G2 blocks and E against the oracle's propagation."""
    from paper_2002_12717_amd import binding as B
    s = jellium_system(dims=dims, lbox=4.0, coupling=4.0, dt=0.02, nsteps=60)
    code, fl = _se(B, se)
    say(f"[jellium trajectory] dims={dims} {se} {prec}, 60 steps in 3 calls")
    stream = torch.cuda.Stream()
    p = B.Jellium(code, dims, s.eps, s.v, s.g1, flags=fl, stream=stream.cuda_stream,
                  precision=B.FP64 if prec == "fp64" else B.MIXED)
    y = None
    t = 0.0
    worst = 0.0
    e_scale = max(abs(p.observables()["E_tot"]), 1.0)
    for k in range(3):
        p.step(s.dt, 20)
        y, rec = OI.propagate_jellium(s, nsteps=20, selfenergy=se, state=y, t0=t, observables_every=20)
        t += 20 * s.dt
        g1, g2, _ = p.get_state()
        o = p.observables()
        e1, e2 = rel(g1, y[0].numpy()), rel(g2, three(y[1]))
        ee = abs(o["E_tot"] - rec[-1]["E_tot"]) / e_scale
        en = abs(o["N"][0] - rec[-1]["N_up"]) + abs(o["N"][1] - rec[-1]["N_dn"])
        say(f"   t={t:.2f} err G1 {e1:.2e}  G2 {e2:.2e}  E {ee:.2e}  N {en:.1e}")
        worst = max(worst, e1, e2, ee)
    p.close()
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert worst < tol
    if prec == "mixed":
        assert worst > 1e-12


@pytest.mark.parametrize("se", ["soa", "gw", "tpp", "tph"])
def test_jellium_full_size_rhs(lib, se):
    """The benchmark grid (6 x 6 x 6 momenta, G2 of 3 x 216^3 elements) at a
    random symmetric state: every element of one right-hand side (the oracle
    needs about 40 s for TPH here)."""
    from paper_2002_12717_amd import binding as B
    dims = (6, 6, 6)
    r = rng(612, len(se))
    gl, g2 = random_jellium_state(dims, r, scale=0.02)
    s = jellium_system(dims=dims)
    code, fl = _se(B, se)
    say(f"[jellium rhs] full size dims={dims} {se}")
    p = B.Jellium(code, dims, s.eps, s.v, gl, flags=fl)
    G1 = torch.as_tensor(gl, dtype=torch.complex128).cuda()
    G2 = torch.as_tensor(three(g2), dtype=torch.complex128).cuda()
    d1, d2 = torch.zeros_like(G1), torch.zeros_like(G2)
    p.rhs(0.0, G1, G2, d1, d2)
    p.close()
    r1, r2 = OJ.rhs(s.eps, s.v, torch.as_tensor(gl), torch.as_tensor(g2), dims, se)
    e1, e2 = rel(d1.cpu().numpy(), r1.numpy()), rel(d2.cpu().numpy(), three(r2))
    say(f"   err dG1 {e1:.2e}  dG2 {e2:.2e}")
    assert e1 < 1e-12 and e2 < 1e-12


@pytest.mark.parametrize("dims,se", [((6, 6, 6), "tpp"), ((6, 6, 6), "tph"), ((2, 3, 2), "tph"), ((10,), "tpp")])
def test_jellium_ladder_rows_agree(lib, dims, se):
    """The ladder transform with two rows per work-group (the form grids of
    more than 512 momenta take, forced here by G1G2_JEL_LAD_ROWS2) against the
    default four: the rows are transformed independently and alike, so the two
    agree to the rounding of the down-spin polarization sums, which are summed
    with atomics (1e-13 relative; a wrong row or momentum index would differ at
    order one).  With the oracle parity of the default this pins the two-row
    form, for one right-hand side and for two steps of the stepper."""
    from paper_2002_12717_amd import binding as B
    r = rng(613, int(np.prod(dims)), len(se))
    gl, g2 = random_jellium_state(dims, r, scale=0.02)
    s = jellium_system(dims=dims)
    code, fl = _se(B, se)
    say(f"[jellium ladder rows] dims={dims} {se}")
    out = []
    for extra in (0, B.JEL_LAD_ROWS2):
        p = B.Jellium(code, dims, s.eps, s.v, gl, flags=fl | extra)
        G1 = torch.as_tensor(gl, dtype=torch.complex128).cuda()
        G2 = torch.as_tensor(three(g2), dtype=torch.complex128).cuda()
        d1, d2 = torch.zeros_like(G1), torch.zeros_like(G2)
        p.rhs(0.0, G1, G2, d1, d2)
        p.set_state(gl, three(g2))
        p.step(0.02, 2)
        a, b, _ = p.get_state()
        p.close()
        out.append((d1.cpu().numpy(), d2.cpu().numpy(), a, b))
    for x, y in zip(out[0], out[1]):
        assert rel(x, y) < 1e-13


def test_jellium_edge_cases_and_graphs(lib):
    """A single momentum (no interaction: v[0] = 0), zero steps, graph-replayed
    steps against eager launches (the down-spin sums use atomics, so the two
    agree to rounding, not bitwise), and the divergence guard."""
    from paper_2002_12717_amd import binding as B
    s1 = jellium_system(dims=(1,), nsteps=10)
    p = B.Jellium(B.GW, (1,), s1.eps, s1.v, s1.g1)
    p.step(0.02, 10)
    g1, g2, t = p.get_state()
    assert np.array_equal(g1, s1.g1) and np.abs(g2).max() == 0.0 and abs(t - 0.2) < 1e-12
    p.step(0.02, 0)
    p.close()
    s = jellium_system(dims=(3, 3, 2), lbox=4.0, coupling=4.0)
    stream = torch.cuda.Stream()
    pg = B.Jellium(B.GW, s.dims, s.eps, s.v, s.g1, stream=stream.cuda_stream)
    pe = B.Jellium(B.GW, s.dims, s.eps, s.v, s.g1)
    for rep in range(3):
        pg.step(s.dt, 8)
        pe.step(s.dt, 8)
        torch.cuda.synchronize()
        (a1, a2, ta), (b1, b2, tb) = pg.get_state(), pe.get_state()
        assert rel(a1, b1) < 1e-13 and rel(a2, b2) < 1e-13 and ta == tb, rep
    pg.close()
    pe.close()
    g = s.g1.copy()
    g[0, 0] = 3j
    p = B.Jellium(B.SOA, s.dims, s.eps, s.v, g)
    with pytest.raises(B.G1G2Error) as e:
        p.step(s.dt, 2)
    assert e.value.status == B.EDIVERGED and p.observables()["diverged_step"] == 1
    p.close()
