"""The allocation-free right-hand side (g1g2_rhs_noalloc) against g1g2_rhs.

Both run the same kernels on the same inputs; the allocation-free call takes
the diagonal gathers of TPH, GW and DSL in the library's static per-GPU
scratch instead of the context's buffer.  Two calls in a row per closure, the
second on a smaller cluster (so the scratch holds the first call's values
where the second does not overwrite them), each compared element by element
with g1g2_rhs at the binary64 bar (they agree bit for bit: same arithmetic).
"""
import numpy as np
import pytest
import torch

from workloads import adjoint_system, chain_hopping, random_g2, random_gless, rng

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _case(ns_side, se, key):
    """An open ns_side x ns_side cluster (8x8: the adjoint workload's lattice)
    or, for ns_side < 0, a chain of -ns_side sites, at a random state."""
    from paper_2002_12717_amd import binding as B
    if ns_side > 0:
        h = adjoint_system(lx=ns_side, ly=ns_side).h0[0]
    else:
        h = chain_hopping(-ns_side)
    ns = h.shape[0]
    r = rng(907, ns, key)
    h0 = np.stack([h + np.diag(r.uniform(-0.3, 0.3, ns)), h + np.diag(r.uniform(-0.3, 0.3, ns))])
    g1 = np.stack([random_gless(ns, r), random_gless(ns, r)])
    nch = 3 if se in ("gw", "dsl") else 1
    g2 = np.stack([random_g2(ns, r, scale=0.05, exchange=False) for _ in range(nch)])
    code = {"tph": B.TPH, "gw": B.GW, "dsl": B.DSL, "soa": B.SOA}[se]
    p = B.Propagator(B.HUBBARD, code, ns, h0, g1, U=1.7)
    G1 = torch.as_tensor(g1, dtype=torch.complex128).cuda()
    G2 = torch.as_tensor(g2 if nch == 3 else g2[0], dtype=torch.complex128).cuda()
    return p, G1, G2


@pytest.mark.parametrize("se", ["tph", "gw", "dsl", "soa"])
def test_rhs_noalloc_matches_rhs(lib, se):
    from paper_2002_12717_amd import binding as B  # noqa: F401
    for call, (side, key) in enumerate([(8, 1), (-10, 2)]):
        p, G1, G2 = _case(side, se, key)
        say(f"[no-alloc rhs] {se} call {call + 1}: ns = {p.nb}")
        ref1, ref2 = torch.zeros_like(G1), torch.zeros_like(G2)
        p.rhs(0.37, G1, G2, ref1, ref2)
        out1, out2 = torch.full_like(G1, float("nan")), torch.full_like(G2, float("nan"))
        p.rhs_noalloc(0.37, G1, G2, out1, out2)
        torch.cuda.synchronize()
        e1 = float((out1 - ref1).abs().max() / ref1.abs().max())
        e2 = float((out2 - ref2).abs().max() / ref2.abs().max())
        say(f"   max rel diff dG1 {e1:.1e}  dG2 {e2:.1e}")
        assert e1 <= 1e-12 and e2 <= 1e-12
        assert torch.equal(out1, ref1) and torch.equal(out2, ref2)
        p.close()


def test_rhs_noalloc_rejects(lib):
    """The general basis and gathers larger than the scratch are refused
    before anything is launched."""
    from paper_2002_12717_amd import binding as B
    from workloads import general_system
    s = general_system(nb=6, rank=4, nocc=2)
    p = B.Propagator(B.GENERAL, B.SOA, s.nb, s.h0, s.g1, w=s.w)
    x = torch.zeros((6, 6), dtype=torch.complex128, device="cuda")
    y = torch.zeros((6,) * 4, dtype=torch.complex128, device="cuda")
    with pytest.raises(B.G1G2Error) as e:
        p.rhs_noalloc(0.0, x, y, x, y)
    assert e.value.status == B.EUNSUPPORTED
    p.close()
    # TPH on a 102-site chain takes the per-element kernel and gathers
    # 2 * 102^3 complex elements (34 MB), more than the 32 MiB scratch
    ns = 102
    h = chain_hopping(ns)
    g1 = np.stack([np.diag([1j] * (ns // 2) + [0] * (ns - ns // 2))] * 2)
    p = B.Propagator(B.HUBBARD, B.TPH, ns, np.stack([h, h]), g1, U=1.0)
    with pytest.raises(B.G1G2Error) as e:
        p.rhs_noalloc(0.0, x, y, x, y)
    assert e.value.status == B.EINVAL and "scratch" in str(e.value)
    p.close()
