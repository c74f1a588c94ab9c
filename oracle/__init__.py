"""Plain FP64 CPU oracle of the G1-G2 scheme (Joost, Schluenzen, Bonitz,
"The G1-G2 scheme", arXiv:2002.12717).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use it.  It shares no code with the HIP path: the only
common module is ``workloads`` (seeded input generators, no method arithmetic).

Everything is written with torch CPU tensors in complex128 / float64 so that
the gradient oracle can differentiate the same code with autograd.  Each
function restates one passage of the paper (cited by section and equation
label) without blocking, fusion or reordering beyond what the equation says;
multi-index sums are evaluated as successive pairwise contractions, which is
how the paper itself evaluates them (Sec. VII.A, eq:soa-skalierung).

Conventions: hbar = 1, fermions (the lower of the +/- signs throughout),
G^< = i n, G^> = G^< - i 1 (Sec. II.B, eq:g-glsymm).  The pair interaction w
is the coefficient of 1/2 c+_i c+_j c_l c_k (eq:h).  The two-particle quantity
G2 is the paper's time-diagonal correlated pair function (eq:gscor-def).

Every function is pinned by ``tests/test_oracle_pins.py`` against something
other than itself: exact diagonalization of small systems, the brute-force
HF-GKBA collision integrals (second Born and GW), the equivalence of the
general-basis equations with the Hubbard reformulations, with the jellium
momentum-space equations and of the direct sums with the reformulated ones,
conservation laws and closed forms (w = 0).  None is parity unpinned.
"""
from . import general, hubbard, integrate, jellium, observables, ed  # noqa: F401
