"""CPU pin of the gradient oracle: the autograd gradient of the discrete RK4
map equals central finite differences of the oracle's own forward map."""
import numpy as np

from oracle import adjoint as OA
from workloads import adjoint_system


def _weights(s):
    ns = s.ns
    lx = s.meta["lx"]
    a = np.full(ns, 1.0 / ns)
    b = np.array([1.0 if (q % lx) < lx / 2 else -1.0 for q in range(ns)]) / ns
    return a, b


def test_oracle_gradient_matches_finite_differences():
    s = adjoint_system(lx=3, ly=2, U=2.0, nmodes=8, T=1.0, dt=0.02)
    a, b = _weights(s)
    L, gc, gU = OA.loss_and_gradient(s, a, b)
    h = 1e-6
    fd_u = (OA.loss_only(s, a, b, U=s.U + h) - OA.loss_only(s, a, b, U=s.U - h)) / (2 * h)
    assert abs(fd_u - gU) < 1e-8 * max(1.0, abs(gU))
    for m in (0, 3, 7):
        c = s.drive.c.copy()
        c[m] += h
        lp = OA.loss_only(s, a, b, c=c)
        c[m] -= 2 * h
        lm = OA.loss_only(s, a, b, c=c)
        assert abs((lp - lm) / (2 * h) - gc[m]) < 1e-8 * max(1.0, abs(gc[m]))
    assert np.abs(gc).max() > 1e-3 and abs(gU) > 1e-4
