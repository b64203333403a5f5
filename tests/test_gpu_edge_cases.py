"""Degenerate and smallest cases of the method on the device, against the
oracle: grids of one segment along some or all axes (a single time step, two
spatial nodes), and identical marginals, whose optimum is the static plan
(objective 0, m = 0, rho(t) = rho0 on every slice)."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

SMALL = [(1, (1, 1)), (1, (6, 1)), (2, (1, 1, 1)), (2, (1, 7, 4)), (2, (5, 1, 3)), (2, (3, 6, 1)),
         (3, (1, 1, 1, 1)), (3, (2, 1, 3, 1)), (3, (1, 4, 1, 5))]


@pytest.mark.parametrize("D,n", SMALL, ids=["x".join(map(str, c[1])) for c in SMALL])
@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_smallest_grids_match_the_oracle(D, n, prec):
    inst = dotgen.tiny_instance(D, n, seed=150 + sum(n), floor=0.02)
    iters = 60
    print(f"[case] small grid {D}d n={n} precision={prec}", flush=True)
    P = O.make_problem(D, n, inst.rho0, inst.rho1)
    ref = O.run_fixed(P, iters)
    plan = B.dot_plan_create(D, n, inst.rho0, inst.rho1, None, tol=-1.0, max_iter=100000, precision=prec)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    rho, m = s.extract()
    assert r.iters == iters and r.checks == len(ref.history)
    scale = max(1.0, float(np.max(np.abs(ref.state.alpha[0]))))
    if prec == B.DOT_FP64:
        assert abs(r.objective - ref.objective) <= 1e-8 * abs(ref.objective) + 1e-14
        assert abs(r.sigma - ref.state.sigma) <= 1e-12 * ref.state.sigma
        assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-6 * scale
        for a, b in zip(m, ref.state.alpha[1:]):
            assert np.max(np.abs(a - b)) <= 1e-6 * scale
    else:
        assert abs(r.objective - ref.objective) <= 1e-5 * abs(ref.objective) + 1e-10
        assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-4 * scale


@pytest.mark.parametrize("D,n", [(1, (8, 16)), (2, (6, 8, 10)), (3, (4, 5, 6, 4))], ids=["1d", "2d", "3d"])
def test_identical_marginals_give_the_static_plan(D, n):
    inst = dotgen.tiny_instance(D, n, seed=3)
    print(f"[case] identical marginals {D}d n={n}", flush=True)
    plan = B.dot_plan_create(D, n, inst.rho0, inst.rho0, None, tol=1e-9, max_iter=40000)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(40000)
    assert B.TERM_NAMES[r.term] == "converged" and r.eta_dot <= 1e-9
    assert abs(r.objective) < 1e-9
    rho, m = s.extract()
    for a in m:
        assert np.max(np.abs(a)) < 1e-6
    vol_x = float(np.prod([1.0 / k for k in n[1:]]))
    dens = inst.rho0 / vol_x
    for t in range(n[0]):
        np.testing.assert_allclose(rho[t], dens, atol=1e-6 * dens.max())
