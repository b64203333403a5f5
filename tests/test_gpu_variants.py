"""Algorithm variants on the same kernels (Rem. 4.2): the dual step length
tau of Algorithm 2 in (0, 2), including the unrelaxed tau = 1, and the
sigma rule switched off. Parity with the oracle run with the same settings."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tau,adapt", [(1.0, 1), (1.5, 1), (1.9, 0)])
@pytest.mark.parametrize("case", ["2d-mask-8x20x24", "3d-6x9x10x7"])
def test_fixed_iterations_match_the_oracle(case, tau, adapt):
    inst = (dotgen.tiny_instance(2, (8, 20, 24), seed=22, floor=0.0, masked=True) if case.startswith("2d")
            else dotgen.tiny_instance(3, (6, 9, 10, 7), seed=23, floor=0.0))
    print(f"[case] {case} tau={tau} adapt={adapt}", flush=True)
    iters = 150
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    ref = O.run_fixed(P, iters, tau=tau, adapt_sigma=bool(adapt))
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=-1.0, max_iter=100000,
                             tau=tau, adapt_sigma=adapt)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    assert r.iters == iters
    assert abs(r.sigma - ref.state.sigma) <= 1e-12 * ref.state.sigma
    assert abs(r.objective - ref.objective) <= 1e-8 * abs(ref.objective)
    rho, m = s.extract()
    assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-6
    for a, b in zip(m, ref.state.alpha[1:]):
        assert np.max(np.abs(a - b)) <= 1e-6


def test_unrelaxed_step_solves_to_tolerance_like_the_oracle():
    inst = dotgen.tiny_instance(2, (6, 10, 12), seed=31, floor=0.01)
    tol = 1e-7
    P = O.make_problem(2, inst.n, inst.rho0, inst.rho1)
    ref = O.solve(P, tol=tol, max_iter=40000, tau=1.0)
    assert ref.converged
    r, rho, m = B.dot_solve(2, inst.n, inst.rho0, inst.rho1, None, tol=tol, max_iter=40000, tau=1.0)
    assert B.TERM_NAMES[r.term] == "converged"
    assert abs(r.iters - ref.iters) <= 5
    assert abs(r.objective - ref.objective) <= 1e-8 * ref.objective
