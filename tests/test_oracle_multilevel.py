"""Pins for the oracle's multilevel initialisation: the data restriction is
the adjoint of linear interpolation between node grids and keeps the mass,
the prolongation reproduces linear functions, and warm-started levels reach
the same optimum as a solve from zero."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from oracle import multilevel as ML


@pytest.mark.parametrize("shape", [(9,), (5, 9), (5, 7, 9)])
def test_restriction_is_the_adjoint_of_node_interpolation(shape):
    rng = np.random.default_rng(1)
    m = rng.standard_normal(shape)
    nf = [k - 1 for k in shape]
    nc = [k // 2 for k in nf]
    v = rng.standard_normal(tuple(k + 1 for k in nc))
    Pv = ML.prolong_array(v, nc, nf, [False] * len(shape))
    assert abs(np.sum(ML.restrict_masses(m) * v) - np.sum(m * Pv)) <= 1e-12 * np.sum(np.abs(m * Pv))


def test_restriction_keeps_mass_and_handles_masks():
    inst = dotgen.tiny_instance(2, (8, 16, 12), seed=5, floor=0.0, masked=True)
    r = ML.restrict_masses(inst.rho0)
    assert abs(r.sum() - inst.rho0.sum()) <= 1e-15
    nc, r0, r1, mk = ML.coarse_data(inst.n, inst.rho0, inst.rho1, inst.mask)
    assert nc == (4, 8, 6) and r0.shape == (9, 7) and mk.shape == (9, 7)
    np.testing.assert_array_equal(mk, inst.mask[::2, ::2])
    assert np.all(r0[mk != 0] == 0) and abs(r0.sum() - 1) < 1e-14 and abs(r1.sum() - 1) < 1e-14


@pytest.mark.parametrize("stag", [False, True])
def test_prolongation_reproduces_linear_functions(stag):
    nc, nf = 6, 12
    xc = (np.arange(nc) + 0.5) / nc if stag else np.arange(nc + 1) / nc
    xf = (np.arange(nf) + 0.5) / nf if stag else np.arange(nf + 1) / nf
    f = lambda x: 0.3 - 2.0 * x
    out = ML.interp_axis(f(xc)[:, None] * np.ones((1, 3)), 0, nc, nf, stag)
    inside = (xf >= xc[0]) & (xf <= xc[-1])
    np.testing.assert_allclose(out[inside, 0], f(xf[inside]), rtol=0, atol=1e-15)
    # constant beyond the outermost coarse positions
    np.testing.assert_allclose(out[xf < xc[0], 0], f(xc[0]), atol=1e-15)
    np.testing.assert_allclose(out[xf > xc[-1], 0], f(xc[-1]), atol=1e-15)


def test_prolonged_state_shapes_and_sigma():
    inst = dotgen.tiny_instance(2, (4, 6, 8), seed=7, floor=0.05)
    P = O.make_problem(2, inst.n, inst.rho0, inst.rho1)
    S = O.run_fixed(P, 12).state
    gf = O.Grid(2, (8, 12, 16))
    T = ML.prolong_state(S, P.g, gf)
    assert T.q[0].shape == gf.cell_shape and T.q[1].shape == gf.q_shape(1) and T.q[2].shape == gf.q_shape(2)
    assert T.beta.shape == (gf.K,) + gf.cell_shape and T.sigma == S.sigma and T.k == 0


def test_multilevel_reaches_the_plain_optimum():
    inst = dotgen.tiny_instance(2, (4, 8, 8), seed=8, floor=0.02, n_comp=2)
    P = O.make_problem(2, inst.n, inst.rho0, inst.rho1)
    plain = O.solve(P, tol=1e-10, max_iter=30000)
    fine, levels = ML.solve_multilevel(2, inst.n, inst.rho0, inst.rho1, None, levels=1, tol=1e-10, max_iter=30000)
    assert plain.converged and fine.converged and len(levels) == 2
    assert abs(fine.objective - plain.objective) <= 1e-8 * plain.objective
    np.testing.assert_allclose(fine.state.alpha[0], plain.state.alpha[0], atol=1e-6)


def test_level_tolerances():
    assert ML.level_tolerances(1e-4, 3) == pytest.approx([1e-6, 1e-6, 1e-5], rel=1e-12)
    assert ML.level_tolerances(1e-6, 2) == pytest.approx([1e-6, 1e-6], rel=1e-12)
