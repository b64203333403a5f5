"""Whole-solver pins for the oracle: brute-force SOCP optimum on tiny grids,
the exact 1D W2^2, the rho0 = rho1 closed form, symmetries that hold at every
iteration, and invariants of the KKT point."""
import json
import math
import os

import numpy as np
import pytest

import dotgen
from oracle import bruteforce as BFS
from oracle import dot_oracle as O
from oracle import w2_1d

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("D,n,masked", [(1, (4, 6), False), (2, (3, 4, 4), False), (2, (3, 4, 4), True)])
def test_bruteforce_socp_optimum(D, n, masked):
    inst = dotgen.tiny_instance(D, n, masked=masked)
    bf = BFS.solve(D, n, inst.rho0, inst.rho1, inst.mask)
    assert bf["eq_residual"] < 1e-10
    P = O.make_problem(D, n, inst.rho0, inst.rho1, inst.mask)
    r = O.solve(P, tol=1e-11, max_iter=20000)
    assert r.converged
    assert abs(r.objective - bf["objective"]) <= 1e-8 * abs(bf["objective"])
    assert abs(r.dual_objective - bf["objective"]) <= 1e-8 * abs(bf["objective"])
    np.testing.assert_allclose(r.state.alpha[0], bf["rho"], atol=1e-5)
    for a, b in zip(r.state.alpha[1:], bf["m"]):
        np.testing.assert_allclose(a, b, atol=1e-5)


def test_w2_closed_form_helper():
    """The exact quantile integral reproduces the Gaussian closed form as the
    sampling is refined (anchor 0.4^2 + 0.03^2 = 0.1609)."""
    gold = json.load(open(os.path.join(GOLD, "w2_gaussians.json")))
    inst = dotgen.config1_instance(n1=4096, floor=0.0)
    w = w2_1d.w2_squared(inst.rho0, inst.rho1)
    assert abs(w - gold["w2_squared"]) < 2e-4
    # identical densities: zero; a shift of a uniform bump by 1/4: (1/4)^2
    r = np.zeros(65)
    r[8:25] = 1.0
    assert w2_1d.w2_squared(r, r) < 1e-20
    assert abs(w2_1d.w2_squared(r, np.roll(r, 16)) - 0.25 ** 2) < 1e-12


def test_1d_objective_converges_to_w2():
    """2 * objective -> W2^2 of the sampled (piecewise-constant) densities as the
    grid is refined; the paper gives no error bound, so the pin is the measured
    decrease of the error (4e-3 at n1 = 32, 2.7e-4 at n1 = 64)."""
    errs = []
    for n1 in (32, 64):
        inst = dotgen.config1_instance(n1=n1, n0=n1 // 2)
        P = O.make_problem(1, inst.n, inst.rho0, inst.rho1)
        r = O.solve(P, tol=1e-9, max_iter=40000)
        assert r.converged
        w = w2_1d.w2_squared(inst.rho0, inst.rho1)
        errs.append(abs(2 * r.objective - w) / w)
    assert errs[0] < 1e-2
    assert errs[1] < errs[0] / 4


@pytest.mark.parametrize("D,n", [(1, (8, 16)), (2, (6, 8, 10))])
def test_identical_marginals_closed_form(D, n):
    """rho0 = rho1: optimal value 0, m = 0, and rho(t) = rho0 on every slice."""
    inst = dotgen.tiny_instance(D, n, seed=3)
    P = O.make_problem(D, n, inst.rho0, inst.rho0)
    r = O.solve(P, tol=1e-10, max_iter=20000)
    assert r.converged
    assert abs(r.objective) < 1e-9
    for m in r.state.alpha[1:]:
        assert np.max(np.abs(m)) < 1e-6
    vol_x = float(np.prod([1.0 / k for k in n[1:]]))
    dens = inst.rho0 / vol_x
    for t in range(n[0]):
        np.testing.assert_allclose(r.state.alpha[0][t], dens, atol=1e-6 * dens.max())


def _flip_time(S, g):
    """Time reversal: nodes t -> n0 - t, cells t -> n0 - 1 - t."""
    return [np.flip(a, axis=0) for a in S]


@pytest.mark.parametrize("D,n", [(1, (6, 9)), (2, (5, 6, 7))])
def test_time_reversal_symmetry_every_iteration(D, n):
    """Swapping rho0 and rho1 maps the iterates by time reversal: phi -> -phi(reversed),
    rho -> rho(reversed), m -> -m(reversed), at every iteration (zero start)."""
    inst = dotgen.tiny_instance(D, n, seed=4, floor=0.0)
    P1 = O.make_problem(D, n, inst.rho0, inst.rho1)
    P2 = O.make_problem(D, n, inst.rho1, inst.rho0)
    S1 = O.zero_state(P1)
    S2 = O.zero_state(P2)
    upd = set(O.sigma_update_points(200))
    for k in range(60):
        S1 = O.iterate(P1, S1)
        S2 = O.iterate(P2, S2)
        sc = 1 + max(np.abs(a).max() for a in S1.alpha)
        np.testing.assert_allclose(S2.phi, -np.flip(S1.phi, 0), atol=1e-10 * (1 + np.abs(S1.phi).max()))
        np.testing.assert_allclose(S2.alpha[0], np.flip(S1.alpha[0], 0), atol=1e-10 * sc)
        for d in range(1, D + 1):
            np.testing.assert_allclose(S2.alpha[d], -np.flip(S1.alpha[d], 0), atol=1e-10 * sc)
            np.testing.assert_allclose(S2.q[d], -np.flip(S1.q[d], 0), atol=1e-10 * sc)
        if S1.k % 5 == 0:
            r1 = O.residuals(P1, S1.phi, S1.z, S1.q, S1.alpha, S1.beta)
            r2 = O.residuals(P2, S2.phi, S2.z, S2.q, S2.alpha, S2.beta)
            assert abs(r1["eta_dot"] - r2["eta_dot"]) <= 1e-9 * r1["eta_dot"]
            if S1.k in upd:
                S1.sigma, d1 = O.sigma_rule(S1.sigma, r1["eta_p_soc"], r1["eta_d_soc"])
                S2.sigma, d2 = O.sigma_rule(S2.sigma, r2["eta_p_soc"], r2["eta_d_soc"])
                assert d1 == d2


@pytest.mark.parametrize("D,n,axis", [(1, (6, 9), 1), (2, (5, 6, 7), 1), (2, (5, 6, 7), 2)])
def test_mirror_symmetry_every_iteration(D, n, axis):
    """Mirroring x_axis -> 1 - x_axis maps rho to its mirror image, m_axis to
    -m_axis mirrored, the other momenta to their mirror images."""
    inst = dotgen.tiny_instance(D, n, seed=5, floor=0.0)
    f0 = np.flip(inst.rho0, axis - 1)
    f1 = np.flip(inst.rho1, axis - 1)
    P1 = O.make_problem(D, n, inst.rho0, inst.rho1)
    P2 = O.make_problem(D, n, f0, f1)
    S1 = O.zero_state(P1)
    S2 = O.zero_state(P2)
    for k in range(40):
        S1 = O.iterate(P1, S1)
        S2 = O.iterate(P2, S2)
        sc = 1 + max(np.abs(a).max() for a in S1.alpha)
        np.testing.assert_allclose(S2.phi, np.flip(S1.phi, axis), atol=1e-10 * (1 + np.abs(S1.phi).max()))
        np.testing.assert_allclose(S2.alpha[0], np.flip(S1.alpha[0], axis), atol=1e-10 * sc)
        for d in range(1, D + 1):
            sgn = -1.0 if d == axis else 1.0
            np.testing.assert_allclose(S2.alpha[d], sgn * np.flip(S1.alpha[d], axis), atol=1e-10 * sc)


def test_kkt_invariants_at_convergence():
    """At the solution: every time slice carries unit mass (sum of the continuity
    equation over space), rho >= 0 up to the tolerance, m = r . q (eta_C small),
    and the duality gap vanishes (strong duality, Prop. 3.1)."""
    inst = dotgen.tiny_instance(2, (8, 12, 12), seed=9, floor=0.0, n_comp=3)
    P = O.make_problem(2, inst.n, inst.rho0, inst.rho1)
    r = O.solve(P, tol=1e-8, max_iter=30000)
    assert r.converged
    vol_x = float(np.prod([1.0 / k for k in inst.n[1:]]))
    masses = r.state.alpha[0].sum(axis=(1, 2)) * vol_x
    np.testing.assert_allclose(masses, 1.0, atol=1e-6)
    assert r.state.alpha[0].min() > -1e-5
    assert O.duality_gap(r.objective, r.dual_objective) < 1e-6
    assert r.res["eta_c"] <= 1e-8


def test_sigma_rule_constants():
    gold = json.load(open(os.path.join(GOLD, "sigma_rule.json")))
    s, d = O.sigma_rule(1.0, 2.0 * gold["s_r"], 1.0)
    assert d == 1 and s == gold["s_sigma"]
    s, d = O.sigma_rule(1.0, 1.0, 2.0 * gold["s_r"])
    assert d == -1 and s == 1.0 / gold["s_sigma"]
    s, d = O.sigma_rule(1.0, 1.0, 1.5)
    assert d == 0 and s == 1.0
    pts = O.sigma_update_points(400)
    assert pts[:6] == [10, 25, 45, 70, 105, 150]
    assert all(p % 5 == 0 for p in pts)


@pytest.mark.parametrize("tau", [1.0, 1.5])
def test_step_length_variants_reach_the_bruteforce_optimum(tau):
    """Rem. 4.2: any dual step length tau in (0, 2) converges to the same
    optimum; tau = 1 is the unrelaxed variant. The oracle with tau = 1 and
    1.5 reaches the brute-force SOCP optimum on a tiny masked 2D grid."""
    inst = dotgen.tiny_instance(2, (3, 4, 4), masked=True)
    bf = BFS.solve(2, (3, 4, 4), inst.rho0, inst.rho1, inst.mask)
    P = O.make_problem(2, (3, 4, 4), inst.rho0, inst.rho1, inst.mask)
    r = O.solve(P, tol=1e-11, max_iter=40000, tau=tau)
    assert r.converged
    assert abs(r.objective - bf["objective"]) <= 1e-8 * abs(bf["objective"])
    np.testing.assert_allclose(r.state.alpha[0], bf["rho"], atol=1e-5)


def test_step_length_scales_only_the_multiplier_steps():
    """tau enters the multiplier steps only: from the same state, one
    iteration gives the same phi, z and q_new for any tau, and the alpha and
    beta increments are proportional to tau."""
    inst = dotgen.tiny_instance(2, (4, 5, 6), seed=3, floor=0.0, n_comp=3)
    P = O.make_problem(2, inst.n, inst.rho0, inst.rho1)
    S = O.zero_state(P)
    for _ in range(7):
        S = O.iterate(P, S)
    a = O.iterate(P, S, tau=1.0)
    b = O.iterate(P, S, tau=1.6)
    np.testing.assert_array_equal(a.phi, b.phi)
    np.testing.assert_array_equal(a.z, b.z)
    for qa, qb in zip(a.q, b.q):
        np.testing.assert_array_equal(qa, qb)
    for x0, xa, xb in zip(S.alpha, a.alpha, b.alpha):
        np.testing.assert_allclose(1.6 * (xa - x0), xb - x0, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(1.6 * (a.beta - S.beta), b.beta - S.beta, rtol=1e-12, atol=1e-14)
