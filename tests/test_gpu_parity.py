"""Parity of the HIP path (through the C ABI) with the FP64 oracle, step by
step and for whole fixed-iteration runs. FP64 mode: steps agree to ~1e-12
relative; whole runs to 1e-8 relative in the objective and 1e-6 in rho, m."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

CASES = {
    "1d-16x32": lambda: dotgen.config1_instance(),
    "2d-ragged-12x70x45": lambda: dotgen.tiny_instance(2, (12, 70, 45), seed=21, floor=0.0, n_comp=3),
    "2d-mask-8x20x24": lambda: dotgen.tiny_instance(2, (8, 20, 24), seed=22, floor=0.0, masked=True),
    "3d-6x9x10x7": lambda: dotgen.tiny_instance(3, (6, 9, 10, 7), seed=23, floor=0.0),
    "2d-32x64x64": lambda: dotgen.config2_instance(),
    "2d-1x1x1": lambda: dotgen.tiny_instance(2, (1, 1, 1), seed=24, floor=0.1),
    "1d-1x5": lambda: dotgen.tiny_instance(1, (1, 5), seed=25, floor=0.1),
    "1d-3x300": lambda: dotgen.tiny_instance(1, (3, 300), seed=26, floor=0.0),
    # last axis of 301 nodes: solved by tridiagonal elimination, not transformed
    "2d-long-last-4x7x300": lambda: dotgen.tiny_instance(2, (4, 7, 300), seed=27, floor=0.0, masked=True),
    # last axis of 2601 nodes: longer than any transform tile holds (the
    # elimination has no length limit)
    "2d-very-long-last-3x5x2600": lambda: dotgen.tiny_instance(2, (3, 5, 2600), seed=28, floor=0.0),
}


def _setup(name):
    inst = CASES[name]()
    print(f"[case] {name} n={inst.n}", flush=True)
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=-1.0, max_iter=100000)
    return inst, P, plan


def _random_state(P, seed):
    rng = np.random.default_rng(seed)
    g = P.g
    q = [rng.standard_normal(s) for s in G.q_shapes(g)]
    al = [rng.uniform(0, 2, s) if i == 0 else rng.standard_normal(s) for i, s in enumerate(G.q_shapes(g))]
    be = rng.standard_normal((g.K,) + g.cell_shape)
    phi = rng.standard_normal(g.node_shape)
    return phi, q, al, be


STEP_CASES = ["1d-16x32", "2d-ragged-12x70x45", "2d-mask-8x20x24", "3d-6x9x10x7", "2d-1x1x1", "1d-1x5", "1d-3x300",
              "2d-long-last-4x7x300", "2d-very-long-last-3x5x2600"]


def _poisson_tol(n):
    """Tolerance of the Poisson step against the oracle's cosine-transform
    solve. Transformed axes: FP64 rounding of the transforms (1e-11). A last
    axis of >= 257 nodes is eliminated line by line; elimination without
    pivoting of these diagonally dominant systems is backward stable, so its
    forward error is bounded by kappa * eps with kappa = (lam + 4 n_D^2) / lam
    for the line with the smallest nonzero eigenvalue sum lam of the other
    axes (4 n_a^2 sin^2(pi / (2 (n_a + 1))) for the axis a that minimises it)."""
    D = len(n) - 1
    if n[D] + 1 < 257:
        return 1e-11
    lam = min(4.0 * k * k * np.sin(np.pi / (2 * (k + 1))) ** 2 for k in n[:D])
    kappa = (lam + 4.0 * n[D] ** 2) / lam
    return max(1e-11, kappa * np.finfo(np.float64).eps)


@pytest.mark.parametrize("name", STEP_CASES)
def test_step_divergence_and_poisson(name):
    inst, P, plan = _setup(name)
    g = P.g
    phi, q, al, be = _random_state(P, 1)
    sigma = 0.8
    st = G.stream_handle()
    qd = G.dev(G.planes_of(q, g.n))
    ad = G.dev(G.planes_of(al, g.n))
    bd = G.dev(np.zeros(g.node_shape))
    B.dot_step_divergence(plan, qd.data_ptr(), ad.data_ptr(), sigma, bd.data_ptr(), st)
    b_ref = O.step_rhs(P, q, al, sigma)
    assert G.rel_err(G.host(bd), b_ref) < 1e-13
    # a4 alone, in place
    B.dot_step_poisson(plan, bd.data_ptr(), st)
    phi_ref = O.poisson(b_ref, g)
    tol = _poisson_tol(inst.n)
    assert G.rel_err(G.host(bd), phi_ref) < tol
    # a3 + a4 fused as the iteration runs it
    pd = G.dev(np.zeros(g.node_shape))
    B.dot_step_rhs_poisson(plan, qd.data_ptr(), ad.data_ptr(), sigma, pd.data_ptr(), st)
    assert G.rel_err(G.host(pd), phi_ref) < tol


@pytest.mark.parametrize("name", STEP_CASES)
def test_step_cone(name):
    inst, P, plan = _setup(name)
    g = P.g
    phi, q, al, be = _random_state(P, 2)
    sigma = 1.3
    st = G.stream_handle()
    qd = G.dev(G.planes_of(q, g.n))
    bed = G.dev(G.planes_of(list(be), g.n))
    zd = G.dev(np.zeros((g.K,) + g.node_shape))
    B.dot_step_cone(plan, qd.data_ptr(), bed.data_ptr(), sigma, zd.data_ptr(), st)
    z_ref = O.proj_soc(O.step_cone_input(P, q, be, sigma))
    z = np.stack([B.from_box(p, g.cell_shape) for p in G.host(zd)])
    assert G.rel_err(z, z_ref) < 1e-13


@pytest.mark.parametrize("name", STEP_CASES)
def test_step_update(name):
    inst, P, plan = _setup(name)
    g = P.g
    phi, q, al, be = _random_state(P, 3)
    sigma, tau = 0.6, 1.9
    st = G.stream_handle()
    pd = G.dev(B.to_box(phi, g.n))
    qd = G.dev(G.planes_of(q, g.n))
    ad = G.dev(G.planes_of(al, g.n))
    bed = G.dev(G.planes_of(list(be), g.n))
    qo = G.dev(np.zeros((g.D + 1,) + g.node_shape))
    wd = G.dev(np.zeros((4 * g.D + 1,) + g.node_shape))
    B.dot_step_update(plan, pd.data_ptr(), qd.data_ptr(), ad.data_ptr(), bed.data_ptr(), sigma, tau,
                      qo.data_ptr(), wd.data_ptr(), st)
    S = O.State(phi, np.zeros_like(be), q, al, be, sigma)
    # the oracle's z-step, q-step and multiplier steps for this phi
    z = O.proj_soc(O.step_cone_input(P, q, be, sigma))
    qn = O.step_q(P, phi, z, al, be, sigma)
    Aphi = O.grad(phi, g)
    al_n = [a + tau * sigma * (ap - qq) for a, ap, qq in zip(al, Aphi, qn)]
    be_n = be + tau * sigma * (z - O.BF(qn, P.omega, g) - O.cone_offset(g))
    shapes = G.q_shapes(g)
    for a, b in zip(G.unpack(G.host(qo), shapes), qn):
        assert G.rel_err(a, b) < 1e-12
    for a, b in zip(G.unpack(G.host(ad), shapes), al_n):
        assert G.rel_err(a, b) < 1e-12
    bn = np.stack([B.from_box(p, g.cell_shape) for p in G.host(bed)])
    assert G.rel_err(bn, be_n) < 1e-12
    # pads stay zero
    assert np.all(G.host(qo)[0][-1] == 0)


@pytest.mark.parametrize("name", STEP_CASES)
def test_step_residuals(name):
    inst, P, plan = _setup(name)
    g = P.g
    S = O.zero_state(P)
    for _ in range(7):
        S = O.iterate(P, S)
    st = G.stream_handle()
    args = [G.dev(B.to_box(S.phi, g.n)), G.dev(G.planes_of(list(S.z), g.n)), G.dev(G.planes_of(S.q, g.n)),
            G.dev(G.planes_of(S.alpha, g.n)), G.dev(G.planes_of(list(S.beta), g.n))]
    r = B.dot_step_residuals(plan, *[a.data_ptr() for a in args], st)
    ref = O.residuals(P, S.phi, S.z, S.q, S.alpha, S.beta)
    for k in ("eta_dot", "eta_p", "eta_d", "eta_c", "eta_p_soc", "eta_d_soc"):
        assert abs(getattr(r, k) - ref[k]) <= 1e-10 * abs(ref[k]) + 1e-300, k
    assert abs(r.objective - O.objective(P, S.phi)) <= 1e-10 * (1e-12 + abs(O.objective(P, S.phi)))
    assert abs(r.dual_objective - O.dual_objective(P, S.alpha)) <= 1e-10 * abs(O.dual_objective(P, S.alpha))


RUN_CASES = [("1d-16x32", 400), ("2d-ragged-12x70x45", 150), ("2d-mask-8x20x24", 200), ("3d-6x9x10x7", 80),
             ("2d-32x64x64", 60), ("1d-1x5", 100), ("2d-long-last-4x7x300", 60),
             ("2d-very-long-last-3x5x2600", 40)]


@pytest.mark.parametrize("name,iters", RUN_CASES)
def test_fixed_iteration_run(name, iters):
    """Whole iterations on the device (sigma rule and checks on the device)
    against the oracle with the same schedule: objective within 1e-8 relative,
    rho and m within 1e-6 in max norm."""
    inst, P, plan = _setup(name)
    ref = O.run_fixed(P, iters)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    assert r.iters == iters
    assert r.checks == len(ref.history)
    assert abs(r.sigma - ref.state.sigma) <= 1e-12 * ref.state.sigma
    assert abs(r.objective - ref.objective) <= 1e-8 * abs(ref.objective) + 1e-14
    assert abs(r.eta_dot - ref.res["eta_dot"]) <= 1e-6 * ref.res["eta_dot"]
    rho, m = s.extract()
    assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-6
    for a, b in zip(m, ref.state.alpha[1:]):
        assert np.max(np.abs(a - b)) <= 1e-6


def test_solve_to_tolerance_1d():
    """The 1D Gaussian pair to eta_dot <= 1e-8 (device-side stop): same stopping
    check as the oracle (within one check) and the same objective."""
    inst, P, plan = _setup("1d-16x32")
    ref = O.solve(P, tol=1e-8, max_iter=20000)
    assert ref.converged
    plan2 = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, None, tol=1e-8, max_iter=20000)
    s = G.GpuState(plan2)
    s.reset()
    r = s.run(20000)
    assert B.TERM_NAMES[r.term] == "converged"
    assert r.eta_dot <= 1e-8
    assert abs(r.iters - ref.iters) <= 5
    assert abs(r.objective - ref.objective) <= 1e-8 * ref.objective


def test_run_is_deterministic():
    inst, P, plan = _setup("2d-ragged-12x70x45")
    outs = []
    for _ in range(2):
        s = G.GpuState(plan)
        s.reset()
        s.run(25)
        outs.append(s.raw().copy())
    assert np.array_equal(outs[0], outs[1])


def test_split_runs_equal_one_run():
    """Running 20 + 17 iterations equals running 37 (state fully on device)."""
    inst, P, plan = _setup("2d-mask-8x20x24")
    a = G.GpuState(plan)
    a.reset()
    a.run(20)
    a.run(17)
    b = G.GpuState(plan)
    b.reset()
    b.run(37)
    assert np.array_equal(a.raw(), b.raw())


def test_dot_solve_one_shot():
    inst = dotgen.tiny_instance(2, (6, 10, 12), seed=31, floor=0.01)
    r, rho, m = B.dot_solve(2, inst.n, inst.rho0, inst.rho1, None, tol=1e-7, max_iter=20000)
    P = O.make_problem(2, inst.n, inst.rho0, inst.rho1)
    ref = O.solve(P, tol=1e-7, max_iter=20000)
    assert B.TERM_NAMES[r.term] == "converged"
    assert abs(r.objective - ref.objective) <= 1e-6 * ref.objective
    assert np.max(np.abs(rho - ref.state.alpha[0])) < 1e-4


@pytest.mark.parametrize("name,iters", [("2d-mask-8x20x24", 137), ("3d-6x9x10x7", 64)])
def test_graph_replay_equals_plain_launches(name, iters):
    """Captured graphs replayed many times, with host polls and syncs between
    replays, give bitwise the iterates of plain launches; so does a run whose
    first two captures fail (forced from the host before they start: the
    blocks fall back to plain launches, and the next run call captures)."""
    inst, P, plan = _setup(name)
    states = []
    for graphs, failures in ((False, 0), (True, 0), (True, 2)):
        B.dot_plan_set_graphs(plan, graphs)
        s = G.GpuState(plan)
        s.reset()
        B.dot_test_fail_captures(failures)
        try:
            s.run(33)
        finally:
            B.dot_test_fail_captures(0)
        s.run(iters - 33)
        states.append(s.raw().copy())
    assert np.array_equal(states[0], states[1])
    assert np.array_equal(states[0], states[2])


def test_headline_solve_matches_the_converged_oracle():
    """The headline workload (2D 32x64^2, three-component mixtures, FP64, default
    settings) solved to eta_dot <= 1e-6 on the device against the oracle's
    converged solve of the same instance (tests/golden/config2_converged.json,
    written by make_config2_golden.py from oracle/ only): the same iteration
    and check counts and sigma sequence, objective and dual objective within
    1e-8 relative, rho and m within 1e-6 at the 4096 stored positions each."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config2_converged.json")))
    inst = dotgen.config2_instance()
    assert inst.label == gold["instance"] and list(inst.n) == gold["n"]
    print("[case] headline solve 2D 32x64x64 FP64 to 1e-6 vs the converged oracle", flush=True)
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=1e-6, max_iter=100000)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(100000)
    assert B.TERM_NAMES[r.term] == "converged"
    assert r.iters == gold["iters"] and r.checks == gold["checks"]
    assert r.sigma_changes == gold["sigma_changes"]
    assert abs(r.sigma - gold["sigma_final"]) <= 1e-12 * gold["sigma_final"]
    assert abs(r.objective - gold["objective"]) <= 1e-8 * abs(gold["objective"])
    assert abs(r.dual_objective - gold["dual_objective"]) <= 1e-8 * abs(gold["dual_objective"])
    assert abs(r.eta_dot - gold["residuals"]["eta_dot"]) <= 1e-6 * gold["residuals"]["eta_dot"]
    rho, m = s.extract()
    mflat = np.concatenate([a.ravel() for a in m])
    assert np.max(np.abs(rho.ravel()[gold["rho_index"]] - np.array(gold["rho_value"]))) <= 1e-6
    assert np.max(np.abs(mflat[gold["m_index"]] - np.array(gold["m_value"]))) <= 1e-6
