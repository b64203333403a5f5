"""Mixed-precision mode (FP32 bulk state and transforms with FP64 defect
correction of phi, FP64 projection / gradients / reductions) against the
FP64 oracle and the FP64 GPU path. Steps are compared with the oracle run on
the same FP32-rounded inputs; tolerances follow from FP32 rounding of the
stored outputs (~1e-7 relative) and of the transform (~1e-6)."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

CASES = {
    "2d-ragged-12x70x45": lambda: dotgen.tiny_instance(2, (12, 70, 45), seed=21, floor=0.0, n_comp=3),
    "2d-mask-8x20x24": lambda: dotgen.tiny_instance(2, (8, 20, 24), seed=22, floor=0.0, masked=True),
    "3d-6x9x10x7": lambda: dotgen.tiny_instance(3, (6, 9, 10, 7), seed=23, floor=0.0),
    "1d-3x300": lambda: dotgen.tiny_instance(1, (3, 300), seed=26, floor=0.0),
}


def _setup(name, **kw):
    inst = CASES[name]() if name in CASES else name
    print(f"[case] {inst.label} n={inst.n} mixed", flush=True)
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    args = dict(tol=-1.0, max_iter=100000, precision=B.DOT_MIXED)
    args.update(kw)
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, **args)
    assert plan.info.scalar_bytes == 4
    return inst, P, plan


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _random_state(P, seed):
    rng = np.random.default_rng(seed)
    g = P.g
    q = [_f32(rng.standard_normal(s)) for s in G.q_shapes(g)]
    al = [_f32(rng.uniform(0, 2, s) if i == 0 else rng.standard_normal(s)) for i, s in enumerate(G.q_shapes(g))]
    be = _f32(rng.standard_normal((g.K,) + g.cell_shape))
    phi = rng.standard_normal(g.node_shape)
    return phi, q, al, be


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_steps(name):
    inst, P, plan = _setup(name)
    g = P.g
    phi, q, al, be = _random_state(P, 5)
    sigma, tau = 0.7, 1.9
    st = G.stream_handle()
    f32 = np.float32
    qd = G.dev(G.planes_of(q, g.n, f32))
    ad = G.dev(G.planes_of(al, g.n))  # alpha is FP64 in both modes
    bed = G.dev(G.planes_of(list(be), g.n, f32))
    # a3: FP64 arithmetic on FP32 inputs
    bd = G.dev(np.zeros(g.node_shape))
    B.dot_step_divergence(plan, qd.data_ptr(), ad.data_ptr(), sigma, bd.data_ptr(), st)
    b_ref = O.step_rhs(P, q, al, sigma)
    assert G.rel_err(G.host(bd), b_ref) < 1e-13
    # a4: FP32 transforms
    B.dot_step_poisson(plan, bd.data_ptr(), st)
    phi_ref = O.poisson(b_ref, g)
    assert G.rel_err(G.host(bd), phi_ref) < 2e-5
    # a1 + a2: FP64 projection, FP32 output
    zd = G.dev(np.zeros((g.K,) + g.node_shape, dtype=f32))
    B.dot_step_cone(plan, qd.data_ptr(), bed.data_ptr(), sigma, zd.data_ptr(), st)
    z_ref = O.proj_soc(O.step_cone_input(P, q, be, sigma))
    z = np.stack([B.from_box(p, g.cell_shape) for p in G.host(zd)])
    assert G.rel_err(z, z_ref) < 1e-6
    # a5 with an FP64 phi
    pd = G.dev(B.to_box(phi, g.n))
    qo = G.dev(np.zeros((g.D + 1,) + g.node_shape, dtype=f32))
    wd = G.dev(np.zeros((4 * g.D + 2,) + g.node_shape, dtype=f32))  # 4D FP32 planes, then one FP64
    B.dot_step_update(plan, pd.data_ptr(), qd.data_ptr(), ad.data_ptr(), bed.data_ptr(), sigma, tau,
                      qo.data_ptr(), wd.data_ptr(), st)
    qn = O.step_q(P, phi, z_ref, al, be, sigma)
    Aphi = O.grad(phi, g)
    al_n = [a + tau * sigma * (ap - qq) for a, ap, qq in zip(al, Aphi, qn)]
    be_n = be + tau * sigma * (z_ref - O.BF(qn, P.omega, g) - O.cone_offset(g))
    shapes = G.q_shapes(g)
    for a, b in zip(G.unpack(G.host(qo), shapes), qn):
        assert G.rel_err(a, b) < 1e-6
    for a, b in zip(G.unpack(G.host(ad), shapes), al_n):
        assert G.rel_err(a, b) < 1e-6
    bn = np.stack([B.from_box(p, g.cell_shape) for p in G.host(bed)])
    assert G.rel_err(bn, be_n) < 1e-6


def test_mixed_residuals_are_fp64_reductions():
    inst, P, plan = _setup("2d-mask-8x20x24")
    g = P.g
    S = O.zero_state(P)
    for _ in range(9):
        S = O.iterate(P, S)
    q = [_f32(a) for a in S.q]
    al = [_f32(a) for a in S.alpha]
    be = _f32(S.beta)
    z = _f32(S.z)
    st = G.stream_handle()
    f32 = np.float32
    args = [G.dev(B.to_box(S.phi, g.n)), G.dev(G.planes_of(list(z), g.n, f32)), G.dev(G.planes_of(q, g.n, f32)),
            G.dev(G.planes_of(al, g.n)), G.dev(G.planes_of(list(be), g.n, f32))]
    r = B.dot_step_residuals(plan, *[a.data_ptr() for a in args], st)
    ref = O.residuals(P, S.phi, z, q, al, be)
    for k in ("eta_dot", "eta_p", "eta_d", "eta_c", "eta_p_soc", "eta_d_soc"):
        assert abs(getattr(r, k) - ref[k]) <= 1e-10 * abs(ref[k]), k


@pytest.mark.parametrize("name,iters", [("2d-ragged-12x70x45", 200), ("2d-mask-8x20x24", 200), ("3d-6x9x10x7", 100)])
def test_mixed_fixed_iterations_track_the_oracle(name, iters):
    inst, P, plan = _setup(name)
    ref = O.run_fixed(P, iters)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    assert r.iters == iters
    assert abs(r.objective - ref.objective) <= 1e-5 * abs(ref.objective)
    rho, m = s.extract()
    scale = np.max(np.abs(ref.state.alpha[0]))
    assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-4 * scale


def test_mixed_solve_matches_fp64_solve():
    """2D 32x64x64 Gaussian mixtures to eta_dot <= 1e-6 in both modes: the
    mixed solve reaches the tolerance and its objective is within 1e-5
    relative of the FP64 GPU solve."""
    inst = dotgen.config2_instance()
    out = {}
    for prec in (B.DOT_FP64, B.DOT_MIXED):
        plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, None, tol=1e-6, max_iter=80000,
                                 precision=prec)
        s = G.GpuState(plan)
        s.reset()
        r = s.run(80000)
        assert B.TERM_NAMES[r.term] == "converged", prec
        assert r.eta_dot <= 1e-6
        out[prec] = (r, s.extract())
    r64, (rho64, _) = out[B.DOT_FP64]
    r32, (rho32, _) = out[B.DOT_MIXED]
    assert abs(r32.objective - r64.objective) <= 1e-5 * r64.objective
    # at eta_dot <= 1e-6 the dual objective is fixed only up to each iterate's
    # own duality gap (primal and dual values meet at the optimum only)
    gaps = abs(r64.objective - r64.dual_objective) + abs(r32.objective - r32.dual_objective)
    assert abs(r32.dual_objective - r64.dual_objective) <= 1e-5 * r64.dual_objective + gaps
    vol_x = 1.0 / (inst.n[1] * inst.n[2])
    np.testing.assert_allclose(rho32.sum(axis=(1, 2)) * vol_x, 1.0, atol=1e-5)
