"""Parity at the full workload sizes, in the launch configuration the
benchmark uses (tile widths, time chunks and graphs chosen by the library for
these grids): 2D 64x256x256 for ten whole iterations (FP64 and mixed) against
the oracle, and the 3D 32x64^3 serving request one step at a time on a
random state (the oracle needs ~13 s per iteration at that size)."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

ITERS = 10


@pytest.fixture(scope="module")
def config3():
    inst = dotgen.config3_instance()
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    print("[case] oracle 2D 64x256x256, 10 iterations", flush=True)
    return inst, P, O.run_fixed(P, ITERS)


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_2d_64x256x256_fixed_iterations(config3, prec):
    inst, P, ref = config3
    print(f"[case] 2D 64x256x256 precision={prec}", flush=True)
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=-1.0, max_iter=100000,
                             precision=prec)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(ITERS)
    assert r.iters == ITERS and r.checks == len(ref.history)
    rho, m = s.extract()
    if prec == B.DOT_FP64:
        assert abs(r.objective - ref.objective) <= 1e-8 * abs(ref.objective)
        # the residuals of the last check: 8,547 workgroup rows, reduced in two stages
        last = ref.history[-1]
        for k in ("eta_dot", "eta_p", "eta_d", "eta_c", "eta_p_soc", "eta_d_soc"):
            assert abs(getattr(r, k) - last[k]) <= 1e-9 * abs(last[k]), (k, getattr(r, k), last[k])
        assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-6
        for a, b in zip(m, ref.state.alpha[1:]):
            assert np.max(np.abs(a - b)) <= 1e-6
    else:
        assert abs(r.objective - ref.objective) <= 1e-5 * abs(ref.objective)
        scale = np.max(np.abs(ref.state.alpha[0]))
        assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-4 * scale


@pytest.fixture(scope="module")
def serving3d():
    inst = dotgen.serving_3d_instance()
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    rng = np.random.default_rng(9)
    g = P.g
    q = [rng.standard_normal(s) for s in G.q_shapes(g)]
    al = [rng.uniform(0, 2, s) if i == 0 else rng.standard_normal(s) for i, s in enumerate(G.q_shapes(g))]
    be = rng.standard_normal((g.K,) + g.cell_shape)
    phi = rng.standard_normal(g.node_shape)
    return inst, P, plan, (phi, q, al, be)


def test_3d_32x64x64x64_steps(serving3d):
    inst, P, plan, (phi, q, al, be) = serving3d
    g = P.g
    print("[case] 3D 32x64^3 steps", flush=True)
    st = G.stream_handle()
    sigma, tau = 0.9, 1.9
    qd = G.dev(G.planes_of(q, g.n))
    ad = G.dev(G.planes_of(al, g.n))
    bed = G.dev(G.planes_of(list(be), g.n))
    # a3 + a4 as the iteration runs them
    pd = G.dev(np.zeros(g.node_shape))
    B.dot_step_rhs_poisson(plan, qd.data_ptr(), ad.data_ptr(), sigma, pd.data_ptr(), st)
    phi_ref = O.poisson(O.step_rhs(P, q, al, sigma), g)
    assert G.rel_err(G.host(pd), phi_ref) < 1e-11
    del pd
    # a1 + a2
    zd = G.dev(np.zeros((g.K,) + g.node_shape))
    B.dot_step_cone(plan, qd.data_ptr(), bed.data_ptr(), sigma, zd.data_ptr(), st)
    z_ref = O.proj_soc(O.step_cone_input(P, q, be, sigma))
    z = np.stack([B.from_box(p, g.cell_shape) for p in G.host(zd)])
    assert G.rel_err(z, z_ref) < 1e-13
    del zd, z
    # a5
    phd = G.dev(B.to_box(phi, g.n))
    qo = G.dev(np.zeros((g.D + 1,) + g.node_shape))
    wd = G.dev(np.zeros((4 * g.D + 1,) + g.node_shape))
    B.dot_step_update(plan, phd.data_ptr(), qd.data_ptr(), ad.data_ptr(), bed.data_ptr(), sigma, tau,
                      qo.data_ptr(), wd.data_ptr(), st)
    qn = O.step_q(P, phi, z_ref, al, be, sigma)
    shapes = G.q_shapes(g)
    for a, b in zip(G.unpack(G.host(qo), shapes), qn):
        assert G.rel_err(a, b) < 1e-12
    Aphi = O.grad(phi, g)
    for a, b, a0, ap, qq in zip(G.unpack(G.host(ad), shapes), al, al, Aphi, qn):
        assert G.rel_err(a, a0 + tau * sigma * (ap - qq)) < 1e-12
    be_n = be + tau * sigma * (z_ref - O.BF(qn, P.omega, g) - O.cone_offset(g))
    bn = np.stack([B.from_box(p, g.cell_shape) for p in G.host(bed)])
    assert G.rel_err(bn, be_n) < 1e-12


def _converged_solve(inst, prec, tol=1e-6, cap=60000):
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=tol, max_iter=cap, precision=prec)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(cap)
    rho, m = s.extract()
    del s
    plan.close()
    return r, rho, m


def test_2d_64x256x256_mixed_against_fp64_at_1e6():
    """The mixed-precision criterion on the 64x256^2 five-component workload:
    both precisions reach eta_dot <= 1e-6; the mixed objective is within 1e-5
    relative of the FP64 one (measured 2.9e-8: both follow the same
    iterates until the FP32 rounding of the stored bulk state matters, and
    stop within one check of each other); every time slice of rho carries unit
    mass (the continuity equation summed over space, to eta_D accuracy); rho
    and m of the two runs agree to 1e-3 of their scale (their distance from the
    exact solution at this tolerance is ~0.4 in max norm on the near-empty
    regions, where they are not unique to that accuracy, so the tight
    comparisons are the objective and the masses)."""
    inst = dotgen.config3_instance()
    out = {}
    for prec in (B.DOT_FP64, B.DOT_MIXED):
        print(f"[case] 2D 64x256x256 to eta_dot <= 1e-6, precision={prec}", flush=True)
        r, rho, m = _converged_solve(inst, prec)
        assert B.TERM_NAMES[r.term] == "converged" and r.eta_dot <= 1e-6, (r.iters, r.eta_dot)
        vx = 1.0 / (inst.n[1] * inst.n[2])
        mass = rho.reshape(rho.shape[0], -1).sum(1) * vx
        assert np.max(np.abs(mass - 1.0)) <= 1e-6
        assert rho.min() > -1e-4 * rho.max()
        out[prec] = (r, rho, m)
    r64, rho64, m64 = out[B.DOT_FP64]
    rmx, rhomx, mmx = out[B.DOT_MIXED]
    rel = abs(rmx.objective - r64.objective) / abs(r64.objective)
    print(f"[result] iterations fp64 {r64.iters} mixed {rmx.iters}; objective rel diff {rel:.3e}", flush=True)
    assert rel <= 1e-5
    assert abs(rmx.iters - r64.iters) <= 200
    assert np.max(np.abs(rhomx - rho64)) <= 1e-3 * np.max(np.abs(rho64))
