"""Axes of 1025 points (1024 segments, the paper's large single instance):
the transforms run on narrow tiles with more work items per wave. Parity with
the oracle on grids that are long along one axis and short along the others,
and one step of each row at the full 32 x 1024 x 1024 size."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [(2, 1024, 5), (3, 6, 1024), (4, 1024)])
@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_long_axis_fixed_iterations(n, prec):
    D = len(n) - 1
    inst = dotgen.tiny_instance(D, n, seed=40 + D, floor=0.0, n_comp=3)
    print(f"[case] long axis n={n} precision={prec}", flush=True)
    iters = 60
    P = O.make_problem(D, n, inst.rho0, inst.rho1)
    ref = O.run_fixed(P, iters)
    plan = B.dot_plan_create(D, n, inst.rho0, inst.rho1, None, tol=-1.0, max_iter=100000, precision=prec)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    rho, m = s.extract()
    if prec == B.DOT_FP64:
        assert abs(r.objective - ref.objective) <= 1e-8 * abs(ref.objective)
        assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-6
        for a, b in zip(m, ref.state.alpha[1:]):
            assert np.max(np.abs(a - b)) <= 1e-6
    else:
        assert abs(r.objective - ref.objective) <= 1e-5 * abs(ref.objective)
        assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-4 * np.max(np.abs(ref.state.alpha[0]))


def test_32x1024x1024_transform_and_cone_steps():
    inst = dotgen.image_like_instance()
    print("[case] 2D 32x1024x1024 steps", flush=True)
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1)
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, None)
    g = P.g
    rng = np.random.default_rng(10)
    q = [rng.standard_normal(s) for s in G.q_shapes(g)]
    al = [rng.standard_normal(s) for s in G.q_shapes(g)]
    sigma = 2.0
    st = G.stream_handle()
    qd = G.dev(G.planes_of(q, g.n))
    ad = G.dev(G.planes_of(al, g.n))
    pd = G.dev(np.zeros(g.node_shape))
    B.dot_step_rhs_poisson(plan, qd.data_ptr(), ad.data_ptr(), sigma, pd.data_ptr(), st)
    phi_ref = O.poisson(O.step_rhs(P, q, al, sigma), g)
    assert G.rel_err(G.host(pd), phi_ref) < 1e-11
    del pd, ad, al, phi_ref
    be = rng.standard_normal((g.K,) + g.cell_shape)
    bed = G.dev(G.planes_of(list(be), g.n))
    zd = G.dev(np.zeros((g.K,) + g.node_shape))
    B.dot_step_cone(plan, qd.data_ptr(), bed.data_ptr(), sigma, zd.data_ptr(), st)
    z_ref = O.proj_soc(O.step_cone_input(P, q, be, sigma))
    z = np.stack([B.from_box(p, g.cell_shape) for p in G.host(zd)])
    assert G.rel_err(z, z_ref) < 1e-13
