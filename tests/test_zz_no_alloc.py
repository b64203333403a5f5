"""The residual entry point that allocates nothing (dot_step_residuals_noalloc)
against dot_step_residuals, through the C ABI: bitwise the same result on
two calls in a row, the second on a smaller grid (the scratch array keeps the
first call's contents), in FP64 and mixed precision; the size limit and the
current-device check are rejected before any device work."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

FIELDS = ("eta_dot", "eta_p", "eta_d", "eta_c", "eta_p_soc", "eta_d_soc", "objective", "dual_objective")


def _case(inst, precision, seed):
    """Plan and device planes of a random iterate of `inst` (seeded)."""
    print(f"[case] {inst.label} n={inst.n} precision={precision} seed={seed}", flush=True)
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=-1.0, max_iter=1000,
                             precision=precision)
    g = P.g
    rng = np.random.default_rng(seed)
    bulk = np.float64 if precision == B.DOT_FP64 else np.float32
    q = [rng.standard_normal(s) for s in G.q_shapes(g)]
    al = [rng.uniform(0, 2, s) if i == 0 else rng.standard_normal(s) for i, s in enumerate(G.q_shapes(g))]
    z = rng.standard_normal((g.K,) + g.cell_shape)
    be = rng.standard_normal((g.K,) + g.cell_shape)
    phi = rng.standard_normal(g.node_shape)
    bufs = [G.dev(B.to_box(phi, g.n)), G.dev(G.planes_of(list(z), g.n, bulk)), G.dev(G.planes_of(q, g.n, bulk)),
            G.dev(G.planes_of(al, g.n)), G.dev(G.planes_of(list(be), g.n, bulk))]
    return plan, bufs


def _same(a, b):
    for k in FIELDS:
        assert getattr(a, k) == getattr(b, k), (k, getattr(a, k), getattr(b, k))
    assert a.term == b.term and a.iters == b.iters == 0


@pytest.mark.parametrize("precision", [B.DOT_FP64, B.DOT_MIXED])
def test_noalloc_residuals_equal_the_allocating_call(precision):
    st = G.stream_handle()
    big = dotgen.config2_instance()                                           # 2D 32x64^2: 561 workgroups
    small = dotgen.tiny_instance(2, (8, 20, 24), seed=22, floor=0.0, masked=True)  # fewer workgroups
    keep = []
    for inst, seed in ((big, 1), (small, 2)):
        plan, bufs = _case(inst, precision, seed)
        keep.append((plan, bufs))
        ptrs = [b.data_ptr() for b in bufs]
        ref = B.dot_step_residuals(plan, *ptrs, st)
        got = B.dot_step_residuals_noalloc(plan, *ptrs, st)
        _same(got, ref)
        assert np.isfinite(got.eta_dot) and got.eta_dot > 0
    # the first plan again after the smaller call: still equal
    plan, bufs = keep[0]
    ptrs = [b.data_ptr() for b in bufs]
    _same(B.dot_step_residuals_noalloc(plan, *ptrs, st), B.dot_step_residuals(plan, *ptrs, st))
    for plan, _ in keep:
        plan.close()


def test_noalloc_rejects_grids_beyond_its_scratch():
    """3D 32x128^3 needs about 75,000 residual workgroups (12 MB of partial
    sums): rejected with DOT_EINVAL before any device work (the plane
    pointers, which are never read, are a small placeholder buffer)."""
    torch = G.torch_mod()
    inst = dotgen.tiny_instance(3, (32, 128, 128, 128), seed=3, floor=0.1)
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, None, tol=-1.0, max_iter=10,
                             precision=B.DOT_MIXED)
    dummy = torch.zeros(256, dtype=torch.float64, device="cuda")
    p = dummy.data_ptr()
    with pytest.raises(B.DotError) as e:
        B.dot_step_residuals_noalloc(plan, p, p, p, p, p, G.stream_handle())
    assert "scratch" in str(e.value)
    plan.close()
