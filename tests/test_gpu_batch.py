"""Batches: heterogeneous instances in one launch per kernel give bitwise the
same iterates as each instance solved alone, stop independently, and match
the oracle."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _insts():
    out = [dotgen.tiny_instance(2, (8, 20, 24), seed=41, floor=0.0, masked=True),
           dotgen.tiny_instance(2, (12, 70, 45), seed=42, floor=0.0, n_comp=3),
           dotgen.tiny_instance(2, (3, 9, 5), seed=43, floor=0.02),
           dotgen.tiny_instance(2, (16, 33, 17), seed=44, floor=0.0, masked=True)]
    out += dotgen.config4_instances(4, seed=4100)
    return out


def _alone(inst, iters, prec, **kw):
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, precision=prec, **kw)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    rho, m = s.extract()
    return r, rho, m


def _torch_ws(nbytes):
    torch = G.torch_mod()
    return torch.zeros(int(nbytes), dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_batch_equals_each_instance_alone(prec):
    insts = _insts()
    print(f"[case] batch of {len(insts)} precision={prec}", flush=True)
    batch = B.dot_batch_create(insts, tol=-1.0, max_iter=100000, precision=prec)
    ws = _torch_ws(batch.workspace_bytes)
    st = G.stream_handle()
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    iters = 60
    res = B.dot_batch_run(batch, ws.data_ptr(), iters, st)
    for i, inst in enumerate(insts):
        r, rho, m = _alone(inst, iters, prec, tol=-1.0, max_iter=100000)
        rb, mb = B.dot_batch_extract(batch, ws.data_ptr(), i, st)
        assert res[i].iters == r.iters == iters
        assert res[i].objective == r.objective, (i, res[i].objective, r.objective)
        assert res[i].eta_dot == r.eta_dot
        assert np.array_equal(rb, rho)
        for a, b in zip(mb, m):
            assert np.array_equal(a, b)


def test_batch_instances_stop_independently_and_match_oracle():
    insts = [dotgen.tiny_instance(2, (6, 10, 12), seed=51, floor=0.05),
             dotgen.tiny_instance(2, (8, 20, 24), seed=52, floor=0.0, masked=True),
             dotgen.tiny_instance(2, (4, 7, 9), seed=53, floor=0.02)]
    tol = 1e-7
    batch = B.dot_batch_create(insts, tol=tol, max_iter=100000)
    ws = _torch_ws(batch.workspace_bytes)
    st = G.stream_handle()
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    res = B.dot_batch_run(batch, ws.data_ptr(), 30000, st)
    iters = [r.iters for r in res]
    assert len(set(iters)) > 1  # different stopping points
    for i, inst in enumerate(insts):
        assert B.TERM_NAMES[res[i].term] == "converged"
        r, rho, _ = _alone(inst, 30000, B.DOT_FP64, tol=tol, max_iter=100000)
        assert res[i].iters == r.iters
        assert res[i].objective == r.objective
        P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
        ref = O.solve(P, tol=tol, max_iter=30000)
        assert abs(res[i].objective - ref.objective) <= 1e-8 * ref.objective
        assert abs(res[i].iters - ref.iters) <= 5


def test_batch_rejects_mixed_dimensions():
    a = dotgen.tiny_instance(2, (3, 4, 4), seed=1)
    b = dotgen.tiny_instance(1, (3, 4), seed=2)
    with pytest.raises(B.DotError):
        B.dot_batch_create([a, b])


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_batch_mixing_tridiagonal_and_transform_last_axes(prec):
    """A long last axis (301 nodes: tridiagonal solve) next to short ones
    (transform, 1/Lambda, transform) in one batch: each instance gives bitwise
    its solve alone."""
    insts = [dotgen.tiny_instance(2, (4, 7, 300), seed=151, floor=0.0, masked=True),
             dotgen.tiny_instance(2, (8, 20, 24), seed=152, floor=0.0)]
    print(f"[case] tridiagonal + transform batch precision={prec}", flush=True)
    batch = B.dot_batch_create(insts, tol=-1.0, max_iter=100000, precision=prec)
    ws = _torch_ws(batch.workspace_bytes)
    st = G.stream_handle()
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    iters = 45
    res = B.dot_batch_run(batch, ws.data_ptr(), iters, st)
    for i, inst in enumerate(insts):
        r, rho, m = _alone(inst, iters, prec, tol=-1.0, max_iter=100000)
        rb, mb = B.dot_batch_extract(batch, ws.data_ptr(), i, st)
        assert res[i].objective == r.objective, i
        assert np.array_equal(rb, rho), i
        for a, b in zip(mb, m):
            assert np.array_equal(a, b), i


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_overlapped_order_gives_the_sequential_bits(prec):
    """From 2^21 grid nodes an executor runs the z-step on a second graph
    branch beside the phi-step and defers beta updates; the same kernels in the
    one-stream order (a kernel class being timed switches to it) give bitwise
    the same iterates. Also a batch large enough to overlap against each member
    solved alone below the threshold (one stream)."""
    big = dotgen.tiny_instance(2, (32, 256, 256), seed=41, floor=0.0, n_comp=3)  # 2.18 M nodes
    small = dotgen.tiny_instance(2, (8, 20, 24), seed=42, floor=0.0, masked=True)
    iters = 60
    st = G.stream_handle()
    print(f"[case] overlapped vs sequential precision={prec}", flush=True)
    plan = B.dot_plan_create(big.D, big.n, big.rho0, big.rho1, big.mask, tol=-1.0, max_iter=10 ** 6, precision=prec)
    a, b = G.GpuState(plan), G.GpuState(plan)
    a.reset()
    ra = a.run(iters)                                    # overlapped (graphs)
    B.dot_profile_select(plan, B.KERNEL_CLASSES["cone"])  # one stream, every class its own launch
    b.reset()
    rb = b.run(iters)
    B.dot_profile_select(plan, -1)
    for k in ("objective", "eta_dot", "sigma", "iters", "checks"):
        assert getattr(ra, k) == getattr(rb, k), k
    assert np.array_equal(G.host(a.buf)[:plan.info.off_w], G.host(b.buf)[:plan.info.off_w])
    # a batch of both (over the threshold) against each alone
    torch = G.torch_mod()
    batch = B.dot_batch_create([big, small], tol=-1.0, max_iter=10 ** 6, precision=prec)
    ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    res = B.dot_batch_run(batch, ws.data_ptr(), iters, st)
    for i, inst in enumerate((big, small)):
        p = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=-1.0, max_iter=10 ** 6,
                              precision=prec)
        s = G.GpuState(p)
        s.reset()
        r = s.run(iters)
        assert res[i].objective == r.objective and res[i].eta_dot == r.eta_dot and res[i].sigma == r.sigma, i
        rho_b, m_b = B.dot_batch_extract(batch, ws.data_ptr(), i, st)
        rho, m = s.extract()
        assert np.array_equal(rho_b, rho), i
        for x, y in zip(m_b, m):
            assert np.array_equal(x, y), i
