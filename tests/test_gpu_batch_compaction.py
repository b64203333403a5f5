"""Batch compaction: once stopped instances hold at least 1/8 of a node
sweep's workgroups, dot_batch_run lays its launches out again over the
instances still running. The members that keep running give bitwise the
iterates of their solves alone, whichever kernels the smaller layout drops
(the tridiagonal pass, the last-axis transform pass, the second graph
branch), and a reset lays every instance out again. Instances stop at
loose per-instance tolerances (the oracle reaches them within 10 to 85
iterations on these grids) while the others run on (tolerance < 0)."""
import numpy as np
import pytest

import dotgen
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _alone(inst, iters, prec, tol):
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, precision=prec, tol=tol,
                             max_iter=10 ** 6)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    rho, m = s.extract()
    return r, rho, m


def _run_batch(insts, tols, prec, iters):
    batch = B.dot_batch_create(insts, per_instance=[{"tol": t} for t in tols], max_iter=10 ** 6, precision=prec)
    torch = G.torch_mod()
    ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
    st = G.stream_handle()
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    assert B.dot_batch_laid_out(batch) == len(insts)
    res = B.dot_batch_run(batch, ws.data_ptr(), iters, st)
    return batch, ws, st, res


def _check_members(batch, ws, st, res, insts, tols, prec, iters):
    for i, inst in enumerate(insts):
        r, rho, m = _alone(inst, iters, prec, tols[i])
        assert res[i].iters == r.iters, (i, res[i].iters, r.iters)
        assert res[i].term == r.term, i
        assert res[i].objective == r.objective, (i, res[i].objective, r.objective)
        assert res[i].eta_dot == r.eta_dot and res[i].sigma == r.sigma, i
        rb, mb = B.dot_batch_extract(batch, ws.data_ptr(), i, st)
        assert np.array_equal(rb, rho), i
        for a, b in zip(mb, m):
            assert np.array_equal(a, b), i


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_compacted_batch_members_equal_their_solves_alone(prec):
    """The tridiagonal instance (301-node last axis, the largest) stops
    first; the transform instances run on in the compacted layout, where no
    instance takes the tridiagonal pass any more."""
    insts = [dotgen.tiny_instance(2, (4, 7, 300), seed=151, floor=0.0, masked=True),
             dotgen.tiny_instance(2, (8, 20, 24), seed=152, floor=0.0),
             dotgen.tiny_instance(2, (3, 9, 5), seed=153, floor=0.02),
             dotgen.tiny_instance(2, (6, 10, 12), seed=154, floor=0.0, masked=True)]
    tols = [0.3, -1.0, 3e-2, -1.0]
    iters = 200
    print(f"[case] compaction, tridiagonal instance stops first, precision={prec}", flush=True)
    batch, ws, st, res = _run_batch(insts, tols, prec, iters)
    assert res[0].iters < 40 and res[2].iters < iters and res[1].iters == res[3].iters == iters
    assert B.dot_batch_laid_out(batch) == 3  # the small one's 4 workgroups stay below 1/8
    _check_members(batch, ws, st, res, insts, tols, prec, iters)
    # a reset lays every instance out again and the same run gives the same bits
    first = [(r.iters, r.objective, r.eta_dot) for r in res]
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    assert B.dot_batch_laid_out(batch) == len(insts)
    res2 = B.dot_batch_run(batch, ws.data_ptr(), iters, st)
    assert [(r.iters, r.objective, r.eta_dot) for r in res2] == first


def test_compaction_down_to_tridiagonal_instances_only():
    """The transform instance stops: the compacted layout holds only the
    tridiagonal instance, so the last-axis transform pass is no longer
    launched."""
    insts = [dotgen.tiny_instance(2, (8, 20, 24), seed=161, floor=0.0),
             dotgen.tiny_instance(2, (4, 7, 300), seed=162, floor=0.0, masked=True)]
    tols = [0.1, -1.0]
    iters = 120
    print("[case] compaction down to the tridiagonal instance", flush=True)
    batch, ws, st, res = _run_batch(insts, tols, B.DOT_FP64, iters)
    assert res[0].iters < 40 and res[1].iters == iters
    assert B.dot_batch_laid_out(batch) == 1
    _check_members(batch, ws, st, res, insts, tols, B.DOT_FP64, iters)


def test_compaction_from_two_branches_to_one_stream():
    """A batch over 2^21 grid nodes runs the z-step on a second graph branch;
    when its large instance stops, the compacted layout falls below the
    threshold and the small instance runs on in the one-stream order."""
    big = dotgen.tiny_instance(2, (32, 256, 256), seed=171, floor=0.0, n_comp=3)  # 2.18 M nodes
    small = dotgen.tiny_instance(2, (8, 20, 24), seed=172, floor=0.0, masked=True)
    insts = [big, small]
    tols = [0.3, -1.0]
    iters = 100
    print("[case] compaction from the overlapped order to one stream (mixed)", flush=True)
    batch, ws, st, res = _run_batch(insts, tols, B.DOT_MIXED, iters)
    assert res[0].iters < 40 and res[1].iters == iters
    assert B.dot_batch_laid_out(batch) == 1
    _check_members(batch, ws, st, res, insts, tols, B.DOT_MIXED, iters)


def test_promoted_members_continue_together_in_an_fp64_batch():
    """Members of a mixed batch promoted into an FP64 batch of their problems
    continue bitwise as dot_batch_promote + dot_run of each; the FP64 batch
    takes the mixed batch's iteration count, and a promotion from another
    count is refused."""
    insts = [dotgen.tiny_instance(2, (8, 20, 24), seed=181, floor=0.0, masked=True),
             dotgen.tiny_instance(2, (4, 7, 300), seed=182, floor=0.0),
             dotgen.tiny_instance(2, (6, 10, 12), seed=183, floor=0.0, masked=True)]
    torch = G.torch_mod()
    st = G.stream_handle()
    print("[case] promotion of mixed batch members into an FP64 batch", flush=True)
    mb = B.dot_batch_create(insts, tol=-1.0, max_iter=10 ** 6, precision=B.DOT_MIXED)
    mws = torch.zeros(int(mb.workspace_bytes), dtype=torch.uint8, device="cuda")
    B.dot_batch_reset(mb, mws.data_ptr(), st)
    B.dot_batch_run(mb, mws.data_ptr(), 120, st)
    picked = [0, 1]
    fb = B.dot_batch_create([insts[i] for i in picked], tol=-1.0, max_iter=10 ** 6, precision=B.DOT_FP64)
    fws = torch.zeros(int(fb.workspace_bytes), dtype=torch.uint8, device="cuda")
    B.dot_batch_reset(fb, fws.data_ptr(), st)
    for slot, i in enumerate(picked):
        B.dot_batch_promote_member(mb, mws.data_ptr(), i, fb, fws.data_ptr(), slot, st)
    res = B.dot_batch_run(fb, fws.data_ptr(), 80, st)
    for slot, i in enumerate(picked):
        inst = insts[i]
        plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=-1.0, max_iter=10 ** 6)
        s = G.GpuState(plan)
        B.dot_batch_promote(mb, mws.data_ptr(), i, plan, s.ptr, st)
        r = s.run(80)
        assert res[slot].iters == r.iters == 200, (slot, res[slot].iters, r.iters)
        assert res[slot].objective == r.objective and res[slot].eta_dot == r.eta_dot, slot
        rho_b, m_b = B.dot_batch_extract(fb, fws.data_ptr(), slot, st)
        rho, m = s.extract()
        assert np.array_equal(rho_b, rho), slot
        for a, b in zip(m_b, m):
            assert np.array_equal(a, b), slot
    # the FP64 batch is now at 200 iterations, the mixed one at 120
    with pytest.raises(B.DotError):
        B.dot_batch_promote_member(mb, mws.data_ptr(), 2, fb, fws.data_ptr(), 0, st)


def test_run_of_a_batch_whose_instances_all_stopped_changes_nothing():
    """Once every instance has stopped, dot_batch_run launches nothing and
    returns the same results."""
    insts = [dotgen.tiny_instance(2, (4, 7, 300), seed=151, floor=0.0, masked=True),
             dotgen.tiny_instance(2, (8, 20, 24), seed=161, floor=0.0)]
    tols = [0.3, 0.1]
    print("[case] run after every instance stopped", flush=True)
    batch, ws, st, res = _run_batch(insts, tols, B.DOT_FP64, 200)
    assert all(B.TERM_NAMES[r.term] == "converged" for r in res)
    before = G.host(ws).copy()
    res2 = B.dot_batch_run(batch, ws.data_ptr(), 200, st)
    assert [(r.iters, r.objective, r.eta_dot) for r in res2] == [(r.iters, r.objective, r.eta_dot) for r in res]
    assert np.array_equal(G.host(ws), before)
