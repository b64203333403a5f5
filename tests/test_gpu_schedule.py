"""Transform schedules (tile width and waves per axis of the cosine-transform
passes of the phi-step) and their autotuner: every schedule an instance can
take gives bitwise the iterates of the rule's schedule, invalid schedules are
rejected before any launch, and autotuned plans and batches keep the results
of untuned ones (a batch member still equals its solve alone)."""
import numpy as np
import pytest

import dotgen
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

ITERS = 30  # six residual checks, both parities of q


def _plan(inst, prec):
    return B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, precision=prec, tol=-1.0,
                             max_iter=100000)


def _run(plan, iters=ITERS):
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    rho, m = s.extract()
    return r, rho, m


def _same(a, b):
    ra, rhoa, ma = a
    rb, rhob, mb = b
    assert ra.iters == rb.iters
    assert ra.objective == rb.objective, (ra.objective, rb.objective)
    assert ra.eta_dot == rb.eta_dot
    assert ra.sigma == rb.sigma
    assert np.array_equal(rhoa, rhob)
    for x, y in zip(ma, mb):
        assert np.array_equal(x, y)


SCHED_CASES = [
    ("1d-6x40", 1, (6, 40)),
    ("2d-8x20x24-masked", 2, (8, 20, 24)),
    ("2d-12x70x45", 2, (12, 70, 45)),
    ("3d-4x6x8x10", 3, (4, 6, 8, 10)),
]


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
@pytest.mark.parametrize("name,D,n", SCHED_CASES, ids=[c[0] for c in SCHED_CASES])
def test_every_schedule_gives_the_rule_bits(name, D, n, prec):
    inst = dotgen.tiny_instance(D, n, seed=61, floor=0.0, masked=(D == 2 and n[1] == 20))
    print(f"[case] {name} precision={prec}", flush=True)
    plan = _plan(inst, prec)
    rule = B.dot_plan_get_schedule(plan)
    assert not rule["tuned"]
    ref = _run(plan)
    tried = 0
    for cw in (16, 32, 64):
        for waves in (0, 16):
            B.dot_plan_set_schedule(plan, cw=[cw] * (D + 1), waves=[waves] * (D + 1))
            got = B.dot_plan_get_schedule(plan)
            assert got["cw"] == [cw] * (D + 1)
            if waves:
                assert got["waves"] == [waves] * (D + 1)
            print(f"[case] {name} cw={cw} waves={got['waves']}", flush=True)
            _same(_run(plan), ref)
            tried += 1
    # one width per axis, different on neighbouring axes
    widths = [(16, 64, 32, 16)[a] for a in range(D + 1)]
    B.dot_plan_set_schedule(plan, cw=widths)
    _same(_run(plan), ref)
    B.dot_plan_set_schedule(plan)  # back to the rule
    assert B.dot_plan_get_schedule(plan)["cw"] == rule["cw"]
    _same(_run(plan), ref)
    assert tried == 6


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
@pytest.mark.parametrize("n", [(4, 7, 300), (3, 5, 1200)], ids=["last-301", "last-1201"])
def test_tridiagonal_last_axis_widths_give_the_same_bits(n, prec):
    # each line is solved by its own lanes in a fixed order: the lines per
    # workgroup change no value. 301 nodes: the partitioned solve with 64
    # lanes per line (4 lines per round); 1201 nodes (longer than a transform
    # tile holds): one lane per line, which takes 16, 32 or 64 lines
    inst = dotgen.tiny_instance(2, n, seed=62, floor=0.0)
    plan = _plan(inst, prec)
    ref = _run(plan, 20)
    assert B.dot_plan_get_schedule(plan)["cw"][2] == (4 if n[2] < 576 else 64)
    for cw in ((4, 8, 16, 32, 64) if n[2] < 576 else (16, 32, 64)):
        B.dot_plan_set_schedule(plan, cw=[16, 32, cw], waves=[8, 16, 0])
        _same(_run(plan, 20), ref)


def test_invalid_schedules_are_rejected():
    inst = dotgen.tiny_instance(2, (8, 20, 24), seed=63, floor=0.02)
    plan = _plan(inst, B.DOT_FP64)
    before = B.dot_plan_get_schedule(plan)
    for cw, waves in (([48, 0, 0], None), ([0, 0, 0], [17, 0, 0]), ([0, 0, 0], [-1, 0, 0]),
                      ([64, 64, 64], [1, 1, 1])):  # 4 work items per 64-line tile, 3 per FP64 wave
        with pytest.raises(B.DotError):
            B.dot_plan_set_schedule(plan, cw=cw, waves=waves)
        assert B.dot_plan_get_schedule(plan) == before


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_plan_autotune_keeps_the_results(prec):
    inst = dotgen.config2_instance()
    print(f"[case] 2d-32x64x64 autotune precision={prec}", flush=True)
    ref = _run(_plan(inst, prec))
    plan = _plan(inst, prec)
    s = G.GpuState(plan)
    s.reset()
    s.run(7)  # the autotuner overwrites and resets the state
    sched = B.dot_plan_autotune(plan, s.ptr, G.stream_handle())
    print(f"[case] schedule {sched}", flush=True)
    assert sched["tuned"]
    assert sched["candidates"] >= 3
    assert 0.0 < sched["us"] <= sched["us_rule"]
    assert B.dot_plan_get_schedule(plan) == sched
    r = s.run(ITERS)
    rho, m = s.extract()
    _same((r, rho, m), ref)


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_batch_autotune_members_equal_their_solves_alone(prec):
    insts = [dotgen.tiny_instance(2, (8, 20, 24), seed=41, floor=0.0, masked=True),
             dotgen.tiny_instance(2, (12, 70, 45), seed=42, floor=0.0, n_comp=3),
             dotgen.tiny_instance(2, (4, 7, 300), seed=45, floor=0.0)]
    insts += dotgen.config4_instances(3, seed=4200)
    print(f"[case] batch autotune of {len(insts)} precision={prec}", flush=True)
    batch = B.dot_batch_create(insts, tol=-1.0, max_iter=100000, precision=prec)
    torch = G.torch_mod()
    ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
    st = G.stream_handle()
    sched = B.dot_batch_autotune(batch, ws.data_ptr(), st)
    print(f"[case] schedule {sched}", flush=True)
    assert sched["tuned"] and 0.0 < sched["us"] <= sched["us_rule"]
    res = B.dot_batch_run(batch, ws.data_ptr(), ITERS, st)
    for i, inst in enumerate(insts):
        r, rho, m = _run(_plan(inst, prec))
        rb, mb = B.dot_batch_extract(batch, ws.data_ptr(), i, st)
        _same((res[i], rb, mb), (r, rho, m))
    # an explicit batch schedule: narrow tiles on every axis
    B.dot_batch_set_schedule(batch, cw=[16, 16, 16])
    assert B.dot_batch_get_schedule(batch)["cw"] == [16, 16, 16]
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    res2 = B.dot_batch_run(batch, ws.data_ptr(), ITERS, st)
    for a, b in zip(res, res2):
        assert a.objective == b.objective and a.eta_dot == b.eta_dot


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
@pytest.mark.parametrize("D,n", [(1, (16, 32)), (3, (8, 12, 16, 20))], ids=["1d-16x32", "3d-8x12x16x20"])
def test_autotune_1d_3d_plans_keep_the_results(D, n, prec):
    inst = dotgen.tiny_instance(D, n, seed=64, floor=0.0)
    print(f"[case] autotune {D}d {n} precision={prec}", flush=True)
    ref = _run(_plan(inst, prec))
    plan = _plan(inst, prec)
    s = G.GpuState(plan)
    sched = B.dot_plan_autotune(plan, s.ptr, G.stream_handle())
    assert sched["tuned"] and len(sched["cw"]) == D + 1
    r = s.run(ITERS)
    rho, m = s.extract()
    _same((r, rho, m), ref)


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_autotuned_3d_batch_members_equal_their_solves_alone(prec):
    insts = [dotgen.tiny_instance(3, (4, 6, 8, 10), seed=71, floor=0.0),
             dotgen.tiny_instance(3, (8, 12, 10, 14), seed=72, floor=0.02),
             dotgen.tiny_instance(3, (6, 16, 8, 9), seed=73, floor=0.0)]
    print(f"[case] 3d batch autotune precision={prec}", flush=True)
    batch = B.dot_batch_create(insts, tol=-1.0, max_iter=100000, precision=prec)
    torch = G.torch_mod()
    ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
    st = G.stream_handle()
    sched = B.dot_batch_autotune(batch, ws.data_ptr(), st)
    assert sched["tuned"] and len(sched["cw"]) == 4
    res = B.dot_batch_run(batch, ws.data_ptr(), ITERS, st)
    for i, inst in enumerate(insts):
        r, rho, m = _run(_plan(inst, prec))
        rb, mb = B.dot_batch_extract(batch, ws.data_ptr(), i, st)
        _same((res[i], rb, mb), (r, rho, m))
