"""Finishing a mixed-precision solve in FP64 (dot_state_promote): promoting the
initial point gives bitwise a plain FP64 run; promoting mid-run continues the
same iterate (the next check's residuals and objective within mixed-precision
distance of the mixed run's); a mixed run that levels off above its tolerance
at the FP32 storage floor converges after promotion; mismatched plans are
rejected."""
import numpy as np
import pytest

import dotgen
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _plan(inst, prec, **kw):
    kw.setdefault("tol", -1.0)
    kw.setdefault("max_iter", 10 ** 6)
    return B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, precision=prec, **kw)


def test_promoting_the_initial_point_gives_the_fp64_run():
    inst = dotgen.tiny_instance(2, (8, 20, 24), seed=81, floor=0.0, masked=True)
    ref_plan = _plan(inst, B.DOT_FP64)
    ref = G.GpuState(ref_plan)
    ref.reset()
    r_ref = ref.run(40)
    rho_ref, m_ref = ref.extract()
    mp, fp = _plan(inst, B.DOT_MIXED), _plan(inst, B.DOT_FP64)
    ms, fs = G.GpuState(mp), G.GpuState(fp)
    ms.reset()
    B.dot_state_promote(mp, ms.ptr, fp, fs.ptr, G.stream_handle())
    r = fs.run(40)
    rho, m = fs.extract()
    assert r.iters == r_ref.iters == 40
    assert r.objective == r_ref.objective and r.eta_dot == r_ref.eta_dot and r.sigma == r_ref.sigma
    assert np.array_equal(rho, rho_ref)
    for a, b in zip(m, m_ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("D,n", [(1, (16, 32)), (2, (12, 30, 26)), (3, (6, 8, 9, 10))], ids=["1d", "2d", "3d"])
def test_promotion_mid_run_continues_the_iterate(D, n):
    inst = dotgen.tiny_instance(D, n, seed=82, floor=0.0)
    print(f"[case] promote {D}d {n}", flush=True)
    mp, fp = _plan(inst, B.DOT_MIXED), _plan(inst, B.DOT_FP64)
    ms, fs = G.GpuState(mp), G.GpuState(fp)
    ms.reset()
    r_mixed0 = ms.run(200)
    B.dot_state_promote(mp, ms.ptr, fp, fs.ptr, G.stream_handle())
    r_f = fs.run(50)
    r_m = ms.run(50)  # the mixed run goes on untouched
    assert r_f.iters == r_m.iters == 250
    assert r_f.checks == r_m.checks == r_mixed0.checks + 10
    # the same trajectory, apart from FP32 storage
    assert abs(r_f.objective - r_m.objective) <= 1e-5 * abs(r_m.objective)
    assert abs(r_f.eta_dot - r_m.eta_dot) <= 0.05 * r_m.eta_dot
    rho_f, _ = fs.extract()
    rho_m, _ = ms.extract()
    assert np.max(np.abs(rho_f - rho_m)) <= 1e-4 * np.max(np.abs(rho_m))


def test_mixed_run_at_its_fp32_floor_converges_in_fp64():
    # a masked batch instance whose mixed run levels off near eta_dot 1.5e-6
    inst = dotgen.config4_instances(12, seed=4000)[11]
    print(f"[case] {inst.label}", flush=True)
    tol = 1e-6
    mp = _plan(inst, B.DOT_MIXED, tol=tol, max_iter=30000)
    fp = _plan(inst, B.DOT_FP64, tol=tol, max_iter=60000)
    ms, fs = G.GpuState(mp), G.GpuState(fp)
    ms.reset()
    r_m = ms.run(30000)
    print(f"[case] mixed: {r_m.iters} iterations, eta {r_m.eta_dot:.3e}", flush=True)
    assert B.TERM_NAMES[r_m.term] == "maxiter" and r_m.eta_dot > tol
    B.dot_state_promote(mp, ms.ptr, fp, fs.ptr, G.stream_handle())
    r_f = fs.run(30000)
    print(f"[case] fp64 after promotion: {r_f.iters} iterations, eta {r_f.eta_dot:.3e}", flush=True)
    assert B.TERM_NAMES[r_f.term] == "converged" and r_f.eta_dot <= tol
    assert r_f.iters < 60000
    assert abs(r_f.objective - r_m.objective) <= 1e-5 * abs(r_f.objective)


def test_promotion_rejects_mismatched_plans():
    a = dotgen.tiny_instance(2, (8, 20, 24), seed=83, floor=0.02)
    b = dotgen.tiny_instance(2, (8, 20, 22), seed=83, floor=0.02)
    mp, fp, fp_other = _plan(a, B.DOT_MIXED), _plan(a, B.DOT_FP64), _plan(b, B.DOT_FP64)
    ms, fs, fs2 = G.GpuState(mp), G.GpuState(fp), G.GpuState(fp_other)
    st = G.stream_handle()
    with pytest.raises(B.DotError):
        B.dot_state_promote(fp, fs.ptr, fp, fs.ptr, st)  # source not mixed
    with pytest.raises(B.DotError):
        B.dot_state_promote(mp, ms.ptr, mp, ms.ptr, st)  # target not FP64
    with pytest.raises(B.DotError):
        B.dot_state_promote(mp, ms.ptr, fp_other, fs2.ptr, st)  # other grid


def test_batch_member_promotion_equals_promoting_its_solve_alone():
    """dot_batch_promote of member 1 of a mixed batch after 200 iterations gives
    bitwise the FP64 state that dot_state_promote gives for the same problem
    solved alone in mixed precision (a batch member equals its solve alone);
    50 FP64 iterations from either are bitwise equal."""
    insts = [dotgen.tiny_instance(2, (12, 30, 26), seed=84, floor=0.0),
             dotgen.tiny_instance(2, (8, 20, 24), seed=85, floor=0.0, masked=True)]
    st = G.stream_handle()
    torch = G.torch_mod()
    batch = B.dot_batch_create(insts, tol=-1.0, max_iter=10 ** 6, precision=B.DOT_MIXED)
    ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    B.dot_batch_run(batch, ws.data_ptr(), 200, st)
    fp_b = _plan(insts[1], B.DOT_FP64)
    fs_b = G.GpuState(fp_b)
    B.dot_batch_promote(batch, ws.data_ptr(), 1, fp_b, fs_b.ptr, st)
    mp, fp = _plan(insts[1], B.DOT_MIXED), _plan(insts[1], B.DOT_FP64)
    ms, fs = G.GpuState(mp), G.GpuState(fp)
    ms.reset()
    ms.run(200)
    B.dot_state_promote(mp, ms.ptr, fp, fs.ptr, st)
    assert np.array_equal(G.host(fs_b.buf), G.host(fs.buf))
    r_b, r = fs_b.run(50), fs.run(50)
    assert r_b.iters == r.iters == 250
    assert r_b.objective == r.objective and r_b.eta_dot == r.eta_dot and r_b.sigma == r.sigma
    with pytest.raises(B.DotError):
        B.dot_batch_promote(batch, ws.data_ptr(), 2, fp_b, fs_b.ptr, st)  # no such member
    with pytest.raises(B.DotError):
        B.dot_batch_promote(batch, ws.data_ptr(), 0, fp_b, fs_b.ptr, st)  # other grid
