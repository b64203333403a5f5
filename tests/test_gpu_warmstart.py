"""Checkpoint / warm start of the iterate (q, alpha, beta, sigma) through the
C ABI: a run started from an imported iterate follows the oracle started from
the same iterate (FP64: objective 1e-8 relative, rho and m 1e-6, sigma equal);
export after import returns what was imported; a solve warm-started from a
converged iterate stops at once; invalid input is rejected."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _plan(inst, prec=B.DOT_FP64, **kw):
    kw.setdefault("tol", -1.0)
    kw.setdefault("max_iter", 10 ** 6)
    return B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, precision=prec, **kw)


def _random_iterate(P, seed):
    rng = np.random.default_rng(seed)
    g = P.g
    q = [0.3 * rng.standard_normal(s) for s in G.q_shapes(g)]
    al = [0.3 * rng.standard_normal(s) for s in G.q_shapes(g)]
    be = 0.3 * rng.standard_normal((g.K,) + g.cell_shape)
    return q, al, be


CASES = [("1d-12x40", 1, (12, 40)), ("2d-8x20x24-masked", 2, (8, 20, 24)), ("3d-4x6x8x10", 3, (4, 6, 8, 10)),
         ("2d-4x7x300-eliminated-last", 2, (4, 7, 300))]


@pytest.mark.parametrize("name,D,n", CASES, ids=[c[0] for c in CASES])
def test_run_from_an_imported_iterate_follows_the_oracle(name, D, n):
    inst = dotgen.tiny_instance(D, n, seed=91, floor=0.0, masked=(D == 2 and n[1] == 20))
    print(f"[case] warm start {name}", flush=True)
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    q, al, be = _random_iterate(P, 5)
    sigma = 0.7
    iters = 40
    S0 = O.State(np.zeros(P.g.node_shape), np.zeros((P.g.K,) + P.g.cell_shape), [a.copy() for a in q],
                 [a.copy() for a in al], be.copy(), sigma, 0)
    ref = O.solve(P, tol=-1.0, max_iter=iters, state=S0)
    plan = _plan(inst)
    s = G.GpuState(plan)
    B.dot_state_import(plan, s.ptr, G.planes_of(q, inst.n), G.planes_of(al, inst.n),
                       G.planes_of(list(be), inst.n), sigma, G.stream_handle())
    r = s.run(iters)
    assert r.iters == iters
    assert abs(r.sigma - ref.state.sigma) <= 1e-12 * ref.state.sigma
    assert abs(r.objective - ref.objective) <= 1e-8 * abs(ref.objective) + 1e-14
    rho, m = s.extract()
    assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-6
    for a, b in zip(m, ref.state.alpha[1:]):
        assert np.max(np.abs(a - b)) <= 1e-6


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_export_after_import_round_trips(prec):
    inst = dotgen.tiny_instance(2, (8, 20, 24), seed=92, floor=0.0, masked=True)
    plan = _plan(inst, prec)
    s = G.GpuState(plan)
    s.reset()
    s.run(33)  # odd count: the newest q sits in the second buffer
    st = G.stream_handle()
    q, al, be, sg = B.dot_state_export(plan, s.ptr, st)
    s2 = G.GpuState(plan)
    B.dot_state_import(plan, s2.ptr, q, al, be, sg, st)
    q2, al2, be2, sg2 = B.dot_state_export(plan, s2.ptr, st)
    assert sg2 == sg
    assert np.array_equal(q2, q) and np.array_equal(al2, al) and np.array_equal(be2, be)
    # the exported iterate is the one the run holds: rho = alpha0 on cells
    rho, _ = s.extract()
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    a0 = B.from_box(al[0].reshape(B.box_shape(inst.n)), P.g.cell_shape)
    assert np.array_equal(a0, rho)


@pytest.mark.parametrize("prec", [B.DOT_FP64, B.DOT_MIXED])
def test_warm_start_from_a_converged_iterate_stops_at_once(prec):
    inst = dotgen.tiny_instance(2, (8, 20, 24), seed=93, floor=0.0)
    tol = 1e-6
    st = G.stream_handle()
    p1 = _plan(inst, B.DOT_FP64, tol=tol, max_iter=100000)
    s1 = G.GpuState(p1)
    s1.reset()
    r1 = s1.run(100000)
    assert B.TERM_NAMES[r1.term] == "converged"
    q, al, be, sg = B.dot_state_export(p1, s1.ptr, st)
    p2 = _plan(inst, prec, tol=tol, max_iter=100000)
    s2 = G.GpuState(p2)
    B.dot_state_import(p2, s2.ptr, q, al, be, sg, st)
    r2 = s2.run(100000)
    print(f"[case] cold {r1.iters} iterations, warm {r2.iters}", flush=True)
    assert B.TERM_NAMES[r2.term] == "converged"
    assert r2.iters <= 50 < r1.iters
    assert abs(r2.objective - r1.objective) <= (1e-8 if prec == B.DOT_FP64 else 1e-5) * abs(r1.objective)


def test_import_rejects_invalid_input():
    inst = dotgen.tiny_instance(2, (8, 20, 24), seed=94, floor=0.02)
    plan = _plan(inst)
    s = G.GpuState(plan)
    s.reset()
    st = G.stream_handle()
    q, al, be, sg = B.dot_state_export(plan, s.ptr, st)
    with pytest.raises(B.DotError):
        B.dot_state_import(plan, s.ptr, q, al, be, 0.0, st)
    with pytest.raises(B.DotError):
        B.dot_state_import(plan, s.ptr, q, al, be, float("nan"), st)
    bad = al.copy()
    bad[0, 3] = np.inf
    with pytest.raises(B.DotError):
        B.dot_state_import(plan, s.ptr, q, bad, be, sg, st)


def test_time_budget_returns_timeout_and_the_state_resumes():
    """A wall-clock budget ends dot_run at its next poll (every 40 iterations)
    with DOT_TIMEOUT; the state goes on where it stopped, bitwise as an
    uninterrupted run."""
    inst = dotgen.config2_instance()
    timed = _plan(inst, tol=1e-6, max_iter=100000, time_limit_s=1e-6)
    s = G.GpuState(timed)
    s.reset()
    r1 = s.run(100000)
    assert B.TERM_NAMES[r1.term] == "timeout" and r1.iters == 40
    r2 = s.run(100000)
    assert B.TERM_NAMES[r2.term] == "timeout" and r2.iters == 80
    plain = _plan(inst, tol=1e-6, max_iter=100000)
    p = G.GpuState(plain)
    p.reset()
    r = p.run(80)
    assert r.iters == 80 and r.objective == r2.objective and r.eta_dot == r2.eta_dot and r.sigma == r2.sigma
    rho, m = s.extract()
    rho_p, m_p = p.extract()
    assert np.array_equal(rho, rho_p)
    # a batch stops at the smallest budget of its instances
    insts = [inst, dotgen.tiny_instance(2, (8, 20, 24), seed=95, floor=0.02)]
    batch = B.dot_batch_create(insts, tol=1e-6, max_iter=100000, time_limit_s=1e-6)
    torch = G.torch_mod()
    ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
    st = G.stream_handle()
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    res = B.dot_batch_run(batch, ws.data_ptr(), 100000, st)
    assert all(B.TERM_NAMES[x.term] == "timeout" and x.iters == 40 for x in res)


def test_invalid_time_budget_is_rejected():
    inst = dotgen.tiny_instance(2, (8, 20, 24), seed=96, floor=0.02)
    for bad in (-1.0, float("inf"), float("nan")):
        with pytest.raises(B.DotError):
            _plan(inst, time_limit_s=bad)


@pytest.mark.parametrize("name,D,n", [("1d-16x32", 1, (16, 32)), ("2d-8x20x24-masked", 2, (8, 20, 24))],
                         ids=["1d-16x32", "2d-8x20x24-masked"])
def test_sigma_history_matches_the_oracle_decisions(name, D, n):
    """Every change of the sigma rule (Sec. 5.3) on the device: the same
    iterations and values as the oracle's decisions, in order; the batch
    keeps each instance's own history."""
    inst = (dotgen.config1_instance() if D == 1 else
            dotgen.tiny_instance(D, n, seed=97, floor=0.0, masked=True))
    iters = 1500
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    ref = O.run_fixed(P, iters)
    expect = [(rec["k"], rec["sigma"] * 1.25 ** rec["decision"]) for rec in ref.history if rec["decision"] != 0]
    plan = _plan(inst)
    s = G.GpuState(plan)
    s.reset()
    r = s.run(iters)
    hist, count = B.dot_sigma_history(plan, s.ptr, 32, G.stream_handle())
    print(f"[case] {name}: {count} sigma changes", flush=True)
    assert count == r.sigma_changes == len(expect) > 0
    tail = expect[-min(count, 32):]
    assert [k for k, _ in hist] == [k for k, _ in tail]
    for (_, a), (_, b) in zip(hist, tail):
        assert abs(a - b) <= 1e-12 * b
    # the same instance inside a batch, next to another one
    other = dotgen.tiny_instance(2 if D == 2 else 1, (6, 10, 12) if D == 2 else (6, 20), seed=98, floor=0.02)
    batch = B.dot_batch_create([other, inst], tol=-1.0, max_iter=10 ** 6)
    torch = G.torch_mod()
    ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
    st = G.stream_handle()
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    B.dot_batch_run(batch, ws.data_ptr(), iters, st)
    hb, cb = B.dot_batch_sigma_history(batch, ws.data_ptr(), 1, 32, st)
    assert cb == count and hb == hist


def test_batch_with_mixed_time_budgets_reports_each_instance():
    """One batch with budgets 0 (none) and 1e-6 s: the call ends at the first
    poll (40 iterations); the instance whose budget ran out reports DOT_TIMEOUT,
    the one without a budget DOT_RUNNING; a further run continues both, and a
    run whose iteration count ends at the same poll as the budget reports the
    iteration cap of the call, not a timeout."""
    insts = [dotgen.config2_instance(), dotgen.tiny_instance(2, (8, 20, 24), seed=97, floor=0.02)]
    batch = B.dot_batch_create(insts, per_instance=[{"time_limit_s": 0.0}, {"time_limit_s": 1e-6}],
                               tol=1e-6, max_iter=100000)
    torch = G.torch_mod()
    ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
    st = G.stream_handle()
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    res = B.dot_batch_run(batch, ws.data_ptr(), 100000, st)
    assert [x.iters for x in res] == [40, 40]
    assert [B.TERM_NAMES[x.term] for x in res] == ["running", "timeout"]
    res = B.dot_batch_run(batch, ws.data_ptr(), 40, st)
    assert [x.iters for x in res] == [80, 80]
    assert [B.TERM_NAMES[x.term] for x in res] == ["maxiter", "maxiter"]
