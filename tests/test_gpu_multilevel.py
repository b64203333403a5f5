"""Multilevel initialisation on the device: the prolongation kernel against
the oracle's interpolation, and level-by-level solves against the oracle's
multilevel solve."""
import numpy as np
import pytest

import dotgen
from oracle import dot_oracle as O
from oracle import multilevel as ML
from paper_2505_05424_amd import binding as B
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _put_planes(state, off, arrs, n, dtype):
    torch = G.torch_mod()
    planes = G.planes_of(arrs, n, dtype)
    raw = np.frombuffer(planes.tobytes(), dtype=np.uint8)
    state.buf[off:off + raw.size] = torch.from_numpy(raw.copy()).to("cuda")


def _get_planes(state, off, count, n, dtype):
    box = B.box_shape(n)
    nbytes = count * int(np.prod(box)) * np.dtype(dtype).itemsize
    raw = G.host(state.buf[off:off + nbytes])
    return np.frombuffer(raw.tobytes(), dtype=dtype).reshape((count,) + box).astype(np.float64)


@pytest.mark.parametrize("D,n,prec", [(2, (4, 6, 5), B.DOT_FP64), (3, (2, 3, 4, 3), B.DOT_FP64),
                                      (2, (3, 7, 4), B.DOT_MIXED), (1, (5, 9), B.DOT_FP64)])
def test_prolongation_matches_the_oracle(D, n, prec):
    print(f"[case] prolong D={D} n={n} prec={prec}", flush=True)
    rng = np.random.default_rng(3)
    ci = dotgen.tiny_instance(D, n, seed=12)
    nf = tuple(2 * k for k in n)
    fi = dotgen.tiny_instance(D, nf, seed=13)
    pc = B.dot_plan_create(D, n, ci.rho0, ci.rho1, None, precision=prec)
    pf = B.dot_plan_create(D, nf, fi.rho0, fi.rho1, None, precision=prec)
    gc, gf = O.Grid(D, n), O.Grid(D, nf)
    shapes = G.q_shapes(gc)
    q = [rng.standard_normal(s) for s in shapes]
    al = [rng.standard_normal(s) for s in shapes]
    be = rng.standard_normal((gc.K,) + gc.cell_shape)
    bulk = np.float64 if prec == B.DOT_FP64 else np.float32
    if bulk == np.float32:  # compare against the oracle on the stored values
        q = [a.astype(np.float32).astype(np.float64) for a in q]
        be = be.astype(np.float32).astype(np.float64)
    sc, sf = G.GpuState(pc), G.GpuState(pf)
    sc.reset()
    ic, fi_ = pc.info, pf.info
    _put_planes(sc, ic.off_q, q, n, bulk)
    _put_planes(sc, ic.off_alpha, al, n, np.float64)
    _put_planes(sc, ic.off_beta, list(be), n, bulk)
    B.dot_prolong(pc, sc.ptr, pf, sf.ptr, G.stream_handle())
    S = O.State(np.zeros(gc.node_shape), np.zeros((gc.K,) + gc.cell_shape), q, al, be, 7.0, 0)
    T = ML.prolong_state(S, gc, gf)
    fshapes = G.q_shapes(gf)
    tol = 1e-14 if bulk == np.float64 else 1e-7
    for got, ref in zip(G.unpack(_get_planes(sf, fi_.off_q, D + 1, nf, bulk), fshapes), T.q):
        assert G.rel_err(got, ref) < tol
    for got, ref in zip(G.unpack(_get_planes(sf, fi_.off_alpha, D + 1, nf, np.float64), fshapes), T.alpha):
        assert G.rel_err(got, ref) < 1e-14
    bet = np.stack([B.from_box(p, gf.cell_shape) for p in _get_planes(sf, fi_.off_beta, gf.K, nf, bulk)])
    assert G.rel_err(bet, T.beta) < tol


@pytest.mark.parametrize("D,n,levels,masked", [(2, (8, 16, 16), 1, False), (2, (8, 16, 16), 2, True),
                                               (3, (4, 8, 8, 8), 1, False), (1, (16, 64), 2, False)])
def test_multilevel_solve_matches_the_oracle(D, n, levels, masked):
    print(f"[case] multilevel D={D} n={n} levels={levels} masked={masked}", flush=True)
    inst = dotgen.tiny_instance(D, n, seed=14, floor=0.0 if masked else 0.01, masked=masked)
    tol = 1e-7
    ref, ref_levels = ML.solve_multilevel(D, n, inst.rho0, inst.rho1, inst.mask, levels=levels, tol=tol,
                                          max_iter=40000)
    r, rho, m, lv = B.dot_solve_multilevel(D, n, inst.rho0, inst.rho1, inst.mask, levels=levels, tol=tol,
                                           max_iter=40000)
    assert B.TERM_NAMES[r.term] == "converged" and ref.converged
    for a, b in zip(lv, ref_levels):
        assert abs(a.iters - b.iters) <= 5, (a.iters, b.iters)
    assert abs(r.objective - ref.objective) <= 1e-8 * abs(ref.objective)
    scale = np.max(np.abs(ref.state.alpha[0]))
    assert np.max(np.abs(rho - ref.state.alpha[0])) <= 1e-5 * scale


def test_prolong_rejects_mismatched_grids():
    a = dotgen.tiny_instance(2, (2, 4, 4), seed=1)
    b = dotgen.tiny_instance(2, (4, 8, 6), seed=2)
    pa = B.dot_plan_create(2, a.n, a.rho0, a.rho1)
    pb = B.dot_plan_create(2, b.n, b.rho0, b.rho1)
    sa, sb = G.GpuState(pa), G.GpuState(pb)
    with pytest.raises(B.DotError):
        B.dot_prolong(pa, sa.ptr, pb, sb.ptr, G.stream_handle())
