"""Pins for the oracle's operators: loop-built matrices, the decoupling
identity, the diagonal of Prop. 3.2, ker A, the Poisson solve and the
strictly feasible points of Prop. 3.1."""
import json
import os

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import dot_oracle as O
from tests import loop_ops as L

GOLD = os.path.join(os.path.dirname(__file__), "golden")
GRIDS = [(1, (3, 5)), (2, (3, 4, 5)), (2, (2, 3, 3)), (3, (2, 3, 2, 4))]


def _flat(arrs):
    return np.concatenate([a.ravel() for a in arrs])


def _rand_q(g, rng):
    return [rng.standard_normal(g.cell_shape)] + [rng.standard_normal(g.q_shape(d)) for d in range(1, g.D + 1)]


@pytest.mark.parametrize("D,n", GRIDS)
def test_grad_matches_loop_matrix_and_adjoint(D, n):
    g = O.Grid(D, n)
    rng = np.random.default_rng(1)
    phi = rng.standard_normal(g.node_shape)
    Ms = L.grad_matrix(D, n)
    for d, (q, M) in enumerate(zip(O.grad(phi, g), Ms)):
        np.testing.assert_allclose(q.ravel(), M @ phi.ravel(), rtol=0, atol=1e-12)
    y = _rand_q(g, rng)
    At = sum(M.T @ yy.ravel() for M, yy in zip(Ms, y))
    np.testing.assert_allclose(O.grad_adj(y, g).ravel(), At, rtol=0, atol=1e-11)


@pytest.mark.parametrize("D,n", GRIDS)
def test_kernel_of_A_is_constants(D, n):
    """eq. kerA: A phi = 0 exactly for constants; the null space has dimension 1."""
    g = O.Grid(D, n)
    for q in O.grad(np.full(g.node_shape, 3.7), g):
        assert np.max(np.abs(q)) == 0.0
    A = np.vstack(L.grad_matrix(D, n))
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.sum(sv < 1e-10 * sv[0]) == 1


@pytest.mark.parametrize("D,n", GRIDS)
def test_interpolations_match_loop_matrices(D, n):
    g = O.Grid(D, n)
    rng = np.random.default_rng(2)
    y = rng.standard_normal(g.node_shape)
    MT = L.avg_matrix(g.node_shape, 0)
    np.testing.assert_allclose(O.LT(y).ravel(), MT @ y.ravel(), atol=1e-14)
    a = rng.standard_normal(g.cell_shape)
    np.testing.assert_allclose(O.LT_adj(a).ravel(), MT.T @ a.ravel(), atol=1e-14)
    for d in range(1, D + 1):
        MX = L.avg_matrix(g.node_shape, d)
        np.testing.assert_allclose(O.LX(y, d).ravel(), MX @ y.ravel(), atol=1e-14)


@pytest.mark.parametrize("D,n", GRIDS)
def test_F_matches_fdetails_and_adjoint(D, n):
    g = O.Grid(D, n)
    rng = np.random.default_rng(3)
    Fm = L.F_matrices(D, n)
    for d in range(1, D + 1):
        qd = rng.standard_normal(g.q_shape(d))
        parts = O.F_d(qd, d, g)
        for v in range(4):
            np.testing.assert_array_equal(parts[v].ravel(), Fm[(d, v + 1)] @ qd.ravel())
        a = [rng.standard_normal(g.cell_shape) for _ in range(4)]
        back = sum(Fm[(d, v + 1)].T @ a[v].ravel() for v in range(4))
        np.testing.assert_allclose(O.F_d_adj(a, d, g).ravel(), back, atol=1e-13)


@pytest.mark.parametrize("D,n", GRIDS)
def test_decoupling_identity(D, n):
    """eq. f1vf2v: L_T L_X^*(q_1; ...; q_D) = 1/4 sum_d sum_v F^d_v q_d, with the
    left side built from the loop matrices of L_T and L_X^d."""
    g = O.Grid(D, n)
    rng = np.random.default_rng(4)
    qb = [rng.standard_normal(g.q_shape(d)) for d in range(1, D + 1)]
    MT = L.avg_matrix(g.node_shape, 0)
    lhs = MT @ sum(L.avg_matrix(g.node_shape, d).T @ qb[d - 1].ravel() for d in range(1, D + 1))
    rhs = 0.25 * sum(sum(O.F_d(qb[d - 1], d, g)) for d in range(1, D + 1))
    np.testing.assert_allclose(rhs.ravel(), lhs, atol=1e-13)


@pytest.mark.parametrize("D,n", GRIDS)
@pytest.mark.parametrize("weighted", [False, True])
def test_prop32_diagonal(D, n, weighted):
    """Prop. 3.2: F^*B^*BF is diagonal; with omega = 1 the diagonal of
    I + F^*B^*BF is 3 on q0 and 2 / 3 / 2 on q_d at the first / inner / last
    time node (paper values in tests/golden/prop32_diagonal.json)."""
    gold = json.load(open(os.path.join(GOLD, "prop32_diagonal.json")))
    g = O.Grid(D, n)
    rng = np.random.default_rng(5)
    sp = g.node_shape[1:]
    om_sp = rng.uniform(0.2, 1.5, size=sp) if weighted else np.ones(sp)
    om = np.broadcast_to(om_sp[None], g.cell_shape).copy()
    BFm = L.BF_matrix(D, n, om.ravel())
    G = BFm.T @ BFm
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) < 1e-14
    diag_or = _flat(O.q_diag(om, g))
    np.testing.assert_allclose(1.0 + np.diag(G), diag_or, rtol=1e-14)
    if not weighted:
        ref = gold["I_plus_FBBF"]
        dg = O.q_diag(om, g)
        assert np.all(dg[0] == ref["q0"])
        for d in range(1, D + 1):
            assert np.all(dg[d][0] == ref["qd_first"])
            assert np.all(dg[d][-1] == ref["qd_last"])
            assert np.all(dg[d][1:-1] == ref["qd_interior"])


@pytest.mark.parametrize("D,n", GRIDS)
def test_BF_and_FtBt_match_loop_matrix(D, n):
    g = O.Grid(D, n)
    rng = np.random.default_rng(6)
    om_sp = rng.uniform(0.1, 1.0, size=g.node_shape[1:])
    om = np.broadcast_to(om_sp[None], g.cell_shape).copy()
    BFm = L.BF_matrix(D, n, om.ravel())
    q = _rand_q(g, rng)
    np.testing.assert_allclose(O.BF(q, om, g).ravel(), BFm @ _flat(q), atol=1e-13)
    u = rng.standard_normal((g.K,) + g.cell_shape)
    np.testing.assert_allclose(_flat(O.FtBt(u, om, g)), BFm.T @ u.ravel(), atol=1e-13)


@pytest.mark.parametrize("D,n", GRIDS)
def test_poisson_against_dense_pseudoinverse(D, n):
    g = O.Grid(D, n)
    rng = np.random.default_rng(7)
    b = rng.standard_normal(g.node_shape)
    A = np.vstack(L.grad_matrix(D, n))
    AtA = A.T @ A
    phi_ref = np.linalg.pinv(AtA) @ b.ravel()
    phi = O.poisson(b, g)
    np.testing.assert_allclose(phi.ravel(), phi_ref, atol=1e-10 * np.max(np.abs(phi_ref)))
    assert abs(phi.mean()) < 1e-13 * np.max(np.abs(phi))
    res = AtA @ phi.ravel() - (b.ravel() - b.mean())
    assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("N", [2, 5, 17, 33])
def test_path_laplacian_eigenpairs_are_dct2(N):
    """Each axis of A^*A is the path-graph Laplacian; its eigenvectors are the
    orthonormal DCT-II basis with eigenvalues 4 sin^2(pi k / (2N)) (times 1/h^2)."""
    T = np.diag(np.r_[1.0, 2.0 * np.ones(N - 2), 1.0]) - np.diag(np.ones(N - 1), 1) - np.diag(np.ones(N - 1), -1)
    C = sfft.dct(np.eye(N), type=2, norm="ortho", axis=0)  # rows = basis vectors
    lam = 4.0 * np.sin(np.pi * np.arange(N) / (2.0 * N)) ** 2
    np.testing.assert_allclose(C @ T @ C.T, np.diag(lam), atol=1e-12)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(T)), np.sort(lam), atol=1e-12)


@pytest.mark.parametrize("D,n", GRIDS)
def test_prop31_strictly_feasible_points(D, n):
    """Proof of Prop. 3.1: phi*_{i0} = -h0 (i0+1) zeta gives A phi* = (-zeta 1; 0),
    and then B F q* + d lies in the interior of Q; xi_0 = h0...hD 1 gives
    -A_0^* xi_0 = +-h1...hD on the first / last time slice, 0 inside."""
    g = O.Grid(D, n)
    zeta = 0.37
    t = np.arange(g.n[0] + 1).reshape((-1,) + (1,) * D)
    phi = np.broadcast_to(-g.h[0] * (t + 1) * zeta, g.node_shape).copy()
    q = O.grad(phi, g)
    np.testing.assert_allclose(q[0], -zeta, rtol=1e-13)
    for d in range(1, D + 1):
        assert np.max(np.abs(q[d])) == 0.0
    u = O.BF(q, np.ones(g.cell_shape), g) + O.cone_offset(g)
    assert np.all(u[0] - np.sqrt(np.sum(u[1:] ** 2, axis=0)) > 0)
    xi0 = np.full(g.cell_shape, g.vol)
    y = [xi0] + [np.zeros(g.q_shape(d)) for d in range(1, D + 1)]
    r = -O.grad_adj(y, g)
    hX = float(np.prod(g.h[1:]))
    np.testing.assert_allclose(r[0], hX, rtol=1e-13)
    np.testing.assert_allclose(r[-1], -hX, rtol=1e-13)
    if g.n[0] > 1:
        assert np.max(np.abs(r[1:-1])) < 1e-15
