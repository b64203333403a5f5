"""Pins of the oracle's residuals (Sec. 5.3): eta_P, eta_D, both eta_C terms,
eta^soc_P and eta^soc_D spelled out again with the loop-built matrices of
loop_ops.py (A from eq. Amap, L_T and L_X from eq. ltlx, B_omega F from
eq. fdetails / eq. bdd), compared with oracle.residuals() on random states of
masked 1D / 2D / 3D grids; and the zero set of the two sigma-rule terms at
the KKT point of eq. kkt (z = B F q + d, F^*B^* beta + alpha = 0), reached by
the oracle on the tiny grids where its optimum equals the brute-force SOCP
solution.

The discrete L2 norm is the cell-volume weighted one, ||x|| = (h0...hD sum
x^2)^(1/2), for every array (a reading; the paper does not fix the weight)."""
import math

import numpy as np
import pytest

import dotgen
from oracle import bruteforce as BFS
from oracle import dot_oracle as O
from tests import loop_ops as LO


def _nrm(vol, *vs):
    return math.sqrt(vol * sum(float(np.dot(v, v)) for v in vs))


def loop_residuals(D, n, omega_sp_flat, c_flat, phi, z, q, alpha, beta):
    """All six ratios of Sec. 5.3 from dense loop-built matrices. Vectors are
    flat in C order: phi / c on nodes, q / alpha as [q0 (cells), q_1, ..., q_D],
    z / beta component-major (K x cells)."""
    node, cell, stag = LO.shapes(D, n)
    vol = float(np.prod([1.0 / k for k in n]))
    nc = int(np.prod(cell))
    ns = [int(np.prod(s)) for s in stag]
    G = np.vstack(LO.grad_matrix(D, n))               # A: nodes -> (G^s_0, ..., G^s_D)
    LT = LO.avg_matrix(node, 0)                         # L_T: nodes -> cells (time average)
    LX = [LO.avg_matrix(node, d) for d in range(1, D + 1)]   # L_X^d: nodes -> G^s_d
    om_cells = np.tile(omega_sp_flat, n[0])             # time-invariant weights on cells
    BF = LO.BF_matrix(D, n, om_cells)
    K = 4 * D + 2
    dvec = np.zeros(K * nc)
    dvec[:nc] = 1.0
    dvec[(K - 1) * nc:] = 1.0
    # split q and alpha into blocks
    cuts = np.cumsum([nc] + ns)[:-1]
    qb = np.split(q, cuts)
    ab = np.split(alpha, cuts)
    Aphi = G @ phi
    eta_p = _nrm(vol, Aphi - q) / (1 + _nrm(vol, Aphi) + _nrm(vol, q))
    eta_d = _nrm(vol, G.T @ alpha + c_flat) / (1 + _nrm(vol, c_flat))
    # f(q) = q0 + 1/2 omega . L_T L_X^*(|q_1|^2; ...; |q_D|^2) (weighted as in Sec. 5.4.5)
    sq = sum(LX[d - 1].T @ (qb[d] ** 2) for d in range(1, D + 1))
    f = qb[0] + 0.5 * om_cells * (LT @ sq)
    c1 = _nrm(vol, ab[0] - np.maximum(0.0, f + ab[0])) / (1 + _nrm(vol, ab[0]) + _nrm(vol, f))
    # g_d = (L_X^d L_T^*(omega . alpha0)) . q_d
    r = LT.T @ (om_cells * ab[0])
    gq = [(LX[d - 1] @ r) * qb[d] for d in range(1, D + 1)]
    abar = ab[1:]
    c2 = _nrm(vol, *[a - b for a, b in zip(abar, gq)]) / (1 + _nrm(vol, *abar) + _nrm(vol, *gq))
    p2 = _nrm(vol, z - BF @ q - dvec) / (1 + _nrm(vol, dvec))
    ftb = BF.T @ beta
    d2 = _nrm(vol, ftb + alpha) / (1 + _nrm(vol, ftb) + _nrm(vol, alpha))
    return dict(eta_p=eta_p, eta_d=eta_d, eta_c1=c1, eta_c2=c2, eta_c=max(c1, c2),
                eta_dot=max(eta_p, eta_d, c1, c2), p2=p2, d2=d2,
                eta_p_soc=max(eta_p, p2), eta_d_soc=max(eta_d, d2))


def _flat_state(P, phi, z, q, alpha, beta):
    return (phi.ravel(), z.reshape(-1), np.concatenate([a.ravel() for a in q]),
            np.concatenate([a.ravel() for a in alpha]), beta.reshape(-1))


def _omega_sp(P):
    return P.omega[0].ravel()


@pytest.mark.parametrize("D,n,masked,seed", [
    (1, (4, 7), False, 1), (1, (3, 6), True, 2),
    (2, (3, 4, 5), False, 3), (2, (3, 5, 4), True, 4),
    (3, (2, 3, 3, 4), False, 5), (3, (2, 4, 3, 3), True, 6)])
def test_residuals_match_the_loop_spelling(D, n, masked, seed):
    inst = dotgen.tiny_instance(D, n, seed=seed, masked=masked)
    P = O.make_problem(D, n, inst.rho0, inst.rho1, inst.mask)
    g = P.g
    rng = np.random.default_rng(100 + seed)
    phi = rng.standard_normal(g.node_shape)
    z = rng.standard_normal((g.K,) + g.cell_shape)
    q = [rng.standard_normal(g.cell_shape)] + [rng.standard_normal(g.q_shape(d)) for d in range(1, D + 1)]
    # alpha0 of both signs, so that both branches of max{0, f + alpha0} occur
    alpha = [rng.standard_normal(a.shape) for a in q]
    beta = rng.standard_normal((g.K,) + g.cell_shape)
    got = O.residuals(P, phi, z, q, alpha, beta)
    ref = loop_residuals(D, n, _omega_sp(P), P.c.ravel(), *_flat_state(P, phi, z, q, alpha, beta))
    for k in ("eta_p", "eta_d", "eta_c1", "eta_c2", "eta_c", "eta_dot", "eta_p_soc", "eta_d_soc"):
        assert got[k] == pytest.approx(ref[k], rel=1e-12), k
    # the sigma-rule terms themselves decide eta^soc on random states (they are not
    # hidden behind eta_P / eta_D), so the comparison above covers p2 and d2
    assert ref["p2"] > ref["eta_p"] and ref["d2"] > 0


def test_sigma_rule_terms_separately():
    """p2 and d2 each checked on states where they are the larger term of the
    max, and against values computed by hand: with q = 0, beta = 0 and z = d,
    p2 = 0 and d2 = |alpha| / (1 + |alpha|); with z = 0, p2 = |d| / (1 + |d|)."""
    D, n = 2, (3, 4, 4)
    inst = dotgen.tiny_instance(D, n, seed=11, masked=True)
    P = O.make_problem(D, n, inst.rho0, inst.rho1, inst.mask)
    g = P.g
    q = [np.zeros(g.cell_shape)] + [np.zeros(g.q_shape(d)) for d in range(1, D + 1)]
    rng = np.random.default_rng(5)
    alpha = [rng.standard_normal(a.shape) for a in q]
    beta = np.zeros((g.K,) + g.cell_shape)
    phi = np.zeros(g.node_shape)
    dv = O.cone_offset(g)
    r = O.residuals(P, phi, dv, q, alpha, beta)
    na = O.l2(alpha, g)
    assert r["eta_d_soc"] == pytest.approx(max(r["eta_d"], na / (1 + na)), rel=1e-13)
    nd = math.sqrt(g.vol * 2 * np.prod(g.cell_shape))  # d has two unit entries per cell
    r0 = O.residuals(P, phi, np.zeros_like(dv), q, alpha, beta)
    assert r0["eta_p_soc"] == pytest.approx(nd / (1 + nd), rel=1e-13)
    assert r["eta_p_soc"] == pytest.approx(r["eta_p"], abs=0.0)


@pytest.mark.parametrize("D,n,masked", [(1, (4, 6), False), (2, (3, 4, 4), False), (2, (3, 4, 4), True)])
def test_sigma_rule_terms_vanish_at_the_kkt_point(D, n, masked):
    """At a solution of eq. kkt, z = B F q + d and F^*B^* beta + alpha = 0. The
    oracle run to eta_dot <= 1e-11 sits at the brute-force SOCP optimum (same
    objective to 1e-8); there both terms, spelled with the loop matrices, are
    <= 1e-8. The same iterate with beta's sign flipped (a plausible slip in
    F^*B^*) leaves d2 of order one, so the zero is not trivial."""
    inst = dotgen.tiny_instance(D, n, masked=masked)
    bf = BFS.solve(D, n, inst.rho0, inst.rho1, inst.mask)
    P = O.make_problem(D, n, inst.rho0, inst.rho1, inst.mask)
    r = O.solve(P, tol=1e-11, max_iter=20000)
    assert r.converged
    assert abs(r.objective - bf["objective"]) <= 1e-8 * abs(bf["objective"])
    S = r.state
    ref = loop_residuals(D, n, _omega_sp(P), P.c.ravel(), *_flat_state(P, S.phi, S.z, S.q, S.alpha, S.beta))
    assert ref["p2"] <= 1e-8 and ref["d2"] <= 1e-8, (ref["p2"], ref["d2"])
    got = O.residuals(P, S.phi, S.z, S.q, S.alpha, S.beta)
    assert got["eta_p_soc"] <= 1e-8 and got["eta_d_soc"] <= 1e-8
    flipped = loop_residuals(D, n, _omega_sp(P), P.c.ravel(),
                             *_flat_state(P, S.phi, S.z, S.q, S.alpha, -S.beta))
    assert flipped["d2"] > 0.1
    # beta in Q and alpha0 = -(F^*B^* beta)_0 >= 0 at the solution (proof of Prop. 3.3)
    y0, yb = S.beta[0], S.beta[1:]
    assert np.all(np.sqrt(np.sum(yb * yb, axis=0)) <= y0 + 1e-9)
