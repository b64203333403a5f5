"""Each explicit step of Algorithm 2 solves the subproblem that Algorithm 1
states, checked with loop-built dense matrices of A and B_omega F (so the
check does not reuse the oracle's operators)."""
import numpy as np
import pytest

from oracle import dot_oracle as O
from tests import loop_ops as L

CASES = [(1, (4, 6)), (2, (3, 4, 5)), (3, (2, 3, 2, 3))]


def _flat(arrs):
    return np.concatenate([a.ravel() for a in arrs])


def _random_state(P, rng):
    g = P.g
    q = [rng.standard_normal(g.cell_shape)] + [rng.standard_normal(g.q_shape(d)) for d in range(1, g.D + 1)]
    al = [rng.standard_normal(a.shape) for a in q]
    be = O.proj_soc(rng.standard_normal((g.K,) + g.cell_shape))
    return q, al, be


@pytest.mark.parametrize("D,n", CASES)
@pytest.mark.parametrize("masked", [False, True])
def test_alg2_steps_minimise_the_augmented_lagrangian(D, n, masked):
    rng = np.random.default_rng(21)
    sp = tuple(k + 1 for k in n[1:])
    r0 = rng.uniform(0.1, 1, sp)
    r0 /= r0.sum()
    r1 = rng.uniform(0.1, 1, sp)
    r1 /= r1.sum()
    mask = None
    if masked:
        mask = np.zeros(sp, dtype=np.uint8)
        mask[(slice(1, 2),) * D] = 1
    P = O.make_problem(D, n, r0, r1, mask)
    g = P.g
    q, al, be = _random_state(P, rng)
    sigma, tau = 0.7, 1.9
    A = np.vstack(L.grad_matrix(D, n))
    BFm = L.BF_matrix(D, n, P.omega.ravel())
    dvec = O.cone_offset(g).ravel()
    c = P.c.ravel()
    qf, af, bf = _flat(q), _flat(al), be.ravel()

    # phi-step: argmin over rge(A^*) of <c,phi> + <A phi - q, alpha> + sigma/2 |A phi - q|^2
    b = O.step_rhs(P, q, al, sigma)
    phi = O.poisson(b, g, P.lam)
    grad_phi = c + A.T @ af + sigma * A.T @ (A @ phi.ravel() - qf)
    grad_phi -= grad_phi.mean()  # component in rge(A^*) (orthogonal to constants)
    assert np.linalg.norm(grad_phi) <= 1e-9 * (1 + np.linalg.norm(c))
    assert abs(phi.mean()) <= 1e-12 * (1 + np.abs(phi).max())

    # z-step: z = Pi_Q(B F q + d - beta/sigma), i.e. z in Q, z - v in Q, <z, z - v> = 0 per cell
    v = (BFm @ qf + dvec - bf / sigma).reshape((g.K, -1))
    z = O.proj_soc(O.step_cone_input(P, q, be, sigma)).reshape((g.K, -1))
    for a in (z, z - v):
        assert np.all(a[0] >= np.linalg.norm(a[1:], axis=0) - 1e-12)
    assert np.max(np.abs(np.sum(z * (z - v), axis=0))) <= 1e-11

    # q-step: gradient of L_sigma in q vanishes at q^{k+1}
    zz = z.reshape((g.K,) + g.cell_shape)
    qn = O.step_q(P, phi, zz, al, be, sigma)
    qnf = _flat(qn)
    Aphi = A @ phi.ravel()
    gq = -af - BFm.T @ bf - sigma * (Aphi - qnf) - sigma * BFm.T @ (zz.ravel() - BFm @ qnf - dvec)
    assert np.linalg.norm(gq) <= 1e-10 * (1 + np.linalg.norm(af) + np.linalg.norm(bf))

    # multipliers: (alpha, beta) += tau sigma (M(phi; z) + N q - (0; d)) as in Algorithm 1
    S1 = O.iterate(P, O.State(np.zeros(g.node_shape), np.zeros_like(be), q, al, be, sigma), tau)
    np.testing.assert_allclose(_flat(S1.alpha), af + tau * sigma * (Aphi - qnf), atol=1e-10)
    np.testing.assert_allclose(S1.beta.ravel(), bf + tau * sigma * (zz.ravel() - BFm @ qnf - dvec), atol=1e-10)
