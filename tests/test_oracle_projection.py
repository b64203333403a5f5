"""Pins for the cone projection (eq. app-proj) and the SOC embedding of the
parabolic constraint (eq. socobservation)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from hypothesis.extra import numpy as hnp

from oracle import dot_oracle as O

finite = st.floats(min_value=-1e3, max_value=1e3, allow_nan=False, allow_infinity=False)


def _in_cone(y, tol=1e-12):
    return y[0] >= np.linalg.norm(y[1:]) - tol * (1 + np.abs(y).max())


@settings(max_examples=300, deadline=None)
@given(hnp.arrays(np.float64, st.integers(2, 14), elements=finite))
def test_projection_properties(y):
    p = O.proj_soc(y[:, None])[:, 0]
    m = -O.proj_soc(-y[:, None])[:, 0]
    scale = 1 + np.abs(y).max()
    assert _in_cone(p)
    # idempotence
    np.testing.assert_allclose(O.proj_soc(p[:, None])[:, 0], p, atol=1e-12 * scale)
    # Moreau decomposition for the self-dual cone: y = P_K(y) - P_K(-y), orthogonal parts
    np.testing.assert_allclose(p + m, y, atol=1e-11 * scale)
    assert abs(np.dot(p, m)) <= 1e-9 * scale * scale


def _nearest_by_bisection(y):
    """Nearest point of the cone by a 1-D search: for y outside K and -K, the
    projection is (s, s ybar/|ybar|) with s minimising (s-y0)^2 + (s-|ybar|)^2
    over s >= 0, and the candidates y (if inside) and 0 complete the search."""
    y0, yb = y[0], y[1:]
    nb = np.linalg.norm(yb)
    cands = [np.zeros_like(y)]
    if y0 >= nb:
        cands.append(y.copy())
    if nb > 0:
        lo, hi = 0.0, max(abs(y0), nb) + 1.0
        f = lambda s: (s - y0) ** 2 + (s - nb) ** 2
        for _ in range(200):
            a = lo + (hi - lo) / 3
            b = hi - (hi - lo) / 3
            if f(a) <= f(b):
                hi = b
            else:
                lo = a
        s = 0.5 * (lo + hi)
        cands.append(np.r_[s, s * yb / nb])
    return min(cands, key=lambda c: np.linalg.norm(c - y))


def test_projection_is_nearest_point():
    rng = np.random.default_rng(11)
    for K in (6, 10, 14):
        for _ in range(200):
            y = rng.standard_normal(K) * rng.uniform(0.1, 10)
            p = O.proj_soc(y[:, None])[:, 0]
            q = _nearest_by_bisection(y)
            assert np.linalg.norm(p - y) <= np.linalg.norm(q - y) + 1e-9
            np.testing.assert_allclose(p, q, atol=1e-7 * (1 + np.abs(y).max()))


def test_projection_cases():
    # inside: unchanged; polar: zero; boundary tie y = 0 gives zero
    y = np.array([3.0, 1.0, 2.0])
    np.testing.assert_array_equal(O.proj_soc(y[:, None])[:, 0], y)
    y = np.array([-3.0, 1.0, 2.0])
    np.testing.assert_array_equal(O.proj_soc(y[:, None])[:, 0], 0 * y)
    np.testing.assert_array_equal(O.proj_soc(np.zeros((5, 1)))[:, 0], np.zeros(5))
    y = np.array([0.0, 3.0, 4.0])
    np.testing.assert_allclose(O.proj_soc(y[:, None])[:, 0], [2.5, 1.5, 2.0])


@pytest.mark.parametrize("D", [1, 2, 3])
def test_socobservation_equivalence(D):
    """x0 + 1/8 sum x_v^2 <= 0  <=>  (1 - x0, sqrt(2)/2 x_v, 1 + x0) in K_soc."""
    rng = np.random.default_rng(12)
    K = 4 * D + 2
    for _ in range(2000):
        x = rng.standard_normal(K - 1) * rng.uniform(0.01, 3)
        lhs = x[0] + np.sum(x[1:] ** 2) / 8.0 <= 0
        y = np.r_[1 - x[0], np.sqrt(2) / 2 * x[1:], 1 + x[0]]
        rhs = y[0] >= np.linalg.norm(y[1:])
        margin = abs(x[0] + np.sum(x[1:] ** 2) / 8.0)
        if margin > 1e-12:
            assert lhs == rhs
