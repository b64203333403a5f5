"""Exact squared 2-Wasserstein distance between two piecewise-constant
densities on [0, 1] (TEST INFRASTRUCTURE).

Each node mass m_i of a grid with n segments is spread uniformly over the
node's cell X_i = [x_i - h/2, x_i + h/2] clipped to [0, 1] (the cube that the
sampling of eq. defc integrates over). In one dimension the W2 distance is
the L2 distance between quantile functions,
    W2^2 = int_0^1 (Q0(s) - Q1(s))^2 ds,
and for piecewise-constant densities both quantile functions are piecewise
linear, so after merging the breakpoints the integrand is a quadratic on each
piece and Simpson's rule integrates it exactly.
"""
from __future__ import annotations

import numpy as np


def _cells(n):
    h = 1.0 / n
    edges = np.concatenate([[0.0], (np.arange(n) + 0.5) * h, [1.0]])
    return edges  # cell i = [edges[i], edges[i+1]], i = 0..n


def _quantile_on(piece_lo, piece_hi, C, edges):
    """Return Q restricted to [piece_lo, piece_hi]: the piece lies inside the
    mass interval [C_i, C_{i+1}] of one cell i of positive mass, where Q runs
    linearly from edges[i] to edges[i+1]. The slope uses C_{i+1} - C_i, the
    same numbers the breakpoints come from, so Q stays inside the cell."""
    mid = 0.5 * (piece_lo + piece_hi)
    i = int(np.searchsorted(C, mid, side="right") - 1)
    i = min(max(i, 0), len(C) - 2)
    while C[i + 1] - C[i] <= 0:
        i += 1
    a, b = edges[i], edges[i + 1]
    dm = C[i + 1] - C[i]

    def Q(s):
        return a + min(max((s - C[i]) / dm, 0.0), 1.0) * (b - a)
    return Q


def w2_squared(rho0, rho1):
    m0 = np.asarray(rho0, dtype=np.float64)
    m1 = np.asarray(rho1, dtype=np.float64)
    assert m0.shape == m1.shape and m0.ndim == 1
    n = m0.size - 1
    m0 = m0 / m0.sum()
    m1 = m1 / m1.sum()
    edges = _cells(n)
    C0 = np.concatenate([[0.0], np.cumsum(m0)])
    C1 = np.concatenate([[0.0], np.cumsum(m1)])
    C0 = np.minimum(C0, 1.0)
    C1 = np.minimum(C1, 1.0)
    C0[-1] = C1[-1] = 1.0
    br = np.unique(np.concatenate([C0, C1]))
    br = br[(br >= 0.0) & (br <= 1.0)]
    total = 0.0
    for lo, hi in zip(br[:-1], br[1:]):
        if hi - lo <= 0:
            continue
        Q0 = _quantile_on(lo, hi, C0, edges)
        Q1 = _quantile_on(lo, hi, C1, edges)
        f = lambda s: (Q0(s) - Q1(s)) ** 2
        total += (hi - lo) / 6.0 * (f(lo) + 4.0 * f(0.5 * (lo + hi)) + f(hi))
    return total
