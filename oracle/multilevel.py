"""Multilevel initialisation for the oracle: restriction of the data to a grid
with half the segments per axis, linear prolongation of a coarse iterate to
the finer grid, and the level-by-level solve.

TEST INFRASTRUCTURE. Only the test suite and the benchmark's CPU-baseline leg
may import this module; the product path never does.

The paper (implementation details of Sec. 5.3 and the experiments of Sec. 5.4)
solves first on grids with n_d / 2^v segments, v = L, ..., 1, interpolates
each coarse solution linearly to the next finer grid and uses it as the
initial point there; each level v is solved to max{Tol * 10^-v, 1e-6}. The
paper gives neither the restriction of the data nor the interpolation
stencil; the readings used here are:
  * data: node masses restricted by the transpose of linear interpolation
    (full weighting): fine node 2i gives all its mass to coarse node i, fine
    node 2i+1 half to coarse nodes i and i+1, per axis; total mass is kept.
    A coarse node is an obstacle node when fine node 2i is one.
  * iterate: q, alpha and beta are interpolated linearly in physical
    coordinates along each axis (tensor product), from the coarse positions
    of their grid (node i/n or staggered (s+1/2)/n) to the fine ones, with
    constant extension beyond the outermost coarse positions. phi and z are
    outputs of the next iteration and start at zero. sigma carries over; the
    iteration count and the sigma schedule restart.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import dot_oracle as O


def restrict_axis(m: np.ndarray, axis: int) -> np.ndarray:
    """Full-weighting transpose along one axis: length 2k+1 -> k+1."""
    nf = m.shape[axis] - 1
    assert nf % 2 == 0, "segment counts must be even to coarsen"
    nc = nf // 2
    shape = list(m.shape)
    shape[axis] = nc + 1
    out = np.zeros(shape)
    for i in range(nc + 1):
        idx = [slice(None)] * m.ndim
        oidx = [slice(None)] * m.ndim
        oidx[axis] = i
        idx[axis] = 2 * i
        out[tuple(oidx)] += m[tuple(idx)]
        if 2 * i - 1 >= 0:
            idx[axis] = 2 * i - 1
            out[tuple(oidx)] += 0.5 * m[tuple(idx)]
        if 2 * i + 1 <= nf:
            idx[axis] = 2 * i + 1
            out[tuple(oidx)] += 0.5 * m[tuple(idx)]
    return out


def restrict_masses(m: np.ndarray) -> np.ndarray:
    out = np.asarray(m, dtype=np.float64)
    for ax in range(out.ndim):
        out = restrict_axis(out, ax)
    return out


def restrict_mask(mask):
    if mask is None:
        return None
    return np.asarray(mask)[tuple(slice(None, None, 2) for _ in range(np.ndim(mask)))].copy()


def coarse_data(n: Sequence[int], rho0, rho1, mask=None):
    """(n / 2, rho0, rho1, mask) of the next coarser grid; obstacle nodes of
    the coarse grid carry no mass (the data are zero there, as on the fine grid)."""
    nc = tuple(k // 2 for k in n)
    assert all(2 * a == b for a, b in zip(nc, n)), "segment counts must be even to coarsen"
    r0 = restrict_masses(rho0)
    r1 = restrict_masses(rho1)
    mk = restrict_mask(mask)
    if mk is not None:
        r0 = np.where(mk != 0, 0.0, r0)
        r1 = np.where(mk != 0, 0.0, r1)
        r0 = r0 / r0.sum()
        r1 = r1 / r1.sum()
    return nc, r0, r1, mk


def _positions(ncells: int, staggered: bool) -> np.ndarray:
    if staggered:
        return (np.arange(ncells) + 0.5) / ncells
    return np.arange(ncells + 1) / ncells


def interp_axis(a: np.ndarray, axis: int, nc: int, nf: int, staggered: bool) -> np.ndarray:
    """Linear interpolation along `axis` from the coarse positions (nc
    segments) to the fine ones (nf segments), constant beyond the ends."""
    xc = _positions(nc, staggered)
    xf = _positions(nf, staggered)
    shape = list(a.shape)
    shape[axis] = len(xf)
    out = np.zeros(shape)
    for j, x in enumerate(xf):
        if x <= xc[0]:
            lo, hi, w = 0, 0, 0.0
        elif x >= xc[-1]:
            lo, hi, w = len(xc) - 1, len(xc) - 1, 0.0
        else:
            hi = int(np.searchsorted(xc, x, side="right"))
            lo = hi - 1
            w = (x - xc[lo]) / (xc[hi] - xc[lo])
        oidx = [slice(None)] * a.ndim
        oidx[axis] = j
        il = [slice(None)] * a.ndim
        il[axis] = lo
        ih = [slice(None)] * a.ndim
        ih[axis] = hi
        out[tuple(oidx)] = (1.0 - w) * a[tuple(il)] + w * a[tuple(ih)]
    return out


def prolong_array(a: np.ndarray, nc: Sequence[int], nf: Sequence[int], stag: Sequence[bool]) -> np.ndarray:
    """Tensor-product linear interpolation; stag[axis] tells whether the
    array lives on the staggered positions of that axis."""
    out = a
    for ax in range(a.ndim):
        out = interp_axis(out, ax, nc[ax], nf[ax], stag[ax])
    return out


def prolong_state(S: O.State, gc: O.Grid, gf: O.Grid) -> O.State:
    D = gc.D
    cell = [True] + [False] * D  # cells: staggered in time, nodes in space
    q = [prolong_array(S.q[0], gc.n, gf.n, cell)]
    al = [prolong_array(S.alpha[0], gc.n, gf.n, cell)]
    for d in range(1, D + 1):
        st = [False] * (D + 1)
        st[d] = True  # q_d: time nodes, staggered on axis d
        q.append(prolong_array(S.q[d], gc.n, gf.n, st))
        al.append(prolong_array(S.alpha[d], gc.n, gf.n, st))
    beta = np.stack([prolong_array(S.beta[k], gc.n, gf.n, cell) for k in range(gc.K)])
    return O.State(np.zeros(gf.node_shape), np.zeros((gf.K,) + gf.cell_shape), q, al, beta, S.sigma, 0)


def level_tolerances(tol: float, levels: int) -> List[float]:
    """Tolerance of coarse levels v = levels, ..., 1 (max{Tol 10^-v, 1e-6})."""
    return [max(tol * 10.0 ** (-v), 1e-6) for v in range(levels, 0, -1)]


def solve_multilevel(D, n, rho0, rho1, mask=None, levels=2, tol=1e-6, max_iter=100000, **kw):
    """Coarsest level from zero, then each finer level from the prolonged
    iterate of the previous one; returns (fine SolveResult, per-level results)."""
    data = [(tuple(n), np.asarray(rho0, float), np.asarray(rho1, float), mask)]
    for _ in range(levels):
        data.append(coarse_data(*data[-1]))
    data = data[::-1]  # coarsest first
    tols = level_tolerances(tol, levels) + [tol]
    state = None
    prev_grid = None
    results = []
    for (nl, r0, r1, mk), tl in zip(data, tols):
        P = O.make_problem(D, nl, r0, r1, mk)
        if state is not None:
            state = prolong_state(state, prev_grid, P.g)
        r = O.solve(P, tol=tl, max_iter=max_iter, state=state, **kw)
        results.append(r)
        state = r.state
        prev_grid = P.g
    return results[-1], results
