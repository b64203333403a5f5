"""Dense matrices of the paper's operators built by explicit index loops.

Used only by the tests, as an independent spelling of the definitions in
Sec. 2.2 (A, L_T, L_X) and Sec. 3.2-3.3 (F, B): the vectorised oracle is
checked against these, so a sign, index or transposition slip in either
shows up as a mismatch.
"""
import itertools

import numpy as np


def shapes(D, n):
    node = tuple(k + 1 for k in n)
    cell = (n[0],) + node[1:]
    stag = []
    for d in range(1, D + 1):
        s = list(node)
        s[d] = n[d]
        stag.append(tuple(s))
    return node, cell, stag


def flat_index(shape):
    return {p: i for i, p in enumerate(itertools.product(*[range(s) for s in shape]))}


def grad_matrix(D, n):
    """Rows: q0 (cells) then q_1..q_D; columns: nodes."""
    h = [1.0 / k for k in n]
    node, cell, stag = shapes(D, n)
    N = flat_index(node)
    blocks = []
    for d, shp in enumerate([cell] + stag):
        Idx = flat_index(shp)
        M = np.zeros((len(Idx), len(N)))
        for p, i in Idx.items():
            hi = tuple(v + (1 if a == d else 0) for a, v in enumerate(p))
            M[i, N[hi]] = 1.0 / h[d]
            M[i, N[p]] = -1.0 / h[d]
        blocks.append(M)
    return blocks


def avg_matrix(shape_from, axis):
    """Average of neighbours along `axis`: output has one entry less on that axis."""
    out_shape = list(shape_from)
    out_shape[axis] -= 1
    src = flat_index(shape_from)
    dst = flat_index(tuple(out_shape))
    M = np.zeros((len(dst), len(src)))
    for p, i in dst.items():
        hi = tuple(v + (1 if a == axis else 0) for a, v in enumerate(p))
        M[i, src[p]] += 0.5
        M[i, src[hi]] += 0.5
    return M


def F_matrices(D, n):
    """F^d_v as dense (cells x G^s_d) matrices, straight from eq. fdetails:
    cell (t, x); v=1: q_d[t, x_d-1] if x_d >= 1; v=2: q_d[t, x_d] if x_d <= n_d-1;
    v=3: q_d[t+1, x_d-1] if x_d >= 1; v=4: q_d[t+1, x_d] if x_d <= n_d-1."""
    node, cell, stag = shapes(D, n)
    C = flat_index(cell)
    out = {}
    for d in range(1, D + 1):
        S = flat_index(stag[d - 1])
        for v in range(1, 5):
            M = np.zeros((len(C), len(S)))
            for p, i in C.items():
                t = p[0]
                xd = p[d]
                if v in (1, 3):
                    if xd < 1:
                        continue
                    s = xd - 1
                else:
                    if xd > n[d] - 1:
                        continue
                    s = xd
                tt = t if v in (1, 2) else t + 1
                qpos = list(p)
                qpos[0] = tt
                qpos[d] = s
                M[i, S[tuple(qpos)]] = 1.0
            out[(d, v)] = M
    return out


def BF_matrix(D, n, omega_cells_flat):
    """B_omega F as a dense matrix: rows = K cone components x cells (component
    major), columns = q0, q_1, ..., q_D."""
    node, cell, stag = shapes(D, n)
    nc = int(np.prod(cell))
    ns = [int(np.prod(s)) for s in stag]
    K = 4 * D + 2
    Fm = F_matrices(D, n)
    cols = nc + sum(ns)
    M = np.zeros((K * nc, cols))
    I = np.eye(nc)
    M[0:nc, 0:nc] = -I
    M[(K - 1) * nc:K * nc, 0:nc] = I
    sc = np.sqrt(omega_cells_flat / 2.0)[:, None]
    off = nc
    for d in range(1, D + 1):
        for v in range(1, 5):
            r = 1 + 4 * (d - 1) + (v - 1)
            M[r * nc:(r + 1) * nc, off:off + ns[d - 1]] = sc * Fm[(d, v)]
        off += ns[d - 1]
    return M
