"""Brute-force reference for tiny grids: the discrete primal (rho, m) problem
solved by a dense log-barrier Newton method.

TEST INFRASTRUCTURE (only tests may use it). It pins the PALM oracle from
outside: it never calls the oracle's operators; every matrix here is built
by explicit loops from the definitions of Sec. 2.2.

Problem (dual of the discretised DOT problem, eq. kkt-dualy, with weights):
    min  sum_d sum_i m_{d,i}^2 / (2 r_{d,i})
    s.t. A^*(alpha0; m) = -c~,  alpha0 >= 0,
         r_d = L_X^d L_T^*(omega . alpha0)
written in epigraph form with rotated cones 2 r_i s_i >= m_i^2, s >= 0:
    min sum s   s.t. the same equality, (r_i, s_i, m_i) in the rotated cone.
The barrier is -sum log(2 r s - m^2) - sum log(alpha0) (degree 2 per cone, 1
per alpha0 entry); the central path is followed with t <- 10 t until the
duality-gap bound nu/t is below 1e-13. The strictly feasible start is
alpha0 = gamma * 1 with gamma = h0 * sum(rho0) / ((h0...hD) prod(n_d + 1)) (the
constant field xi_0 of the proof of Prop. 3.1, rescaled so that the mass of
every time slice equals that of rho0 in the scaled units), m the
minimum-norm solution of the remaining spatial divergence equations.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, Optional

import numpy as np


def _index_maps(D, n):
    """Flat index maps for nodes, cells and staggered sets, built by loops."""
    node_shape = tuple(k + 1 for k in n)
    nodes = {p: i for i, p in enumerate(itertools.product(*[range(s) for s in node_shape]))}
    cell_shape = (n[0],) + node_shape[1:]
    cells = {p: i for i, p in enumerate(itertools.product(*[range(s) for s in cell_shape]))}
    stag = []
    for d in range(1, D + 1):
        sh = list(node_shape)
        sh[d] = n[d]
        stag.append({p: i for i, p in enumerate(itertools.product(*[range(s) for s in sh]))})
    return node_shape, nodes, cell_shape, cells, stag


def build_matrices(D, n, omega_sp):
    """Dense matrices of A_0 (cells <- nodes), A_d (G^s_d <- nodes), and of the
    interpolated density maps R_d = L_X^d L_T^* diag(omega) (G^s_d <- cells)."""
    h = [1.0 / k for k in n]
    node_shape, nodes, cell_shape, cells, stag = _index_maps(D, n)
    Nn = len(nodes)
    A0 = np.zeros((len(cells), Nn))
    for p, i in cells.items():
        # cell (t, x) is the time point t+1/2 between nodes t and t+1
        lo = p
        hi = (p[0] + 1,) + p[1:]
        A0[i, nodes[hi]] += 1.0 / h[0]
        A0[i, nodes[lo]] -= 1.0 / h[0]
    Ad = []
    for d in range(1, D + 1):
        M = np.zeros((len(stag[d - 1]), Nn))
        for p, i in stag[d - 1].items():
            # staggered point s+1/2 on axis d lies between nodes s and s+1
            lo = p
            hi = tuple(v + (1 if a == d else 0) for a, v in enumerate(p))
            M[i, nodes[hi]] += 1.0 / h[d]
            M[i, nodes[lo]] -= 1.0 / h[d]
        Ad.append(M)
    # L_T: cells <- nodes (average of the two time neighbours)
    LT = np.zeros((len(cells), Nn))
    for p, i in cells.items():
        LT[i, nodes[p]] += 0.5
        LT[i, nodes[(p[0] + 1,) + p[1:]]] += 0.5
    R = []
    om_cells = np.array([omega_sp[p[1:]] for p in cells])
    for d in range(1, D + 1):
        LX = np.zeros((len(stag[d - 1]), Nn))
        for p, i in stag[d - 1].items():
            hi = tuple(v + (1 if a == d else 0) for a, v in enumerate(p))
            LX[i, nodes[p]] += 0.5
            LX[i, nodes[hi]] += 0.5
        R.append(LX @ LT.T @ np.diag(om_cells))
    return dict(A0=A0, Ad=Ad, R=R, nodes=nodes, cells=cells, stag=stag,
                node_shape=node_shape, cell_shape=cell_shape, h=h)


def solve(D, n, rho0, rho1, mask=None, omega_obstacle=1e-6, gap_tol=1e-13,
          max_newton=200, verbose=False) -> Dict:
    n = tuple(int(k) for k in n)
    h = [1.0 / k for k in n]
    vol = float(np.prod(h))
    sp_shape = tuple(k + 1 for k in n[1:])
    omega_sp = np.ones(sp_shape)
    if mask is not None:
        omega_sp = np.where(np.asarray(mask) != 0, omega_obstacle, 1.0)
    M = build_matrices(D, n, omega_sp)
    nodes = M["nodes"]
    # scaled boundary vector c~ (eq. defc divided by h0...hD)
    c = np.zeros(len(nodes))
    for p, i in nodes.items():
        if p[0] == 0:
            c[i] = rho0[p[1:]] / vol
        elif p[0] == n[0]:
            c[i] = -rho1[p[1:]] / vol
    nC = M["A0"].shape[0]
    nm = [a.shape[0] for a in M["Ad"]]
    Nm = sum(nm)
    # equality E [alpha0; m] = -c with E = [A0^T, A1^T, ...]; drop the last row
    E_full = np.hstack([M["A0"].T] + [a.T for a in M["Ad"]])
    E = E_full[:-1]
    e = -c[:-1]
    Rmat = np.vstack(M["R"])  # r = Rmat @ alpha0, stacked over d
    # strictly feasible start
    gamma = h[0] * float(np.sum(rho0)) / (vol * float(np.prod(sp_shape)))
    a0 = np.full(nC, gamma)
    Em = E[:, nC:]
    rhs = e - E[:, :nC] @ a0
    m, *_ = np.linalg.lstsq(Em, rhs, rcond=None)
    if np.linalg.norm(Em @ m - rhs) > 1e-9 * (1 + np.linalg.norm(rhs)):
        raise RuntimeError("no feasible start (unequal masses?)")
    r = Rmat @ a0
    s = (m * m + 1.0) / (2.0 * r)
    x = np.concatenate([a0, m, s])
    Efull = np.hstack([E, np.zeros((E.shape[0], Nm))])
    nvar = x.size
    nu = 2 * Nm + nC

    def split(xx):
        return xx[:nC], xx[nC:nC + Nm], xx[nC + Nm:]

    def feasible(xx):
        a, mm, ss = split(xx)
        rr = Rmat @ a
        return np.all(a > 0) and np.all(rr > 0) and np.all(ss > 0) and np.all(2 * rr * ss - mm * mm > 0)

    def fval(xx, t):
        a, mm, ss = split(xx)
        rr = Rmat @ a
        psi = 2 * rr * ss - mm * mm
        return t * ss.sum() - np.sum(np.log(psi)) - np.sum(np.log(a))

    def grad_hess(xx, t):
        a, mm, ss = split(xx)
        rr = Rmat @ a
        psi = 2 * rr * ss - mm * mm
        # derivatives of psi with respect to (r, m, s), per cone
        dr, dm, ds = 2 * ss, -2 * mm, 2 * rr
        ip = 1.0 / psi
        g_r = -ip * dr
        g_m = -ip * dm
        g_s = -ip * ds + t
        g_a = Rmat.T @ g_r - 1.0 / a
        grad = np.concatenate([g_a, g_m, g_s])
        # Hessian blocks: ip^2 * dpsi dpsi^T - ip * d2psi, d2psi: (r,s)=2, (m,m)=-2
        ip2 = ip * ip
        Hrr = ip2 * dr * dr
        Hrm = ip2 * dr * dm
        Hrs = ip2 * dr * ds - 2 * ip
        Hmm = ip2 * dm * dm + 2 * ip
        Hms = ip2 * dm * ds
        Hss = ip2 * ds * ds
        H = np.zeros((nvar, nvar))
        ia = slice(0, nC)
        im = slice(nC, nC + Nm)
        is_ = slice(nC + Nm, nvar)
        H[ia, ia] = Rmat.T @ (Hrr[:, None] * Rmat) + np.diag(1.0 / (a * a))
        H[ia, im] = Rmat.T * Hrm[None, :]
        H[ia, is_] = Rmat.T * Hrs[None, :]
        H[im, ia] = H[ia, im].T
        H[is_, ia] = H[ia, is_].T
        H[im, im] = np.diag(Hmm)
        H[im, is_] = np.diag(Hms)
        H[is_, im] = np.diag(Hms)
        H[is_, is_] = np.diag(Hss)
        return grad, H

    # feasible directions: orthonormal basis Z of the null space of the equality
    _, sv, Vt = np.linalg.svd(Efull)
    rank = int(np.sum(sv > sv[0] * 1e-12))
    Z = Vt[rank:].T
    t = 1.0
    total_newton = 0
    while True:
        for _ in range(max_newton):
            gr, H = grad_hess(x, t)
            gy = Z.T @ gr
            Hy = Z.T @ H @ Z
            dy = -np.linalg.solve(Hy, gy)
            dx = Z @ dy
            lam2 = float(-gy @ dy)
            total_newton += 1
            if lam2 / 2 <= 1e-12:
                break
            step = 1.0
            f0 = fval(x, t)
            accepted = False
            while step > 1e-14:
                xn = x + step * dx
                if feasible(xn) and fval(xn, t) <= f0 - 0.25 * step * lam2:
                    accepted = True
                    break
                step *= 0.5
            if not accepted:
                break
            x = xn
        if verbose:
            a, mm, ss = split(x)
            print(f"t={t:.1e} obj={vol * ss.sum():.12e} newton={total_newton}")
        if nu / t < gap_tol:
            break
        t *= 10.0
    a, mm, ss = split(x)
    rr = Rmat @ a
    obj = vol * float(np.sum(mm * mm / (2 * rr)))
    # reshape outputs onto the paper's grids
    rho = np.zeros(M["cell_shape"])
    for p, i in M["cells"].items():
        rho[p] = a[i]
    mom = []
    off = 0
    for d in range(1, D + 1):
        sh = list(M["node_shape"])
        sh[d] = n[d]
        arr = np.zeros(sh)
        for p, i in M["stag"][d - 1].items():
            arr[p] = mm[off + i]
        mom.append(arr)
        off += nm[d - 1]
    return dict(objective=obj, rho=rho, m=mom, newton=total_newton,
                eq_residual=float(np.linalg.norm(E_full @ np.concatenate([a, mm]) + c)))
