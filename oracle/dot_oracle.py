"""FP64 CPU oracle of the inexact proximal ALM for dynamic OT as a linear SOCP.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.

It follows Chen, Lin & Zhou, "An efficient SOCP approach for dynamic optimal
transport on staggered grid discretization" (arXiv 2505.05424) and is written
for a reader who has the paper beside it: plain numpy, exact array shapes,
no fusion, no blocking, one function per operator of the paper.

Array conventions (0-based, time axis first, last spatial axis fastest):
  nodes  G^c    : phi, b, c          shape (n0+1, n1+1, ..., nD+1)
  cells  G^s_0  : q0, alpha0, omega  shape (n0,   n1+1, ..., nD+1)
  G^s_d (d>=1)  : q_d, alpha_d       node shape with n_d (not n_d+1) on axis d
  cones         : z, beta            shape (K, n0, n1+1, ...), K = 4D+2
A cell (t, x) sits at time (t+1/2)h0 and spatial node x; q_d[t, s] sits at
time node t and at the staggered point s+1/2 on axis d.

Readings of points the paper leaves open (each is a parameter here):
  * data scaling: c~ = c/(h0 h1...hD), so alpha0 and alpha_bar come out as
    density and momentum density; objective = -(h0...hD) <c~, phi>.
  * sigma0 = 30 (the penalty acts on data scaled to density units), tau = 1.9,
    zero initial point; residuals checked every 5
    iterations (after iterations 5, 10, 15, ...); sigma reconsidered only at
    the checks listed by sigma_update_points (gaps 10, 15, 20, 25, 35, ...
    growing by about 1.2x), since changing sigma at every check stalls the
    method near 1e-5 on the 1D Gaussian pair.
  * discrete L2 norm ||x|| = sqrt(h0 h1...hD sum x_i^2) for every array.
  * obstacle weights omega live on cells and do not depend on time; the
    weighted residuals f, g and the dual objective carry omega the way the
    weighted constraint set P_omega (Sec. 5.4.5) carries it.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.fft as sfft

OMEGA_OBSTACLE = 1e-6  # weight on obstacle cells (Sec. 5.4.5, Ex-heart / Ex-maze)


# ---------------------------------------------------------------------------
# Grid (Sec. 2.2)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Grid:
    D: int
    n: tuple  # (n0, n1, ..., nD): segment counts

    @property
    def h(self):
        return tuple(1.0 / k for k in self.n)

    @property
    def vol(self):
        return float(np.prod(self.h))

    @property
    def K(self):
        return 4 * self.D + 2

    @property
    def node_shape(self):
        return tuple(k + 1 for k in self.n)

    @property
    def cell_shape(self):
        return (self.n[0],) + tuple(k + 1 for k in self.n[1:])

    def q_shape(self, d):
        s = list(self.node_shape)
        s[d] = self.n[d]
        return tuple(s)


def _sl(ndim, axis, s):
    idx = [slice(None)] * ndim
    idx[axis] = s
    return tuple(idx)


def _pad0(a, axis):
    """Zero extension by one entry at both ends of `axis`."""
    pad = [(0, 0)] * a.ndim
    pad[axis] = (1, 1)
    return np.pad(a, pad)


# ---------------------------------------------------------------------------
# Discrete gradient A (eq. Amap) and divergence A^*
# ---------------------------------------------------------------------------
def grad(phi, g: Grid):
    """(A_d phi)_i = (phi_{i+e_d/2} - phi_{i-e_d/2}) / h_d, i in G^s_d."""
    return [np.diff(phi, axis=d) / g.h[d] for d in range(g.D + 1)]


def grad_adj(y, g: Grid):
    """A^* y: at node j, sum_d (y_d[j - e_d/2] - y_d[j + e_d/2]) / h_d, zero outside G^s_d."""
    out = np.zeros(g.node_shape)
    for d in range(g.D + 1):
        yp = _pad0(y[d], d)
        nd = yp.ndim
        out += (yp[_sl(nd, d, slice(None, -1))] - yp[_sl(nd, d, slice(1, None))]) / g.h[d]
    return out


# ---------------------------------------------------------------------------
# Interpolations L_T, L_X^d and adjoints (eq. ltlx)
# ---------------------------------------------------------------------------
def avg(y, axis):
    nd = y.ndim
    return 0.5 * (y[_sl(nd, axis, slice(None, -1))] + y[_sl(nd, axis, slice(1, None))])


def avg_adj(a, axis):
    ap = _pad0(a, axis)
    nd = ap.ndim
    return 0.5 * (ap[_sl(nd, axis, slice(None, -1))] + ap[_sl(nd, axis, slice(1, None))])


def LT(y):
    return avg(y, 0)


def LT_adj(a):
    return avg_adj(a, 0)


def LX(y, d):
    return avg(y, d)


def LX_adj_sum(v, g: Grid):
    """L_X^* (v_1; ...; v_D) = sum_d (L_X^d)^* v_d."""
    return sum(avg_adj(v[d - 1], d) for d in range(1, g.D + 1))


# ---------------------------------------------------------------------------
# Decoupling operator F (eq. operatorF, fdetails)
# ---------------------------------------------------------------------------
def F_d(qd, d, g: Grid):
    """The four maps F^d_1..F^d_4 applied to q_d; each result lives on the cells.
    F^d_1: q_d at (t, x_d - 1/2)   (zero when x_d = 0)
    F^d_2: q_d at (t, x_d + 1/2)   (zero when x_d = n_d)
    F^d_3: q_d at (t+1, x_d - 1/2) (zero when x_d = 0)
    F^d_4: q_d at (t+1, x_d + 1/2) (zero when x_d = n_d)"""
    n0 = g.n[0]
    nd = len(g.cell_shape)
    lo_t = qd[:n0]
    hi_t = qd[1:]
    out = [np.zeros(g.cell_shape) for _ in range(4)]
    out[0][_sl(nd, d, slice(1, None))] = lo_t
    out[1][_sl(nd, d, slice(None, -1))] = lo_t
    out[2][_sl(nd, d, slice(1, None))] = hi_t
    out[3][_sl(nd, d, slice(None, -1))] = hi_t
    return out


def F_d_adj(parts, d, g: Grid):
    """sum_v (F^d_v)^* parts[v]: each cell value goes back to the q_d entry it was read from."""
    n0 = g.n[0]
    nd = len(g.cell_shape)
    qd = np.zeros(g.q_shape(d))
    qd[:n0] += parts[0][_sl(nd, d, slice(1, None))]
    qd[:n0] += parts[1][_sl(nd, d, slice(None, -1))]
    qd[1:] += parts[2][_sl(nd, d, slice(1, None))]
    qd[1:] += parts[3][_sl(nd, d, slice(None, -1))]
    return qd


# ---------------------------------------------------------------------------
# SOC embedding B (eq. bdd), offset d, weighted by omega (Sec. 5.4.5)
# ---------------------------------------------------------------------------
def BF(q, omega_cells, g: Grid):
    """B_omega F q as K cone components per cell:
    [ -q0, sqrt(omega/2) F^1_1 q1, ..., sqrt(omega/2) F^D_4 qD, q0 ]."""
    s = np.sqrt(omega_cells / 2.0)
    comps = [-q[0]]
    for d in range(1, g.D + 1):
        for part in F_d(q[d], d, g):
            comps.append(s * part)
    comps.append(q[0].copy())
    return np.stack(comps)


def cone_offset(g: Grid):
    """d = (1; 0; ...; 0; 1) on every cell."""
    dv = np.zeros((g.K,) + g.cell_shape)
    dv[0] = 1.0
    dv[-1] = 1.0
    return dv


def FtBt(u, omega_cells, g: Grid):
    """F^* B_omega^* u (eq. operFB): q0 <- u_{K-1} - u_0,
    q_d <- sqrt(omega/2) * sum_v (F^d_v)^* u_{d,v}."""
    s = np.sqrt(omega_cells / 2.0)
    out = [u[-1] - u[0]]
    for d in range(1, g.D + 1):
        base = 1 + 4 * (d - 1)
        out.append(F_d_adj([s * u[base + v] for v in range(4)], d, g))
    return out


def q_diag(omega_cells, g: Grid):
    """Diagonal of I + F^* B_omega^* B_omega F (Prop. 3.2 with weights):
    3 on q0; on q_d at (t, s): 1 + 1/2 * sum of omega over the cells adjacent
    to that point (cells (t-1,.) exist for t >= 1, cells (t,.) for t < n0; on
    axis d the adjacent spatial nodes are s and s+1). With omega = 1 this is
    2 at t = 0 and t = n0 and 3 in between."""
    out = [np.full(g.cell_shape, 3.0)]
    n0 = g.n[0]
    om = omega_cells[0]  # time-invariant weights
    for d in range(1, g.D + 1):
        ax = d - 1  # axis of `om` (spatial only)
        pair = avg(om, ax) * 2.0  # omega[s] + omega[s+1]
        shp = g.q_shape(d)
        count = np.full(n0 + 1, 2.0)
        count[0] = 1.0
        count[n0] = 1.0
        dd = 1.0 + 0.5 * count.reshape((n0 + 1,) + (1,) * g.D) * pair[None]
        out.append(np.broadcast_to(dd, shp).copy())
    return out


# ---------------------------------------------------------------------------
# Projection onto the second-order cone (eq. app-proj), per cell
# ---------------------------------------------------------------------------
def proj_soc(y):
    """y has shape (K, ...): y[0] is the scalar part, y[1:] the vector part."""
    y0 = y[0]
    yb = y[1:]
    nrm = np.sqrt(np.sum(yb * yb, axis=0))
    out = np.zeros_like(y)
    inside = nrm <= y0
    polar = (~inside) & (nrm <= -y0)
    other = ~(inside | polar)
    out[:, inside] = y[:, inside]
    a = 0.5 * (y0[other] + nrm[other])
    out[0, other] = a
    out[1:, other] = a * yb[:, other] / nrm[other]
    return out


# ---------------------------------------------------------------------------
# Poisson solve A^*A phi = b on rge(A^*) by cosine transforms (Sec. 4, Alg. 2)
# ---------------------------------------------------------------------------
def laplacian_eigs(g: Grid):
    """Eigenvalues of A^*A: sum_d (4/h_d^2) sin^2(pi k_d / (2 (n_d+1))); the
    eigenvectors are the tensor products of orthonormal DCT-II basis vectors."""
    lam = np.zeros(g.node_shape)
    for d in range(g.D + 1):
        N = g.n[d] + 1
        k = np.arange(N)
        ld = 4.0 / g.h[d] ** 2 * np.sin(np.pi * k / (2.0 * N)) ** 2
        shape = [1] * (g.D + 1)
        shape[d] = N
        lam = lam + ld.reshape(shape)
    return lam


def poisson(b, g: Grid, lam=None):
    """The unique solution in rge(A^*) (mean zero) of A^*A phi = b - mean(b)."""
    if lam is None:
        lam = laplacian_eigs(g)
    bh = sfft.dctn(b, type=2, norm="ortho")
    ph = np.zeros_like(bh)
    nz = lam > 0
    ph[nz] = bh[nz] / lam[nz]
    return sfft.idctn(ph, type=2, norm="ortho")


# ---------------------------------------------------------------------------
# Problem data (eq. defc) with the density scaling
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    g: Grid
    c: np.ndarray            # scaled boundary vector c~ = c / (h0...hD) on nodes
    omega: np.ndarray        # cell weights, shape g.cell_shape
    diag: List[np.ndarray]
    lam: np.ndarray


def make_problem(D, n, rho0, rho1, mask=None, omega_obstacle=OMEGA_OBSTACLE) -> Problem:
    """c_i = rho0 mass at t = 0, -rho1 mass at t = n0, 0 elsewhere (eq. defc),
    divided by h0...hD. Obstacle nodes carry weight omega_obstacle."""
    g = Grid(D, tuple(int(k) for k in n))
    rho0 = np.asarray(rho0, dtype=np.float64)
    rho1 = np.asarray(rho1, dtype=np.float64)
    assert rho0.shape == g.node_shape[1:] and rho1.shape == g.node_shape[1:]
    c = np.zeros(g.node_shape)
    c[0] = rho0
    c[-1] = -rho1
    c /= g.vol
    om_sp = np.ones(g.node_shape[1:])
    if mask is not None:
        om_sp = np.where(np.asarray(mask) != 0, omega_obstacle, 1.0)
    omega = np.broadcast_to(om_sp[None], g.cell_shape).copy()
    return Problem(g, c, omega, q_diag(omega, g), laplacian_eigs(g))


# ---------------------------------------------------------------------------
# Residuals (Sec. 5.3) and objectives
# ---------------------------------------------------------------------------
def l2(arrs, g: Grid):
    if isinstance(arrs, np.ndarray):
        arrs = [arrs]
    return math.sqrt(g.vol * sum(float(np.sum(a * a)) for a in arrs))


def f_of_q(q, omega, g: Grid):
    """f(q) = q0 + 1/2 omega . L_T L_X^*(|q_1|^2; ...; |q_D|^2)."""
    return q[0] + 0.5 * omega * LT(LX_adj_sum([q[d] ** 2 for d in range(1, g.D + 1)], g))


def g_of(alpha0, q, omega, g: Grid):
    """g_d = (L_X^d L_T^*(omega . alpha0)) . q_d, d = 1..D."""
    r = LT_adj(omega * alpha0)
    return [LX(r, d) * q[d] for d in range(1, g.D + 1)]


def interp_density(alpha0, omega, g: Grid):
    """r_d = L_X^d L_T^*(omega . alpha0) on G^s_d, d = 1..D."""
    r = LT_adj(omega * alpha0)
    return [LX(r, d) for d in range(1, g.D + 1)]


def residuals(P: Problem, phi, z, q, alpha, beta) -> Dict[str, float]:
    g = P.g
    Aphi = grad(phi, g)
    eta_p = l2([a - b for a, b in zip(Aphi, q)], g) / (1 + l2(Aphi, g) + l2(q, g))
    dres = grad_adj(alpha, g) + P.c
    eta_d = l2(dres, g) / (1 + l2(P.c, g))
    fq = f_of_q(q, P.omega, g)
    a0 = alpha[0]
    c1 = l2(a0 - np.maximum(0.0, fq + a0), g) / (1 + l2(a0, g) + l2(fq, g))
    gq = g_of(a0, q, P.omega, g)
    abar = alpha[1:]
    c2 = l2([a - b for a, b in zip(abar, gq)], g) / (1 + l2(abar, g) + l2(gq, g))
    eta_c = max(c1, c2)
    dv = cone_offset(g)
    bfq = BF(q, P.omega, g)
    p2 = l2(z - bfq - dv, g) / (1 + l2(dv, g))
    ftb = FtBt(beta, P.omega, g)
    d2 = l2([a + b for a, b in zip(ftb, alpha)], g) / (1 + l2(ftb, g) + l2(alpha, g))
    return dict(eta_p=eta_p, eta_d=eta_d, eta_c=eta_c, eta_c1=c1, eta_c2=c2,
                eta_dot=max(eta_p, eta_d, eta_c),
                eta_p_soc=max(eta_p, p2), eta_d_soc=max(eta_d, d2))


def objective(P: Problem, phi) -> float:
    """-<c, phi> in the unscaled units (approximately W2^2 / 2)."""
    return -P.g.vol * float(np.sum(P.c * phi))


def dual_objective(P: Problem, alpha) -> float:
    """1/2 sum_d sum_{r_d > 0} alpha_d^2 / r_d, r_d = L_X^d L_T^*(omega alpha0), unscaled."""
    g = P.g
    rs = interp_density(alpha[0], P.omega, g)
    tot = 0.0
    for d in range(1, g.D + 1):
        r = rs[d - 1]
        m = alpha[d]
        pos = r > 0
        tot += 0.5 * float(np.sum(m[pos] ** 2 / r[pos]))
    return g.vol * tot


# ---------------------------------------------------------------------------
# Algorithm 2 (explicit steps of Algorithm 1)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class State:
    phi: np.ndarray
    z: np.ndarray
    q: List[np.ndarray]
    alpha: List[np.ndarray]
    beta: np.ndarray
    sigma: float
    k: int = 0  # iterations done


def zero_state(P: Problem, sigma0=30.0) -> State:
    g = P.g
    q = [np.zeros(g.cell_shape)] + [np.zeros(g.q_shape(d)) for d in range(1, g.D + 1)]
    alpha = [np.zeros_like(a) for a in q]
    return State(np.zeros(g.node_shape), np.zeros((g.K,) + g.cell_shape), q, alpha,
                 np.zeros((g.K,) + g.cell_shape), float(sigma0))


def step_rhs(P: Problem, q, alpha, sigma):
    """b = A^*(q - alpha/sigma) - c/sigma."""
    return grad_adj([a - b / sigma for a, b in zip(q, alpha)], P.g) - P.c / sigma


def step_cone_input(P: Problem, q, beta, sigma):
    """B F q + d - beta/sigma (argument of the projection)."""
    return BF(q, P.omega, P.g) + cone_offset(P.g) - beta / sigma


def step_q(P: Problem, phi, z, alpha, beta, sigma):
    """q = (I + F^*B^*BF)^{-1} (A phi + alpha/sigma + F^*B^*(z - d + beta/sigma))."""
    g = P.g
    Aphi = grad(phi, g)
    w = z - cone_offset(g) + beta / sigma
    back = FtBt(w, P.omega, g)
    return [(a + al / sigma + bk) / dg for a, al, bk, dg in zip(Aphi, alpha, back, P.diag)]


def iterate(P: Problem, S: State, tau=1.9) -> State:
    """One pass of Algorithm 2."""
    g = P.g
    sigma = S.sigma
    b = step_rhs(P, S.q, S.alpha, sigma)
    phi = poisson(b, g, P.lam)
    z = proj_soc(step_cone_input(P, S.q, S.beta, sigma))
    qn = step_q(P, phi, z, S.alpha, S.beta, sigma)
    Aphi = grad(phi, g)
    alpha = [a + tau * sigma * (ap - qq) for a, ap, qq in zip(S.alpha, Aphi, qn)]
    beta = S.beta + tau * sigma * (z - BF(qn, P.omega, g) - cone_offset(g))
    return State(phi, z, qn, alpha, beta, sigma, S.k + 1)


def sigma_update_points(limit, first_gap=10, growth=1.2, cadence=5):
    """Iteration counts (1-based, multiples of `cadence`) at which the sigma
    rule is applied: k_1 = first_gap, k_{j+1} = k_j + g_{j+1} with
    g_{j+1} = cadence * floor((floor(growth * g_j) + cadence) / cadence)."""
    pts = []
    k = 0
    gap = first_gap
    while k + gap <= limit:
        k += gap
        pts.append(k)
        nxt = int(math.floor(growth * gap)) + cadence
        gap = nxt - nxt % cadence
    return pts


def sigma_rule(sigma, eta_p_soc, eta_d_soc, s_sigma=1.25, s_r=2.0):
    """Sec. 5.3: multiply sigma by s_sigma when eta_P^soc / eta_D^soc > s_r,
    divide when below 1/s_r. Returns (new sigma, decision in {-1, 0, 1})."""
    ratio = eta_p_soc / eta_d_soc if eta_d_soc > 0 else math.inf
    if ratio > s_r:
        return sigma * s_sigma, 1
    if ratio < 1.0 / s_r:
        return sigma / s_sigma, -1
    return sigma, 0


@dataclasses.dataclass
class SolveResult:
    state: State
    iters: int
    converged: bool
    res: Dict[str, float]
    objective: float
    dual_objective: float
    history: List[Dict]
    seconds: float


def solve(P: Problem, tol=1e-6, max_iter=10000, tau=1.9, sigma0=30.0, check_every=5,
          adapt_sigma=True, state: Optional[State] = None, on_check=None,
          sigma_gap0=10, sigma_growth=1.2) -> SolveResult:
    """Run Algorithm 2 from zero (or `state`), checking eta_dot and adapting
    sigma every `check_every` iterations; stop at eta_dot <= tol."""
    S = state if state is not None else zero_state(P, sigma0)
    upd = set(sigma_update_points(S.k + max_iter + 1, sigma_gap0, sigma_growth, check_every))
    hist = []
    res = {}
    conv = False
    t0 = time.perf_counter()
    start = S.k
    while S.k - start < max_iter:
        S = iterate(P, S, tau)
        if S.k % check_every == 0:
            res = residuals(P, S.phi, S.z, S.q, S.alpha, S.beta)
            rec = dict(k=S.k, sigma=S.sigma, **res)
            if res["eta_dot"] <= tol:
                rec["decision"] = 0
                hist.append(rec)
                conv = True
                break
            if adapt_sigma and S.k in upd:
                S.sigma, dec = sigma_rule(S.sigma, res["eta_p_soc"], res["eta_d_soc"])
            else:
                dec = 0
            rec["decision"] = dec
            hist.append(rec)
            if on_check is not None:
                on_check(rec)
    if not res:
        res = residuals(P, S.phi, S.z, S.q, S.alpha, S.beta)
    secs = time.perf_counter() - t0
    return SolveResult(S, S.k - start, conv, res, objective(P, S.phi),
                       dual_objective(P, S.alpha), hist, secs)


def run_fixed(P: Problem, iters, tau=1.9, sigma0=30.0, check_every=5, adapt_sigma=True,
              sigma_gap0=10, sigma_growth=1.2) -> SolveResult:
    """Exactly `iters` iterations with the same check/sigma schedule and no stop."""
    return solve(P, tol=-1.0, max_iter=iters, tau=tau, sigma0=sigma0, check_every=check_every,
                 adapt_sigma=adapt_sigma, sigma_gap0=sigma_gap0, sigma_growth=sigma_growth)


def duality_gap(p, d):
    return abs(p - d) / (1.0 + abs(p) + abs(d))
