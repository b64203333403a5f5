"""Algorithmic byte counts of the solver's kernels (exact array shapes, each
input element read once and each output element written once), used for
roofline fractions. `w` is the bytes per scalar of the bulk state."""
from __future__ import annotations

import math
from typing import Dict, Sequence

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def sizes(D: int, n: Sequence[int]) -> Dict[str, int]:
    n = [int(k) for k in n[:D + 1]]
    N = [k + 1 for k in n]
    Nc = math.prod(N)
    nx = Nc // N[0]
    S = n[0] * nx
    Qd = [Nc // N[d] * n[d] for d in range(1, D + 1)]
    return dict(Nc=Nc, S=S, nx=nx, Qbar=sum(Qd), Q=S + sum(Qd), K=4 * D + 2, D=D)


def kernel_bytes(D: int, n: Sequence[int], w: int) -> Dict[str, float]:
    """Compulsory bytes per launch of each kernel class; w is the bulk scalar
    size (8 FP64, 4 mixed); phi and alpha are always FP64 (8 bytes)."""
    z = sizes(D, n)
    Nc, S, Q, Qb, K = z["Nc"], z["S"], z["Q"], z["Qbar"], z["K"]
    mixed = w != 8
    a = 8  # alpha
    last_inv = (w + 16) * Nc if mixed else 2 * w * Nc  # time-axis inverse adds into phi (mixed)
    rhs = w * Q + a * Q + w * Nc + (8 * Nc if mixed else 0)
    beta = w * (2 * Q + 2 * K * S)
    beta_cone = w * (2 * Q + 2 * K * S + 4 * D * S) + 8 * S
    cone = w * (Q + K * S + 4 * D * S) + 8 * S
    return {
        # b (FP64) or b - A^*A phi (mixed): read q, alpha (and phi); write the work plane
        "rhs": rhs,
        "dct_first": 2 * w * Nc,
        "dct_mid": 2 * w * Nc,
        "dct_last": 2 * w * Nc,
        # D launches: D-1 plain inverse passes and the time-axis one
        "dct_inv": ((D - 1) * 2 * w * Nc + last_inv) / D,
        # cone (z-step): read q, beta; write 4D weighted w planes and w_{K-1} - w_0 (FP64)
        "cone": cone,
        # the z-step and the right-hand side of one iteration in one launch (q counted once)
        "cone_rhs": cone + rhs - w * Q,
        # q-step: read phi, alpha, the 4D w planes and w_{K-1} - w_0; write q, alpha
        "qd": w * (Q + 4 * D * S) + 8 * S + 2 * a * Q + 8 * Nc,
        # beta: read q_old, q_new, beta; write beta
        "beta": beta,
        # beta update and the next z-step in one sweep: read q_old, q_new, beta;
        # write beta, the 4D w planes and w_{K-1} - w_0
        "beta_cone": beta_cone,
        # the fused launches with the next right-hand side (q_new counted once)
        "beta_rhs": beta + rhs - w * Q,
        "beta_cone_rhs": beta_cone + rhs - w * Q,
        # residual partials: read phi, q, alpha, beta
        "resid": w * (Q + K * S) + a * Q + 8 * Nc,
        "final": 0.0,
    }


def iteration_min_bytes(D: int, n: Sequence[int], w: int) -> float:
    """Fused lower bound per PALM iteration: read phi, q, alpha, beta and write
    q, alpha, beta, b once, plus one read of b and one write of phi in the
    Poisson solve (phi, b and alpha in FP64)."""
    z = sizes(D, n)
    return 8 * 4 * z["Nc"] + (2 * w + 16) * z["Q"] + w * 2 * z["K"] * z["S"]


def launches_per_iteration(D: int) -> Dict[str, int]:
    return {"rhs": 1, "dct_first": 1, "dct_mid": max(D - 1, 0), "dct_last": 1, "dct_inv": D,
            "cone": 1, "qd": 1, "beta": 1}
