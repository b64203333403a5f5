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
    """Compulsory bytes per launch of each kernel class."""
    z = sizes(D, n)
    Nc, S, Q, Qb, K = z["Nc"], z["S"], z["Q"], z["Qbar"], z["K"]
    return {
        # divergence of (q, alpha) fused into the time-axis forward pass
        "dct_first": w * (2 * Q + Nc),
        "dct_mid": w * 2 * Nc,
        "dct_last": w * 2 * Nc,
        "dct_inv": w * 2 * Nc,
        # cone: read q, beta, phi, alpha0; write q0_new, alpha0, 4D weighted w planes
        "cone": w * (Q + K * S + Nc + S + 2 * S + 4 * D * S),
        # q_d: read phi, alpha_d, w planes; write q_d, alpha_d
        "qd": w * (Nc + Qb + 4 * D * S + 2 * Qb),
        # beta: read q_old, q_new, beta; write beta
        "beta": w * (2 * Q + 2 * K * S),
        # residual partials: read phi, q, alpha, beta
        "resid": w * (Nc + 2 * Q + K * S),
        "final": 0.0,
    }


def iteration_min_bytes(D: int, n: Sequence[int], w: int) -> float:
    """Fused lower bound per PALM iteration: read phi, q, alpha, beta and write
    q, alpha, beta, b once, plus one read of b and one write of phi in the
    Poisson solve."""
    z = sizes(D, n)
    return w * (4 * z["Nc"] + 4 * z["Q"] + 2 * z["K"] * z["S"])


def launches_per_iteration(D: int) -> Dict[str, int]:
    return {"dct_first": 1, "dct_mid": max(D - 1, 0), "dct_last": 1, "dct_inv": D,
            "cone": 1, "qd": 1, "beta": 1}
