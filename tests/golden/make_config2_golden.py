"""Writes config2_converged.json: the FP64 oracle's converged solve of the
2D 32x64^2 Gaussian-mixture instance (seed 2000) at eta_dot <= 1e-6 with the
default settings (tau 1.9, sigma0 30, checks every 5 iterations, sigma rule on
the growing schedule), as the reference of the headline GPU solve.

Calls only oracle/ and the seeded input generator dotgen/. Stored: the
scalars of the result, and rho / m at 4096 seeded positions each (the full
arrays would be several MB); the comparison of the GPU solve reads the same
positions from its own rho / m.

  python tests/golden/make_config2_golden.py     (about 5 minutes on one core)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import dotgen  # noqa: E402
from oracle import dot_oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_converged.json")
SAMPLE_SEED = 20250505
NSAMPLE = 4096


def main():
    inst = dotgen.config2_instance()
    P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
    t0 = time.perf_counter()
    r = O.solve(P, tol=1e-6, max_iter=100000)
    secs = time.perf_counter() - t0
    rho = r.state.alpha[0]
    m = np.concatenate([a.ravel() for a in r.state.alpha[1:]])
    rng = np.random.default_rng(SAMPLE_SEED)
    i_rho = np.sort(rng.choice(rho.size, NSAMPLE, replace=False))
    i_m = np.sort(rng.choice(m.size, NSAMPLE, replace=False))
    rec = {
        "instance": inst.label, "D": inst.D, "n": list(inst.n), "seed": 2000,
        "settings": {"tol": 1e-6, "tau": 1.9, "sigma0": 30.0, "check_every": 5,
                     "sigma_gap0": 10, "sigma_growth": 1.2, "adapt_sigma": True},
        "converged": bool(r.converged), "iters": int(r.iters),
        "checks": len(r.history),
        "sigma_final": r.state.sigma,
        "sigma_changes": int(sum(1 for h in r.history if h["decision"] != 0)),
        "objective": r.objective, "dual_objective": r.dual_objective,
        "residuals": {k: float(v) for k, v in r.res.items()},
        "rho_max_abs": float(np.max(np.abs(rho))), "m_max_abs": float(np.max(np.abs(m))),
        "rho_sum_per_slice_times_hx": [float(s) for s in rho.reshape(rho.shape[0], -1).sum(1) * P.g.vol / P.g.h[0]],
        "sample_seed": SAMPLE_SEED,
        "rho_index": i_rho.tolist(), "rho_value": rho.ravel()[i_rho].tolist(),
        "m_index": i_m.tolist(), "m_value": m[i_m].tolist(),
        "oracle_seconds": secs,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=0)
    print(f"{OUT}: {r.iters} iterations, objective {r.objective:.12f}, {secs:.0f} s")


if __name__ == "__main__":
    main()
