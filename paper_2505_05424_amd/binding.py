"""ctypes binding of libdotsocp (include/dotsocp.h), one Python function per C
entry point with the same name. Only argument marshalling happens here:
every step of the solver runs in the library's HIP kernels. Device buffers
are passed as raw pointers (for instance torch.Tensor.data_ptr() of a CUDA
tensor) and streams as the integer handle of a hipStream_t (0 = default).

Loading fails loudly if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libdotsocp.so")

DOT_FP64 = 0
DOT_MIXED = 1
TERM_NAMES = {-1: "running", 0: "converged", 1: "maxiter", 2: "timeout", 3: "diverged"}

EXPORTED = [
    "dot_last_error", "dot_plan_create", "dot_plan_destroy", "dot_plan_get_info",
    "dot_state_reset", "dot_run", "dot_extract",
    "dot_step_divergence", "dot_step_poisson", "dot_step_rhs_poisson", "dot_step_cone",
    "dot_step_update", "dot_step_residuals", "dot_profile_select", "dot_profile_read", "dot_solve",
    "dot_batch_create", "dot_batch_destroy", "dot_batch_workspace_bytes", "dot_batch_size",
    "dot_batch_laid_out", "dot_batch_reset",
    "dot_batch_run", "dot_batch_extract", "dot_batch_profile_select", "dot_batch_profile_read",
    "dot_plan_set_graphs", "dot_batch_set_graphs",
    "dot_plan_set_schedule", "dot_batch_set_schedule", "dot_plan_get_schedule", "dot_batch_get_schedule",
    "dot_plan_autotune", "dot_batch_autotune", "dot_state_promote", "dot_state_export", "dot_state_import",
    "dot_sigma_history", "dot_batch_sigma_history",
    "dot_footprint_bytes", "dot_ctx_create", "dot_ctx_destroy", "dot_ctx_submit", "dot_ctx_submit_ml", "dot_ctx_step", "dot_ctx_poll",
    "dot_ctx_fetch", "dot_ctx_stats", "dot_coarsen_data", "dot_prolong", "dot_solve_multilevel",
    "dot_step_residuals_noalloc", "dot_ctx_export", "dot_ctx_import", "dot_ctx_last_error", "dot_batch_promote",
    "dot_ctx_keep_capped", "dot_batch_promote_member", "dot_test_fail_captures",
]
NOALLOC_SCRATCH_BYTES = 8 << 20

CTX_QUEUED, CTX_RUNNING, CTX_DONE = 0, 1, 2

KERNEL_CLASSES = {"rhs": 9, "dct_first": 0, "dct_mid": 1, "dct_last": 2, "dct_inv": 3, "cone": 4, "qd": 5,
                  "beta": 6, "resid": 7, "final": 8}


class dot_problem(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32),
        ("n", ctypes.c_int32 * 4),
        ("rho0", ctypes.POINTER(ctypes.c_double)),
        ("rho1", ctypes.POINTER(ctypes.c_double)),
        ("mask", ctypes.POINTER(ctypes.c_uint8)),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("sigma0", ctypes.c_double),
        ("check_every", ctypes.c_int32),
        ("adapt_sigma", ctypes.c_int32),
        ("sigma_gap0", ctypes.c_int32),
        ("sigma_growth", ctypes.c_double),
        ("time_limit_s", ctypes.c_double),
    ]


class dot_result(ctypes.Structure):
    _fields_ = [
        ("objective", ctypes.c_double),
        ("dual_objective", ctypes.c_double),
        ("eta_dot", ctypes.c_double),
        ("eta_p", ctypes.c_double),
        ("eta_d", ctypes.c_double),
        ("eta_c", ctypes.c_double),
        ("eta_p_soc", ctypes.c_double),
        ("eta_d_soc", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("iters", ctypes.c_int32),
        ("term", ctypes.c_int32),
        ("checks", ctypes.c_int32),
        ("sigma_changes", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dot_plan_info(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("n", ctypes.c_int32 * 4),
        ("nb", ctypes.c_int64),
        ("scalar_bytes", ctypes.c_int32),
        ("n_planes", ctypes.c_int32),
        ("state_bytes", ctypes.c_size_t),
        ("off_phi", ctypes.c_uint64),
        ("off_scratch", ctypes.c_uint64),
        ("off_q", ctypes.c_uint64),
        ("off_qn", ctypes.c_uint64),
        ("off_alpha", ctypes.c_uint64),
        ("off_beta", ctypes.c_uint64),
        ("off_w", ctypes.c_uint64),
    ]


class dot_schedule(ctypes.Structure):
    _fields_ = [
        ("cw", ctypes.c_int32 * 4),
        ("waves", ctypes.c_int32 * 4),
        ("tuned", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("us", ctypes.c_double),
        ("us_rule", ctypes.c_double),
    ]


_lib = None


def load(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libdotsocp.so (built by paper_2505_05424_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libdotsocp.so not built at {p}; run python -m paper_2505_05424_amd.build")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Loading torch first makes the dynamic linker bind this library to that
    # runtime, so torch's device pointers and streams are valid here; loading
    # a second runtime into the process would leave torch without a device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.dot_last_error.restype = ctypes.c_char_p
    lib.dot_plan_create.argtypes = [ctypes.POINTER(dot_problem), ctypes.POINTER(vp)]
    lib.dot_plan_destroy.argtypes = [vp]
    lib.dot_plan_destroy.restype = None
    lib.dot_plan_get_info.argtypes = [vp, ctypes.POINTER(dot_plan_info)]
    lib.dot_state_reset.argtypes = [vp, vp, vp]
    lib.dot_run.argtypes = [vp, vp, i32, vp, ctypes.POINTER(dot_result)]
    lib.dot_extract.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), vp]
    lib.dot_step_divergence.argtypes = [vp, vp, vp, dbl, vp, vp]
    lib.dot_step_poisson.argtypes = [vp, vp, vp]
    lib.dot_step_rhs_poisson.argtypes = [vp, vp, vp, dbl, vp, vp]
    lib.dot_step_cone.argtypes = [vp, vp, vp, dbl, vp, vp]
    lib.dot_step_update.argtypes = [vp, vp, vp, vp, vp, dbl, dbl, vp, vp, vp]
    lib.dot_step_residuals.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(dot_result), vp]
    lib.dot_step_residuals_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(dot_result), vp]
    lib.dot_profile_select.argtypes = [vp, i32]
    lib.dot_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.dot_solve.argtypes = [ctypes.POINTER(dot_problem), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(dot_result)]
    lib.dot_batch_create.argtypes = [ctypes.POINTER(dot_problem), i32, ctypes.POINTER(vp)]
    lib.dot_batch_destroy.argtypes = [vp]
    lib.dot_batch_destroy.restype = None
    lib.dot_batch_workspace_bytes.argtypes = [vp]
    lib.dot_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.dot_batch_size.argtypes = [vp]
    lib.dot_batch_size.restype = i32
    lib.dot_batch_laid_out.argtypes = [vp]
    lib.dot_batch_laid_out.restype = i32
    lib.dot_batch_reset.argtypes = [vp, vp, vp]
    lib.dot_batch_run.argtypes = [vp, vp, i32, vp, ctypes.POINTER(dot_result)]
    lib.dot_batch_extract.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), vp]
    lib.dot_plan_set_graphs.argtypes = [vp, i32]
    lib.dot_batch_set_graphs.argtypes = [vp, i32]
    lib.dot_test_fail_captures.argtypes = [i32]
    for fn in ("dot_plan_set_schedule", "dot_batch_set_schedule", "dot_plan_get_schedule",
               "dot_batch_get_schedule"):
        getattr(lib, fn).argtypes = [vp, ctypes.POINTER(dot_schedule)]
    lib.dot_plan_autotune.argtypes = [vp, vp, vp, ctypes.POINTER(dot_schedule)]
    lib.dot_batch_autotune.argtypes = [vp, vp, vp, ctypes.POINTER(dot_schedule)]
    lib.dot_batch_profile_select.argtypes = [vp, i32]
    lib.dot_batch_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.dot_footprint_bytes.argtypes = [ctypes.POINTER(dot_problem)]
    lib.dot_footprint_bytes.restype = ctypes.c_size_t
    lib.dot_ctx_create.argtypes = [i32, i32, i32, ctypes.c_size_t, i32, ctypes.POINTER(vp)]
    lib.dot_ctx_export.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t), vp]
    lib.dot_ctx_import.argtypes = [vp, ctypes.POINTER(dot_problem), i32, vp, ctypes.c_size_t,
                                   ctypes.POINTER(ctypes.c_uint64)]
    lib.dot_ctx_last_error.argtypes = [vp]
    lib.dot_ctx_keep_capped.argtypes = [vp, i32]
    lib.dot_ctx_last_error.restype = ctypes.c_char_p
    lib.dot_ctx_destroy.argtypes = [vp]
    lib.dot_ctx_destroy.restype = None
    lib.dot_ctx_submit.argtypes = [vp, ctypes.POINTER(dot_problem), ctypes.POINTER(ctypes.c_uint64)]
    lib.dot_ctx_submit_ml.argtypes = [vp, ctypes.POINTER(dot_problem), i32, ctypes.POINTER(ctypes.c_uint64)]
    lib.dot_ctx_step.argtypes = [vp, i32, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.dot_ctx_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32)]
    lib.dot_ctx_fetch.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(dot_result)]
    lib.dot_ctx_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64)]
    lib.dot_coarsen_data.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint8),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_uint8)]
    lib.dot_prolong.argtypes = [vp, vp, vp, vp, vp]
    lib.dot_state_promote.argtypes = [vp, vp, vp, vp, vp]
    lib.dot_batch_promote.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.dot_batch_promote_member.argtypes = [vp, vp, i32, vp, vp, i32, vp]
    pd = ctypes.POINTER(ctypes.c_double)
    lib.dot_state_export.argtypes = [vp, vp, pd, pd, pd, pd, vp]
    lib.dot_state_import.argtypes = [vp, vp, pd, pd, pd, dbl, vp]
    pi = ctypes.POINTER(ctypes.c_int32)
    lib.dot_sigma_history.argtypes = [vp, vp, pd, pi, i32, pi, vp]
    lib.dot_batch_sigma_history.argtypes = [vp, vp, i32, pd, pi, i32, pi, vp]
    lib.dot_solve_multilevel.argtypes = [ctypes.POINTER(dot_problem), i32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(dot_result),
                                         ctypes.POINTER(dot_result)]
    for name in EXPORTED:
        if name not in ("dot_last_error", "dot_plan_destroy", "dot_batch_destroy", "dot_batch_workspace_bytes",
                        "dot_batch_size", "dot_batch_laid_out", "dot_footprint_bytes", "dot_ctx_destroy",
                        "dot_ctx_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class DotError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        msg = load().dot_last_error().decode(errors="replace")
        raise DotError(f"dotsocp error {rc}: {msg}")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_problem(D: int, n: Sequence[int], rho0, rho1, mask=None, tol=1e-6, max_iter=10000,
                 precision=DOT_FP64, tau=0.0, sigma0=0.0, check_every=0, adapt_sigma=1,
                 sigma_gap0=0, sigma_growth=0.0, time_limit_s=0.0):
    """Fill a dot_problem; returns (struct, keepalive) — keep both alive while in use."""
    r0 = np.ascontiguousarray(rho0, dtype=np.float64).ravel()
    r1 = np.ascontiguousarray(rho1, dtype=np.float64).ravel()
    keep = [r0, r1]
    p = dot_problem()
    p.D = D
    for i in range(4):
        p.n[i] = int(n[i]) if i <= D else 0
    p.rho0 = _dptr(r0)
    p.rho1 = _dptr(r1)
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
        keep.append(mk)
        p.mask = mk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    p.tol = tol
    p.max_iter = max_iter
    p.precision = precision
    p.tau = tau
    p.sigma0 = sigma0
    p.check_every = check_every
    p.adapt_sigma = adapt_sigma
    p.sigma_gap0 = sigma_gap0
    p.sigma_growth = sigma_growth
    p.time_limit_s = time_limit_s
    return p, keep


class Plan:
    """Owns a dot_plan handle; `info` describes the state-buffer layout."""

    def __init__(self, handle, info: dot_plan_info, D: int, n):
        self.handle = handle
        self.info = info
        self.D = D
        self.n = tuple(int(k) for k in n[:D + 1])

    def close(self):
        if self.handle:
            load().dot_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dot_plan_create(D, n, rho0, rho1, mask=None, **kw) -> Plan:
    lib = load()
    p, keep = make_problem(D, n, rho0, rho1, mask, **kw)
    h = ctypes.c_void_p()
    _check(lib.dot_plan_create(ctypes.byref(p), ctypes.byref(h)))
    info = dot_plan_info()
    _check(lib.dot_plan_get_info(h, ctypes.byref(info)))
    return Plan(h, info, D, n)


def dot_plan_destroy(plan: Plan):
    plan.close()


def dot_state_reset(plan: Plan, state_ptr: int, stream: int = 0):
    _check(load().dot_state_reset(plan.handle, ctypes.c_void_p(state_ptr), ctypes.c_void_p(stream)))


def dot_run(plan: Plan, state_ptr: int, max_iters: int, stream: int = 0) -> dot_result:
    r = dot_result()
    _check(load().dot_run(plan.handle, ctypes.c_void_p(state_ptr), int(max_iters), ctypes.c_void_p(stream),
                          ctypes.byref(r)))
    return r


def dot_extract(plan: Plan, state_ptr: int, stream: int = 0):
    """Returns (rho, [m_1..m_D]) as numpy arrays in the paper's exact shapes."""
    D, n = plan.D, plan.n
    sp = tuple(k + 1 for k in n[1:])
    rho = np.zeros((n[0],) + sp)
    shapes = []
    for d in range(1, D + 1):
        s = [n[0] + 1] + list(sp)
        s[d] = n[d]
        shapes.append(tuple(s))
    m = np.zeros(sum(int(np.prod(s)) for s in shapes))
    _check(load().dot_extract(plan.handle, ctypes.c_void_p(state_ptr), _dptr(rho), _dptr(m),
                              ctypes.c_void_p(stream)))
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(m[o:o + k].reshape(s))
        o += k
    return rho, out


def dot_step_divergence(plan, q_ptr, alpha_ptr, sigma, b_ptr, stream=0):
    _check(load().dot_step_divergence(plan.handle, ctypes.c_void_p(q_ptr), ctypes.c_void_p(alpha_ptr),
                                      float(sigma), ctypes.c_void_p(b_ptr), ctypes.c_void_p(stream)))


def dot_step_poisson(plan, b_ptr, stream=0):
    _check(load().dot_step_poisson(plan.handle, ctypes.c_void_p(b_ptr), ctypes.c_void_p(stream)))


def dot_step_rhs_poisson(plan, q_ptr, alpha_ptr, sigma, phi_ptr, stream=0):
    _check(load().dot_step_rhs_poisson(plan.handle, ctypes.c_void_p(q_ptr), ctypes.c_void_p(alpha_ptr),
                                       float(sigma), ctypes.c_void_p(phi_ptr), ctypes.c_void_p(stream)))


def dot_step_cone(plan, q_ptr, beta_ptr, sigma, z_ptr, stream=0):
    _check(load().dot_step_cone(plan.handle, ctypes.c_void_p(q_ptr), ctypes.c_void_p(beta_ptr), float(sigma),
                                ctypes.c_void_p(z_ptr), ctypes.c_void_p(stream)))


def dot_step_update(plan, phi_ptr, q_ptr, alpha_ptr, beta_ptr, sigma, tau, q_out_ptr, w_ptr, stream=0):
    _check(load().dot_step_update(plan.handle, ctypes.c_void_p(phi_ptr), ctypes.c_void_p(q_ptr),
                                  ctypes.c_void_p(alpha_ptr), ctypes.c_void_p(beta_ptr), float(sigma), float(tau),
                                  ctypes.c_void_p(q_out_ptr), ctypes.c_void_p(w_ptr), ctypes.c_void_p(stream)))


def dot_step_residuals(plan, phi_ptr, z_ptr, q_ptr, alpha_ptr, beta_ptr, stream=0) -> dot_result:
    r = dot_result()
    _check(load().dot_step_residuals(plan.handle, ctypes.c_void_p(phi_ptr), ctypes.c_void_p(z_ptr),
                                     ctypes.c_void_p(q_ptr), ctypes.c_void_p(alpha_ptr), ctypes.c_void_p(beta_ptr),
                                     ctypes.byref(r), ctypes.c_void_p(stream)))
    return r


def dot_step_residuals_noalloc(plan, phi_ptr, z_ptr, q_ptr, alpha_ptr, beta_ptr, stream=0) -> dot_result:
    r = dot_result()
    _check(load().dot_step_residuals_noalloc(plan.handle, ctypes.c_void_p(phi_ptr), ctypes.c_void_p(z_ptr),
                                             ctypes.c_void_p(q_ptr), ctypes.c_void_p(alpha_ptr),
                                             ctypes.c_void_p(beta_ptr), ctypes.byref(r), ctypes.c_void_p(stream)))
    return r


def dot_plan_set_graphs(plan, enable: bool):
    _check(load().dot_plan_set_graphs(plan.handle, int(bool(enable))))


def dot_test_fail_captures(count: int):
    """The next `count` graph captures fail before they start (testing the
    fallback to plain launches)."""
    _check(load().dot_test_fail_captures(int(count)))


def dot_batch_set_graphs(batch, enable: bool):
    _check(load().dot_batch_set_graphs(batch.handle, int(bool(enable))))


def _schedule_dict(s: dot_schedule, D: int) -> dict:
    return {"cw": list(s.cw)[:D + 1], "waves": list(s.waves)[:D + 1], "tuned": bool(s.tuned),
            "candidates": int(s.candidates), "us": float(s.us), "us_rule": float(s.us_rule)}


def _schedule_struct(cw=None, waves=None) -> dot_schedule:
    s = dot_schedule()
    for a, v in enumerate(cw or []):
        s.cw[a] = int(v)
    for a, v in enumerate(waves or []):
        s.waves[a] = int(v)
    return s


def dot_plan_set_schedule(plan, cw=None, waves=None):
    """cw / waves: per-axis lists (0 keeps the rule's); both None restores the rule."""
    s = None if cw is None and waves is None else ctypes.byref(_schedule_struct(cw, waves))
    _check(load().dot_plan_set_schedule(plan.handle, s))


def dot_batch_set_schedule(batch, cw=None, waves=None):
    s = None if cw is None and waves is None else ctypes.byref(_schedule_struct(cw, waves))
    _check(load().dot_batch_set_schedule(batch.handle, s))


def dot_plan_get_schedule(plan) -> dict:
    s = dot_schedule()
    _check(load().dot_plan_get_schedule(plan.handle, ctypes.byref(s)))
    return _schedule_dict(s, plan.D)


def dot_batch_get_schedule(batch) -> dict:
    s = dot_schedule()
    _check(load().dot_batch_get_schedule(batch.handle, ctypes.byref(s)))
    return _schedule_dict(s, batch.insts[0].D)


def dot_plan_autotune(plan, state_ptr: int, stream: int = 0) -> dict:
    s = dot_schedule()
    _check(load().dot_plan_autotune(plan.handle, ctypes.c_void_p(state_ptr), ctypes.c_void_p(stream),
                                    ctypes.byref(s)))
    return _schedule_dict(s, plan.D)


def dot_batch_autotune(batch, ws_ptr: int, stream: int = 0) -> dict:
    s = dot_schedule()
    _check(load().dot_batch_autotune(batch.handle, ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream),
                                     ctypes.byref(s)))
    return _schedule_dict(s, batch.insts[0].D)


def dot_profile_select(plan, kernel_class: int):
    _check(load().dot_profile_select(plan.handle, int(kernel_class)))


def dot_profile_read(plan):
    """Returns (total_ms, launches) of the selected kernel class since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().dot_profile_read(plan.handle, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def dot_solve(D, n, rho0, rho1, mask=None, **kw):
    """One-shot blocking solve from host arrays; returns (result, rho, [m_d])."""
    lib = load()
    p, keep = make_problem(D, n, rho0, rho1, mask, **kw)
    sp = tuple(int(k) + 1 for k in n[1:D + 1])
    rho = np.zeros((int(n[0]),) + sp)
    shapes = []
    for d in range(1, D + 1):
        s = [int(n[0]) + 1] + list(sp)
        s[d] = int(n[d])
        shapes.append(tuple(s))
    m = np.zeros(sum(int(np.prod(s)) for s in shapes))
    r = dot_result()
    _check(lib.dot_solve(ctypes.byref(p), _dptr(rho), _dptr(m), ctypes.byref(r)))
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(m[o:o + k].reshape(s))
        o += k
    return r, rho, out


class Batch:
    """Owns a dot_batch handle; instances are described by dotgen-like objects
    with D, n, rho0, rho1, mask."""

    def __init__(self, handle, insts):
        self.handle = handle
        self.insts = list(insts)

    @property
    def workspace_bytes(self):
        return int(load().dot_batch_workspace_bytes(self.handle))

    def close(self):
        if self.handle:
            load().dot_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dot_batch_create(insts, per_instance=None, **kw) -> Batch:
    """Batch of problems (objects with D, n, rho0, rho1, mask); kw as make_problem,
    per_instance: optional list of dicts of further make_problem settings, one per instance."""
    lib = load()
    structs, keep = [], []
    for i, inst in enumerate(insts):
        kwi = dict(kw)
        if per_instance is not None:
            kwi.update(per_instance[i])
        p, k = make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, **kwi)
        structs.append(p)
        keep.append(k)
    arr = (dot_problem * len(structs))(*structs)
    h = ctypes.c_void_p()
    _check(lib.dot_batch_create(arr, len(structs), ctypes.byref(h)))
    return Batch(h, insts)


def dot_batch_destroy(batch: Batch):
    batch.close()


def dot_batch_reset(batch: Batch, ws_ptr: int, stream: int = 0):
    _check(load().dot_batch_reset(batch.handle, ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream)))


def dot_batch_laid_out(batch: Batch) -> int:
    """Instances with workgroups in the batch's launches (fewer than the batch
    after a run that compacted the layout around stopped instances)."""
    return int(load().dot_batch_laid_out(batch.handle))


def dot_batch_run(batch: Batch, ws_ptr: int, max_iters: int, stream: int = 0):
    n = len(batch.insts)
    res = (dot_result * n)()
    _check(load().dot_batch_run(batch.handle, ctypes.c_void_p(ws_ptr), int(max_iters), ctypes.c_void_p(stream), res))
    return list(res)


def dot_batch_extract(batch: Batch, ws_ptr: int, index: int, stream: int = 0):
    inst = batch.insts[index]
    D, n = inst.D, tuple(int(k) for k in inst.n)
    sp = tuple(k + 1 for k in n[1:])
    rho = np.zeros((n[0],) + sp)
    shapes = []
    for d in range(1, D + 1):
        s = [n[0] + 1] + list(sp)
        s[d] = n[d]
        shapes.append(tuple(s))
    m = np.zeros(sum(int(np.prod(s)) for s in shapes))
    _check(load().dot_batch_extract(batch.handle, ctypes.c_void_p(ws_ptr), int(index), _dptr(rho), _dptr(m),
                                    ctypes.c_void_p(stream)))
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(m[o:o + k].reshape(s))
        o += k
    return rho, out


def dot_batch_profile_select(batch: Batch, kernel_class: int):
    _check(load().dot_batch_profile_select(batch.handle, int(kernel_class)))


def dot_batch_profile_read(batch: Batch):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().dot_batch_profile_read(batch.handle, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def _solution_buffers(D, n):
    """Host buffers for (rho, packed m) in the paper's shapes, and the m shapes."""
    n = tuple(int(k) for k in n[:D + 1])
    sp = tuple(k + 1 for k in n[1:])
    rho = np.zeros((n[0],) + sp)
    shapes = []
    for d in range(1, D + 1):
        s = [n[0] + 1] + list(sp)
        s[d] = n[d]
        shapes.append(tuple(s))
    m = np.zeros(sum(int(np.prod(s)) for s in shapes))
    return rho, m, shapes


def _split(m, shapes):
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(m[o:o + k].reshape(s))
        o += k
    return out


# ---- multilevel initialisation ---------------------------------------------
def dot_coarsen_data(D, n, rho0, rho1, mask=None):
    """(n / 2, rho0, rho1, mask) of the next coarser grid (host arithmetic)."""
    n = [int(k) for k in n[:D + 1]]
    nc = tuple(k // 2 for k in n)
    shape = tuple(k + 1 for k in nc[1:])
    r0 = np.ascontiguousarray(rho0, dtype=np.float64).ravel()
    r1 = np.ascontiguousarray(rho1, dtype=np.float64).ravel()
    o0 = np.zeros(shape)
    o1 = np.zeros(shape)
    mk = mo = None
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
        mo = np.zeros(shape, dtype=np.uint8)
    narr = (ctypes.c_int32 * 4)(*(n + [0] * (4 - len(n))))
    u8 = ctypes.POINTER(ctypes.c_uint8)
    _check(load().dot_coarsen_data(int(D), narr, _dptr(r0), _dptr(r1),
                                   mk.ctypes.data_as(u8) if mk is not None else None, _dptr(o0), _dptr(o1),
                                   mo.ctypes.data_as(u8) if mo is not None else None))
    return nc, o0, o1, mo


def dot_state_export(plan, state_ptr: int, stream: int = 0):
    """Returns (q, alpha, beta, sigma): padded-box planes, shapes (D+1, nb), (D+1, nb), (K, nb)."""
    nb, D, K = int(plan.info.nb), plan.D, int(plan.info.K)
    q = np.zeros((D + 1, nb))
    alpha = np.zeros((D + 1, nb))
    beta = np.zeros((K, nb))
    sigma = ctypes.c_double()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    _check(load().dot_state_export(plan.handle, ctypes.c_void_p(state_ptr), dp(q), dp(alpha), dp(beta),
                                   ctypes.byref(sigma), ctypes.c_void_p(stream)))
    return q, alpha, beta, float(sigma.value)


def dot_state_import(plan, state_ptr: int, q, alpha, beta, sigma: float, stream: int = 0):
    nb, D, K = int(plan.info.nb), plan.D, int(plan.info.K)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(D + 1, nb)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64).reshape(D + 1, nb)
    beta = np.ascontiguousarray(beta, dtype=np.float64).reshape(K, nb)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    _check(load().dot_state_import(plan.handle, ctypes.c_void_p(state_ptr), dp(q), dp(alpha), dp(beta),
                                   float(sigma), ctypes.c_void_p(stream)))


def _history(call, cap):
    sig = np.zeros(cap)
    its = np.zeros(cap, dtype=np.int32)
    n = ctypes.c_int32()
    _check(call(sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(n)))
    k = min(int(n.value), cap, 32)
    return [(int(its[j]), float(sig[j])) for j in range(k)], int(n.value)


def dot_sigma_history(plan, state_ptr: int, cap: int = 32, stream: int = 0):
    """Returns ([(iteration, sigma) of the kept changes, oldest first], changes overall)."""
    return _history(lambda s, i, n: load().dot_sigma_history(plan.handle, ctypes.c_void_p(state_ptr), s, i, cap, n,
                                                             ctypes.c_void_p(stream)), cap)


def dot_batch_sigma_history(batch, ws_ptr: int, index: int, cap: int = 32, stream: int = 0):
    return _history(lambda s, i, n: load().dot_batch_sigma_history(batch.handle, ctypes.c_void_p(ws_ptr), int(index),
                                                                   s, i, cap, n, ctypes.c_void_p(stream)), cap)


def dot_state_promote(mixed_plan, mixed_state_ptr: int, fp64_plan, fp64_state_ptr: int, stream: int = 0):
    _check(load().dot_state_promote(mixed_plan.handle, ctypes.c_void_p(mixed_state_ptr), fp64_plan.handle,
                                    ctypes.c_void_p(fp64_state_ptr), ctypes.c_void_p(stream)))


def dot_batch_promote(batch, ws_ptr: int, index: int, fp64_plan, fp64_state_ptr: int, stream: int = 0):
    _check(load().dot_batch_promote(batch.handle, ctypes.c_void_p(ws_ptr), int(index), fp64_plan.handle,
                                    ctypes.c_void_p(fp64_state_ptr), ctypes.c_void_p(stream)))


def dot_batch_promote_member(batch, ws_ptr: int, index: int, fp64_batch, fp64_ws_ptr: int, slot: int,
                             stream: int = 0):
    """Promote member `index` of a mixed batch into member `slot` of an FP64
    batch of the same problems (see include/dotsocp.h)."""
    _check(load().dot_batch_promote_member(batch.handle, ctypes.c_void_p(ws_ptr), int(index), fp64_batch.handle,
                                           ctypes.c_void_p(fp64_ws_ptr), int(slot), ctypes.c_void_p(stream)))


def dot_prolong(coarse: Plan, coarse_state_ptr: int, fine: Plan, fine_state_ptr: int, stream: int = 0):
    _check(load().dot_prolong(coarse.handle, ctypes.c_void_p(coarse_state_ptr), fine.handle,
                              ctypes.c_void_p(fine_state_ptr), ctypes.c_void_p(stream)))


def dot_solve_multilevel(D, n, rho0, rho1, mask=None, levels=2, **kw):
    """Multilevel one-shot solve; returns (result, rho, [m_d], level_results coarsest first)."""
    p, keep = make_problem(D, n, rho0, rho1, mask, **kw)
    rho, m, shapes = _solution_buffers(D, n)
    r = dot_result()
    lv = (dot_result * (levels + 1))()
    _check(load().dot_solve_multilevel(ctypes.byref(p), int(levels), _dptr(rho), _dptr(m), ctypes.byref(r), lv))
    return r, rho, _split(m, shapes), list(lv)


# ---- serving context ---------------------------------------------------------
def dot_footprint_bytes(D, n, precision=DOT_FP64) -> int:
    """Device bytes one instance of this size takes in a serving context."""
    p = dot_problem()
    p.D = D
    for i in range(4):
        p.n[i] = int(n[i]) if i <= D else 0
    p.precision = precision
    return int(load().dot_footprint_bytes(ctypes.byref(p)))


class Ctx:
    """Owns a dot_ctx handle and the shapes of the requests submitted to it."""

    def __init__(self, handle, D, precision):
        self.handle = handle
        self.D = D
        self.precision = precision
        self.shapes = {}

    def close(self):
        if self.handle:
            load().dot_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dot_ctx_create(D, precision, hbm_budget_bytes, max_slots, device: int = -1) -> Ctx:
    """Serving context on HIP device `device` (-1: the current one)."""
    h = ctypes.c_void_p()
    _check(load().dot_ctx_create(int(device), int(D), int(precision), int(hbm_budget_bytes), int(max_slots),
                                 ctypes.byref(h)))
    return Ctx(h, D, precision)


def dot_ctx_destroy(ctx: Ctx):
    ctx.close()


def dot_ctx_submit(ctx: Ctx, inst, **kw) -> int:
    """Queue one problem (object with D, n, rho0, rho1, mask); returns its ticket."""
    p, keep = make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, precision=ctx.precision, **kw)
    t = ctypes.c_uint64()
    _check(load().dot_ctx_submit(ctx.handle, ctypes.byref(p), ctypes.byref(t)))
    ctx.shapes[t.value] = (inst.D, tuple(int(k) for k in inst.n))
    return t.value


def dot_ctx_submit_ml(ctx: Ctx, inst, levels: int, **kw) -> int:
    """Queue one multilevel solve (levels coarser grids first); returns its ticket."""
    p, keep = make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, precision=ctx.precision, **kw)
    t = ctypes.c_uint64()
    _check(load().dot_ctx_submit_ml(ctx.handle, ctypes.byref(p), int(levels), ctypes.byref(t)))
    ctx.shapes[t.value] = (inst.D, tuple(int(k) for k in inst.n))
    return t.value


def dot_ctx_step(ctx: Ctx, iters: int, stream: int = 0):
    """Admit, run `iters` iterations (a multiple of 10), retire; returns (active, queued)."""
    a = ctypes.c_int32()
    q = ctypes.c_int32()
    _check(load().dot_ctx_step(ctx.handle, int(iters), ctypes.c_void_p(stream), ctypes.byref(a), ctypes.byref(q)))
    return a.value, q.value


def dot_ctx_poll(ctx: Ctx, ticket: int) -> int:
    s = ctypes.c_int32()
    _check(load().dot_ctx_poll(ctx.handle, ctypes.c_uint64(ticket), ctypes.byref(s)))
    return s.value


def dot_ctx_fetch(ctx: Ctx, ticket: int):
    """Result of a finished request as (dot_result, rho, [m_d]); releases the ticket."""
    D, n = ctx.shapes[ticket]
    rho, m, shapes = _solution_buffers(D, n)
    r = dot_result()
    _check(load().dot_ctx_fetch(ctx.handle, ctypes.c_uint64(ticket), _dptr(rho), _dptr(m), ctypes.byref(r)))
    del ctx.shapes[ticket]
    return r, rho, _split(m, shapes)


def dot_ctx_stats(ctx: Ctx):
    """(free arena bytes, admitted, retired)."""
    f = ctypes.c_size_t()
    a = ctypes.c_int64()
    r = ctypes.c_int64()
    _check(load().dot_ctx_stats(ctx.handle, ctypes.byref(f), ctypes.byref(a), ctypes.byref(r)))
    return f.value, a.value, r.value


def dot_ctx_export(ctx: Ctx, ticket: int, stream: int = 0) -> bytes:
    """Checkpoint of a running request (opaque bytes, see dotsocp.h)."""
    lib = load()
    need = ctypes.c_size_t()
    _check(lib.dot_ctx_export(ctx.handle, ctypes.c_uint64(ticket), None, 0, ctypes.byref(need),
                              ctypes.c_void_p(stream)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib.dot_ctx_export(ctx.handle, ctypes.c_uint64(ticket), buf, need.value, ctypes.byref(need),
                              ctypes.c_void_p(stream)))
    return buf.raw[:need.value]


def dot_ctx_import(ctx: Ctx, inst, checkpoint: bytes, levels: int = 0, **kw) -> int:
    """Queue a request that resumes from a checkpoint of dot_ctx_export; returns its ticket."""
    p, keep = make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, precision=ctx.precision, **kw)
    t = ctypes.c_uint64()
    buf = ctypes.create_string_buffer(bytes(checkpoint), len(checkpoint))
    _check(load().dot_ctx_import(ctx.handle, ctypes.byref(p), int(levels), buf, len(checkpoint),
                                 ctypes.byref(t)))
    ctx.shapes[t.value] = (inst.D, tuple(int(k) for k in inst.n))
    return t.value


def dot_ctx_keep_capped(ctx: Ctx, keep: bool = True):
    """Requests that stop at their iteration cap keep a checkpoint of their
    final state until fetched (dot_ctx_export returns it)."""
    _check(load().dot_ctx_keep_capped(ctx.handle, int(bool(keep))))


def dot_ctx_last_error(ctx: Ctx) -> str:
    return load().dot_ctx_last_error(ctx.handle).decode(errors="replace")


# ---- padded-box marshalling (host side, numpy) -----------------------------
def box_shape(n):
    return tuple(int(k) + 1 for k in n)


def to_box(arr, n):
    """Zero-pad an exact-shape array (cells or G^s_d) to the node box."""
    full = box_shape(n)
    a = np.asarray(arr)
    pad = [(0, f - s) for s, f in zip(a.shape, full)]
    return np.pad(a, pad)


def from_box(plane, shape):
    return np.asarray(plane)[tuple(slice(0, s) for s in shape)]
