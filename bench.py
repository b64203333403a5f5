#!/usr/bin/env python3
"""Benchmark: solves/s and PALM iterations/s of the MI355X solver at KKT
residual eta_dot <= 1e-6 on the single-instance FP64 workload (2D, 64x64
spatial segments, 32 time steps, 3-component Gaussian mixtures without a
floor), inputs resident in HBM.

One step = one complete solve: state reset on the device, then PALM
iterations (every hot-path kernel, residual checks and the sigma rule on the
device) until eta_dot <= 1e-6. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import dotgen  # noqa: E402
from paper_2505_05424_amd import binding as B  # noqa: E402
from paper_2505_05424_amd import perfmodel as PM  # noqa: E402

TOL = 1e-6
MAX_ITER = 100000
BATCH_MAX_ITER = 60000   # mixed-precision batch iterations before the FP64 finish
FINISH_MAX_ITER = 100000  # cap per instance in all (batch + FP64 finish; plain FP64 solves)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def section(name, fn, *a, **kw):
    """Run one section after the headline; an error in it is reported in its
    place in the line (the headline measured above stands)."""
    try:
        return fn(*a, **kw)
    except Exception as e:  # noqa: BLE001
        log(f"{name}: failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# The paper's own CPU figures (MATLAB with a C++ projection on an Intel Core
# i9-9900KF, 8 cores, 3.6 GHz; Table 4, single-level inpALM, tolerance 1e-4),
# as seconds per iteration = total time / iterations over its rows. Context only.
PAPER_CPU_S_PER_ITER = {"(32,128,128)": [0.105, 0.120], "(64,256,256)": [0.829, 0.921]}


def cpu_baseline(iters_per_solve_cfg2, cfg3_iters=3):
    """The FP64 oracle as it stands, timed on this host: the cosine transforms
    (scipy.fft) on all cores (workers = os.cpu_count()) and on one core (the
    rest of the oracle is single-threaded numpy either way). Per leg: ms per
    iteration over a 50-iteration block on the headline 2D 32x64^2 instance
    (after one warm-up iteration; residuals every 5 as in a solve) and over a
    `cfg3_iters`-iteration block on 2D 64x256^2 (a full 50-iteration block
    would take minutes); a full solve of the 1D 16x32 instance to
    eta_dot <= 1e-8. value = headline solves/s with all cores = 1 / (ms per
    iteration x the iterations a solve takes)."""
    import scipy.fft as sfft
    from oracle import dot_oracle as O
    ncpu = os.cpu_count() or 1

    def ms_per_iter(inst, n_iter, workers):
        P = O.make_problem(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask)
        S = O.zero_state(P)
        with sfft.set_workers(workers):
            S = O.iterate(P, S)
            t0 = time.perf_counter()
            for _ in range(n_iter):
                S = O.iterate(P, S)
                if S.k % 5 == 0:
                    O.residuals(P, S.phi, S.z, S.q, S.alpha, S.beta)
            return 1e3 * (time.perf_counter() - t0) / n_iter

    c2, c3 = dotgen.config2_instance(), dotgen.config3_instance()
    legs = {}
    for workers, name in ((ncpu, "all_cores"), (1, "one_core")):
        log(f"cpu baseline: {name}")
        legs[name] = {"threads": workers,
                      "2d_32x64x64_ms_per_iter_50": ms_per_iter(c2, 50, workers),
                      f"2d_64x256x256_ms_per_iter_{cfg3_iters}": ms_per_iter(c3, cfg3_iters, workers)}
    c1 = dotgen.config1_instance()
    P1 = O.make_problem(c1.D, c1.n, c1.rho0, c1.rho1, c1.mask)
    with sfft.set_workers(1):
        r1 = O.solve(P1, tol=1e-8, max_iter=200000)
    ms_all = legs["all_cores"]["2d_32x64x64_ms_per_iter_50"]
    return {
        "value": 1e3 / ms_all / iters_per_solve_cfg2,
        "unit": "solves/s",
        "cores": ncpu,
        "kind": "oracle",
        "sample": (f"50 consecutive oracle iterations (numpy/scipy FP64) of the 32x64x64 headline instance with "
                   f"the transforms on {ncpu} threads: {ms_all:.1f} ms per iteration, times the "
                   f"{iters_per_solve_cfg2} iterations one solve takes"),
        "legs": legs,
        "config1_full_solve": {"workload": "1d-16x32, tol 1e-8", "iters": r1.iters, "converged": r1.converged,
                               "seconds": r1.seconds, "objective": r1.objective},
        "paper_table4_s_per_iter_i9_9900kf_8_cores": PAPER_CPU_S_PER_ITER,
        "cpu_model": cpu_model(),
        "host_cpus": ncpu,
    }


def headline_error(rho, m, r):
    """The headline solve against the oracle's converged solve of the same
    instance (tests/golden/config2_converged.json, written from the oracle):
    iteration counts, relative objective error, max |rho|, |m| errors at the
    stored positions."""
    path = os.path.join(ROOT, "tests", "golden", "config2_converged.json")
    try:
        gold = json.load(open(path))
    except (OSError, ValueError):
        return None
    mflat = np.concatenate([a.ravel() for a in m])
    return {"reference": "tests/golden/config2_converged.json (FP64 oracle, same settings)",
            "iters": r.iters, "oracle_iters": gold["iters"],
            "objective_rel_err": abs(r.objective - gold["objective"]) / abs(gold["objective"]),
            "dual_objective_rel_err": abs(r.dual_objective - gold["dual_objective"]) / abs(gold["dual_objective"]),
            "rho_max_abs_err_sampled": float(np.max(np.abs(rho.ravel()[gold["rho_index"]] - np.array(gold["rho_value"])))),
            "m_max_abs_err_sampled": float(np.max(np.abs(mflat[gold["m_index"]] - np.array(gold["m_value"])))),
            "samples": len(gold["rho_index"]) + len(gold["m_index"])}


def mixed_vs_fp64_config3(torch, st):
    """2D 64x256^2 (5-component mixtures) solved to eta_dot <= 1e-6 in FP64 and
    in mixed precision: iterations, seconds, relative objective difference."""
    inst = dotgen.config3_instance()
    out = {"workload": "2d-64x256x256-gaussmix5, tol 1e-6"}
    for prec, name in ((B.DOT_FP64, "fp64"), (B.DOT_MIXED, "mixed")):
        plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=TOL, max_iter=MAX_ITER,
                                 precision=prec)
        buf = torch.zeros(int(plan.info.state_bytes), dtype=torch.uint8, device="cuda")
        el, r = time_solves(plan, buf.data_ptr(), st, 1, torch)
        rho, _ = B.dot_extract(plan, buf.data_ptr(), st)
        mass = rho.reshape(rho.shape[0], -1).sum(1) / (inst.n[1] * inst.n[2])
        out[name] = {"iters": r[0].iters, "term": B.TERM_NAMES[r[0].term], "seconds": el,
                     "eta_dot": r[0].eta_dot, "objective": r[0].objective,
                     "ms_per_iter": 1e3 * el / r[0].iters, "slice_mass_max_err": float(np.max(np.abs(mass - 1)))}
        del buf
        plan.close()
    out["objective_rel_diff_mixed_vs_fp64"] = (abs(out["mixed"]["objective"] - out["fp64"]["objective"])
                                               / abs(out["fp64"]["objective"]))
    out["speedup_mixed_vs_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    return out


def solve_plain(plan, ptr, st, cap=MAX_ITER):
    B.dot_state_reset(plan, ptr, st)
    return B.dot_run(plan, ptr, cap, st)


def time_solves(plan, ptr, st, k, torch, cap=MAX_ITER):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [solve_plain(plan, ptr, st, cap) for _ in range(k)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, res


def kernel_breakdown(plan, ptr, st):
    """Per-class event times over one solve (graphs are off while timing)."""
    out = {}
    for name, cls in B.KERNEL_CLASSES.items():
        B.dot_profile_select(plan, cls)
        solve_plain(plan, ptr, st)
        ms, cnt = B.dot_profile_read(plan)
        if cnt:
            out[name] = {"ms_total": ms, "launches": cnt, "us_per_launch": 1e3 * ms / cnt}
    B.dot_profile_select(plan, -1)
    return out


def kernel_sources_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2505_05424_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(workload, kernel_class):
    """HBM bytes per launch of one kernel class from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE runs scaled by a copy calibration), or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"kernels_{workload}.md")
    try:
        text = open(path).read()
        blk = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blk.get("source_sha256") != kernel_sources_hash():
        return None
    b = blk["per_launch_bytes"].get(kernel_class)
    if not b:
        return None
    return {"bytes": b["fetch"] + b["write"], "fetch": b["fetch"], "write": b["write"],
            "copy_factor_fetch": blk["copy_factor_fetch"], "copy_factor_write": blk["copy_factor_write"],
            "source": f"profiles/kernels_{workload}.md"}


def large_roofline(torch, st, iters=60):
    """Per-class HIP-event timing on the bandwidth-bound size: 2D 64x256x256,
    mixed precision, `iters` iterations per class after a warm-up."""
    inst = dotgen.config3_instance()
    plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=-1.0, max_iter=10 ** 6,
                             precision=B.DOT_MIXED)
    buf = torch.zeros(int(plan.info.state_bytes), dtype=torch.uint8, device="cuda")
    B.dot_state_reset(plan, buf.data_ptr(), st)
    B.dot_run(plan, buf.data_ptr(), 20, st)
    kb = PM.kernel_bytes(inst.D, inst.n, 4)
    classes = {}
    for name, cls in B.KERNEL_CLASSES.items():
        if name in ("resid", "final"):
            continue
        B.dot_profile_select(plan, cls)
        B.dot_run(plan, buf.data_ptr(), iters, st)
        ms, cnt = B.dot_profile_read(plan)
        if cnt:
            us = 1e3 * ms / cnt
            classes[name] = {"avg_launch_us": us, "algorithmic_bytes": kb[name],
                             "achieved_GBs": kb[name] / (us * 1e-6) / 1e9,
                             "frac": kb[name] / (us * 1e-6) / 1e9 / PM.HBM_PEAK_GBS}
    B.dot_profile_select(plan, -1)
    plan.close()
    lp = PM.launches_per_iteration(inst.D)
    dom = max(classes, key=lambda k: classes[k]["avg_launch_us"] * lp.get(k, 1))
    return {"workload": "2d-64x256x256-gaussmix5-mixed", "dominant": dom, "peak_GBs": PM.HBM_PEAK_GBS,
            "classes": classes}



def variants_section(torch, st, inst):
    """Algorithm variants on the same kernels (Rem. 4.2): dual step length tau
    in {1, 1.5, 1.9} on the single-instance workload, FP64, to eta_dot <= 1e-6."""
    out = {}
    for tau in (1.0, 1.5, 1.9):
        plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=TOL, max_iter=MAX_ITER,
                                 tau=tau)
        buf = torch.zeros(int(plan.info.state_bytes), dtype=torch.uint8, device="cuda")
        el, r = time_solves(plan, buf.data_ptr(), st, 1, torch)
        out[f"tau={tau}"] = {"iters": r[0].iters, "term": B.TERM_NAMES[r[0].term], "seconds": el,
                             "solves_per_s": 1.0 / el, "objective": r[0].objective}
        plan.close()
    return out


def multilevel_section(torch, inst):
    """Multilevel initialisation (coarse grids n / 2^v, each level started from
    the interpolated coarser solution), one-shot calls (plans and states
    allocated inside, as dot_solve does): the single-instance workload in FP64
    with 0..3 coarse levels, and 2D 64x256x256 (5-component mixtures) in mixed
    precision without and with 3 coarse levels."""
    def one(i, levels, prec):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r, rho, m, lv = B.dot_solve_multilevel(i.D, i.n, i.rho0, i.rho1, i.mask, levels=levels, tol=TOL,
                                               max_iter=MAX_ITER, precision=prec)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return {"seconds": el, "solves_per_s": 1.0 / el, "term": B.TERM_NAMES[r.term],
                "iters_per_level_coarsest_first": [x.iters for x in lv], "objective": r.objective,
                "eta_dot": r.eta_dot}
    out = {"2d-32x64x64-fp64": {f"levels={v}": one(inst, v, B.DOT_FP64) for v in (0, 1, 2, 3)}}
    big = dotgen.config3_instance()
    log("multilevel at 2D 64x256x256 (mixed)")
    out["2d-64x256x256-mixed"] = {f"levels={v}": one(big, v, B.DOT_MIXED) for v in (0, 3)}
    return out


def large_section(torch, st, iters=40, max_solve_s=60.0):
    """The paper's large single-instance size, 2D 32x1024x1024 (image-like
    mixtures of 16 narrow Gaussians stand in for its image pair): state size,
    ms per iteration (after a warm-up, graphs on) in both modes, and a mixed
    solve to eta_dot <= 1e-4 (the tolerance of the paper's 1024^2 runs),
    stopped after `max_solve_s` seconds."""
    inst = dotgen.image_like_instance()
    out = {"workload": "2d-32x1024x1024-image-like", "nodes": int(np.prod([k + 1 for k in inst.n]))}
    for prec, name in ((B.DOT_MIXED, "mixed"), (B.DOT_FP64, "fp64")):
        plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, None, tol=1e-4, max_iter=10 ** 6,
                                 precision=prec)
        buf = torch.zeros(int(plan.info.state_bytes), dtype=torch.uint8, device="cuda")

        def ms_per_iter():
            B.dot_state_reset(plan, buf.data_ptr(), st)
            B.dot_run(plan, buf.data_ptr(), 20, st)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.dot_run(plan, buf.data_ptr(), iters, st)
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t0) / iters

        ms_rule = ms_per_iter()
        # transform schedule measured on this instance (setup, before the timed runs)
        t0 = time.perf_counter()
        sched = B.dot_plan_autotune(plan, buf.data_ptr(), st)
        tune_s = time.perf_counter() - t0
        ms = ms_per_iter()
        rec = {"state_GB": plan.info.state_bytes / 1e9, "ms_per_iter": ms, "ms_per_iter_rule_schedule": ms_rule,
               "transform_schedule": sched, "autotune_s": tune_s,
               "min_bytes_frac_of_hbm_peak": PM.iteration_min_bytes(inst.D, inst.n, 8 if name == "fp64" else 4)
               / (ms * 1e-3) / 1e9 / PM.HBM_PEAK_GBS}
        if name == "mixed":
            B.dot_state_reset(plan, buf.data_ptr(), st)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while True:
                r = B.dot_run(plan, buf.data_ptr(), 1000, st)
                el = time.perf_counter() - t0
                log(f"large: {r.iters} iterations, eta {r.eta_dot:.2e}, {el:.1f} s")
                if B.TERM_NAMES[r.term] != "maxiter" or el > max_solve_s:
                    break
            rec["solve_tol_1e-4"] = {"iters": r.iters, "term": B.TERM_NAMES[r.term], "seconds": el,
                                     "eta_dot": r.eta_dot, "objective": r.objective}
        out[name] = rec
        del buf
        plan.close()
    return out


def _converged(r):
    return B.TERM_NAMES[r.term] == "converged" and r.eta_dot <= TOL


def batched_section(torch, st, count, seed=4000):
    """Config-4 batch: `count` instances (grid sides from {32..128}, n0 from
    {16, 32, 64}, half masked), mixed precision, one launch per kernel for all
    instances, to eta_dot <= 1e-6 with a cap of BATCH_MAX_ITER iterations;
    members still above the tolerance at the cap (masked instances that need
    more iterations, or that level off at their FP32 storage floor) are then
    promoted into one FP64 batch of their problems (dot_batch_promote_member)
    and finished together up to FINISH_MAX_ITER iterations in all. Against
    it: the same `count` instances solved one at a time in plain FP64 (cap
    FINISH_MAX_ITER). Only results with eta_dot <= 1e-6 count as solves."""
    insts = dotgen.config4_instances(count, seed=seed)
    batch = B.dot_batch_create(insts, tol=TOL, max_iter=FINISH_MAX_ITER, precision=B.DOT_MIXED)
    ws = torch.zeros(batch.workspace_bytes, dtype=torch.uint8, device="cuda")
    # transform schedule of this batch's launches, measured before the timed run
    t0 = time.perf_counter()
    sched = B.dot_batch_autotune(batch, ws.data_ptr(), st)
    tune_s = time.perf_counter() - t0
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    log(f"batched: {count} instances, workspace {batch.workspace_bytes / 2**30:.2f} GiB, schedule {sched}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < BATCH_MAX_ITER:
        res = B.dot_batch_run(batch, ws.data_ptr(), 5000, st)
        done += 5000
        conv = sum(1 for r in res if _converged(r))
        log(f"batched: {done} iterations, {conv}/{count} converged, {time.perf_counter() - t0:.1f} s")
        if conv == count:
            break
    torch.cuda.synchronize()
    el_batch = time.perf_counter() - t0
    conv_batch = sum(1 for r in res if _converged(r))
    # FP64 finish of the members still running (inside the timed region): all
    # of them promoted into one FP64 batch of their problems, run together
    finished = {}
    pending = [i for i, r in enumerate(res) if not _converged(r)]
    if pending:
        fb = B.dot_batch_create([insts[i] for i in pending], tol=TOL, max_iter=FINISH_MAX_ITER,
                                precision=B.DOT_FP64)
        fws = torch.zeros(fb.workspace_bytes, dtype=torch.uint8, device="cuda")
        B.dot_batch_reset(fb, fws.data_ptr(), st)
        for slot, i in enumerate(pending):
            B.dot_batch_promote_member(batch, ws.data_ptr(), i, fb, fws.data_ptr(), slot, st)
        left = FINISH_MAX_ITER - done
        k = 0
        rf_all = None
        while k < left:
            step = min(5000, left - k)
            rf_all = B.dot_batch_run(fb, fws.data_ptr(), step, st)
            k += step
            nconv = sum(1 for r in rf_all if _converged(r))
            log(f"batched: fp64 finish batch of {len(pending)}: {k} iterations, {nconv} converged, "
                f"{time.perf_counter() - t0:.1f} s")
            if all(B.TERM_NAMES[r.term] in ("converged", "diverged") for r in rf_all):
                break
        for slot, i in enumerate(pending):
            r, rf = res[i], rf_all[slot]
            finished[insts[i].label] = {"mixed_iters": r.iters, "mixed_eta_dot": r.eta_dot,
                                        "fp64_iters_after": rf.iters - r.iters, "eta_dot": rf.eta_dot,
                                        "term": B.TERM_NAMES[rf.term],
                                        "objective_change_rel": abs(rf.objective - r.objective) / abs(rf.objective)}
            res[i] = rf
            log(f"batched: fp64 finish {insts[i].label}: {r.iters} mixed + {rf.iters - r.iters} fp64 iterations, "
                f"eta {rf.eta_dot:.2e}")
        del fws
        fb.close()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    conv = sum(1 for r in res if _converged(r))
    inst_iters = sum(r.iters for r in res)
    nodes = sum(int(np.prod([k + 1 for k in i.n])) for i in insts)
    # dominant kernel of the batch, timed with events in a second run
    log("batched: beta-kernel timing")
    B.dot_batch_reset(batch, ws.data_ptr(), st)
    B.dot_batch_profile_select(batch, B.KERNEL_CLASSES["beta"])
    B.dot_batch_run(batch, ws.data_ptr(), 400, st)
    ms, cnt = B.dot_batch_profile_read(batch)
    B.dot_batch_profile_select(batch, -1)
    del ws
    batch.close()
    kb = sum(PM.kernel_bytes(i.D, i.n, 4)["beta"] for i in insts)
    avg_us = 1e3 * ms / max(cnt, 1)
    out = {
        "workload": f"{count} 2D instances, sides {{32,48,64,96,128}}, n0 {{16,32,64}}, half masked, mixed precision",
        "instances": count,
        "converged": conv,
        "converged_in_batch": conv_batch,
        "batch_iteration_cap": BATCH_MAX_ITER,
        "finished_in_fp64": finished,
        "total_iteration_cap": FINISH_MAX_ITER,
        "seconds": el,
        "seconds_batch_part": el_batch,
        "solves_per_s": conv / el,
        "instance_iters_per_s": inst_iters / el,
        "max_iters": max(r.iters for r in res),
        "mean_iters": inst_iters / count,
        "nodes_total": nodes,
        "transform_schedule": sched,
        "autotune_s": tune_s,
        "beta_kernel": {"avg_launch_us_first_400_iters": avg_us, "algorithmic_bytes": kb,
                        "achieved_GBs": kb / (avg_us * 1e-6) / 1e9,
                        "frac_of_hbm_peak": kb / (avg_us * 1e-6) / 1e9 / PM.HBM_PEAK_GBS},
    }
    # the same instances one at a time in plain FP64
    t_tot, its, conv_p = 0.0, 0, 0
    for k, inst in enumerate(insts):
        plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=TOL,
                                 max_iter=FINISH_MAX_ITER)
        buf = torch.zeros(int(plan.info.state_bytes), dtype=torch.uint8, device="cuda")
        el1, r = time_solves(plan, buf.data_ptr(), st, 1, torch, cap=FINISH_MAX_ITER)
        t_tot += el1
        its += r[0].iters
        conv_p += int(_converged(r[0]))
        if k % 8 == 7:
            log(f"plain fp64: {k + 1}/{count} solved, {t_tot:.1f} s")
        del buf
        plan.close()
    out["plain_fp64_one_at_a_time"] = {"instances": count, "converged": conv_p, "seconds": t_tot,
                                       "solves_per_s": conv_p / t_tot, "iters_per_s": its / t_tot}
    out["speedup_batched_mixed_vs_plain_fp64"] = (conv / el) / (conv_p / t_tot)
    return out


def serving_section(torch, rate, seconds, drain_s, seed=5000):
    """Serving stream: Poisson arrivals at `rate` requests/s for `seconds` of
    2D solves (sides log-uniform in [32, 256], n0 from {16, 32, 64}, every
    second one masked) and 10% 3D solves (32 x 64^3), mixed precision, tol
    1e-6; continuous batching with admission by HBM footprint and backfill
    (one context per D, each on its own thread and stream). A request still
    above 1e-6 at the mixed cap continues in an FP64 context of its
    dimension from its final state (promoted exactly) for up to
    FINISH_MAX_ITER iterations in all. Latency is arrival -> result in host
    memory. Requests still running `drain_s` after the last arrival are
    reported as unfinished (their latency is censored)."""
    from paper_2505_05424_amd.serving import Server
    rng = np.random.default_rng(seed)
    t_arr = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * seconds * 2) + 10))
    t_arr = t_arr[t_arr < seconds]
    log(f"serving: generating {len(t_arr)} requests (rate {rate:.3f}/s over {seconds:.0f} s)")
    reqs = [dotgen.serving_request(i, seed=seed) for i in range(len(t_arr))]
    srv = Server(precision=B.DOT_MIXED, budgets={2: 96 << 30, 3: 64 << 30}, slots={2: 160, 3: 32},
                 step_iters=40, tol=TOL, max_iter=BATCH_MAX_ITER, finish_fp64=True,
                 finish_iters=FINISH_MAX_ITER - BATCH_MAX_ITER, finish_budgets={2: 24 << 30, 3: 32 << 30},
                 finish_slots={2: 32, 3: 8})
    # warm-up: one small request per context (first launches, module loads)
    warm = [srv.submit(dotgen.tiny_instance(2, (8, 16, 16), seed=1)),
            srv.submit(dotgen.tiny_instance(3, (4, 8, 8, 8), seed=2))]
    for w in warm:
        w.done.wait(120)
    srv.check()
    lanes = {D: (ln.steps, ln.active_sum) for D, ln in srv.lanes.items()}
    log("serving: arrivals start")
    handles = []
    t0 = time.perf_counter()
    last_log = t0
    for i, ta in enumerate(t_arr):
        while True:
            now = time.perf_counter()
            if now - t0 >= ta:
                break
            time.sleep(min(0.01, ta - (now - t0)))
        h = srv.submit(reqs[i])
        h.t_arrival = t0 + ta  # scheduled arrival time
        handles.append(h)
        if now - last_log > 10:
            last_log = now
            log(f"serving: t={now - t0:.0f} s, submitted {len(handles)}, "
                f"done {sum(x.done.is_set() for x in handles)}, in flight {srv.in_flight()}")
        srv.check()
    t_end_arr = time.perf_counter()
    while time.perf_counter() - t_end_arr < drain_s and not all(h.done.is_set() for h in handles):
        time.sleep(0.05)
        now = time.perf_counter()
        if now - last_log > 10:
            last_log = now
            log(f"serving: draining, t={now - t0:.0f} s, done {sum(x.done.is_set() for x in handles)} "
                f"of {len(handles)}")
    t_stop = time.perf_counter()
    stats_lanes = {D: {"steps": ln.steps - lanes[D][0],
                       "mean_active": (ln.active_sum - lanes[D][1]) / max(1, ln.steps - lanes[D][0])}
                   for D, ln in srv.lanes.items()}
    srv.abandon()
    fin = [h for h in handles if h.done.is_set() and h.result is not None]
    conv = [h for h in fin if _converged(h.result)]
    lat = np.array([h.latency for h in fin]) if fin else np.zeros(1)
    wall = (max(h.t_done for h in fin) if fin else t_stop) - t0
    by_d = {}
    for D in (2, 3):
        hs = [h for h in fin if h.inst.D == D]
        if hs:
            ld = np.array([h.latency for h in hs])
            by_d[f"{D}d"] = {"finished": len(hs), "p50_s": float(np.percentile(ld, 50)),
                             "p99_s": float(np.percentile(ld, 99)),
                             "mean_iters": float(np.mean([h.result.iters for h in hs]))}
    return {
        "workload": ("Poisson arrivals; 2D sides log-uniform in [32,256], n0 {16,32,64}, every second 2D "
                     "request masked; 10% 3D 32x64^3; mixed precision; tol 1e-6"),
        "rate_per_s": rate,
        "arrival_window_s": seconds,
        "submitted": len(handles),
        "finished": len(fin),
        "converged": len(conv),
        "hit_iteration_cap": len(fin) - len(conv),
        "unfinished_at_cutoff": len(handles) - len(fin),
        "iteration_cap": BATCH_MAX_ITER,
        "finished_in_fp64": {f"r{i}-" + "x".join(str(k) for k in h.inst.n) + ("-mask" if h.inst.mask is not None
                                                                             else ""):
                             {"mixed_iters": h.mixed_result.iters, "mixed_eta_dot": h.mixed_result.eta_dot,
                              "iters": h.result.iters, "eta_dot": h.result.eta_dot,
                              "term": B.TERM_NAMES[h.result.term], "latency_s": h.latency}
                             for i, h in enumerate(handles) if h.result is not None and h.finished_in_fp64},
        "total_iteration_cap": FINISH_MAX_ITER,
        "wall_s": wall,
        "solves_per_s": len(conv) / wall,
        "instance_iters_per_s": sum(h.result.iters for h in fin) / wall,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "latency_note": "over finished requests; unfinished ones are censored (p99 is then a lower bound)",
        "by_dimension": by_d,
        "lanes": stats_lanes,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cfg3-iters", type=int, default=3,
                    help="oracle iterations timed on 2D 64x256^2 per leg of the CPU baseline")
    ap.add_argument("--batch", type=int, default=64, help="instances of the batched section (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=50.0, help="serving arrival window (0: skip)")
    ap.add_argument("--serve-drain", type=float, default=90.0)
    # about 80% of the serving mix's capacity on one MI355X: a 3D request
    # (32 x 64^3, ~1.3 ms per iteration) costs ~15 GPU-seconds and an average
    # 2D request ~1.5, so the 90/10 mix needs ~3 GPU-seconds per request
    ap.add_argument("--serve-rate", type=float, default=0.25, help="Poisson arrivals per second")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(instances are independent: several GPUs would each take their own instances)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.init()
    st = torch.cuda.current_stream().cuda_stream

    inst = dotgen.config2_instance()
    D, n = inst.D, inst.n
    plan = B.dot_plan_create(D, n, inst.rho0, inst.rho1, inst.mask, tol=TOL, max_iter=MAX_ITER)
    w = int(plan.info.scalar_bytes)
    state = torch.zeros(int(plan.info.state_bytes), dtype=torch.uint8, device="cuda")
    ptr = state.data_ptr()

    log("warmup")
    for _ in range(args.warmup):
        solve_plain(plan, ptr, st)
    log("timed solves")

    # timed region: K complete solves, graphs on, no events
    el, results = time_solves(plan, ptr, st, args.steps, torch)
    iters = [r.iters for r in results]
    assert all(B.TERM_NAMES[r.term] == "converged" for r in results), [r.term for r in results]
    last = results[-1]
    rho_h, m_h = B.dot_extract(plan, ptr, st)
    err = headline_error(rho_h, m_h, last)

    # roofline: the same solves again with events around the dominant kernel
    log("kernel breakdown")
    breakdown = kernel_breakdown(plan, ptr, st)
    dominant = max(breakdown, key=lambda k: breakdown[k]["ms_total"])
    B.dot_profile_select(plan, B.KERNEL_CLASSES[dominant])
    n_ev = min(args.steps, 5)
    el_ev, _ = time_solves(plan, ptr, st, n_ev, torch)
    dom_ms, dom_cnt = B.dot_profile_read(plan)
    B.dot_profile_select(plan, -1)
    kb = PM.kernel_bytes(D, n, w)
    avg_us = 1e3 * dom_ms / max(dom_cnt, 1)
    achieved = kb[dominant] / (avg_us * 1e-6) / 1e9
    it_min = PM.iteration_min_bytes(D, n, w)
    traffic = profiled_traffic("2d_32x64x64_fp64", dominant)
    log("roofline at 2D 64x256x256 (mixed)")
    large = section("roofline at 2D 64x256x256", large_roofline, torch, st)

    out = {
        "metric": "solves/s at KKT residual 1e-6 (plain FP64, one instance)",
        "value": args.steps / el,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2d-{n[0]}x{n[1]}x{n[2]}-gaussmix3-fp64", "D": D, "n": list(n),
                   "tol": TOL, "precision": "fp64", "instances": 1, "hip_graphs": True},
        "palm_iters_per_s": sum(iters) / el,
        # the launch-size rule's schedule (the autotuner gains < 1% at this size and its
        # choice may vary run to run; the roofline kernel must match the committed profile)
        "transform_schedule": B.dot_plan_get_schedule(plan),
        "iters_per_solve": iters[0],
        "eta_dot": last.eta_dot,
        "objective": last.objective,
        "dual_objective": last.dual_objective,
        "error_vs_oracle": err,
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": achieved,
            "peak": PM.HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / PM.HBM_PEAK_GBS,
            "traffic": traffic["bytes"] if traffic else None,
            "traffic_detail": traffic,
            "algorithmic_bytes_per_launch": kb[dominant],
            "avg_launch_us": avg_us,
            "launches": dom_cnt,
            "timed_region": f"{n_ev} further solves of the same instance with HIP events around every "
                            f"launch of this kernel on the solver's stream (graphs off), {el_ev:.2f} s",
        },
        "iteration": {
            "us_per_iter": 1e6 * el / sum(iters),
            "min_bytes_per_iter": it_min,
            "min_bytes_frac_of_hbm_peak": it_min / (el / sum(iters)) / 1e9 / PM.HBM_PEAK_GBS,
        },
        "kernel_breakdown_one_solve": breakdown,
        "kernel_breakdown_note": ("one solve per class with HIP events around every launch of that class: "
                                  "graphs off and the fused launches split into their classes (beta + next z-step "
                                  "+ next right-hand side; z-step + right-hand side), so the classes sum to more "
                                  "than the timed solve (which runs graphs and the fused launches)"),
        "roofline_bandwidth_bound_size": large,
    }
    log("large instance 32x1024x1024")
    out["large_instance"] = section("large instance", large_section, torch, st)
    log("multilevel")
    out["multilevel"] = section("multilevel", multilevel_section, torch, inst)
    log("mixed vs fp64 at 2D 64x256x256")
    out["mixed_vs_fp64_2d_64x256x256"] = section("mixed vs fp64", mixed_vs_fp64_config3, torch, st)
    log("variants (tau)")
    out["variants_tau"] = section("variants", variants_section, torch, st, inst)
    if args.batch > 0:
        out["batched"] = section("batched", batched_section, torch, st, args.batch)
    if args.serve_seconds > 0:
        out["serving"] = section("serving", serving_section, torch, args.serve_rate, args.serve_seconds,
                                 args.serve_drain)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = section("cpu baseline", cpu_baseline, iters[0], args.cpu_cfg3_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
