"""Fixed-iteration runs of named workloads, for rocprofv3 kernel traces and
counter collection:

  rocprofv3 --kernel-trace --stats --output-format csv -d OUT -- \
      python3 -m paper_2505_05424_amd.profile_run --workload 2d-32x64x64 --iters 500

Workloads: 1d-16x32, 2d-32x64x64, 2d-64x256x256, 3d-32x64x64x64, 2d-32x1024x1024 (add
--mixed for the mixed-precision mode). --copy-mib M first runs one plain
device-to-device copy of M MiB (torch), the calibration of the HBM byte
counters. --cw / --waves install an explicit transform schedule (comma lists
over the axes, 0 keeps the rule's; e.g. one the autotuner chose in another
run), so that no tuning launches enter the trace. --batch K runs K instances of
the heterogeneous 2D batch (grid sides from {32..128}, n0 from {16, 32, 64},
every second one masked; seed --seed) as one batch for --iters iterations
(the schedule options apply to it)."""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import dotgen  # noqa: E402
from paper_2505_05424_amd import binding as B  # noqa: E402

WORKLOADS = {
    "1d-16x32": dotgen.config1_instance,
    "2d-32x64x64": dotgen.config2_instance,
    "2d-64x256x256": dotgen.config3_instance,
    "3d-32x64x64x64": dotgen.serving_3d_instance,
    "2d-32x1024x1024": dotgen.image_like_instance,
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", action="append", default=[])
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--iters", type=int, action="append")
    ap.add_argument("--mixed", action="store_true")
    ap.add_argument("--cw", type=str, default="")
    ap.add_argument("--waves", type=str, default="")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--seed", type=int, default=4000)
    a = ap.parse_args()
    import torch
    st = torch.cuda.current_stream().cuda_stream
    if a.copy_mib:
        nbytes = a.copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy {nbytes} bytes", flush=True)
        del src, dst
    cw = [int(v) for v in a.cw.split(",")] if a.cw else None
    waves = [int(v) for v in a.waves.split(",")] if a.waves else None
    if a.batch:
        its = (a.iters or [20])[0]
        insts = dotgen.config4_instances(a.batch, seed=a.seed)
        batch = B.dot_batch_create(insts, tol=-1.0, max_iter=its, precision=B.DOT_MIXED if a.mixed else B.DOT_FP64)
        if cw or waves:
            B.dot_batch_set_schedule(batch, cw=cw, waves=waves)
        sched = B.dot_batch_get_schedule(batch)
        print(f"batch of {a.batch} schedule cw={sched['cw']} waves={sched['waves']}", flush=True)
        ws = torch.zeros(int(batch.workspace_bytes), dtype=torch.uint8, device="cuda")
        B.dot_batch_reset(batch, ws.data_ptr(), st)
        res = B.dot_batch_run(batch, ws.data_ptr(), its, st)
        torch.cuda.synchronize()
        print(f"batch of {a.batch} iters={res[0].iters}", flush=True)
        batch.close()
        return
    iters = a.iters or [100] * len(a.workload)
    for name, its in zip(a.workload, iters):
        inst = WORKLOADS[name]()
        plan = B.dot_plan_create(inst.D, inst.n, inst.rho0, inst.rho1, inst.mask, tol=-1.0, max_iter=its,
                                 precision=B.DOT_MIXED if a.mixed else B.DOT_FP64)
        if cw or waves:
            B.dot_plan_set_schedule(plan, cw=cw, waves=waves)
        sched = B.dot_plan_get_schedule(plan)
        print(f"{name} schedule cw={sched['cw']} waves={sched['waves']}", flush=True)
        s = torch.zeros(int(plan.info.state_bytes), dtype=torch.uint8, device="cuda")
        B.dot_state_reset(plan, s.data_ptr(), st)
        r = B.dot_run(plan, s.data_ptr(), its, st)
        torch.cuda.synchronize()
        print(f"{name} iters={r.iters} eta={r.eta_dot:.3e}", flush=True)
        plan.close()


if __name__ == "__main__":
    main()
