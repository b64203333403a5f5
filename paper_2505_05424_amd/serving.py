"""Host driver of the serving contexts: one dot_ctx per spatial dimension, each
stepped by its own host thread on its own HIP stream, so that 2D and 3D work
overlap on the device. Requests are queued from any thread; a context admits
them as its HBM budget and slots allow, steps every running instance together
and retires (then backfills) the ones that stop. With an FP64 finish, a
mixed-precision request that stops at its iteration cap without converging
(its FP32 state has levelled off above the tolerance) is handed, as a
checkpoint of its final state, to an FP64 context of the same dimension,
which continues that iterate (promoted exactly) up to a second cap. All
solver work runs inside the library; this module only moves requests,
checkpoints and timestamps.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

from . import binding as B


@dataclass
class Request:
    inst: object
    t_arrival: float = 0.0   # host clock when submitted
    t_done: float = 0.0      # host clock when the result reached host memory
    result: Optional[object] = None
    rho: Optional[object] = None
    m: Optional[List[object]] = None
    error: Optional[str] = None   # set when the context refused the request
    mixed_result: Optional[object] = None  # result at the mixed cap, when finished in FP64
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def finished_in_fp64(self) -> bool:
        return self.mixed_result is not None


class _Lane:
    """One context, its stream and the thread that steps it. `finish`: the
    FP64 lane that continues this lane's requests stopped at the cap."""

    def __init__(self, D, precision, budget, slots, step_iters, tol, max_iter, keep_solution, device,
                 finish: Optional["_Lane"] = None):
        import torch
        self.D = D
        self.precision = precision
        self.ctx = B.dot_ctx_create(D, precision, budget, slots, device=device)
        self.stream = torch.cuda.Stream()  # default priority
        self.step_iters = step_iters
        self.tol = tol
        self.max_iter = max_iter
        self.keep = keep_solution
        self.finish = finish
        if finish is not None:
            B.dot_ctx_keep_capped(self.ctx, True)
        self.inbox: List[Tuple[Request, Optional[bytes]]] = []
        self.running: Dict[int, Request] = {}
        self.cv = threading.Condition()
        self.stop = False
        self.abort = False
        self.error: Optional[BaseException] = None
        self.steps = 0
        self.active_sum = 0
        self.thread = threading.Thread(target=self._loop, daemon=True)

    def put(self, req: Request, checkpoint: Optional[bytes] = None):
        with self.cv:
            self.inbox.append((req, checkpoint))
            self.cv.notify()

    def pending(self) -> int:
        with self.cv:
            return len(self.inbox) + len(self.running)

    def _loop(self):
        try:
            h = self.stream.cuda_stream
            while True:
                with self.cv:
                    while not self.inbox and not self.running and not self.stop and not self.abort:
                        self.cv.wait(0.05)
                    if self.abort or (self.stop and not self.inbox and not self.running):
                        return
                    new, self.inbox = self.inbox, []
                for r, ck in new:
                    try:
                        if ck is None:
                            t = B.dot_ctx_submit(self.ctx, r.inst, tol=self.tol, max_iter=self.max_iter)
                        else:
                            t = B.dot_ctx_import(self.ctx, r.inst, ck, tol=self.tol, max_iter=self.max_iter)
                    except B.DotError as e:
                        r.error = str(e)
                        r.t_done = time.perf_counter()
                        r.done.set()
                        continue
                    with self.cv:
                        self.running[t] = r
                active, _ = B.dot_ctx_step(self.ctx, self.step_iters, h)
                self.steps += 1
                self.active_sum += active
                for t, r in list(self.running.items()):
                    if B.dot_ctx_poll(self.ctx, t) != B.CTX_DONE:
                        continue
                    ck = None
                    if self.finish is not None:
                        try:  # kept only for a request stopped at its cap
                            ck = B.dot_ctx_export(self.ctx, t, h)
                        except B.DotError:
                            ck = None
                    res, rho, m = B.dot_ctx_fetch(self.ctx, t)
                    if ck is not None and B.TERM_NAMES[res.term] == "maxiter":
                        r.mixed_result = res
                        with self.cv:
                            del self.running[t]
                        self.finish.put(r, ck)
                        continue
                    r.t_done = time.perf_counter()
                    r.result = res
                    if self.keep:
                        r.rho, r.m = rho, m
                    with self.cv:
                        del self.running[t]
                    r.done.set()
        except BaseException as e:  # surfaced by Server.check()
            self.error = e
            for r in self.running.values():
                r.done.set()


class Server:
    """Continuous-batching solver service on one GPU.

    budgets / slots: per spatial dimension D, the device bytes reserved for
    iterate state and the number of concurrently running instances.
    step_iters: iterations per context step (a multiple of 10); requests are
    admitted and retired between steps. device: HIP device of the contexts
    (-1: the current one). finish_fp64 (mixed precision only): requests that
    stop at max_iter without converging continue in an FP64 context of their
    dimension (finish_budgets / finish_slots) for up to finish_iters more
    iterations (max_iter and finish_iters multiples of 10)."""

    def __init__(self, precision=B.DOT_MIXED, budgets=None, slots=None, step_iters=40, tol=1e-6,
                 max_iter=40000, keep_solution=False, device=-1, finish_fp64=False, finish_iters=40000,
                 finish_budgets=None, finish_slots=None):
        budgets = budgets or {2: 64 << 30, 3: 24 << 30}
        slots = slots or {2: 128, 3: 16}
        self.finish_lanes: Dict[int, _Lane] = {}
        if finish_fp64 and precision == B.DOT_MIXED:
            if max_iter % 10 or finish_iters % 10:
                raise ValueError("max_iter and finish_iters must be multiples of 10")
            fb = finish_budgets or {D: b for D, b in budgets.items()}
            fs = finish_slots or {D: max(1, s // 4) for D, s in slots.items()}
            self.finish_lanes = {D: _Lane(D, B.DOT_FP64, fb[D], fs[D], step_iters, tol, max_iter + finish_iters,
                                          keep_solution, device) for D in budgets}
        self.lanes = {D: _Lane(D, precision, budgets[D], slots[D], step_iters, tol, max_iter, keep_solution, device,
                               finish=self.finish_lanes.get(D))
                      for D in budgets}
        for ln in self._all():
            ln.thread.start()

    def _all(self) -> List[_Lane]:
        return list(self.lanes.values()) + list(self.finish_lanes.values())

    def submit(self, inst) -> Request:
        r = Request(inst=inst, t_arrival=time.perf_counter())
        lane = self.lanes.get(inst.D)
        if lane is None:
            raise ValueError(f"no serving context for D={inst.D}")
        lane.put(r)
        return r

    def check(self):
        for ln in self._all():
            if ln.error is not None:
                raise ln.error

    def in_flight(self) -> int:
        return sum(ln.pending() for ln in self._all())

    def close(self):
        """Finish every submitted request (FP64 finishes included), then free
        the contexts."""
        self._stop(list(self.lanes.values()), abort=False)
        self._stop(list(self.finish_lanes.values()), abort=False)
        self._free()

    def abandon(self):
        """Stop stepping now; requests still queued or running stay unfinished."""
        self._stop(self._all(), abort=True)
        self._free()

    @staticmethod
    def _stop(lanes: List[_Lane], abort: bool):
        for ln in lanes:
            with ln.cv:
                if abort:
                    ln.abort = True
                else:
                    ln.stop = True
                ln.cv.notify()
        for ln in lanes:
            ln.thread.join()

    def _free(self):
        for ln in self._all():
            ln.ctx.close()
        self.check()
