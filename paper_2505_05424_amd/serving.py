"""Host driver of the serving contexts: one dot_ctx per spatial dimension, each
stepped by its own host thread on its own HIP stream, so that 2D and 3D work
overlap on the device. Requests are queued from any thread; a context admits
them as its HBM budget and slots allow, steps every running instance together
and retires (then backfills) the ones that stop. All solver work runs inside
the library; this module only moves requests and timestamps.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

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
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class _Lane:
    """One context, its stream and the thread that steps it."""

    def __init__(self, D, precision, budget, slots, step_iters, tol, max_iter, keep_solution, device):
        import torch
        self.D = D
        self.ctx = B.dot_ctx_create(D, precision, budget, slots, device=device)
        self.stream = torch.cuda.Stream()  # default priority
        self.step_iters = step_iters
        self.tol = tol
        self.max_iter = max_iter
        self.keep = keep_solution
        self.inbox: List[Request] = []
        self.running: Dict[int, Request] = {}
        self.cv = threading.Condition()
        self.stop = False
        self.abort = False
        self.error: Optional[BaseException] = None
        self.steps = 0
        self.active_sum = 0
        self.thread = threading.Thread(target=self._loop, daemon=True)

    def put(self, req: Request):
        with self.cv:
            self.inbox.append(req)
            self.cv.notify()

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
                for r in new:
                    try:
                        t = B.dot_ctx_submit(self.ctx, r.inst, tol=self.tol, max_iter=self.max_iter)
                    except B.DotError as e:
                        r.error = str(e)
                        r.t_done = time.perf_counter()
                        r.done.set()
                        continue
                    self.running[t] = r
                active, _ = B.dot_ctx_step(self.ctx, self.step_iters, h)
                self.steps += 1
                self.active_sum += active
                for t, r in list(self.running.items()):
                    if B.dot_ctx_poll(self.ctx, t) == B.CTX_DONE:
                        res, rho, m = B.dot_ctx_fetch(self.ctx, t)
                        r.t_done = time.perf_counter()
                        r.result = res
                        if self.keep:
                            r.rho, r.m = rho, m
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
    (-1: the current one)."""

    def __init__(self, precision=B.DOT_MIXED, budgets=None, slots=None, step_iters=40, tol=1e-6,
                 max_iter=40000, keep_solution=False, device=-1):
        budgets = budgets or {2: 64 << 30, 3: 24 << 30}
        slots = slots or {2: 128, 3: 16}
        self.lanes = {D: _Lane(D, precision, budgets[D], slots[D], step_iters, tol, max_iter, keep_solution, device)
                      for D in budgets}
        for ln in self.lanes.values():
            ln.thread.start()

    def submit(self, inst) -> Request:
        r = Request(inst=inst, t_arrival=time.perf_counter())
        lane = self.lanes.get(inst.D)
        if lane is None:
            raise ValueError(f"no serving context for D={inst.D}")
        lane.put(r)
        return r

    def check(self):
        for ln in self.lanes.values():
            if ln.error is not None:
                raise ln.error

    def in_flight(self) -> int:
        return sum(len(ln.inbox) + len(ln.running) for ln in self.lanes.values())

    def close(self):
        """Finish every submitted request, then free the contexts."""
        for ln in self.lanes.values():
            with ln.cv:
                ln.stop = True
                ln.cv.notify()
        self._join()

    def abandon(self):
        """Stop stepping now; requests still queued or running stay unfinished."""
        for ln in self.lanes.values():
            with ln.cv:
                ln.abort = True
                ln.cv.notify()
        self._join()

    def _join(self):
        for ln in self.lanes.values():
            ln.thread.join()
            ln.ctx.close()
        self.check()
