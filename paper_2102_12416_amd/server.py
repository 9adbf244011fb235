"""A solve server: continuous batching of independent Jacobi3D solves.

Requests (cubic grids of different sizes, binary64 or binary32-refined)
arrive over time.  The loop keeps every admitted solve's fields, halos and
face buffers resident in HBM and sweeps all of them in shared launches (a
libjc group).  At every window boundary (every `window` sweeps) it:

  1. admits queued requests, oldest first, while their device footprint
     fits the free HBM budget (the head of the queue waits for memory;
     a request larger than the whole budget is rejected);
  2. computes every member's residual norm in one batched pass (for the
     refined solves this is their binary64 outer step);
  3. retires members that reached the relative tolerance or the sweep cap
     (their result is copied out, their arena freed);
  4. rebuilds the group if membership changed and runs the next window.

Latency = retirement time - arrival time.  The schedule of a solve (its
windows, checks and stop) depends only on its own data, and a group's
tile shape is fixed, so every result is bitwise the same alone and in any
mix.
"""
from __future__ import annotations

import sys
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from .solver import Group, Solver, synth_field


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    n: int                  # cubic interior edge
    precision: str          # "f64" (plain Jacobi) or "f32" (binary32-refined)
    seed: int


@dataclass
class Result:
    id: int
    n: int
    precision: str
    arrival: float
    admitted: float = 0.0
    finished: float = 0.0
    iters: int = 0
    rel_resid: float = float("nan")
    converged: bool = False
    rejected: bool = False
    field: object = None    # host numpy array of the final iterate (keep_fields)

    @property
    def latency(self):
        return self.finished - self.arrival


def request_footprint(n: int, precision: str) -> int:
    """Device bytes of one admitted solve (its context arena): one block of
    n^3 with a source, plus binary32 refinement buffers for "f32"."""
    import ctypes

    from . import _lib as L
    opt = L.Options()
    opt.mode = L.JC_MODE_FUSED
    opt.with_source = 1
    opt.ir_dtype = L.JC_NONE
    if precision == "f32":
        opt.ir_enable = 1
        opt.ir_dtype = L.JC_F32
    fp = ctypes.c_size_t()
    L.check(L.lib.jc_footprint(L.i64((n, n, n)), L.i64((n, n, n)), ctypes.byref(opt), ctypes.byref(fp)))
    return int(fp.value)


@dataclass
class _Live:
    req: Request
    solver: Solver
    res: Result
    bytes: int
    r0: float = -1.0


class Server:
    """Continuous-batching Jacobi3D solve server on one GPU."""

    def __init__(self, budget_bytes: int, window: int = 50, rtol: float = 1e-10, max_iter: int = 20000,
                 device: str = "cuda:0", keep_fields: bool = False, use_graphs: bool = True,
                 progress_every: float = 0.0):
        if window < 1 or max_iter % window:
            raise ValueError("max_iter must be a multiple of the window")
        self.budget = int(budget_bytes)
        self.window = int(window)
        self.rtol = float(rtol)
        self.max_iter = int(max_iter)
        self.device = torch.device(device)
        self.keep_fields = keep_fields
        self.use_graphs = use_graphs
        self.stream = torch.cuda.Stream(device=self.device)
        self.max_members = 4096
        self.stats = dict(windows=0, group_builds=0, peak_members=0, peak_bytes=0)
        self.progress_every = float(progress_every)   # seconds between progress lines (0: none)

    # ---------------------------------------------------------------- admit
    def _admit(self, req: Request, now: float) -> _Live:
        n = req.n
        ir = "f32" if req.precision == "f32" else None
        s = Solver((n, n, n), mode="fused", with_source=True, ir_dtype=ir, device=str(self.device),
                   use_graphs=False)
        with torch.cuda.stream(s.stream):
            g = synth_field((n, n, n), req.seed, 0, device=str(self.device), stream=s.stream)
            b = synth_field((n, n, n), req.seed, 1, device=str(self.device), stream=s.stream)
        s.load(g, b)
        g.record_stream(s.stream)
        b.record_stream(s.stream)
        del g, b
        res = Result(id=req.id, n=n, precision=req.precision, arrival=req.arrival, admitted=now)
        return _Live(req=req, solver=s, res=res, bytes=s.footprint)

    def _retire(self, live: _Live, now: float, rel: float):
        live.res.finished = now
        live.res.iters = live.solver.iterations
        live.res.rel_resid = rel
        live.res.converged = rel <= self.rtol
        if self.keep_fields:
            live.res.field = live.solver.store().cpu().numpy()
        live.solver.close()

    # ------------------------------------------------------------------ run
    def run(self, requests, realtime: bool = True):
        """Serve `requests` (Request objects); returns the list of Results.

        realtime: requests become visible at their arrival time on the wall
        clock; otherwise all are queued at once (closed-loop capacity)."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.id))
        incoming = deque(reqs)
        queue: deque = deque()
        active: list[_Live] = []
        done: list[Result] = []
        used = 0
        group = None
        members_key = None
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        last_report = 0.0
        while incoming or queue or active:
            now = clock()
            if self.progress_every > 0 and now - last_report >= self.progress_every:
                last_report = now
                print("[serve] t=%.1fs done=%d active=%d queued=%d arriving=%d windows=%d"
                      % (now, len(done), len(active), len(queue), len(incoming), self.stats["windows"]),
                      file=sys.stderr, flush=True)
            while incoming and (not realtime or incoming[0].arrival <= now):
                queue.append(incoming.popleft())
            # admission by footprint, oldest first
            changed = False
            while queue and len(active) < self.max_members:
                head = queue[0]
                need = request_footprint(head.n, head.precision)
                if need > self.budget:
                    queue.popleft()
                    done.append(Result(id=head.id, n=head.n, precision=head.precision, arrival=head.arrival,
                                       finished=clock(), rejected=True))
                    continue
                if used + need > self.budget:
                    break
                queue.popleft()
                if group is not None:
                    group.close()
                    group = None
                live = self._admit(head, clock())
                active.append(live)
                used += live.bytes
                changed = True
            self.stats["peak_members"] = max(self.stats["peak_members"], len(active))
            self.stats["peak_bytes"] = max(self.stats["peak_bytes"], used)
            if not active:
                if incoming and realtime:
                    time.sleep(max(0.0, min(0.05, incoming[0].arrival - clock())))
                continue
            key = tuple(l.req.id for l in active)
            if group is None or key != members_key:
                if group is not None:
                    group.close()
                group = Group([l.solver for l in active], use_graphs=self.use_graphs, stream=self.stream)
                members_key = key
                self.stats["group_builds"] += 1
            # window boundary: residuals of everyone, retire finished solves
            norms = group.residuals()
            now = clock()
            keep = []
            for live, r in zip(active, norms):
                if live.r0 < 0:
                    live.r0 = r
                rel = r / live.r0 if live.r0 > 0 else 0.0
                if rel <= self.rtol or live.solver.iterations >= self.max_iter:
                    keep.append(None)
                    self._retire(live, now, rel)
                    used -= live.bytes
                    done.append(live.res)
                else:
                    keep.append(live)
            if any(k is None for k in keep):
                active = [k for k in keep if k is not None]
                group.close()
                group = None
                if not active:
                    continue
                group = Group([l.solver for l in active], use_graphs=self.use_graphs, stream=self.stream)
                members_key = tuple(l.req.id for l in active)
                self.stats["group_builds"] += 1
            # every active solve has done a whole number of windows and is
            # below its cap, which is a multiple of the window
            group.iterate(self.window)
            self.stats["windows"] += 1
        if group is not None:
            group.close()
        torch.cuda.synchronize(self.device)
        return sorted(done, key=lambda r: r.id)


def summarize(results, makespan: float):
    """p50/p99 latency, solves/s and the converged / capped / rejected split."""
    served = [r for r in results if not r.rejected]
    lat = np.array([r.latency for r in served]) if served else np.zeros(1)
    return dict(
        requests=len(results),
        served=len(served),
        rejected=sum(r.rejected for r in results),
        converged=sum(r.converged for r in served),
        capped=sum((not r.converged) for r in served),
        p50_s=float(np.percentile(lat, 50)),
        p99_s=float(np.percentile(lat, 99)),
        mean_s=float(lat.mean()),
        solves_per_s=len(served) / makespan if makespan > 0 else 0.0,
        makespan_s=makespan,
    )
