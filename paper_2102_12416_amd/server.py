"""A solve server: continuous batching of independent Jacobi3D solves.

Requests (cubic grids of different sizes, binary64 or binary32-refined)
arrive over time.  The loop keeps every admitted solve's fields, halos and
face buffers resident in HBM and sweeps them in shared launches (libjc
groups).  Requests are split into size lanes; each lane has its own stream,
group and window cadence, so the windows of small solves (tens of
microseconds) never wait behind those of large ones (milliseconds), and
the lanes' launches overlap on the device.

The loop admits queued requests, oldest first, while their device
footprint fits the free HBM budget (the head of the queue waits for memory;
a request larger than the whole budget is rejected) and hands each to its
lane.  At every window boundary of a lane (every `window` sweeps) it:

  1. lets the lane's newly admitted requests join;
  2. computes every member's residual norm in one batched pass (for the
     refined solves this is their binary64 outer step);
  3. retires members that reached the relative tolerance or the sweep cap
     (their result is copied out, their arena freed);
  4. rebuilds the lane's group if membership changed and enqueues the next
     window.

Latency = retirement time - arrival time.  The schedule of a solve (its
windows, checks and stop) depends only on its own data, and every group
uses the same tile shape, so every result is bitwise the same alone, in
any mix and in any lane.
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


# the largest cubic edge a resident block takes: at most 32 planes, (n + 1) / 2 * n
# <= 512 cell pairs and 8 (4 n n' + 2 n n + 2 n n') <= 64 KiB of LDS (n' = n rounded up to even)
RESIDENT_MAX_EDGE = 32


class _Lane:
    """Requests of one size class: their own stream, group and window
    cadence, so a small solve never waits for the windows of large ones."""

    def __init__(self, max_edge, device, resident=False):
        self.max_edge = max_edge          # largest edge in this lane (None: unbounded)
        self.resident = resident          # resident sweeps: one work-group per member, one launch per window
        self.stream = torch.cuda.Stream(device=device)
        self.active: list[_Live] = []
        self.pending: list[_Live] = []    # admitted, joining at the next window boundary
        self.group = None
        self.key = None
        self.done = None                  # event: the last enqueued window has finished
        self.windows = 0

    def busy(self):
        return self.done is not None and not self.done.query()

    def close(self):
        if self.group is not None:
            self.group.close()
            self.group = None


class Server:
    """Continuous-batching Jacobi3D solve server on one GPU.

    lanes: ascending edge bounds of the size classes; a request of edge n
    joins the first lane with n <= bound, else the last (unbounded) lane.
    An empty tuple serves everything in one group.  temporal: every size
    class gets a lane per precision, and every lane sweeps twice (True) or
    three times (3) per launch (results bitwise the same).  resident: binary64
    requests whose grid fits one compute unit (edges up to 32) go to a lane
    of their own that sweeps each window in one launch with one work-group
    per request (results bitwise the same)."""

    def __init__(self, budget_bytes: int, window: int = 50, rtol: float = 1e-10, max_iter: int = 20000,
                 device: str = "cuda:0", keep_fields: bool = False, use_graphs: bool = True,
                 progress_every: float = 0.0, lanes=(64, 160), tile=None, temporal: bool = False,
                 resident: bool = False):
        if window < 1 or max_iter % window:
            raise ValueError("max_iter must be a multiple of the window")
        bounds = [int(v) for v in lanes]
        if any(b < 1 for b in bounds) or bounds != sorted(set(bounds)):
            raise ValueError("lane bounds must be ascending positive edges")
        self.budget = int(budget_bytes)
        self.window = int(window)
        self.rtol = float(rtol)
        self.max_iter = int(max_iter)
        self.device = torch.device(device)
        self.keep_fields = keep_fields
        self.use_graphs = use_graphs
        self.lane_bounds = tuple(bounds)
        # one tile shape for every group (None: the library's group default,
        # 64 x 8 x 32, which measured best for the served mix): a member's
        # residual norms, and so its stopping check, then do not depend on
        # who else is in the group
        self.tile = None if tile is None else tuple(int(v) for v in tile)
        # temporal: every lane's group sweeps twice (True) or three times (3)
        # per launch (bitwise the same results), and the size lanes are kept
        # per precision
        self.temporal = 3 if temporal == 3 else bool(temporal)
        if self.temporal is True and self.window % 2:
            raise ValueError("two sweeps per launch need an even window")
        self.resident = bool(resident)
        self.max_members = 4096
        self.stats = dict(windows=0, group_builds=0, peak_members=0, peak_bytes=0, lane_windows=[])
        self.progress_every = float(progress_every)   # seconds between progress lines (0: none)

    # ---------------------------------------------------------------- admit
    def _admit(self, req: Request, now: float, stream) -> _Live:
        n = req.n
        ir = "f32" if req.precision == "f32" else None
        s = Solver((n, n, n), mode="fused", with_source=True, ir_dtype=ir, device=str(self.device),
                   use_graphs=False, stream=stream)
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

    def _lane_of(self, lanes, n):
        for lane in lanes[:-1]:
            if n <= lane.max_edge:
                return lane
        return lanes[-1]

    def _regroup(self, lane):
        lane.close()
        if lane.active:
            # a resident lane's window is one launch per kernel variant: a
            # graph of it would save nothing and cost an instantiation per
            # membership change
            lane.group = Group([l.solver for l in lane.active], use_graphs=self.use_graphs and not lane.resident,
                               stream=lane.stream, tile=self.tile, temporal=False if lane.resident else self.temporal,
                               resident=lane.resident)
            lane.key = tuple(l.req.id for l in lane.active)
            self.stats["group_builds"] += 1

    def _boundary(self, lane, clock, done) -> int:
        """One window boundary of an idle lane: members join, every member's
        residual is taken, finished ones retire, the next window is
        enqueued.  Returns the device bytes released."""
        if lane.pending:
            lane.active += lane.pending
            lane.pending = []
        if lane.group is None or lane.key != tuple(l.req.id for l in lane.active):
            self._regroup(lane)
        # the stopping rule runs in the library: |r| / |r_0| <= rtol or the cap
        checks = lane.group.check(self.rtol, self.max_iter)
        now = clock()
        freed = 0
        keep = []
        for live, (rel, stop) in zip(lane.active, checks):
            if stop:
                self._retire(live, now, rel)
                freed += live.bytes
                done.append(live.res)
            else:
                keep.append(live)
        if len(keep) != len(lane.active):
            lane.active = keep
            self._regroup(lane)
        if lane.active:
            # every active solve has done a whole number of windows and is
            # below its cap, which is a multiple of the window
            lane.group.iterate(self.window)
            lane.done = torch.cuda.Event()
            lane.done.record(lane.stream)
            lane.windows += 1
            self.stats["windows"] += 1
        return freed

    # ------------------------------------------------------------------ run
    def run(self, requests, realtime: bool = True):
        """Serve `requests` (Request objects); returns the list of Results.

        realtime: requests become visible at their arrival time on the wall
        clock; otherwise all are queued at once (closed-loop capacity)."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.id))
        incoming = deque(reqs)
        queue: deque = deque()
        keys = ("f64", "f32") if self.temporal else (None,)
        lane_sets = {k: [_Lane(b, self.device) for b in self.lane_bounds] + [_Lane(None, self.device)]
                     for k in keys}
        lanes = [lane for k in keys for lane in lane_sets[k]]
        small = _Lane(RESIDENT_MAX_EDGE, self.device, resident=True) if self.resident else None
        if small is not None:
            lanes.append(small)
        done: list[Result] = []
        used = 0
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        def members():
            return sum(len(l.active) + len(l.pending) for l in lanes)

        last_report = 0.0
        while incoming or queue or any(l.active or l.pending for l in lanes):
            now = clock()
            if self.progress_every > 0 and now - last_report >= self.progress_every:
                last_report = now
                print("[serve] t=%.1fs done=%d active=%d queued=%d arriving=%d windows=%s"
                      % (now, len(done), members(), len(queue), len(incoming), [l.windows for l in lanes]),
                      file=sys.stderr, flush=True)
            while incoming and (not realtime or incoming[0].arrival <= now):
                queue.append(incoming.popleft())
            # admission by footprint, oldest first; a request joins its
            # lane at that lane's next window boundary
            while queue and members() < self.max_members:
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
                if small is not None and head.precision == "f64" and head.n <= RESIDENT_MAX_EDGE:
                    lane = small
                else:
                    lane = self._lane_of(lane_sets[head.precision if self.temporal else None], head.n)
                live = self._admit(head, clock(), lane.stream)
                lane.pending.append(live)
                used += live.bytes
            self.stats["peak_members"] = max(self.stats["peak_members"], members())
            self.stats["peak_bytes"] = max(self.stats["peak_bytes"], used)
            progressed = False
            for lane in lanes:
                if (lane.active or lane.pending) and not lane.busy():
                    used -= self._boundary(lane, clock, done)
                    progressed = True
            if not progressed:
                if not any(l.active or l.pending for l in lanes):
                    if incoming and realtime:
                        time.sleep(max(0.0, min(0.05, incoming[0].arrival - clock())))
                else:
                    time.sleep(0)
        for lane in lanes:
            lane.close()
        torch.cuda.synchronize(self.device)
        self.stats["lane_windows"] = [l.windows for l in lanes]
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
