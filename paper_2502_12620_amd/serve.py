"""Continuous-batching request loop for DG solves on one GPU.

Requests (a forest and a step count) arrive over time.  Each (dim, degree)
class has a pool: a device-resident arena of leaf slots whose size is the
class's share of an HBM budget.  A request is admitted as soon as its class
pool has a free member id and a contiguous free slot range for its leaves
(first come, first served within a class); its initial state is projected
straight into the arena.  Every tick advances every admitted member of every
pool by one SSP-RK3 step, each pool on its own HIP stream so the pools'
kernels overlap on the device; members that reach their step count are
copied out (optionally), released, and their slots admit waiting requests
at the next tick.  A member's arithmetic does not depend on the other
members, so each result is the same alone and in the mix.

Argument marshalling and scheduling only: every step runs in the HIP
library through the pool C-ABI.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import torch

from . import dgamr as G


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    workload: object        # workloads.Workload (dim, degree, n_cell, roots, ... steps, cfl)
    admitted: float = -1.0
    done: float = -1.0
    dofs: int = 0
    result: object = None   # device tensor of the final state when kept


@dataclass
class _Member:
    req: Request
    forest: object
    member: int
    first: int
    n_leaves: int
    steps_left: int


@dataclass
class _Class:
    pool: object
    stream: object
    waiting: collections.deque = field(default_factory=collections.deque)
    members: dict = field(default_factory=dict)


class Server:
    """Pools for the given classes [(dim, degree, n_cell), ...], each sized
    to an equal share of hbm_budget bytes (state arena + work buffer)."""

    def __init__(self, classes, hbm_budget: float, max_members: int = 512, precision=G.FP64,
                 keep_results: bool = False, tune: bool = False):
        self.keep = keep_results
        self.precision = precision
        self.classes = {}
        share = hbm_budget / len(classes)
        for dim, degree, n_cell in classes:
            nb = {2: [1, 3, 6, 10], 3: [1, 4, 10, 20]}[dim][degree]
            leaf = 8 * (dim + 2) * nb * n_cell ** dim
            guard = 8 * 2 * dim * (dim + 2) * nb * n_cell ** (dim - 1)
            per_leaf = 3 * leaf + guard + 8  # arena + two stage buffers + guard + leaf maximum
            cap = max(1, int(share // per_leaf))
            pool = G.Pool(dim, degree, n_cell, cap, max_members, precision=precision)
            self.classes[(dim, degree, n_cell)] = _Class(pool, torch.cuda.Stream())
        self.tuned = {}
        self.tune = tune
        self.full_waits = 0  # admissions deferred for lack of slots or member ids
        self._forests = {}   # topology of waiting requests, built once

    def _admit(self, c: _Class, now: float) -> bool:
        req = c.waiting[0]
        w = req.workload
        f = self._forests.get(req.rid)
        if f is None:
            f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma,
                         precision=self.precision)
            self._forests[req.rid] = f
        try:
            mid, first = c.pool.admit(f, w.cfl, stream=c.stream)
        except G.DgamrError as e:
            if e.code == G.EFULL:
                self.full_waits += 1
                return False
            raise
        with torch.cuda.stream(c.stream):
            f.project_ic(w.ic_kind, w.ic_params, u=c.pool.view(first, f.n_leaves), stream=c.stream)
        c.waiting.popleft()
        del self._forests[req.rid]
        req.admitted = now
        req.dofs = f.n_leaves * (w.dim + 2) * f.nb * f.ncell
        c.members[mid] = _Member(req, f, mid, first, f.n_leaves, w.steps)
        return True

    def run(self, requests, clock=time.perf_counter, on_done=None):
        """Serve the requests (sorted by arrival) until all are done; returns
        them with admitted / done times (seconds after the start).  on_done,
        if given, is called with each finished request."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        total = len(pending)
        finished = []
        t0 = clock()
        self.ticks = 0
        for c in self.classes.values():
            c.pool.u.zero_()
        torch.cuda.synchronize()
        while len(finished) < total:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                w = r.workload
                key = (w.dim, w.degree, w.n_cell)
                if key not in self.classes:
                    raise ValueError(f"no pool for class {key}")
                self.classes[key].waiting.append(r)
            for c in self.classes.values():
                while c.waiting and self._admit(c, now):
                    pass
            active = [c for c in self.classes.values() if c.members]
            if not active:
                if pending:
                    wait = pending[0].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                    continue
                stuck = [c.waiting[0].rid for c in self.classes.values() if c.waiting]
                raise RuntimeError(f"requests {stuck} never fit their pool")
            if self.tune:
                for key, c in self.classes.items():
                    if c.members and key not in self.tuned:
                        torch.cuda.synchronize()
                        self.tuned[key] = c.pool.autotune(stream=c.stream)
            for c in active:
                c.pool.step(stream=c.stream)
            for c in active:
                c.stream.synchronize()
            self.ticks += 1
            now = clock() - t0
            for c in active:
                for mid in list(c.members):
                    m = c.members[mid]
                    m.steps_left -= 1
                    if m.steps_left == 0:
                        if self.keep:
                            with torch.cuda.stream(c.stream):
                                m.req.result = c.pool.view(m.first, m.n_leaves).clone()
                        c.pool.release(mid, stream=c.stream)
                        m.req.done = now
                        finished.append(m.req)
                        del c.members[mid]
                        if on_done is not None:
                            on_done(m.req)
            if self.keep:
                for c in active:
                    c.stream.synchronize()
        self.makespan = clock() - t0
        return finished
