"""Continuous-batching request loop for DG solves on one GPU.

Requests (a forest and a step count) arrive over time.  Each (dim, degree,
n_cell) class has a pool: a device-resident arena of leaf slots, stepped as
one.  All pools share one HBM budget, counted in bytes of arena and work
buffer per leaf slot: a class's pool is created at its first admission,
grows when a request of the class does not fit (rebuilt larger, its members
moved over), and pools that hold more slots than they use give them back
when another class needs the room.  Waiting requests are admitted in
arrival order across all classes: the oldest one as soon as its footprint
fits the budget (growing its pool), later ones meanwhile only into free
slots of their pools, so a large request is not starved by small ones.
The initial state is projected straight into the arena.

Each class advances on its own HIP stream: the host keeps up to `depth`
steps of every active pool queued on that pool's stream and never waits on
all of them at once; it waits only on the oldest queued step of some class
when there is nothing else to do.  A member's last step is followed on the
class's stream by the copy of its result (when kept) and its release, so its
slots take new requests without stopping the other classes.  A request is
done when the host sees the event after its last step complete.  A member's
arithmetic does not depend on the other members, so each result is the same
alone and in the mix.

Argument marshalling and scheduling only: every step runs in the HIP
library through the pool C-ABI.
"""
from __future__ import annotations

import collections
import math
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
    key: tuple
    stream: object
    per_leaf: int           # bytes of arena + work per leaf slot
    pool: object = None
    capacity: int = 0       # leaf slots of the current pool
    members: dict = field(default_factory=dict)
    inflight: collections.deque = field(default_factory=collections.deque)  # (event, finished requests, seq)
    version: int = 0        # bumped when slots are released or the pool is rebuilt
    fail: tuple = (-1, 0)   # (version, fewest leaves that did not fit at that version)

    def used(self) -> int:
        return sum(m.n_leaves for m in self.members.values())


def slot_bytes(dim: int, degree: int, n_cell: int) -> int:
    """Bytes per leaf slot of a pool: the arena's state, the two stage
    states and the guard traces of the work buffer, and the leaf maximum."""
    nb = {2: [1, 3, 6, 10], 3: [1, 4, 10, 20]}[dim][degree]
    leaf = 8 * (dim + 2) * nb * n_cell ** dim
    guard = 8 * 2 * dim * (dim + 2) * nb * n_cell ** (dim - 1)
    return 3 * leaf + guard + 8


class Server:
    """Pools for the given classes [(dim, degree, n_cell), ...] within one
    budget of hbm_budget bytes (arenas and work buffers)."""

    def __init__(self, classes, hbm_budget: float, max_members: int = 512, precision=G.FP64,
                 keep_results: bool = False, tune: bool = False, depth: int = 2):
        self.keep = keep_results
        self.precision = precision
        self.budget = int(hbm_budget)
        self.max_members = max_members
        self.depth = max(1, depth)
        self.classes = {tuple(k): _Class(tuple(k), torch.cuda.Stream(), slot_bytes(*k)) for k in classes}
        self.tuned = {}
        self.tune = tune
        self.full_waits = 0  # admission attempts deferred for lack of room or member ids
        self.rebuilds = 0    # pools created, or rebuilt to grow or give back slots
        self.moved = 0       # members moved by rebuilds
        self.peak_bytes = 0
        self._forests = {}   # topology of waiting requests, built once

    # ------------------------------------------------------------ budget
    def allocated(self, skip=None) -> int:
        return sum(c.capacity * c.per_leaf for c in self.classes.values() if c is not skip)

    def _rebuild(self, c: _Class, capacity: int):
        """Replace c's pool by one of `capacity` slots, its members re-admitted
        (packed from slot 0) with their states copied over on c's stream."""
        c.stream.synchronize()
        old, members = c.pool, sorted(c.members.values(), key=lambda m: m.first)
        c.pool, c.capacity, c.members = None, 0, {}
        if capacity > 0:
            dim, degree, n_cell = c.key
            pool = G.Pool(dim, degree, n_cell, capacity, self.max_members, precision=self.precision)
            for m in members:
                mid, first = pool.admit(m.forest, m.req.workload.cfl, stream=c.stream)
                with torch.cuda.stream(c.stream):
                    pool.view(first, m.n_leaves).copy_(old.view(m.first, m.n_leaves))
                m.member, m.first = mid, first
                c.members[mid] = m
                self.moved += 1
            c.pool, c.capacity = pool, capacity
            self.tuned.pop(c.key, None)
        c.version += 1
        c.stream.synchronize()  # the old arena is no longer read
        del old
        self.rebuilds += 1

    def _make_room(self, c: _Class, need: int) -> bool:
        """Give c's pool room for `need` more leaves within the budget: grow
        it (by half again at least, as far as the budget allows), shrinking
        other pools to what they use only when that makes the request fit,
        idle pools first and no more of them than needed.  Nothing is rebuilt
        when it would not fit anyway."""
        used = c.used()
        free = self.budget - self.allocated(skip=c)
        if free // c.per_leaf < used + need:
            spare = sum((o.capacity - o.used()) * o.per_leaf for o in self.classes.values() if o is not c)
            if (free + spare) // c.per_leaf < used + need:
                return False
            # give back only what is missing: idle pools first (nothing to
            # move), then the pools with the most spare bytes
            others = sorted((o for o in self.classes.values() if o is not c and o.capacity > o.used()),
                            key=lambda o: (len(o.members) > 0, -(o.capacity - o.used()) * o.per_leaf))
            for o in others:
                if free // c.per_leaf >= used + need:
                    break
                self._rebuild(o, o.used())
                free = self.budget - self.allocated(skip=c)
        self._rebuild(c, min(max(used + need, math.ceil(1.5 * c.capacity)), free // c.per_leaf))
        return True

    # ------------------------------------------------------------ admission
    def _admit(self, req: Request, now: float, may_grow: bool) -> bool:
        w = req.workload
        c = self.classes.get((w.dim, w.degree, w.n_cell))
        if c is None:
            raise ValueError(f"no pool for class {(w.dim, w.degree, w.n_cell)}")
        f = self._forests.get(req.rid)
        if f is None:
            f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma,
                         precision=self.precision)
            self._forests[req.rid] = f
        if f.n_leaves * c.per_leaf > self.budget:
            raise RuntimeError(f"request {req.rid} ({f.n_leaves} leaves) exceeds the whole HBM budget")
        if not may_grow and c.fail[0] == c.version and f.n_leaves >= c.fail[1]:
            return False  # a request this large did not fit the pool as it is
        for attempt in range(2):
            if c.pool is not None and len(c.members) < self.max_members:
                try:
                    mid, first = c.pool.admit(f, w.cfl, stream=c.stream)
                    break
                except G.DgamrError as e:
                    if e.code != G.EFULL:
                        raise
            if (attempt == 1 or not may_grow or len(c.members) >= self.max_members
                    or not self._make_room(c, f.n_leaves)):
                self.full_waits += 1
                if c.fail[0] != c.version or f.n_leaves < c.fail[1]:
                    c.fail = (c.version, f.n_leaves)
                return False
        with torch.cuda.stream(c.stream):
            f.project_ic(w.ic_kind, w.ic_params, u=c.pool.view(first, f.n_leaves), stream=c.stream)
        del self._forests[req.rid]
        req.admitted = now
        req.dofs = f.n_leaves * (w.dim + 2) * f.nb * f.ncell
        c.members[mid] = _Member(req, f, mid, first, f.n_leaves, w.steps)
        self.peak_bytes = max(self.peak_bytes, self.allocated())
        return True

    # ------------------------------------------------------------ stepping
    def _enqueue_step(self, c: _Class):
        c.pool.step(stream=c.stream)
        finished = []
        for mid in list(c.members):
            m = c.members[mid]
            m.steps_left -= 1
            if m.steps_left == 0:
                if self.keep:
                    with torch.cuda.stream(c.stream):
                        m.req.result = c.pool.view(m.first, m.n_leaves).clone()
                c.pool.release(mid, stream=c.stream)
                del c.members[mid]
                c.version += 1
                finished.append(m.req)
        ev = torch.cuda.Event()
        ev.record(c.stream)
        c.inflight.append((ev, finished, self.steps_enqueued))
        self.steps_enqueued += 1

    def run(self, requests, clock=time.perf_counter, on_done=None):
        """Serve the requests until all are done; returns them with admitted /
        done times (seconds after the start).  on_done, if given, is called
        with each finished request."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        total = len(pending)
        waiting = []  # arrived, not admitted, in arrival order
        finished = []
        self.steps_enqueued = 0
        torch.cuda.synchronize()
        t0 = clock()

        def complete(c, block):
            ev, reqs, _ = c.inflight[0]
            if block:
                ev.synchronize()
            elif not ev.query():
                return False
            c.inflight.popleft()
            t = clock() - t0
            for r in reqs:
                r.done = t
                finished.append(r)
                if on_done is not None:
                    on_done(r)
            return True

        while len(finished) < total:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            progressed = False
            for c in self.classes.values():
                while c.inflight and complete(c, False):
                    progressed = True
            if waiting:
                # arrival order; only the oldest waiting request may grow a
                # pool (and shrink others), later ones fill free slots
                still = []
                for r in waiting:
                    if self._admit(r, now, may_grow=not still):
                        progressed = True
                    else:
                        still.append(r)
                waiting = still
            if self.tune:
                for key, c in self.classes.items():
                    if c.members and key not in self.tuned:
                        c.stream.synchronize()
                        self.tuned[key] = c.pool.autotune(stream=c.stream)
            for c in self.classes.values():
                while c.members and len(c.inflight) < self.depth:
                    self._enqueue_step(c)
                    progressed = True
            if progressed:
                continue
            busy = [c for c in self.classes.values() if c.inflight]
            if busy:
                # nothing to do until some queued step completes: wait on the
                # class whose oldest queued step was queued first
                complete(min(busy, key=lambda c: c.inflight[0][2]), True)
                continue
            if pending:
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
                continue
            stuck = [r.rid for r in waiting]
            raise RuntimeError(f"requests {stuck} never fit the HBM budget")
        self.makespan = clock() - t0
        torch.cuda.synchronize()
        return finished
