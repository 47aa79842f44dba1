"""Serving loop: continuous batching of rebuild requests for moving particle
systems.

The paper motivates fast data-structure construction by dynamic problems in
which particles move every time step and the structures are rebuilt each step
(Section 1, Section 2.5). This module serves a stream of such rebuild requests
on one GPU:

- every request names a system; it displaces the system's points by
  N(0, sigma^2) per coordinate (fmmds_displace: counter-based normals seeded
  by system and step, clamped into the unit cube) and rebuilds its tables
  and lists;
- requests wait in arrival order; whenever one of `n_slots` streams is free,
  the waiting requests (at most one per system, since a system's steps are
  sequential) are packed into one batched build (fmmds_batch_*) and launched
  on that stream, so work from different ticks overlaps on the device;
- a batch of the same systems on the same slot is planned once and kept: its
  input buffer and its HIP graph (captured at the first launch) are reused by
  every later batch of those systems there, so a repeated batch costs one
  displacement and one graph launch on the host;
- a new plan is admitted only if its device footprint (fmmds_batch_footprint
  plus its input buffer) fits the HBM budget next to everything resident;
  planned batches are freed least recently used first, first those that hold
  no system's current tables, then (with nothing in flight) any idle one
  (their systems are rebuilt from scratch on their next request); a request
  that does not fit an empty budget fails with ERR_NOMEM;
- each system keeps its latest tables resident on the GPU (a view into the
  batch that built them) until its next request reuses that batch or the
  batch is freed.

All compute is the library's; this is host scheduling only. The sequential
baseline replays the same arrival trace with one fmmds_build per request on
one stream.
"""
from __future__ import annotations

import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I

ONE_MINUS_ULP = 1.0 - 2.0 ** -24


@dataclass
class Request:
    rid: int
    system: int
    arrival: float
    step: int = -1
    launched: float = -1.0
    done: float = -1.0


@dataclass
class _Entry:
    """A planned batch for one (slot, system tuple), kept for reuse: its
    input buffer and, after the first launch, its captured graph are replayed
    by later batches of the same systems on the same slot."""
    key: tuple
    slot: int
    batch: object
    xbuf: object
    nbytes: int
    refs: int = 0          # systems whose resident tables are this batch's
    in_flight: bool = False
    launches: int = 0


@dataclass
class _Slot:
    stream: object
    entry: object = None
    event: object = None
    reqs: list = field(default_factory=list)


class Server:
    def __init__(self, systems, levels, *, n_slots: int = 4, hbm_budget: int | None = None,
                 max_batch_points: int = 1 << 24, max_batch_sets: int = 64,
                 sigma: float = 1e-3, seed: int = 8, keep_inputs=(),
                 stall_seconds: float = 60.0, graphs: bool = True):
        import torch
        import paper_1301_1704_amd as F
        self.torch, self.F = torch, F
        self.levels = [int(v) for v in levels]
        self.x0 = [np.ascontiguousarray(p, dtype=np.float32) for p in systems]
        self.n = [p.shape[0] for p in self.x0]
        self.sigma, self.seed = sigma, seed
        self.max_batch_points, self.max_batch_sets = max_batch_points, max_batch_sets
        self.slots = [_Slot(stream=torch.cuda.Stream()) for _ in range(n_slots)]
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.5 * free)
        self.budget = hbm_budget
        self.keep_inputs = set(keep_inputs)  # request ids whose inputs are kept (tests)
        self.stall_seconds = stall_seconds
        self.graphs = graphs
        self._prewarm()
        self.reset()

    def _prewarm(self):
        """One-time initialization (the displacement and batched-build code on
        every stream) before any request is timed."""
        torch, F = self.torch, self.F
        pts = np.ascontiguousarray(I.uniform_points(1, 300))
        for slot in self.slots:
            with torch.cuda.stream(slot.stream):
                x = torch.from_numpy(pts).cuda()
                F.displace([(x, 1, 0)], 0.0, stream=slot.stream)
            b = F.Batch(np.asarray([0, 100, 300], np.uint64), np.asarray([2, 3], np.uint8),
                        stream=slot.stream)
            b.launch(x, capture=self.graphs)
            b.wait()
            b.free()
        torch.cuda.synchronize()

    # ------------------------------------------------------------- state
    def reset(self, keep_plans: bool = False):
        """Systems back to their initial points; with keep_plans the planned
        batches (and their graphs) stay for reuse, holding no tables."""
        torch = self.torch
        torch.cuda.synchronize()
        entries = getattr(self, "entries", None) or OrderedDict()
        if keep_plans:
            for e in entries.values():
                e.refs, e.in_flight = 0, False
        else:
            for e in entries.values():
                e.batch.free()
            entries = OrderedDict()
        self.x = [torch.from_numpy(p).cuda() for p in self.x0]
        self.step = [0] * len(self.x0)
        self.latest = [None] * len(self.x0)     # (entry, set index) of resident tables
        self.entries = entries                  # (slot, systems) -> _Entry, least recent first
        self.resident = sum(e.nbytes for e in entries.values())
        self.kept_inputs = {}
        self.results = {}                       # rid -> (entry, set index, launch number)
        self.evictions = 0                      # systems that lost resident tables
        self.reused = 0                         # launches that replayed a planned batch
        self.host_ms = {"create": [], "stage": [], "launch": [], "wait": []}
        torch.cuda.synchronize()

    def _step(self, reqs, off, out, stream):
        """Advance each request's system by one displacement step on the GPU
        (one fmmds_displace for the whole batch) and assemble the batch input
        `out` in the same pass."""
        items = []
        for i, r in enumerate(reqs):
            r.step = self.step[r.system]
            items.append((self.x[r.system], I.displacement_seed(self.seed, r.system, r.step),
                          int(off[i])))
            self.step[r.system] += 1
        self.F.displace(items, self.sigma, out=out, stream=stream)

    def _drop(self, e: _Entry):
        """Free a planned batch; systems whose tables it held lose them."""
        del self.entries[(e.slot, e.key)]
        for s, v in enumerate(self.latest):
            if v is not None and v[0] is e:
                self.latest[s] = None
                self.evictions += 1
        e.batch.free()
        self.resident -= e.nbytes

    def _make_room(self, need: int) -> bool:
        """Free planned batches, least recently used first, until `need`
        more bytes fit the budget: first those no system's tables live in,
        then (only with nothing in flight) any idle one. False if it cannot."""
        for held in (False, True):
            if held and any(sl.entry is not None for sl in self.slots):
                break
            for e in list(self.entries.values()):
                if self.resident + need <= self.budget:
                    return True
                if not e.in_flight and (held or e.refs == 0):
                    self._drop(e)
        return self.resident + need <= self.budget

    # ------------------------------------------------------------- batches
    def _entry_bytes(self, off, lev) -> int:
        return self.F.batch_footprint(off, lev) + 12 * int(off[-1])

    def _plan(self, si: int, key: tuple, off, lev) -> _Entry:
        torch, F = self.torch, self.F
        slot = self.slots[si]
        tc = time.perf_counter()
        b = F.Batch(off, lev, stream=slot.stream)
        with torch.cuda.stream(slot.stream):
            xbuf = torch.empty((int(off[-1]), 3), dtype=torch.float32, device="cuda")
        e = _Entry(key, si, b, xbuf, b.nbytes + 12 * int(off[-1]))
        self.entries[(si, key)] = e
        self.resident += e.nbytes
        self.host_ms["create"].append((time.perf_counter() - tc) * 1e3)
        return e

    def _launch(self, si: int, e: _Entry, reqs: list, off, now: float):
        torch = self.torch
        slot = self.slots[si]
        tc = time.perf_counter()
        self._step(reqs, off, e.xbuf, slot.stream)
        for r in reqs:
            r.launched = now
            if r.rid in self.keep_inputs:
                with torch.cuda.stream(slot.stream):
                    self.kept_inputs[r.rid] = self.x[r.system].clone()
        self.host_ms["stage"].append((time.perf_counter() - tc) * 1e3)
        tc = time.perf_counter()
        e.batch.launch(e.xbuf, capture=self.graphs)
        self.host_ms["launch"].append((time.perf_counter() - tc) * 1e3)
        ev = torch.cuda.Event()
        ev.record(slot.stream)
        e.in_flight = True
        e.launches += 1
        self.entries.move_to_end((si, e.key))
        slot.entry, slot.event, slot.reqs = e, ev, reqs

    def _finish(self, slot: _Slot, t0: float):
        e = slot.entry
        tc = time.perf_counter()
        e.batch.wait()
        self.host_ms["wait"].append((time.perf_counter() - tc) * 1e3)
        done = time.perf_counter() - t0
        e.in_flight = False
        for i, r in enumerate(slot.reqs):
            r.done = done
            old = self.latest[r.system]
            if old is None or old[0] is not e:
                if old is not None:
                    old[0].refs -= 1
                e.refs += 1
            self.latest[r.system] = (e, i)
            self.results[r.rid] = (e, i, e.launches)
        slot.entry, slot.event, slot.reqs = None, None, []

    def tree_of(self, rid: int):
        """The tree a request produced, while it is still resident (until its
        system's next request reuses the same planned batch, or the batch is
        freed for memory)."""
        e, i, n = self.results[rid]
        if self.entries.get((e.slot, e.key)) is not e or e.launches != n:
            raise KeyError("tables of this request were replaced")
        return e.batch.tree(i)

    # ------------------------------------------------------------- loop
    def run(self, arrivals, systems, *, on_complete=None):
        """Serve requests arriving at `arrivals` (seconds from the start) for
        `systems`. Returns the list of Requests with launch and done times."""
        reqs = [Request(i, int(s), float(a)) for i, (a, s) in enumerate(zip(arrivals, systems))]
        pending = deque()
        nxt = 0
        busy = set()           # systems with a build in flight
        t0 = time.perf_counter()
        n_done = 0
        last_progress = t0
        while n_done < len(reqs):
            now = time.perf_counter() - t0
            if time.perf_counter() - last_progress > self.stall_seconds:
                raise RuntimeError(f"serving loop made no progress for {self.stall_seconds} s "
                                   f"({n_done}/{len(reqs)} done, {len(pending)} pending)")
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            progressed = False
            for slot in self.slots:
                if slot.entry is not None and slot.event.query():
                    fin = slot.reqs
                    self._finish(slot, t0)
                    for r in fin:
                        busy.discard(r.system)
                        if on_complete is not None:
                            on_complete(self, r)
                    n_done += len(fin)
                    progressed = True
            while pending:
                free = [si for si, sl in enumerate(self.slots) if sl.entry is None]
                if not free:
                    break
                take, pts, seen = [], 0, set()
                for r in pending:
                    if r.system in busy or r.system in seen:
                        continue
                    if take and (pts + self.n[r.system] > self.max_batch_points or
                                 len(take) >= self.max_batch_sets):
                        break
                    take.append(r)
                    seen.add(r.system)
                    pts += self.n[r.system]
                if not take:
                    break
                e = si = None
                while True:
                    # systems in set order: the key of a reusable planned batch,
                    # on whichever free slot holds one
                    take.sort(key=lambda r: r.system)
                    key = tuple(r.system for r in take)
                    off = np.zeros(len(take) + 1, dtype=np.uint64)
                    off[1:] = np.cumsum([self.n[r.system] for r in take])
                    si = next((k for k in free if (k, key) in self.entries), None)
                    if si is not None:
                        e = self.entries[(si, key)]
                        self.reused += 1
                        break
                    si = free[0]
                    lev = np.asarray([self.levels[r.system] for r in take], dtype=np.uint8)
                    need = self._entry_bytes(off, lev)
                    if self._make_room(need):
                        e = self._plan(si, key, off, lev)
                        break
                    if len(take) > 1:
                        take.pop()  # admit fewer
                        continue
                    if any(sl.entry is not None for sl in self.slots):
                        break  # wait: a completion will free memory
                    raise self.F.FmmdsError(self.F.ERR_NOMEM,
                                            f"request {take[0].rid} needs {need} bytes, "
                                            f"budget {self.budget}")
                if e is None:
                    break
                for r in take:
                    pending.remove(r)
                    busy.add(r.system)
                self._launch(si, e, take, off, time.perf_counter() - t0)
                progressed = True
            if progressed or (nxt < len(reqs) and not pending):
                last_progress = time.perf_counter()
            if not progressed:
                if nxt < len(reqs) and not pending and all(s.entry is None for s in self.slots):
                    wait = reqs[nxt].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.001))
                else:
                    time.sleep(0)
        return reqs

    def close(self):
        self.torch.cuda.synchronize()
        for slot in self.slots:
            if slot.entry is not None:
                slot.entry.batch.wait()
                slot.entry.in_flight = False
                slot.entry = None
        for e in list(self.entries.values()):
            e.batch.free()
        self.entries.clear()
        self.latest = [None] * len(self.x0)
        self.resident = 0


def run_sequential(systems, levels, arrivals, picks, *, sigma=1e-3, seed=8, final=None):
    """Baseline: the same trace served one request at a time with fmmds_build
    on one stream. Returns the list of Requests; when `final` is a list, the
    systems' final coordinates (host arrays) are appended to it."""
    import torch
    import paper_1301_1704_amd as F
    x = [torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda() for p in systems]
    step = [0] * len(x)
    latest = [None] * len(x)
    reqs = [Request(i, int(s), float(a)) for i, (a, s) in enumerate(zip(arrivals, picks))]
    F.displace([(x[0], 1, 0)], 0.0)  # one-time initialization, untimed
    F.build(torch.from_numpy(I.uniform_points(1, 300)).cuda(), None, max_level=3).free()
    torch.cuda.synchronize()
    x[0].copy_(torch.from_numpy(np.ascontiguousarray(systems[0], dtype=np.float32)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            pass
        r.launched = time.perf_counter() - t0
        r.step = step[r.system]
        F.displace([(x[r.system], I.displacement_seed(seed, r.system, r.step), 0)], sigma)
        step[r.system] += 1
        t = F.build(x[r.system], None, max_level=int(levels[r.system]), key_bits=64)
        torch.cuda.synchronize()
        r.done = time.perf_counter() - t0
        if latest[r.system] is not None:
            latest[r.system].free()
        latest[r.system] = t
    for t in latest:
        if t is not None:
            t.free()
    if final is not None:
        final.extend(v.cpu().numpy() for v in x)
    return reqs


def latency_stats(reqs, skip: int = 0) -> dict:
    rs = reqs[skip:]
    lat = np.asarray([r.done - r.arrival for r in rs]) * 1e3
    span = max(r.done for r in rs) - min(r.arrival for r in rs)
    wait = np.asarray([r.launched - r.arrival for r in rs]) * 1e3
    serve = np.asarray([r.done - r.launched for r in rs]) * 1e3
    return {"requests": len(rs), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "builds_per_s": len(rs) / span if span > 0 else float("nan"),
            "p99_queue_ms": float(np.percentile(wait, 99)),
            "p99_service_ms": float(np.percentile(serve, 99))}
