"""Continuous-batching render server over one resident scene.

The scene stays in HBM for the server's lifetime.  Requests (one camera
each: model, intrinsics, pose, BEAP grid size) wait in a FIFO queue.  The
device is divided into `slots`; a slot is one stream, one workspace arena of
`slot_bytes` and one output arena.  Whenever a slot is free the scheduler
admits queued requests in arrival order while the workspace of the growing
batch (geer_plan_workspace_bytes: per-(Gaussian, view) records and sort
buffers plus the association-list capacity) still fits the slot's arena, up
to `max_views`; requests that arrive while other batches are on the GPU are
admitted as soon as a slot frees.  A batch renders with one replay of a
graph captured for its shape (the tuple of grid sizes, cached per slot), so
batches on different slots run concurrently on the device.  Results are
copied out of the slot's arena on its stream; a batch whose association list
overflowed the capacity is re-rendered eagerly (the eager path sizes itself).

Latency runs from a request's arrival (host clock) to the completion of its
batch on the device: an event recorded after the batch's result copies, put
on the host clock through a reference event that the host waited for when
the run started.  A batch whose association sort stalled
(a bounded device-side wait gave up) is re-rendered eagerly like an
overflowed one.  The same cameras rendered alone give the
same bits: a view's tiles only ever hold that view's Gaussians, sorted by the
same (depth key, index) order.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import renderer


@dataclass
class Request:
    rid: int
    cam: dict
    t_arrive: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    t_done_host: float = 0.0
    rgb: torch.Tensor | None = None
    depth: torch.Tensor | None = None
    trans: torch.Tensor | None = None
    retried: bool = False

    @property
    def shape(self):
        return int(self.cam["width"]), int(self.cam["height"])

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


@dataclass
class _Slot:
    index: int
    stream: torch.cuda.Stream
    workspace: torch.Tensor
    out: tuple
    plans: dict = field(default_factory=dict)
    batch: list = field(default_factory=list)
    plan: object = None
    ev_start: torch.cuda.Event | None = None
    ev_done: torch.cuda.Event | None = None

    @property
    def busy(self) -> bool:
        return bool(self.batch)


def tiles_of(shape) -> int:
    w, h = shape
    return ((w + 15) // 16) * ((h + 15) // 16)


class Server:
    """slots: concurrent batches (streams); slot_views: the workspace arena of
    a slot holds that many views of the largest shape (or give slot_bytes);
    entries_per_tile: capacity of PBF (tile, Gaussian) pairs per 16x16 tile
    of a view;
    max_views: largest batch."""

    def __init__(self, scene: dict, shapes, entries_per_tile: float, slots: int = 3, slot_views: int = 1,
                 slot_bytes: int | None = None, max_views: int = 4, opts: dict | None = None):
        self.scene = scene
        self.opts = opts
        self.max_views = max_views
        self.entries_per_tile = float(entries_per_tile)
        self.dev = scene["mean"].device
        shapes = sorted({(int(w), int(h)) for w, h in shapes})
        self._ws_cache = {}
        largest = max(shapes, key=lambda s: s[0] * s[1])
        biggest = max(self.workspace_bytes([s]) for s in shapes)
        self.slot_bytes = int(slot_bytes) if slot_bytes else self.workspace_bytes([largest] * slot_views)
        if self.slot_bytes < biggest:
            raise ValueError("slot_bytes %d cannot hold one view of the largest shape (%d)" % (self.slot_bytes,
                                                                                              biggest))
        max_pix = max(w * h for w, h in shapes) * max_views
        self.slots = []
        for i in range(slots):
            st = torch.cuda.Stream(device=self.dev)  # default priority
            with torch.cuda.stream(st):
                ws = torch.empty(self.slot_bytes + 256, dtype=torch.uint8, device=self.dev)
                out = (torch.empty(3 * max_pix, device=self.dev), torch.empty(max_pix, device=self.dev),
                       torch.empty(max_pix, device=self.dev))
            self.slots.append(_Slot(i, st, ws, out))
        self.stats = dict(batches=0, overflows=0, stalls=0, views=0, overlapped=0)
        self.intervals = []  # (slot, start event, end event) per batch
        self.evaluated = 0   # evaluated (ray, entry) pairs of the render kernel, over retired batches
        self._ref = None     # (event, host time) pairing the device clock with the host clock

    # ------------------------------------------------------------ sizing --
    def capacity(self, shapes) -> int:
        return max(1, int(math.ceil(sum(tiles_of(s) for s in shapes) * self.entries_per_tile)))

    def _dummy_cams(self, shapes):
        return [dict(model="pinhole", width=w, height=h, fx=w / 2, fy=w / 2, cx=w / 2, cy=h / 2, k=[0, 0, 0, 0],
                     fov_x=math.pi / 2, fov_y=2 * math.atan(h / w), R=np.eye(3), t=np.zeros(3)) for w, h in shapes]

    def workspace_bytes(self, shapes) -> int:
        key = tuple(shapes)
        if key not in self._ws_cache:
            self._ws_cache[key] = renderer.plan_workspace_bytes(self.scene, self._dummy_cams(shapes),
                                                                self.capacity(shapes), self.opts)
        return self._ws_cache[key]

    def admit(self, queue: list) -> list:
        """Pops the batch for a free slot: queued requests in arrival order
        while the batch's workspace fits the slot."""
        batch = [queue.pop(0)]
        while queue and len(batch) < self.max_views:
            shapes = sorted([r.shape for r in batch] + [queue[0].shape])
            if self.workspace_bytes(shapes) > self.slot_bytes:
                break
            batch.append(queue.pop(0))
        batch.sort(key=lambda r: r.shape)
        return batch

    def prepare(self, shapes) -> int:
        """Captures, on every slot, the graph of every batch shape that the
        admission rule can form from `shapes`; returns the count per slot."""
        import itertools

        shapes = sorted({(int(w), int(h)) for w, h in shapes})
        count = 0
        for k in range(1, self.max_views + 1):
            for combo in itertools.combinations_with_replacement(shapes, k):
                combo = list(combo)
                if self.workspace_bytes(combo) <= self.slot_bytes:
                    for s in self.slots:
                        self._plan(s, combo)
                    count += 1
        return count

    # ---------------------------------------------------------- batches --
    def _plan(self, slot: _Slot, shapes):
        key = tuple(shapes)
        if key not in slot.plans:
            npix = sum(w * h for w, h in shapes)
            out = (slot.out[0][: 3 * npix], slot.out[1][:npix], slot.out[2][:npix])
            ws = slot.workspace
            off = (-ws.data_ptr()) % 256
            slot.plans[key] = renderer.Plan(self.scene, self._dummy_cams(shapes), self.capacity(shapes), self.opts,
                                            workspace=ws[off: off + self.slot_bytes], out=out)
        return slot.plans[key]

    def launch(self, slot: _Slot, batch: list, now: float):
        shapes = [r.shape for r in batch]
        plan = self._plan(slot, shapes)
        if any(s.busy for s in self.slots if s is not slot):
            self.stats["overlapped"] += 1
        slot.ev_start = torch.cuda.Event(enable_timing=True)
        slot.ev_done = torch.cuda.Event(enable_timing=True)
        slot.ev_start.record(slot.stream)
        plan.launch([r.cam for r in batch], slot.stream)
        with torch.cuda.stream(slot.stream):
            off = 0
            for r in batch:
                hw = r.shape[0] * r.shape[1]
                r.rgb = plan.rgb[3 * off: 3 * (off + hw)].clone()
                r.depth = plan.depth[off: off + hw].clone()
                r.trans = plan.trans[off: off + hw].clone()
                r.t_start = now
                off += hw
        slot.ev_done.record(slot.stream)
        slot.batch, slot.plan = batch, plan
        self.stats["batches"] += 1
        self.stats["views"] += len(batch)

    def _device_time(self, ev) -> float:
        """Host-clock time of a completed device event."""
        ref, t_ref = self._ref
        return t_ref + ref.elapsed_time(ev) * 1e-3

    def retire(self, slot: _Slot, now: float) -> list:
        batch, plan = slot.batch, slot.plan
        st = plan.status()
        t_dev = self._device_time(slot.ev_done)
        if st["overflow"] or st["stalled"]:
            # the batch's outputs are invalid: render its views again eagerly
            # (the eager path sizes its list exactly)
            self.stats["overflows" if st["overflow"] else "stalls"] += 1
            with torch.cuda.stream(slot.stream):
                for r in batch:
                    r.rgb, r.depth, r.trans, _ = renderer.render(self.scene, [r.cam], opts=self.opts)
                    r.retried = True
            slot.stream.synchronize()
            now = t_dev = time.perf_counter()
        else:
            self.evaluated += plan.stats()["n_evaluated"]
        for r in batch:
            r.t_done = t_dev
            r.t_done_host = now
        self.intervals.append((slot.index, slot.ev_start, slot.ev_done))
        slot.batch, slot.plan = [], None
        return batch

    # -------------------------------------------------------------- loop --
    def run(self, requests: list, arrivals=None) -> list:
        """Serves `requests` (arrival offsets in seconds from the start, or
        all at once).  Returns the completed requests in completion order."""
        arrivals = np.zeros(len(requests)) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
        order = np.argsort(arrivals, kind="stable")
        queue, done = [], []
        nxt = 0
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(self.slots[0].stream)
        ref.synchronize()
        self._ref = (ref, time.perf_counter())
        t0 = time.perf_counter()
        while len(done) < len(requests):
            now = time.perf_counter()
            while nxt < len(order) and t0 + arrivals[order[nxt]] <= now:
                r = requests[order[nxt]]
                r.t_arrive = t0 + arrivals[order[nxt]]
                queue.append(r)
                nxt += 1
            progressed = False
            for s in self.slots:
                if s.busy and s.ev_done.query():
                    done.extend(self.retire(s, time.perf_counter()))
                    progressed = True
            for s in self.slots:
                if not s.busy and queue:
                    self.launch(s, self.admit(queue), time.perf_counter())
                    progressed = True
            if not progressed and not queue and nxt < len(order) and not any(s.busy for s in self.slots):
                time.sleep(max(0.0, min(t0 + arrivals[order[nxt]] - time.perf_counter(), 1e-3)))
        return done

    def device_overlap(self) -> float:
        """Fraction of batch GPU time that overlapped another slot's batch
        (from the events bracketing each batch on its stream)."""
        if len(self.intervals) < 2:
            return 0.0
        ref = self.intervals[0][1]
        spans = [(s, ref.elapsed_time(a), ref.elapsed_time(b)) for s, a, b in self.intervals]
        total = sum(b - a for _, a, b in spans)
        ev = sorted([(a, 1, s) for s, a, _ in spans] + [(b, -1, s) for s, _, b in spans])
        busy, last, over = 0, None, 0.0
        for t, d, _ in ev:
            if last is not None and busy >= 2:
                over += (t - last) * busy
            busy += d
            last = t
        return over / total if total > 0 else 0.0

    def close(self):
        torch.cuda.synchronize(self.dev)
        for s in self.slots:
            for p in s.plans.values():
                p.destroy()
            s.plans.clear()


def poisson_arrivals(count: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival offsets (s) of a Poisson process with `rate` requests/s."""
    return np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, count))


def latency_summary(done: list) -> dict:
    """Latency percentiles (arrival to device completion) and throughput over
    the span from the first arrival to the last completion."""
    lat = np.array([r.latency for r in done]) * 1e3
    span = max(r.t_done for r in done) - min(r.t_arrive for r in done)
    rays = sum(r.shape[0] * r.shape[1] for r in done)
    return dict(requests=len(done), p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()), req_per_s=len(done) / span,
                mrays_per_s=rays / span / 1e6, retried=sum(r.retried for r in done))
