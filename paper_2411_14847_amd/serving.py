"""Novel-view render serving beside streaming training.

Requests (camera, arrival time) are served by continuous batching: whenever a render slot is
free, the engine admits the oldest pending requests that fit the slot's reserved tiles, tile
keys and output images, and renders them in one render_fwd on the slot's own stream; requests
that arrive while others are on the GPU wait only for a free slot.  Several slots (contexts +
streams) keep batches overlapping on the device, and training runs on yet another stream.
The scene is read from a published snapshot (double-buffered), so renders never see a
half-updated timestep.  Every request's image is the same alone and in any batch (the forward
has no cross-view interaction and no atomics).  Latency = completion time of the batch's HIP
event (polled) minus the request's arrival time.

Each slot's stream and the training stream need hardware queues of their own: streams that share
a hardware queue run in submission order, so a slot sharing the training stream's queue waits
behind its kernels.  HIP maps streams onto GPU_MAX_HW_QUEUES queues (4 by default, read when the
runtime starts): a serving process should start with at least MIN_HW_QUEUES.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from ._ffi import DASS_E_CAPACITY
from .api import Context, DassError, GaussianBuffers, RenderOut

# hardware queues a serving process wants (default stream, training, three slots, spare)
MIN_HW_QUEUES = 8


def tiles_of(cam) -> int:
    return ((int(cam.width) + 15) // 16) * ((int(cam.height) + 15) // 16)


class SceneSnapshots:
    """Two device copies of the scene.  `publish` copies the live scene into the idle copy on the
    caller's stream, after every render still reading that copy has finished, and then flips;
    `read` enqueues work on the newest complete copy and registers its completion event as a
    reader of that copy.  Safe to call from a training thread and a serving thread at once."""

    def __init__(self, like: GaussianBuffers):
        self.bufs = [like.clone(), like.clone()]
        self.ready = [torch.cuda.Event(), torch.cuda.Event()]
        for e in self.ready:
            e.record()
        self.readers = [[], []]
        self.cur = 0
        self.version = 0
        self.lock = threading.Lock()

    def publish(self, g: GaussianBuffers, stream: Optional[torch.cuda.Stream] = None):
        s = stream or torch.cuda.current_stream()
        with self.lock:
            nxt = 1 - self.cur
            readers, self.readers[nxt] = self.readers[nxt], []
        dst = self.bufs[nxt]
        with torch.cuda.stream(s):
            for ev in readers:
                s.wait_event(ev)
            for d, src in zip(dst.planes(), g.planes()):
                d.copy_(src, non_blocking=True)
            self.ready[nxt].record(s)
        with self.lock:
            dst.n, dst.n_base = g.n, g.n_base
            self.cur = nxt
            self.version += 1

    def read(self, stream: torch.cuda.Stream, enqueue):
        """Enqueues `enqueue(scene_copy)` on `stream` after the newest copy is complete and returns
        (its result, an event recorded after it).  The event is registered as a reader of that
        copy, so the publish that would overwrite the copy waits for it."""
        with self.lock:
            i = self.cur
            stream.wait_event(self.ready[i])
            res = enqueue(self.bufs[i])
            ev = torch.cuda.Event()
            ev.record(stream)
            if len(self.readers[i]) >= 64:
                self.readers[i] = [e for e in self.readers[i] if not e.query()]
            self.readers[i].append(ev)
        return res, ev

    def current(self):
        with self.lock:
            return self.bufs[self.cur], self.ready[self.cur]


@dataclass
class Request:
    rid: int
    arrival: float     # seconds on the engine clock
    camera: object


@dataclass
class Slot:
    ctx: Context
    stream: torch.cuda.Stream
    outs: List[RenderOut]
    max_tiles: int
    max_keys: int
    busy: bool = False
    event: Optional[torch.cuda.Event] = None
    batch: List[Request] = field(default_factory=list)


class RenderServer:
    def __init__(self, snapshots: SceneSnapshots, max_gaussians: int, n_slots: int = 3, max_batch: int = 8,
                 max_tiles: int = 8 * 8160, keys_per_tile: int = 1200, max_w: int = 1920, max_h: int = 1080,
                 bg=(0.0, 0.0, 0.0)):
        self.snap = snapshots
        self.bg = bg
        self.max_w, self.max_h = max_w, max_h
        self.max_batch = max_batch
        self.keys_per_tile = keys_per_tile
        self.slots: List[Slot] = []
        for _ in range(n_slots):
            ctx = Context(max_gaussians=max_gaussians, max_views=max_batch, max_keys=max_tiles * keys_per_tile,
                          max_tiles=max_tiles)
            outs = [RenderOut(torch.empty(3 * max_h * max_w, device="cuda"), torch.empty(max_h * max_w, device="cuda"),
                              torch.empty(max_h * max_w, dtype=torch.int32, device="cuda")) for _ in range(max_batch)]
            self.slots.append(Slot(ctx, torch.cuda.Stream(), outs, max_tiles, max_tiles * keys_per_tile))
        self.pending = collections.deque()
        self.latencies = []
        self.completed = 0
        self.retried = 0

    @staticmethod
    def _view(buf: RenderOut, cam) -> RenderOut:
        H, W = int(cam.height), int(cam.width)
        return RenderOut(buf.rgb[:3 * H * W].view(3, H, W), buf.t_final[:H * W].view(H, W),
                         buf.n_contrib[:H * W].view(H, W))

    def submit(self, req: Request):
        cam = req.camera
        if int(cam.width) > self.max_w or int(cam.height) > self.max_h or tiles_of(cam) > self.slots[0].max_tiles:
            raise ValueError(f"request {req.rid}: {cam.width}x{cam.height} exceeds the server's slot size")
        self.pending.append(req)

    def _admit(self, slot: Slot) -> List[Request]:
        batch, tiles = [], 0
        while self.pending and len(batch) < self.max_batch:
            t = tiles_of(self.pending[0].camera)
            if tiles + t > slot.max_tiles:
                break
            tiles += t
            batch.append(self.pending.popleft())
        return batch

    def launch(self, slot: Slot, batch: List[Request]):
        cams = [r.camera for r in batch]
        outs = [self._view(o, c) for o, c in zip(slot.outs, cams)]
        _, ev = self.snap.read(slot.stream, lambda g: slot.ctx.render_fwd(g, cams, self.bg, out=outs,
                                                                            stream=slot.stream))
        slot.busy, slot.event, slot.batch = True, ev, batch

    def poll(self, now_fn) -> int:
        """Retires finished batches, then admits pending requests into free slots."""
        done = 0
        for slot in self.slots:
            if slot.busy and slot.event.query():
                t_done = now_fn()
                try:
                    slot.ctx.sync(slot.stream)  # already complete: returns at once; reports key overflow
                    for r in slot.batch:
                        self.latencies.append(t_done - r.arrival)
                    self.completed += len(slot.batch)
                    done += len(slot.batch)
                except DassError as e:
                    if e.status != DASS_E_CAPACITY:
                        raise
                    # key budget exceeded: put the batch back at the front and admit smaller batches
                    self.retried += len(slot.batch)
                    for r in reversed(slot.batch):
                        self.pending.appendleft(r)
                    self.max_batch = max(1, self.max_batch // 2)
                slot.busy, slot.event, slot.batch = False, None, []
        for slot in self.slots:
            if not slot.busy and self.pending:
                batch = self._admit(slot)
                if batch:
                    self.launch(slot, batch)
        return done

    def render_alone(self, cam) -> RenderOut:
        """One request rendered by itself (reference for the alone-vs-batched identity)."""
        slot = self.slots[0]
        out = RenderOut.allocate(cam)
        self.snap.read(slot.stream, lambda g: slot.ctx.render_fwd(g, [cam], self.bg, out=[out], stream=slot.stream))
        slot.stream.synchronize()
        slot.ctx.sync(slot.stream)
        return out

    def stats(self, wall_s: float) -> dict:
        lat = np.array(self.latencies) * 1e3
        return {"frames": self.completed, "frames_per_s": self.completed / wall_s if wall_s > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
                "p99_ms": float(np.percentile(lat, 99)) if lat.size else None, "retried": self.retried}


def serve_requests(server: RenderServer, requests: List[Request], time_scale: float = 1.0,
                   deadline_s: float = 600.0, poll_s: float = 2e-4) -> dict:
    """Feeds requests at their arrival times (engine clock = wall clock / time_scale) and serves
    until every request has completed.  Between polls with nothing to admit the loop sleeps
    `poll_s`, which releases the interpreter to a training thread."""
    t0 = time.perf_counter()
    now = lambda: (time.perf_counter() - t0) / time_scale
    i = 0
    while server.completed < len(requests) and now() < deadline_s:
        t = now()
        while i < len(requests) and requests[i].arrival <= t:
            server.submit(requests[i])
            i += 1
        server.poll(now)
        if server.completed >= len(requests):
            break
        can_admit = server.pending and any(not s.busy for s in server.slots)
        if not can_admit:
            wait = poll_s
            if i < len(requests):
                wait = min(wait, max(0.0, requests[i].arrival - now()) * time_scale)
            time.sleep(wait)
    return server.stats(time.perf_counter() - t0)
