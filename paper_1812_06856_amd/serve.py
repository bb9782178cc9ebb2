"""Serving loop over a rig pool: light-field video frames from several rigs
arrive over time; each rig keeps its images, superpixels and previous planes
on the device; frames are admitted into the pool's stages as rigs free up
(continuous batching: a frame that arrives while others are on the GPU joins
at the next stage boundary); latency runs from arrival to the frame's depth
maps in device memory.

Frames come with label maps or are segmented on the GPU when admitted
(slf_segment, Sec. III-A / III-E).  A rig's first frame is solved in full (the sweep, Sec. III-B, then
`cold_iters` refinement iterations, Sec. III-C); later frames start from the
rig's previous planes (slf_warm_start: each grid cell keeps its 3D plane and
takes the depth at its new centroid; the paper treats frames independently,
so this is a serving form) and run `warm_iters` iterations.  Optionally each
frame's depth maps are fused (Sec. III-D) before the frame counts as done.

All GPU work runs in libslf (the pool, the kernels); this module only orders
host-side calls: arrivals, the per-rig frame queue, admission and the
latency clock.  Admission by memory happens when a rig is attached to the
pool (slf_pool_attach compares its footprint with the pool's HBM budget).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import torch

from . import slf


@dataclass
class Completed:
    rig: int
    frame: object        # the caller's frame id
    arrival: float       # seconds on the server clock
    done: float          # when the depth maps were in device memory
    cold: bool           # solved in full (first frame of the rig)

    @property
    def latency_ms(self) -> float:
        return (self.done - self.arrival) * 1e3


@dataclass
class _Rig:
    ctx: "slf.Context"
    stream: torch.cuda.Stream
    depth: Sequence[torch.Tensor]
    cold_iters: int
    warm_iters: int
    fused: Optional[Sequence[torch.Tensor]] = None
    queue: collections.deque = field(default_factory=collections.deque)
    busy: Optional[tuple] = None       # (frame, arrival, tag, cold) of the request in the pool
    has_state: bool = False


class Server:
    """Frames of several rigs served through one slf.Pool.

    latest_only: when a rig frees up with several frames waiting, it takes the
    newest and drops the older ones (bounded latency under overload);
    otherwise every frame is served in arrival order.
    fuse_tol: if not None, each frame's depth maps are fused with this
    agreement tolerance (written to the rig's `fused` buffers)."""

    def __init__(self, pool: "slf.Pool", latest_only: bool = False, fuse_tol: Optional[float] = None,
                 clock: Callable[[], float] = time.perf_counter, segment: Optional[tuple] = None):
        """segment: (iterations, compactness) of the GPU SLIC for frames
        submitted without labels (the rig's label grid is kept)."""
        self.pool = pool
        self.segment = segment
        self.latest_only = latest_only
        self.fuse_tol = fuse_tol
        self.clock = clock
        self.rigs: List[_Rig] = []
        self._tag = 0
        self._reading = {}     # tag -> (rig, frame, arrival, cold, event)
        self.dropped = 0

    def add_rig(self, ctx: "slf.Context", stream: torch.cuda.Stream, depth: Sequence[torch.Tensor],
                cold_iters: int, warm_iters: int = 2, fused: Optional[Sequence[torch.Tensor]] = None) -> int:
        """Registers a rig already attached to the pool, with the device buffers
        its depth maps (and fused maps) are written to.  Returns its index."""
        if self.fuse_tol is not None and fused is None:
            raise ValueError("fusion is on: give the rig fused depth buffers")
        self.rigs.append(_Rig(ctx, stream, depth, cold_iters, warm_iters, fused))
        return len(self.rigs) - 1

    def submit(self, rig: int, frame, images: Sequence[torch.Tensor], labels: Optional[Sequence[torch.Tensor]],
               arrival: Optional[float] = None) -> None:
        """Queues a frame of `rig`: device uint8 images [H, W, 3] and int32 label
        maps [H, W] per view (kept alive by the caller until served).  With
        labels None the frame is segmented on the GPU (slf_segment, with the
        server's `segment` settings) when it is admitted."""
        if labels is None and self.segment is None:
            raise ValueError("no labels and no GPU segmentation configured")
        self.rigs[rig].queue.append((frame, self.clock() if arrival is None else arrival, images, labels))

    def busy(self) -> bool:
        return bool(self._reading) or any(r.busy is not None or r.queue for r in self.rigs)

    def _admit(self, j: int, r: _Rig) -> None:
        while self.latest_only and len(r.queue) > 1:
            r.queue.popleft()
            self.dropped += 1
        frame, arrival, images, labels = r.queue.popleft()
        for v, img in enumerate(images):
            gw, gh = r.ctx.grids[v]
            r.ctx.set_image(v, img)
            if labels is None:
                r.ctx.segment(v, gw, gh, *self.segment)
            else:
                r.ctx.set_labels(v, labels[v], gw, gh)
        cold = not r.has_state
        if cold:
            self.pool.submit(r.ctx, slf.SLF_POOL_SOLVE, 1, r.cold_iters, self._tag)
        else:
            r.ctx.warm_start()
            self.pool.submit(r.ctx, slf.SLF_POOL_PROPAGATE, 1, r.warm_iters, self._tag)
        r.has_state = True
        r.busy = (frame, arrival, self._tag, cold)
        self._tag += 1

    def tick(self) -> List[Completed]:
        """Admits waiting frames of idle rigs, launches one stage of the pool's
        active requests, starts the depth readout of finished requests and
        returns the frames whose depth maps have landed."""
        for j, r in enumerate(self.rigs):
            if r.busy is None and r.queue:
                self._admit(j, r)
        if self.pool.usage()["active"]:
            self.pool.step()
        for tag in self.pool.poll():
            j = next(i for i, r in enumerate(self.rigs) if r.busy is not None and r.busy[2] == tag)
            r = self.rigs[j]
            frame, arrival, _, cold = r.busy
            r.busy = None
            for v in range(len(r.depth)):
                r.ctx.get_depth(v, out=r.depth[v])
            if self.fuse_tol is not None:
                r.ctx.fuse(self.fuse_tol)
                for v in range(len(r.fused)):
                    r.ctx.get_fused_depth(v, out=r.fused[v])
            ev = torch.cuda.Event()
            ev.record(r.stream)
            self._reading[tag] = (j, frame, arrival, cold, ev)
        done = []
        for tag in list(self._reading):
            j, frame, arrival, cold, ev = self._reading[tag]
            if ev.query():
                done.append(Completed(j, frame, arrival, self.clock(), cold))
                del self._reading[tag]
        return done

    def drain(self, idle_sleep_s: float = 0.0002) -> List[Completed]:
        """Serves every queued frame to the end."""
        out = []
        while self.busy():
            out += self.tick()
            if not self.pool.usage()["active"] and self._reading:
                time.sleep(idle_sleep_s)
        return out


def poisson_arrivals(rate: float, horizon_s: float, n_rigs: int, rng) -> List[tuple]:
    """(time, rig) pairs of a Poisson stream of `rate` frames per second over
    `horizon_s` seconds, the rig of each frame drawn uniformly."""
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= horizon_s:
            return out
        out.append((t, int(rng.integers(0, n_rigs))))
