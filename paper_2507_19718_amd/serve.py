"""Serving loop: frame requests from many viewers over several resident scenes.

Two drivers replay the same request log (arrival time, scene, viewer camera, resolution):

  * plain  -- one frame at a time in arrival order: gsc_render_frame, wait for completion.
  * served -- continuous batching: requests that arrive while others are on the GPU wait in a
    queue and are admitted as slots and HBM budget free up.  A batch holds at most one request
    per scene (each frame trains its scene, so a scene's frames apply in arrival order) and runs
    as one gsc_render_frames call: one launch per stage over all (request, level) pairs.  Up to
    `slots` batches are in flight at once, each on its own context and HIP stream, so their work
    overlaps on the device; a scene is never in two in-flight batches.

Admission charges each request its scene's transient frame footprint
(gsc_frame_footprint_bytes with an instance estimate) against an HBM budget; scenes stay resident
for the whole run.  Latency = completion - arrival (queueing included).  Both drivers apply
every scene's frames in the same order, so they reach the same cache state up to float-atomic
summation order.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

from . import (Context, Scene, frame_request, gsc_render_frame, gsc_render_frames)


@dataclasses.dataclass
class Request:
    idx: int
    t_arrival: float
    scene: int
    viewer: int
    cam: object
    frame: int
    seed: int
    t_view: int = 1
    t_start: float = math.nan
    t_done: float = math.nan


@dataclasses.dataclass
class SceneSpec:
    scene: Scene
    K: int
    max_bounces: int
    loss: int
    lr: Sequence[float]
    weight_decay: float
    C: float


def percentile(xs: Sequence[float], q: float) -> float:
    """Nearest-rank percentile."""
    if not xs:
        return math.nan
    s = sorted(xs)
    k = max(1, int(math.ceil(q / 100.0 * len(s))))
    return s[k - 1]


def summarize(reqs: Sequence[Request], t0: float, t_end: float, skip_s: float = 0.0) -> dict:
    """Frames/s over the whole run; latency percentiles over the requests that arrived at or
    after skip_s (the warm-up of the first seconds left out)."""
    lat = [1000.0 * (r.t_done - r.t_arrival) for r in reqs if r.t_arrival >= skip_s]
    return {"frames": len(reqs), "wall_s": t_end - t0, "latency_from_s": skip_s,
            "frames_per_s": len(reqs) / max(t_end - t0, 1e-9),
            "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "mean_ms": float(np.mean(lat)) if lat else math.nan}


def _req_struct(spec: SceneSpec, r: Request):
    return frame_request(r.cam, r.seed, r.frame, spec.K, spec.max_bounces, loss=spec.loss,
                         train=True, viewport_frames=r.t_view, lr=spec.lr,
                         weight_decay=spec.weight_decay, C=spec.C)


def run_plain(ctx: Context, scenes: Sequence[SceneSpec], reqs: Sequence[Request],
              realtime: bool = True, skip_s: float = 0.0) -> dict:
    """One frame at a time in arrival order.  realtime=False is the closed loop (every request
    has arrived at time 0): frames/s is then the loop's capacity."""
    images = {}
    t0 = time.perf_counter()
    for r in reqs:
        if realtime:
            now = time.perf_counter() - t0
            if now < r.t_arrival:
                time.sleep(r.t_arrival - now)
        key = (r.cam.h, r.cam.w)
        if key not in images:
            images[key] = torch.empty((r.cam.h, r.cam.w, 3), device="cuda")
        r.t_start = time.perf_counter() - t0
        gsc_render_frame(ctx, scenes[r.scene].scene, _req_struct(scenes[r.scene], r), images[key])
        ctx.synchronize()
        r.t_done = time.perf_counter() - t0
    return summarize(reqs, 0.0, time.perf_counter() - t0, skip_s)


class ContinuousBatcher:
    """Admission by HBM footprint, at most one request per scene per batch, `slots` batches in
    flight on separate contexts/streams."""

    def __init__(self, scenes: Sequence[SceneSpec], slots: int = 2, hbm_budget: Optional[int] = None,
                 instance_estimate: Callable[[Request], int] = lambda r: 0,
                 max_batch: int = 8,
                 before_launch: Optional[Callable[[int, List[Request]], None]] = None,
                 executor: Optional[Callable[[int, List[Request]], None]] = None,
                 footprint: Optional[Callable[[Request], int]] = None,
                 after_batch: Optional[Callable[[int, List[Request], List[torch.Tensor]], None]] = None,
                 deterministic: bool = False):
        """executor(slot, batch) runs a batch to completion (default: gsc_render_frames on the
        slot's context, then a stream synchronise); footprint(r) gives a request's transient
        bytes (default: gsc_frame_footprint_bytes of its scene).  before_launch(slot, batch)
        runs on the scheduler thread before a batch starts; after_batch(slot, batch, images)
        after the default executor finished it (for snapshots in tests).  deterministic: the
        slots' contexts sum the splat adjoint in fixed point (bit-reproducible training)."""
        self.scenes = scenes
        self.n_slots = slots
        self.budget = hbm_budget
        self.estimate = instance_estimate
        self.max_batch = max_batch
        self.before_launch = before_launch
        self.after_batch = after_batch
        self._footprint = footprint
        self.executor = executor if executor is not None else self._gpu_executor
        self.slots = [Context(0, torch.cuda.Stream()) for _ in range(slots)] if executor is None else []
        for c in self.slots:
            c.set_deterministic(deterministic)
        self.images: Dict[tuple, torch.Tensor] = {}
        self.batches: List[List[int]] = []

    def footprint(self, r: Request) -> int:
        if self._footprint is not None:
            return self._footprint(r)
        sc = self.scenes[r.scene].scene
        return sc.frame_footprint_bytes(r.cam.w, r.cam.h, self.estimate(r))

    def _gpu_executor(self, slot: int, batch: List[Request]):
        ctx = self.slots[slot]
        images = []
        for k, r in enumerate(batch):
            key = (slot, k, r.cam.h, r.cam.w)
            if key not in self.images:
                self.images[key] = torch.empty((r.cam.h, r.cam.w, 3), device="cuda")
            images.append(self.images[key])
        with torch.cuda.stream(ctx.stream):
            gsc_render_frames(ctx, [self.scenes[r.scene].scene for r in batch],
                              [_req_struct(self.scenes[r.scene], r) for r in batch], images)
            ctx.synchronize()
            if self.after_batch:
                self.after_batch(slot, batch, images)

    def run(self, reqs: Sequence[Request], realtime: bool = True, skip_s: float = 0.0) -> dict:
        """Replays the log (realtime) or serves it as a closed loop (every request has arrived
        at time 0: frames/s is then the capacity); latencies of requests that arrived before
        skip_s are left out of the percentiles."""
        pending = collections.deque()                 # arrived, not started (arrival order)
        upcoming = collections.deque(reqs)
        busy_scenes = set()
        in_use = 0
        lock = threading.Condition()
        free_slots = list(range(self.n_slots))
        done_batches = collections.deque()
        errors = []
        t0 = time.perf_counter()

        def worker(slot: int, batch: List[Request]):
            try:
                self.executor(slot, batch)
            except Exception as e:  # surfaced after the run
                errors.append(e)
            t = time.perf_counter() - t0
            with lock:
                for r in batch:
                    r.t_done = t
                done_batches.append((slot, batch))
                lock.notify_all()

        threads = []
        n_done = 0
        while n_done < len(reqs):
            with lock:
                now = time.perf_counter() - t0
                while upcoming and (not realtime or upcoming[0].t_arrival <= now):
                    pending.append(upcoming.popleft())
                while done_batches:
                    slot, batch = done_batches.popleft()
                    free_slots.append(slot)
                    for r in batch:
                        busy_scenes.discard(r.scene)
                        in_use -= self.footprint(r)
                    n_done += len(batch)
                if n_done >= len(reqs):
                    break
                launched = False
                if free_slots and pending:
                    batch, seen, keep = [], set(), collections.deque()
                    budget_left = None if self.budget is None else self.budget - in_use
                    while pending:
                        r = pending.popleft()
                        fp = self.footprint(r)
                        ok = (r.scene not in seen and r.scene not in busy_scenes
                              and len(batch) < self.max_batch
                              and (budget_left is None or fp <= budget_left or (not batch and in_use == 0)))
                        if ok:
                            batch.append(r)
                            seen.add(r.scene)
                            if budget_left is not None:
                                budget_left -= fp
                        else:
                            keep.append(r)
                            seen.add(r.scene)        # keep later frames of a scene behind it
                    pending.extendleft(reversed(keep))
                    if batch:
                        slot = free_slots.pop(0)
                        for r in batch:
                            busy_scenes.add(r.scene)
                            in_use += self.footprint(r)
                            r.t_start = now
                        self.batches.append([r.idx for r in batch])
                        if self.before_launch:
                            self.before_launch(slot, batch)
                        th = threading.Thread(target=worker, args=(slot, batch), daemon=True)
                        th.start()
                        threads.append(th)
                        launched = True
                if not launched:
                    wait = None
                    if upcoming and realtime:
                        wait = max(0.0, upcoming[0].t_arrival - now)
                    lock.wait(timeout=wait if wait is not None else 0.05)
        for th in threads:
            th.join()
        if errors:
            raise errors[0]
        return summarize(reqs, 0.0, time.perf_counter() - t0, skip_s)


def make_requests(log: Sequence[dict], cams: Callable[[dict], object], duration_s: Optional[float] = None,
                  scene_frames: Optional[Dict[int, int]] = None) -> List[Request]:
    """From a synth.poisson_requests log: per-scene frame counters give each request its RNG
    frame index; a viewer's viewport counter t (Eq. 5) restarts on every pose change, so an
    orbiting viewer always trains at t = 1."""
    out = []
    sf = dict(scene_frames or {})
    for i, e in enumerate(log):
        if duration_s is not None and e["t_arrival"] >= duration_s:
            break
        f = sf.get(e["scene"], 0)
        sf[e["scene"]] = f + 1
        out.append(Request(idx=i, t_arrival=e["t_arrival"], scene=e["scene"], viewer=e["viewer"],
                           cam=cams(e), frame=f, seed=e["seed"]))
    return out
