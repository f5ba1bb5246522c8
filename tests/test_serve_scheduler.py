"""The continuous-batching scheduler on the CPU with a fake executor: every request completes,
a batch holds at most one request per scene, no scene is in two in-flight batches, each scene's
requests run in arrival order, admission respects the HBM budget, and work overlaps across
slots.  Plus the nearest-rank percentile."""
import threading
import time
import types

import pytest

import synth
from paper_2507_19718_amd import serve


def fake_requests(n=120, scenes=4, seed=3, rate=400.0):
    log = synth.poisson_requests(rate, n / rate * 1.5, 16, scenes, seed)[:n]
    cams = lambda e: types.SimpleNamespace(w=e["width"], h=e["height"])
    return serve.make_requests(log, cams)


class FakeGPU:
    def __init__(self, slots):
        self.lock = threading.Lock()
        self.active = {}
        self.max_concurrent = 0
        self.order = []

    def __call__(self, slot, batch):
        with self.lock:
            for r in batch:
                assert r.scene not in self.active, "scene in two in-flight batches"
                self.active[r.scene] = slot
            self.max_concurrent = max(self.max_concurrent, len(set(self.active.values())))
            self.order.extend(r.idx for r in batch)
        time.sleep(0.002 + 1e-9 * sum(r.cam.w * r.cam.h for r in batch))
        with self.lock:
            for r in batch:
                del self.active[r.scene]


def test_scheduler_invariants():
    reqs = fake_requests()
    gpu = FakeGPU(3)
    fp = lambda r: r.cam.w * r.cam.h * 100
    budget = 1920 * 1080 * 100 * 2
    b = serve.ContinuousBatcher([None] * 4, slots=3, hbm_budget=budget, executor=gpu, footprint=fp)
    res = b.run(reqs, realtime=True)
    assert res["frames"] == len(reqs)
    assert all(r.t_done >= r.t_start >= r.t_arrival - 1e-6 for r in reqs)
    by_idx = {r.idx: r for r in reqs}
    for batch in b.batches:
        scenes = [by_idx[i].scene for i in batch]
        assert len(scenes) == len(set(scenes))
        assert sum(fp(by_idx[i]) for i in batch) <= budget or len(batch) == 1
    for s in range(4):
        seq = [i for i in gpu.order if by_idx[i].scene == s]
        assert seq == sorted(seq), "a scene's frames must apply in arrival order"
    assert gpu.max_concurrent >= 2


def test_scheduler_tight_budget_still_progresses():
    reqs = fake_requests(n=40)
    gpu = FakeGPU(2)
    b = serve.ContinuousBatcher([None] * 4, slots=2, hbm_budget=1, executor=gpu,
                                footprint=lambda r: 10)
    res = b.run(reqs, realtime=False)
    assert res["frames"] == 40
    assert all(len(x) == 1 for x in b.batches)


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert serve.percentile(xs, 50) == 50
    assert serve.percentile(xs, 99) == 99
    assert serve.percentile([5.0], 99) == 5.0
