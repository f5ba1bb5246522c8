"""JSON Lines metrics (CPU only): frame records from a frame's statistics, request records from
served requests, and the nearest-rank latency summary read back from them."""
import json
import math

import numpy as np

from paper_2507_19718_amd import metrics
from paper_2507_19718_amd.serve import Request, percentile, summarize


def _stats(loss=0.25, skipped=0):
    return {"ms_project_bin": 1.5, "ms_forward": 2.0, "ms_trace": 1.25, "ms_loss": 0.125,
            "ms_backward": 3.0, "ms_adam": 0.375, "ms_total": 7.0, "gaussians": 4_000_000,
            "instances": 61_000_000, "tiles": 8160, "pixels": 2_073_600, "paths": 2_073_600,
            "path_vertices": 3_000_000, "loss": loss, "adam_skipped": skipped}


def test_frame_records_round_trip(tmp_path):
    p = tmp_path / "frames.jsonl"
    with metrics.JsonlLog(str(p)) as log:
        log.write(metrics.frame_record(0, _stats(), l2=[1e-3, 2e-3, 4e-3], phase=0, t_view=1))
        log.write(metrics.frame_record(1, _stats(loss=math.inf, skipped=1), phase=0, t_view=2))
        assert log.records == 2
    lines = p.read_text().splitlines()
    assert len(lines) == 2
    r0, r1 = (json.loads(x) for x in lines)
    assert r0["kind"] == "frame" and r0["frame"] == 0 and r0["l2"] == [1e-3, 2e-3, 4e-3]
    assert r0["ms"]["total"] == 7.0 and r0["ms"]["backward"] == 3.0
    assert r0["counters"]["instances"] == 61_000_000 and r0["loss"] == 0.25
    assert r0["adam_skipped"] is False and r0["t_view"] == 1
    # A non-finite loss is written as null (JSON has no infinity), and the skip is recorded.
    assert r1["loss"] is None and r1["adam_skipped"] is True and "l2" not in r1


def test_request_records_and_latency_summary(tmp_path):
    rng = np.random.default_rng(7)
    reqs = []
    t = 0.0
    for i in range(500):
        t += float(rng.exponential(1 / 240))
        r = Request(idx=i, t_arrival=t, scene=i % 4, viewer=i % 32, cam=None, frame=i // 4, seed=1)
        r.t_start = t + float(rng.exponential(0.002))
        r.t_done = r.t_start + float(rng.uniform(0.002, 0.02))
        reqs.append(r)
    p = tmp_path / "requests.jsonl"
    assert metrics.write_requests(str(p), reqs) == len(reqs)
    recs = list(metrics.read_jsonl(str(p)))
    assert [r["idx"] for r in recs] == list(range(500))
    assert all(r["t_start"] >= r["t_arrival"] and r["t_done"] >= r["t_start"] for r in recs)
    # The percentiles read back from the file equal the serving summary's (nearest rank), with
    # and without the first two seconds left out.
    for skip in (0.0, 1.0):
        got = metrics.latency_percentiles(recs, skip_s=skip)
        want = summarize(reqs, 0.0, t, skip_s=skip)
        assert got["p50_ms"] == want["p50_ms"] and got["p99_ms"] == want["p99_ms"]
    lat = [1000.0 * (r.t_done - r.t_arrival) for r in reqs]
    assert metrics.latency_percentiles(recs)["p99_ms"] == percentile(lat, 99)


def test_unfinished_request_has_no_latency():
    r = Request(idx=3, t_arrival=0.5, scene=0, viewer=1, cam=None, frame=0, seed=1)
    rec = metrics.request_record(r)
    assert rec["t_start"] is None and rec["t_done"] is None and rec["latency_ms"] is None
    assert metrics.latency_percentiles([rec]) == {"n": 0, "p50_ms": None, "p99_ms": None}
