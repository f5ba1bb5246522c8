"""Per-frame and per-request metrics as JSON Lines (host side only).

One record per line, so a long run can be followed while it is written and cut at any line.

  * frame records: the frame number, the stage times of gsc_render_frame's statistics (ms), its
    work counters (Gaussians, tile instances, tiles, pixels, paths, path vertices), the loss,
    whether the AdamW step was skipped, and, when the caller measured it, the per-level cache
    error against a reference;
  * request records (serving): arrival, start and completion times of one request, its scene and
    viewer, and its latency (completion - arrival).

`read_jsonl` reads either kind back; `latency_percentiles` computes the serving summary's
nearest-rank p50 / p99 from request records.
"""
import json
import math
from typing import Dict, Iterable, Iterator, List, Optional, Sequence

STAGES = ("ms_project_bin", "ms_forward", "ms_trace", "ms_loss", "ms_backward", "ms_adam", "ms_total")
COUNTERS = ("gaussians", "instances", "tiles", "pixels", "paths", "path_vertices")


def _num(x):
    """JSON has no NaN or infinity: non-finite floats are written as null."""
    if isinstance(x, float) and not math.isfinite(x):
        return None
    return x


class JsonlLog:
    """Appends one JSON object per line to `path` (mode "w" starts the file afresh)."""

    def __init__(self, path: str, mode: str = "w"):
        if mode not in ("w", "a"):
            raise ValueError("mode must be 'w' or 'a'")
        self.path = path
        self._f = open(path, mode, encoding="utf-8")
        self.records = 0

    def write(self, record: Dict) -> None:
        self._f.write(json.dumps(record, allow_nan=False, separators=(",", ":")) + "\n")
        self._f.flush()
        self.records += 1

    def close(self) -> None:
        if not self._f.closed:
            self._f.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def frame_record(frame: int, stats: Dict, l2: Optional[Sequence[float]] = None, **extra) -> Dict:
    """A frame's record from gsc_render_frame(..., stats=True)'s dictionary."""
    rec = {"kind": "frame", "frame": int(frame),
           "ms": {k[3:]: _num(float(stats[k])) for k in STAGES if k in stats},
           "counters": {k: int(stats[k]) for k in COUNTERS if k in stats},
           "loss": _num(float(stats["loss"])) if "loss" in stats else None,
           "adam_skipped": bool(stats.get("adam_skipped", 0))}
    if l2 is not None:
        rec["l2"] = [_num(float(x)) for x in l2]
    for k, v in extra.items():
        rec[k] = _num(v) if isinstance(v, float) else v
    return rec


def request_record(r, t0: float = 0.0) -> Dict:
    """A served request's record (times in seconds from t0; latency in ms)."""
    done = r.t_done - t0 if math.isfinite(r.t_done) else None
    start = r.t_start - t0 if math.isfinite(r.t_start) else None
    lat = 1000.0 * (r.t_done - r.t_arrival) if math.isfinite(r.t_done) else None
    return {"kind": "request", "idx": int(r.idx), "scene": int(r.scene), "viewer": int(r.viewer),
            "frame": int(r.frame), "t_arrival": r.t_arrival - t0, "t_start": start, "t_done": done,
            "latency_ms": lat}


def write_requests(path: str, reqs: Iterable, t0: float = 0.0) -> int:
    with JsonlLog(path) as log:
        for r in reqs:
            log.write(request_record(r, t0))
        return log.records


def read_jsonl(path: str) -> Iterator[Dict]:
    with open(path, encoding="utf-8") as f:
        for line in f:
            line = line.strip()
            if line:
                yield json.loads(line)


def latency_percentiles(records: Iterable[Dict], skip_s: float = 0.0) -> Dict[str, Optional[float]]:
    """Nearest-rank p50 / p99 latency (ms) of the completed requests that arrived at or after
    skip_s seconds."""
    lat: List[float] = sorted(r["latency_ms"] for r in records
                              if r.get("kind") == "request" and r["latency_ms"] is not None
                              and r["t_arrival"] >= skip_s)

    def rank(q):
        if not lat:
            return None
        return lat[max(0, math.ceil(q / 100.0 * len(lat)) - 1)]

    return {"n": len(lat), "p50_ms": rank(50), "p99_ms": rank(99)}
