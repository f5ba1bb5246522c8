"""The cache follows a change of optics while frames keep training (Abstract; Introduction):
after the transfer function is replaced, and again after the light is moved, the cache's error
against the new optics' reference jumps, then falls as frames train on the new targets."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def test_cache_readapts_after_transfer_function_swap_and_light_move(tmp_path):
    import paper_2507_19718_amd as gsc
    from paper_2507_19718_amd import metrics
    from paper_2507_19718_amd.experiments import study_adapt
    ctx = gsc.Context(0)
    wl = synth.workload("tiny")
    cam = wl.camera()
    gv = gsc.Volume.from_synth(wl.volume())
    lv = [gsc.level_to_device(g) for g in wl.gaussians()]
    path = str(tmp_path / "adapt_frames.jsonl")
    with metrics.JsonlLog(path) as log:
        r = study_adapt(ctx, wl, gv, lv, cam, frames=360, changes=(160, 260), ref_spp=256, log=log)
    # One record per frame: the frame's statistics and the per-level error measured after it.
    recs = list(metrics.read_jsonl(path))
    assert [x["frame"] for x in recs] == list(range(360))
    assert [x["l2"] for x in recs] == [x["l2"] for x in r["per_frame"]]
    assert all(x["counters"]["instances"] > 0 and x["ms"]["total"] > 0 and x["loss"] is not None
               and not x["adam_skipped"] for x in recs)
    assert [x["t_view"] for x in recs if x["frame"] in (159, 160, 259, 260)] == [160, 1, 100, 1]
    ph = r["phases"]
    print({"phases": ph})
    print({"per_frame_total_l2": [round(sum(x["l2"]), 6) for x in r["per_frame"]]})
    assert len(ph) == 3 and len(r["per_frame"]) == 360
    assert all(torch.isfinite(torch.tensor(x["l2"])).all() for x in r["per_frame"])
    for p in (1, 2):
        before = sum(ph[p - 1]["l2_end"])
        stale = sum(ph[p]["l2_stale"])
        end = sum(ph[p]["l2_end"])
        # The change makes the trained cache wrong: its error against the new reference is
        # well above what it had reached under the old optics.
        assert stale > 1.5 * before, (p, stale, before)
        # Training on the new targets brings it down again, by half within 40 frames.
        assert end < 0.5 * stale, (p, end, stale)
        assert ph[p]["frames_to_halve_stale"] is not None and ph[p]["frames_to_halve_stale"] <= 40
