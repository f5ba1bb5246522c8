"""Binning at the size limits: a 16384x16384 window (the largest the library takes, 2^20 tiles)
and large splats, so that one level holds more than 2^32 tile instances and the runs of many
tiles start beyond the 32-bit range.  The instance count, every tile's run length and the run
partition are checked against the oracle's projection over all tiles; the runs of sampled
tiles, among them tiles whose runs start beyond 2^32 and the last tile, are compared with the
brute-force depth-sorted list of the Gaussians whose tile rectangle contains the tile."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


def tile_counts(pr, TX, TY):
    r = pr["rect"][pr["tiles"] > 0].astype(np.int64)       # inclusive tile rectangles
    d = np.zeros((TY + 1, TX + 1), np.int64)
    np.add.at(d, (r[:, 2], r[:, 0]), 1)
    np.add.at(d, (r[:, 2], r[:, 1] + 1), -1)
    np.add.at(d, (r[:, 3] + 1, r[:, 0]), -1)
    np.add.at(d, (r[:, 3] + 1, r[:, 1] + 1), 1)
    return d.cumsum(0).cumsum(1)[:TY, :TX].ravel()


def oracle_tile_list(pr, tx, ty):
    r = pr["rect"]
    hit = (pr["tiles"] > 0) & (r[:, 0] <= tx) & (tx <= r[:, 1]) & (r[:, 2] <= ty) & (ty <= r[:, 3])
    ids = np.nonzero(hit)[0]
    bits = pr["depth"][ids].view(np.uint32)
    return ids[np.lexsort((ids, bits))].astype(np.uint32)


def test_binning_beyond_2_32_instances(gsc):
    cam = synth.orbit_camera(16384, 16384, azimuth_deg=25.0)
    g = synth.frustum_gaussians(cam, 160_000, seed=77, radius_px=(1100.0, 1500.0))
    pr = oracle.project(g, cam)
    total = int(pr["tiles"].astype(np.int64).sum())
    assert total > 2 ** 32, total                         # the premise of the test
    TX, TY = oracle.tiles_x(cam), oracle.tiles_y(cam)
    print(f"maxsize: {TX}x{TY} tiles, {total} instances", flush=True)
    ctx = gsc.Context(0)
    b = gsc.gsc_project_bin(ctx, [gsc.level_to_device(g)], cam)
    view = gsc.gsc_binning_view(ctx, b)
    assert view["n_instances"] == total
    ranges = to_np(view["ranges"]).view(np.uint64).astype(np.int64)
    cnt = ranges[:, 1] - ranges[:, 0]
    assert np.array_equal(cnt, tile_counts(pr, TX, TY))
    live = cnt > 0
    starts = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    assert np.array_equal(ranges[live, 0], starts[live]) and ranges[live, 1].max() == total
    rng = np.random.default_rng(1)
    beyond = np.nonzero(live & (ranges[:, 0] >= 2 ** 32))[0]
    assert beyond.size > 0
    live_ids = np.nonzero(live)[0]
    picks = np.unique(np.concatenate([rng.choice(live_ids, 6, replace=False),
                                      rng.choice(beyond, 6, replace=False), live_ids[-1:]]))
    values = view["values"]
    for t in picks:
        s, e = int(ranges[t, 0]), int(ranges[t, 1])
        got = values[s:e].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, oracle_tile_list(pr, int(t % TX), int(t // TX))), (int(t), s, e)
    print(f"maxsize: {picks.size} sampled tiles equal, {beyond.size} runs start beyond 2^32", flush=True)
