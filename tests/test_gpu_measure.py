"""The measurement side through the C ABI: the splat kernels' work counters and the ceiling
micro-benchmarks the rooflines are held against."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


@pytest.fixture(scope="module")
def gctx(gsc):
    return gsc.Context(0)


def test_work_counters_of_a_training_frame(gsc, gctx):
    """The adjoint blends exactly the pairs the forward blended (it walks each pixel up to its
    last blended entry and re-takes the same fp32 decisions); every count is consistent with the
    pairs evaluated, and the counting variants render the same frame as the plain kernels."""
    wl = synth.workload("tiny")
    cam = wl.camera()
    vol = wl.volume()
    lv = [gsc.level_to_device(g) for g in wl.gaussians()]
    scenes = [gsc.Scene(gctx, gsc.Volume.from_synth(vol), lv) for _ in range(2)]
    images = [torch.empty((cam.h, cam.w, 3), device="cuda") for _ in range(2)]
    req = gsc.frame_request(cam, wl.seed, 0, wl.K, wl.max_bounces, loss=wl.loss, lr=wl.lr,
                            weight_decay=wl.weight_decay, C=wl.C)
    s0 = gsc.gsc_render_frame(gctx, scenes[0], req, images[0], stats=True)
    c0 = gctx.counters()
    gctx.set_work_counters(True)
    try:
        s1 = gsc.gsc_render_frame(gctx, scenes[1], req, images[1], stats=True)
    finally:
        gctx.set_work_counters(False)
    c1 = gctx.counters()
    d = {k: c1[k] - c0[k] for k in c1}
    assert torch.equal(images[0], images[1]) and s0["loss"] == s1["loss"]
    assert d["blended"] > 0
    assert d["bwd_blended"] == d["blended"]
    assert d["blended"] <= d["fwd_tested"] <= 64 * d["fwd_slots"]
    assert d["bwd_blended"] <= d["bwd_tested"] <= 64 * d["bwd_slots"]
    assert d["fwd_tested"] <= d["evaluations"]
    # (The adjoint's wavefronts of one frame tile walk its list from the tile's last
    # contributor, so they may walk more entries than the forward's wavefronts evaluated.)
    assert d["bwd_entries"] > 0
    # At most nine float atomics per walked (tile, entry) pair, at least one per pair that
    # blended anything; they go out as one record of up to nine adds per such pair.
    assert 0 < d["bwd_atomics"] <= 9 * d["bwd_entries"]
    assert 0 < d["bwd_records"] <= d["bwd_entries"]
    assert d["bwd_records"] <= d["bwd_atomics"] <= 9 * d["bwd_records"]


def test_ceiling_probes(gsc, gctx):
    buf = torch.zeros(1 << 20, dtype=torch.float32, device="cuda")
    threads, per = 256 * 64, 8
    ms = gctx.probe_atomics(buf, threads, per)
    assert ms > 0.0
    # Every add of 1.0 lands exactly (no element is near 2^24).
    assert float(buf.double().sum().item()) == threads * per
    cells = torch.ones(32 * 4096, dtype=torch.uint8, device="cuda")
    assert gctx.probe_gather(cells, 256 * 16, 16) > 0.0
    for mode in (0, 1):
        assert gctx.probe_valu(256 * 16, 64, mode) > 0.0
    with pytest.raises(gsc.GscError):
        gctx.probe_valu(100, 64, 0)                 # threads not a multiple of 256
    with pytest.raises(gsc.GscError):
        gctx.probe_gather(cells, 256, 12)           # per_thread not a multiple of 8
