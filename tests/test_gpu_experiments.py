"""The experiment harness runs end to end on the tiny workload through the library calls, its
reference converges, and its metrics are finite."""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import paper_2507_19718_amd as gsc
    from paper_2507_19718_amd import experiments as ex
    wl = synth.workload("tiny")
    vol = wl.volume()
    ctx = gsc.Context(0)
    gv = gsc.Volume.from_synth(vol)
    init = gsc.gsc_cache_init(ctx, gv, 8192, wl.K, wl.seed)
    return dict(gsc=gsc, ex=ex, wl=wl, vol=vol, ctx=ctx, gv=gv, init=init, cam=wl.camera())


def test_reference_converges(env):
    ex, e = env["ex"], env
    a = ex.reference_radiance(e["ctx"], e["gv"], e["cam"], e["wl"].K, e["wl"].max_bounces, 1, spp=256)
    b = ex.reference_radiance(e["ctx"], e["gv"], e["cam"], e["wl"].K, e["wl"].max_bounces, 2, spp=256)
    rel = float((a - b).norm() / (0.5 * (a + b)).norm())
    assert rel < 0.2, rel
    # 4x the samples halves the difference (Monte Carlo rate), up to noise.
    c = ex.reference_radiance(e["ctx"], e["gv"], e["cam"], e["wl"].K, e["wl"].max_bounces, 3, spp=1024)
    d = ex.reference_radiance(e["ctx"], e["gv"], e["cam"], e["wl"].K, e["wl"].max_bounces, 4, spp=1024)
    rel4 = float((c - d).norm() / (0.5 * (c + d)).norm())
    assert 0.3 < rel4 / rel < 0.75, (rel, rel4)


def test_studies_run(env):
    ex, e = env["ex"], env
    ref = ex.reference_radiance(e["ctx"], e["gv"], e["cam"], e["wl"].K, e["wl"].max_bounces, 5, spp=128)
    r = ex.study_C(e["ctx"], e["wl"], e["vol"], e["gv"], e["init"], ref, e["cam"], Cs=(0.5, math.inf),
                   warm=2, measure=4)
    assert len(r["cached"]) == 2
    for row in r["cached"]:
        assert all(math.isfinite(row[k]) for k in ("bias2", "variance", "mse"))
        assert row["mse"] >= row["bias2"] * 0.5
    c = ex.study_cold_start(e["ctx"], e["wl"], e["vol"], e["gv"], e["init"], ref, e["cam"], frames=8,
                            marks=(1, 4, 8))
    assert set(c["mse_after_frames"]) == {1, 4, 8}
    a = ex.study_ablation(e["ctx"], e["wl"], e["vol"], e["gv"], e["init"], ref, e["cam"], orbit=6,
                          still=4, marks=(1, 4))
    assert set(a["mse_at_still_frames"]) == {"ours", "-REG", "-CO", "-CO,-REG"}
    for v in a["mse_at_still_frames"].values():
        assert all(math.isfinite(x) for x in v.values())


def test_estimator_study_with_area_lights(env):
    """Under area lights both uncached estimators and the cache produce finite errors, and
    MIS next-event estimation beats phase sampling alone at 1 spp."""
    ex, e, gsc = env["ex"], env, env["gsc"]
    vol = e["wl"].volume()
    vol.lights = vol.lights[:0]
    vol.spheres = synth.sphere_lights(2)
    gv = gsc.Volume.from_synth(vol)
    ref = ex.reference_radiance(e["ctx"], gv, e["cam"], e["wl"].K, e["wl"].max_bounces, 6, spp=256)
    assert float(ref.max()) > 0
    r = ex.study_estimators(e["ctx"], e["wl"], gv, e["init"], ref, e["cam"], warm=4, measure=4)
    res = r["results"]
    assert set(res) == {"PT_uniform", "PT_nee", "GSCache"}
    assert all(math.isfinite(v["mse"]) for v in res.values())
    assert res["PT_nee"]["mse"] < res["PT_uniform"]["mse"]


def test_spp_study_cache_cost_constant(env):
    """Several samples per pixel: the cache stages cost the same at 1 and 8 spp (they run once
    per frame), the trace does not."""
    ex, e = env["ex"], env
    ref = ex.reference_radiance(e["ctx"], e["gv"], e["cam"], e["wl"].K, e["wl"].max_bounces, 7, spp=128)
    r = ex.study_spp(e["ctx"], e["wl"], e["gv"], e["init"], ref, e["cam"], spps=(1, 8), warm=2, measure=3)
    a, b = r["rows"]
    assert (a["spp"], b["spp"]) == (1, 8)
    assert all(math.isfinite(x["mse_cached"]) and math.isfinite(x["mse_path_traced"]) for x in (a, b))
    assert b["mse_path_traced"] < a["mse_path_traced"]
