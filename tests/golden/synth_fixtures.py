"""SHA-256 of every seeded input generator's output at small sizes (the byte-stability fixture of
the synthetic inputs).  Run as a script to rewrite synth_sha256.json; the test recomputes the
same digests.  Calls only synth/."""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_sha256.json")


def _digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def _gauss(g) -> str:
    return _digest(g.pos, g.rot, g.log_scale, g.rgb, g.opacity_logit)


def _cam(c) -> str:
    return _digest(c.R, c.t, np.array([c.fx, c.fy, c.cx, c.cy, c.znear], np.float64),
                   np.array([c.full_w, c.full_h, c.x0, c.y0, c.w, c.h], np.int64))


def fixtures() -> dict:
    seed = 0x47534301
    fbm = synth.fbm_volume(32, seed)
    slabs = synth.slab_volume(fbm.copy(), seed)
    cam = synth.orbit_camera(320, 200, azimuth_deg=35.0)
    return {
        "blob_volume(32)": _digest(synth.blob_volume(32, seed)),
        "fbm_volume(32)": _digest(fbm),
        "slab_volume(fbm 32)": _digest(slabs),
        "transfer_function(16)": _digest(synth.transfer_function(16, seed)),
        "transfer_function(16, index 1)": _digest(synth.transfer_function(16, seed, 1)),
        "point_lights(2)": _digest(synth.point_lights(2)),
        "sphere_lights(2)": _digest(synth.sphere_lights(2)),
        "tiny_gaussians(256)": _gauss(synth.tiny_gaussians(256, seed)),
        "random_gaussians(1000, level 1)": _gauss(synth.random_gaussians(1000, seed, 1)),
        "frustum_gaussians(500)": _gauss(synth.frustum_gaussians(cam, 500, seed)),
        "orbit_camera(320x200, 35 deg)": _cam(cam),
        "crop_camera": _cam(cam.crop(17, 9, 100, 80)),
        "poisson_requests(240 Hz, 0.5 s)": _digest(np.array(
            [[r["t_arrival"], r["viewer"], r["scene"], r["width"], r["height"], r["azimuth"],
              r["elevation"], r["radius"], r["seed"]]
             for r in synth.poisson_requests(240.0, 0.5, 8, 3, seed)], np.float64)),
    }


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(fixtures(), f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", OUT)
