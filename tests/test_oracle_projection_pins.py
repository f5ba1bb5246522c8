"""Pins of the oracle's projection against definitions outside the oracle (CPU).

The rasteriser the paper delegates to (Method: a path space radiance cache) projects each 3D
Gaussian by the EWA splatting approximation: the 3D covariance R(q) S^2 R(q)^T, moved into the
camera frame, mapped by the Jacobian of the perspective map evaluated at the Gaussian's centre
(clamped to 1.3x the field of view), plus 0.3 px^2 on the diagonal.  Two parts of that are
pinned here against something other than a second statement of the same formulas:

* R(q), the rotation matrix of a unit quaternion (w, x, y, z), by scipy's
  ``Rotation.from_quat`` (scalar-last input order) -- a conjugated quaternion or a wrong sign
  would swap R and R^T, which anisotropic scales expose;
* the EWA Jacobian, by fp64 central differences of the perspective map
  (x, y, z) -> (fx x / z, fy y / z) at the clamped point, inside and outside the clamp.

Both the fp32 C++ oracle (the bit-exact projection contract) and the fp64 statement used by the
gradient oracle are compared with the independent covariance.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth


def perspective(cam, p):
    return np.array([cam.fx * p[0] / p[2], cam.fy * p[1] / p[2]])


def fd_jacobian(cam, p, rel=1e-6):
    """Central differences of the perspective map at p (2 x 3)."""
    J = np.zeros((2, 3))
    for k in range(3):
        h = rel * max(abs(p[2]), 1.0)
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (perspective(cam, p + e) - perspective(cam, p - e)) / (2 * h)
    return J


def independent_conic(g, cam):
    """(A, B, C, u, v, clamped) per Gaussian from scipy's rotation and the differenced Jacobian."""
    Rc = np.asarray(cam.R, np.float64).reshape(3, 3)
    tc = np.asarray(cam.t, np.float64)
    limx = 1.3 * cam.full_w / (2.0 * cam.fx)
    limy = 1.3 * cam.full_h / (2.0 * cam.fy)
    out = np.zeros((g.n, 6))
    q = np.asarray(g.rot, np.float64)
    Rq = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()       # scipy: (x, y, z, w)
    for i in range(g.n):
        S = np.diag(np.exp(2.0 * np.asarray(g.log_scale[i], np.float64)))
        S3 = Rq[i] @ S @ Rq[i].T
        xc = Rc @ np.asarray(g.pos[i], np.float64) + tc
        x, y, z = xc
        cx_ = min(max(x / z, -limx), limx)
        cy_ = min(max(y / z, -limy), limy)
        clamped = (cx_ != x / z) or (cy_ != y / z)
        J = fd_jacobian(cam, np.array([cx_ * z, cy_ * z, z]))
        S2 = J @ Rc @ S3 @ Rc.T @ J.T + 0.3 * np.eye(2)
        inv = np.linalg.inv(S2)
        uv = perspective(cam, xc) + np.array([cam.cx - 0.5, cam.cy - 0.5])
        out[i] = (inv[0, 0], inv[0, 1], inv[1, 1], uv[0], uv[1], float(clamped))
    return out


def pin_cases():
    cam = synth.orbit_camera(320, 240, azimuth_deg=70.0)
    inside = synth.random_gaussians(400, 91, log_scale_mean=-3.0, log_scale_std=0.8)
    # Gaussians placed at 1.1x .. 2.5x of the half field of view (outside the 1.3x clamp for
    # most), so the Jacobian is taken at the clamped point.
    rng = np.random.default_rng(5)
    n = 200
    Rc = np.asarray(cam.R, np.float64).reshape(3, 3)
    tc = np.asarray(cam.t, np.float64)
    z = rng.uniform(1.0, 2.5, n)
    k = rng.uniform(1.1, 2.5, n) * rng.choice([-1.0, 1.0], n)
    ky = rng.uniform(-1.5, 1.5, n)
    xc = np.stack([k * cam.full_w / (2 * cam.fx) * z, ky * cam.full_h / (2 * cam.fy) * z, z], 1)
    pos = (xc - tc) @ Rc
    outside = synth.random_gaussians(n, 92, log_scale_mean=-2.5, log_scale_std=0.8)
    outside.pos[:] = pos.astype(np.float32)
    return cam, inside, outside


@pytest.mark.parametrize("which", ["inside", "outside"])
def test_conic_pinned_by_scipy_rotation_and_differenced_jacobian(ora, which):
    import torch
    from oracle import backward as B
    cam, inside, outside = pin_cases()
    g = inside if which == "inside" else outside
    ref = independent_conic(g, cam)
    clamped = ref[:, 5] > 0
    if which == "outside":
        assert clamped.mean() > 0.5          # the clamp branch is what this case exercises
    else:
        assert not clamped.all()
    pr = ora.project(g, cam)
    z_ok = pr["depth"] > cam.znear
    assert z_ok.sum() > 0.9 * g.n
    # fp32 oracle (bit-exact contract): rounding of a well-conditioned 2x2 inverse.
    scr = pr["screen"].astype(np.float64)
    for col, k in ((2, 0), (3, 1), (4, 2)):
        got, want = scr[z_ok, col], ref[z_ok, k]
        scale = np.maximum(np.abs(want), 1e-3 * np.abs(ref[z_ok, 0]) + 1e-3 * np.abs(ref[z_ok, 2]))
        assert np.max(np.abs(got - want) / scale) < 1e-4, (which, col)
    assert np.max(np.abs(scr[z_ok, 0] - ref[z_ok, 3])) < 2e-3
    assert np.max(np.abs(scr[z_ok, 1] - ref[z_ok, 4])) < 2e-3
    # fp64 statement used by the gradient oracle.
    t = [torch.tensor(np.asarray(a, np.float64)) for a in (g.pos, g.rot, g.log_scale, g.opacity_logit)]
    P = B.project_f64(t[0], t[1], t[2], t[3], cam)
    for name, k in (("A", 0), ("B", 1), ("Cc", 2)):
        got = P[name].numpy()[z_ok]
        want = ref[z_ok, k]
        scale = np.abs(ref[z_ok, 0]) + np.abs(ref[z_ok, 2])
        assert np.max(np.abs(got - want) / scale) < 1e-8, (which, name)
    assert np.max(np.abs(P["u"].numpy()[z_ok] - ref[z_ok, 3])) < 1e-8
    assert np.max(np.abs(P["v"].numpy()[z_ok] - ref[z_ok, 4])) < 1e-8


def test_pin_detects_a_conjugated_quaternion_and_a_flipped_jacobian_term(ora):
    """The independent covariance differs from what a conjugated quaternion (R^T in place of R)
    or a sign error in the depth column of the Jacobian would give, by far more than the
    tolerances above, on these inputs."""
    cam, inside, _ = pin_cases()
    g = inside
    ref = independent_conic(g, cam)
    Rc = np.asarray(cam.R, np.float64).reshape(3, 3)
    tc = np.asarray(cam.t, np.float64)
    q = np.asarray(g.rot, np.float64)
    Rq = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    worst_conj, worst_sign = 0.0, 0.0
    for i in range(g.n):
        S = np.diag(np.exp(2.0 * np.asarray(g.log_scale[i], np.float64)))
        xc = Rc @ np.asarray(g.pos[i], np.float64) + tc
        if xc[2] <= cam.znear:
            continue
        J = fd_jacobian(cam, xc)
        Jbad = J.copy()
        Jbad[:, 2] = -Jbad[:, 2]
        for Rm, Jm, tag in ((Rq[i].T, J, "conj"), (Rq[i], Jbad, "sign")):
            S2 = Jm @ Rc @ (Rm @ S @ Rm.T) @ Rc.T @ Jm.T + 0.3 * np.eye(2)
            inv = np.linalg.inv(S2)
            d = max(abs(inv[0, 0] - ref[i, 0]), abs(inv[0, 1] - ref[i, 1]),
                    abs(inv[1, 1] - ref[i, 2])) / (abs(ref[i, 0]) + abs(ref[i, 2]))
            if tag == "conj":
                worst_conj = max(worst_conj, d)
            else:
                worst_sign = max(worst_sign, d)
    assert worst_conj > 1e-2 and worst_sign > 1e-3, (worst_conj, worst_sign)
