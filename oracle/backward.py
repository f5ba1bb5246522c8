"""Exact fp64 gradient of the splat forward -- TEST INFRASTRUCTURE ONLY (part of the oracle).

The forward that the paper rasterises each cache level with (Method: a path space radiance
cache; the 3D Gaussian splatting rasteriser) is restated here in plain PyTorch CPU ops in
float64, for *given* blended sets (the ordered list of Gaussians each pixel blended, as the fp32
brute-force forward decided them).  Its gradient with respect to the 14 per-Gaussian
parameters is then taken by reverse mode (torch.autograd) -- the plain definition of "the exact
gradient of that forward".  No tiling, no transmittance recovery by division, no atomics.

Also: `forward_f64` (the C++ oracle's independent fp64 forward, used to finite-difference the
result of this module) and `fd_gradient`.
"""
from __future__ import annotations

import ctypes
from typing import Dict

import numpy as np
import torch

from . import _cam_args, _f32, _p, lib

PARAM_NAMES = ("pos", "rot", "log_scale", "rgb", "opacity_logit")


def project_f64(pos, rot, log_scale, logit, cam) -> Dict[str, torch.Tensor]:
    """Activations, 3D covariance M M^T with M = R(q) diag(exp s), camera transform, EWA
    Jacobian (with the 1.3x frustum clamp on x/z and y/z), 2D covariance + 0.3 I, conic and the
    screen-space mean u = fx x/z + cx - 1/2 (pixel-index coordinates)."""
    d = torch.float64
    Rc = torch.as_tensor(np.asarray(cam.R, np.float64).reshape(3, 3), dtype=d)
    tc = torch.as_tensor(np.asarray(cam.t, np.float64), dtype=d)
    q = rot / torch.linalg.vector_norm(rot, dim=1, keepdim=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    Rq = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], dim=1)                                                       # (n, 3, 3)
    s = torch.exp(log_scale)
    M = Rq * s[:, None, :]
    S3 = M @ M.transpose(1, 2)
    xc = pos @ Rc.T + tc
    X, Y, Z = xc[:, 0], xc[:, 1], xc[:, 2]
    fx, fy = float(cam.fx), float(cam.fy)
    limx = 1.3 * (cam.full_w / (2.0 * fx))
    limy = 1.3 * (cam.full_h / (2.0 * fy))
    tx = torch.clamp(X / Z, -limx, limx) * Z
    ty = torch.clamp(Y / Z, -limy, limy) * Z
    zero = torch.zeros_like(Z)
    J = torch.stack([torch.stack([fx / Z, zero, -fx * tx / (Z * Z)], -1),
                     torch.stack([zero, fy / Z, -fy * ty / (Z * Z)], -1)], dim=1)   # (n, 2, 3)
    T = J @ Rc
    S2 = T @ S3 @ T.transpose(1, 2)
    a = S2[:, 0, 0] + 0.3
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + 0.3
    det = a * c - b * b
    return dict(u=fx * (X / Z) + (float(cam.cx) - 0.5), v=fy * (Y / Z) + (float(cam.cy) - 0.5),
                A=c / det, B=-b / det, Cc=a / det, o=torch.sigmoid(logit))


def render_lists_f64(proj: Dict[str, torch.Tensor], rgb: torch.Tensor, cam, list_off: np.ndarray,
                     list_ids: np.ndarray) -> torch.Tensor:
    """Front-to-back blending of each pixel's given ordered list:
    C = sum_k c_k alpha_k T_k, T_k = prod_{j<k} (1 - alpha_j), alpha = min(0.99, o e^power)."""
    H, W = cam.h, cam.w
    P = H * W
    counts = np.diff(list_off).astype(np.int64)
    Lmax = int(counts.max()) if P else 0
    if Lmax == 0:
        return torch.zeros((H, W, 3), dtype=torch.float64) + 0.0 * rgb.sum()
    idx = np.full((P, Lmax), 0, dtype=np.int64)
    mask = np.zeros((P, Lmax), dtype=bool)
    rows = np.repeat(np.arange(P), counts)
    cols = np.arange(list_ids.size) - np.repeat(list_off[:-1], counts)
    idx[rows, cols] = list_ids
    mask[rows, cols] = True
    idx_t = torch.from_numpy(idx)
    m = torch.from_numpy(mask).to(torch.float64)
    pi = torch.from_numpy((np.arange(P) % W + cam.x0).astype(np.float64))[:, None]
    pj = torch.from_numpy((np.arange(P) // W + cam.y0).astype(np.float64))[:, None]
    dx = proj["u"][idx_t] - pi
    dy = proj["v"][idx_t] - pj
    power = -0.5 * (proj["A"][idx_t] * dx * dx + proj["Cc"][idx_t] * dy * dy) \
        - proj["B"][idx_t] * dx * dy
    alpha = torch.clamp(proj["o"][idx_t] * torch.exp(power), max=0.99) * m
    one_minus = 1.0 - alpha
    T = torch.cumprod(torch.cat([torch.ones((P, 1), dtype=torch.float64), one_minus[:, :-1]], 1), 1)
    wgt = alpha * T                                                        # (P, Lmax)
    C = torch.einsum("pk,pkc->pc", wgt, rgb[idx_t])
    return C.reshape(H, W, 3)


def params_f64(g, requires_grad=True):
    ts = [torch.tensor(np.asarray(a, np.float64), requires_grad=requires_grad)
          for a in (g.pos, g.rot, g.log_scale, g.rgb, g.opacity_logit)]
    return ts


def backward(g, cam, fwd: dict, dL_dimage: np.ndarray) -> Dict[str, np.ndarray]:
    """Gradient of sum_p sum_c dL_dimage[p, c] * image[p, c] with respect to the 14 parameters
    of every Gaussian, in fp64, for the blended lists in `fwd` (oracle.forward(lists=True))."""
    pos, rot, ls, rgb, logit = params_f64(g)
    proj = project_f64(pos, rot, ls, logit, cam)
    img = render_lists_f64(proj, rgb, cam, fwd["list_off"], fwd["list_ids"])
    G = torch.as_tensor(np.asarray(dL_dimage, np.float64))
    (img * G).sum().backward()
    out = {}
    for name, t in zip(PARAM_NAMES, (pos, rot, ls, rgb, logit)):
        out[name] = (t.grad if t.grad is not None else torch.zeros_like(t)).numpy().copy()
    return out


def image_f64(g, cam, fwd: dict) -> np.ndarray:
    with torch.no_grad():
        pos, rot, ls, rgb, logit = params_f64(g, requires_grad=False)
        proj = project_f64(pos, rot, ls, logit, cam)
        return render_lists_f64(proj, rgb, cam, fwd["list_off"], fwd["list_ids"]).numpy()


def forward_f64(g, cam):
    """The C++ oracle's independent fp64 forward (decisions in double; `g` may hold float64
    arrays, which are used as given).  Returns the image
    [h][w][3] and a per-pixel signature of the blended set and 0.99-clamp states."""
    keep, cargs = _cam_args(cam)
    arrs = [np.ascontiguousarray(a, dtype=np.float64)
            for a in (g.pos, g.rot, g.log_scale, g.opacity_logit, g.rgb)]
    image = np.zeros((cam.h, cam.w, 3), dtype=np.float64)
    sig = np.zeros((cam.h, cam.w), dtype=np.uint64)
    lib().ora_forward_f64(*[_p(a) for a in arrs], ctypes.c_int64(g.n), *cargs, _p(image), _p(sig))
    return image, sig
