"""Shared helpers of the GPU parity tests (inputs and comparisons; no method arithmetic)."""
import numpy as np
import torch

import synth


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def u32(t: torch.Tensor) -> np.ndarray:
    return to_np(t).view(np.uint32)


def u64(t: torch.Tensor) -> np.ndarray:
    return to_np(t).view(np.uint64)


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def forward_close(got: np.ndarray, ref: np.ndarray, mask: np.ndarray, tol: float = 1e-5):
    """The forward criterion: relative L2 and max-abs (relative to max |ref|) within `tol`
    over the pixels of `mask`."""
    g = got[mask].astype(np.float64)
    r = ref[mask].astype(np.float64)
    l2 = rel_l2(g, r)
    mx = float(np.abs(g - r).max()) if g.size else 0.0
    scale = float(np.abs(r).max()) if r.size else 1.0
    return l2 <= tol and mx <= tol * max(scale, 1e-30), (l2, mx, scale)


def grads_close(got: np.ndarray, ref: np.ndarray, tol: float = 1e-4):
    """Per parameter group: ||d|| / ||ref|| <= tol (the 1e-4 relative bar on gradients), and
    elementwise |d_i| <= tol |ref_i| + 2 tol rms(ref).  The absolute floor covers elements whose
    gradient is a strongly cancelling sum: the fp32 path evaluates every pair at screen
    coordinates rounded to fp32 (u ~ 1e3 px carries ~1e-4 px of rounding, which moves a small
    splat's alpha by ~1e-4 relative), so a sum of terms of size ~rms that cancels to ~0 keeps an
    absolute error of order 1e-4 rms."""
    g = np.asarray(got, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    if rms == 0.0:
        return float(np.abs(g).max() if g.size else 0.0) == 0.0, (0.0, 0.0)
    l2 = rel_l2(g, r)
    bound = tol * np.abs(r) + 2.0 * tol * rms
    worst = float(np.max(np.abs(g - r) / bound))
    return l2 <= tol and worst <= 1.0, (l2, worst)
