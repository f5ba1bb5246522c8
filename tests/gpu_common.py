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
    """Per parameter group: ||d||/||ref|| <= tol and elementwise |d_i| <= tol * max(|ref_i|,
    1e-2 rms(ref)) + a floor of 1e-7 rms(ref) for fp32 atomic accumulation of cancelling sums."""
    g = np.asarray(got, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    if rms == 0.0:
        return float(np.abs(g).max() if g.size else 0.0) == 0.0, (0.0, 0.0)
    l2 = rel_l2(g, r)
    bound = tol * np.maximum(np.abs(r), 1e-2 * rms)
    worst = float(np.max(np.abs(g - r) / bound))
    return l2 <= tol and worst <= 1.0, (l2, worst)
