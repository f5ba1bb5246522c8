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
    gradient is a strongly cancelling sum: every fp32 path evaluates the pairs at the fp32
    screen values of the bit-exact projection (u ~ 1e3 px carries ~6e-5 px of rounding), and
    the exact gradient at those rounded values already differs from the reference by up to
    0.58 of this bound, and by up to 115x the bound 1e-4 max(|ref_i|, 1e-2 rms)
    (tests/test_oracle_gradient_conditioning.py measures it on the backward parity cases)."""
    g = np.asarray(got, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    if rms == 0.0:
        return float(np.abs(g).max() if g.size else 0.0) == 0.0, (0.0, 0.0)
    l2 = rel_l2(g, r)
    bound = tol * np.abs(r) + 2.0 * tol * rms
    worst = float(np.max(np.abs(g - r) / bound))
    return l2 <= tol and worst <= 1.0, (l2, worst)


GROUP_OFFSETS = (0, 3, 7, 10, 13, 14)     # pos, rot, log_scale, rgb, opacity_logit (x n)


def adamw_params_close(got, want, before, grads_ref, lrs, n, frac=2e-3):
    """Parameters after a training frame's AdamW step, per group with learning rate lr:
    where the oracle's gradient is well above the gradient tolerance, |got - want| <= frac lr (a
    gradient within 1e-4 relative moves the normalised AdamW step by ~1e-4 lr); elsewhere AdamW
    normalises rounding noise into a step of up to lr on either side, so only |got - before|
    <= 4 lr is required there.  A group with lr 0 must not move at all.  Returns (ok, info)."""
    got, want, before, g = (np.asarray(a, np.float64).ravel() for a in (got, want, before, grads_ref))
    gmax_all = float(np.abs(g).max()) if g.size else 0.0
    for k in range(5):
        s = slice(GROUP_OFFSETS[k] * n, GROUP_OFFSETS[k + 1] * n)
        lr = float(lrs[k])
        if lr == 0.0:
            if not (np.array_equal(got[s], before[s]) and np.array_equal(want[s], before[s])):
                return False, (k, "moved with lr 0")
            continue
        ga = np.abs(g[s])
        # A group whose exact gradient vanishes (the rotation of isotropic Gaussians) holds only
        # fp64 rounding noise: only the step bound applies to it.
        if ga.size == 0 or ga.max() <= 1e-9 * gmax_all:
            if ga.size and float(np.max(np.abs(got[s] - before[s]))) > 4.0 * lr:
                return False, (k, "step bound")
            continue
        # Tight elements: above 1e-3 of the group's largest and above 0.1 rms, where the
        # gradient bound (1e-4 |g| + 2e-4 rms) is at most 2.1e-3 |g| relative.
        tight = (ga > 1e-3 * ga.max()) & (ga > 0.1 * float(np.sqrt(np.mean(ga * ga))))
        if tight.mean() <= 0.05:
            return False, (k, "few tight elements", float(tight.mean()))
        err = float(np.max(np.abs(got[s] - want[s])[tight]))
        if err > frac * lr:
            return False, (k, "tight", err / lr)
        if float(np.max(np.abs(got[s] - before[s]))) > 4.0 * lr:
            return False, (k, "step bound")
    return True, None
