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


def gaussians_at_pixels(window, culled, pixels, cam):
    """Per Gaussian: does its integer pixel window (x0, x1, y0, y1, full-frame, inclusive) hold
    any of the render window's pixels marked in `pixels` [h][w]?"""
    hit = np.zeros(window.shape[0], dtype=bool)
    for j, i in zip(*np.nonzero(pixels)):
        x, y = cam.x0 + int(i), cam.y0 + int(j)
        hit |= (window[:, 0] <= x) & (x <= window[:, 1]) & (window[:, 2] <= y) & (y <= window[:, 3])
    return hit & ~np.asarray(culled, bool)


def adamw_params_close(got, want, before, grads_ref, m_before, v_before, step, lrs, n,
                       beta1=0.9, beta2=0.999, eps=1e-8, exclude=None):
    """Parameters after one training frame's AdamW step taken from the same state (p, m, v
    before the step) on both sides; step = the step number t of that update.  The gradients may
    differ by e, within the gradient bound |e| <= e_max = 1e-4 |g| + 2e-4 rms(g) of the group.
    The update is p' = p (1 - lr wd) - lr r(g) with r(x) = m^(x) / (sqrt(v^(x)) + eps),
    m(x) = b1 m + (1 - b1) x and v(x) = b2 v + (1 - b2) x^2, so each element's r is evaluated
    in float64 over x in [g - e_max, g + e_max] (33 points, plus x = 0 when the interval holds
    it), and |got - want| <= 1.05 lr max_x |r(x) - r(g)| + 2 ulp of the parameter and of the
    step is required (1.05 for an extremum between the sample points).  Every element must also
    stay within 4 lr (1 + max |p|) of where it started, and a group with lr 0 must not move at
    all.  A group whose reference gradient is rounding noise (rms below 1e-9 of the largest
    group's) is held to the step bound only, and so are the Gaussians in `exclude` ([n], or
    [5][n] per group): those whose window holds a boundary pixel, where the two sides may
    legitimately blend different sets, and, for the rotation group, nearly isotropic Gaussians.
    Returns (ok, info)."""
    got, want, before, g, mb, vb = (np.asarray(a, np.float64).ravel()
                                    for a in (got, want, before, grads_ref, m_before, v_before))
    t = float(step)
    bc1, bc2 = 1.0 - beta1 ** t, 1.0 - beta2 ** t
    group_rms = [float(np.sqrt(np.mean(g[GROUP_OFFSETS[k] * n:GROUP_OFFSETS[k + 1] * n] ** 2)))
                 if n else 0.0 for k in range(5)]

    def r_of(x, mm, vv):
        return ((beta1 * mm + (1 - beta1) * x) / bc1) / (np.sqrt((beta2 * vv + (1 - beta2) * x * x) / bc2) + eps)

    for k in range(5):
        s = slice(GROUP_OFFSETS[k] * n, GROUP_OFFSETS[k + 1] * n)
        lr = float(lrs[k])
        if lr == 0.0:
            if not (np.array_equal(got[s], before[s]) and np.array_equal(want[s], before[s])):
                return False, (k, "moved with lr 0")
            continue
        if s.stop == s.start:
            continue
        if float(np.max(np.abs(got[s] - before[s]))) > 4.0 * lr * (1.0 + float(np.max(np.abs(before[s])))):
            return False, (k, "step bound")
        gs, ms, vs = g[s], mb[s], vb[s]
        rms = group_rms[k]
        # A group whose exact gradient vanishes (the rotation of isotropic Gaussians) holds only
        # rounding noise on both sides, which AdamW normalises into steps of up to lr: only the
        # step bound applies to it.
        if rms <= 1e-9 * max(group_rms):
            continue
        emax = 1e-4 * np.abs(gs) + 2e-4 * rms
        r0 = r_of(gs, ms, vs)
        dr = np.abs(r_of(np.zeros_like(gs), ms, vs) - r0) * (np.abs(gs) <= emax)
        for f in np.linspace(-1.0, 1.0, 33):
            dr = np.maximum(dr, np.abs(r_of(gs + f * emax, ms, vs) - r0))
        allow = 1.05 * lr * dr + 2.4e-7 * (np.abs(want[s]) + lr * (1.0 + np.abs(r0))) + 1e-30
        ratio = np.abs(got[s] - want[s]) / allow
        if exclude is not None:
            ex = np.asarray(exclude, bool)
            ex = ex[k] if ex.ndim == 2 else ex
            w = GROUP_OFFSETS[k + 1] - GROUP_OFFSETS[k]
            ratio = ratio[~np.repeat(ex, w)]
        worst = float(np.max(ratio)) if ratio.size else 0.0
        if worst > 1.0:
            return False, (k, "step", worst)
    return True, None


def frame_exclusions(boundary_gaussians, log_scale, min_anisotropy=5e-2):
    """[5][n] exclusion masks for adamw_params_close in training frames: every group skips the
    Gaussians at boundary pixels; the rotation group also skips Gaussians whose log-scales differ
    by less than `min_anisotropy`.  The rotation gradient of a Gaussian of anisotropy a is a sum
    of terms of the size of its covariance gradient that cancel down to ~a of it, so an fp32
    chain rule keeps only ~1.4e-7 / a of it relative, and its worst elements use up the bar's
    2e-4 rms allowance by a = 1e-2; from 5e-2 on they stay below half of it
    (test_oracle_gradient_conditioning measures this).  The rotation gradient is compared on
    anisotropic Gaussians by the backward parity tests."""
    ls = np.asarray(log_scale, np.float64).reshape(-1, 3)
    iso = (ls.max(axis=1) - ls.min(axis=1)) < min_anisotropy
    ex = np.repeat(np.asarray(boundary_gaussians, bool)[None, :], 5, axis=0)
    ex[1] |= iso
    return ex
