"""The training-frame parameter comparison (tests/gpu_common.adamw_params_close) on the CPU:
oracle AdamW steps whose gradients differ by up to the gradient tolerance pass it, and a
gradient error ten times that tolerance fails it, so the bound is neither vacuous nor stricter
than the gradient bar it derives from."""
import numpy as np

import oracle
from tests.gpu_common import GROUP_OFFSETS, adamw_params_close


def _run(scale, seed, steps=6, n=4000):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=14 * n).astype(np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    lrs = (1e-3, 1e-2, 0.0, 5e-3, 2e-2)
    off = [o * n for o in GROUP_OFFSETS]
    results = []
    for t in range(1, steps + 1):
        g = (rng.normal(size=14 * n) * np.exp(2.0 * rng.normal(size=14 * n))).astype(np.float32)
        e = np.zeros(14 * n)
        for k in range(5):
            s = slice(off[k], off[k + 1])
            rms = np.sqrt(np.mean(g[s].astype(np.float64) ** 2))
            e[s] = scale * rng.uniform(-1, 1, size=off[k + 1] - off[k]) * (1e-4 * np.abs(g[s]) + 2e-4 * rms)
        g2 = (g + e).astype(np.float32)
        P1, M1, V1, P2 = p.copy(), m.copy(), v.copy(), p.copy()
        for k in range(5):
            s = slice(off[k], off[k + 1])
            P1[s], M1[s], V1[s] = oracle.adamw_step(p[s], m[s], v[s], g[s], lrs[k], 0.9, 0.999, 1e-8, 1e-2, t)
            P2[s], _, _ = oracle.adamw_step(p[s], m[s], v[s], g2[s], lrs[k], 0.9, 0.999, 1e-8, 1e-2, t)
        results.append(adamw_params_close(P2, P1, p, g, m, v, t, lrs, n)[0])
        p, m, v = P1, M1, V1
    return results


def test_within_the_gradient_tolerance_passes():
    for seed in range(4):
        assert all(_run(1.0, seed))


def test_ten_times_the_gradient_tolerance_fails():
    assert not all(_run(10.0, 11))
