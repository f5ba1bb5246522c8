"""Pins of the oracle's random numbers and portable transcendentals (CPU).

Philox4x32-10 (Salmon et al., SC'11) is pinned through structure: a width-generic Philox
written here reproduces numpy's Philox4x64-10 bit generator (a library routine) exactly, and
the same generic code with the 32-bit multipliers and Weyl constants reproduces the oracle's
C++ Philox4x32-10.  The exp / log / sincos used by the bit-exact projection and by the tracer
are checked against float64 libm to <= 3 ulp over dense sweeps of their actual domains.
"""
import math

import numpy as np
import pytest

M64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
W64 = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
M32 = (0xD2511F53, 0xCD9E8D57)
W32 = (0x9E3779B9, 0xBB67AE85)


def philox_generic(ctr, key, width, mult, weyl, rounds=10):
    mask = (1 << width) - 1
    c, k = list(ctr), list(key)
    for r in range(rounds):
        if r:
            k = [(k[0] + weyl[0]) & mask, (k[1] + weyl[1]) & mask]
        p0, p1 = mult[0] * c[0], mult[1] * c[2]
        c = [(p1 >> width) ^ c[1] ^ k[0], p1 & mask, (p0 >> width) ^ c[3] ^ k[1], p0 & mask]
    return c


def test_generic_philox_matches_numpy_4x64():
    g = np.random.default_rng(1)
    for _ in range(20):
        key = [int(x) for x in g.integers(0, 2**63, size=2)]
        ctr = [int(x) for x in g.integers(0, 2**62, size=4)]
        bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
        raw = [int(x) for x in bg.random_raw(4)]
        nxt = list(ctr)
        nxt[0] += 1                         # numpy increments the counter before each block
        assert raw == philox_generic(nxt, key, 64, M64, W64)


def test_oracle_philox4x32_matches_generic(ora):
    g = np.random.default_rng(2)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)]
    for _ in range(200):
        cases.append(([int(x) for x in g.integers(0, 2**32, size=4)],
                      [int(x) for x in g.integers(0, 2**32, size=2)]))
    for ctr, key in cases:
        assert [int(x) for x in ora.philox4x32_10(ctr, key)] == \
            philox_generic(ctr, key, 32, M32, W32)


def test_path_stream_layout(ora):
    """Draw k of a path is word k % 4 of block k // 4, counter (pixel, sample, frame, block),
    key (lo32(seed), hi32(seed)); u = (w >> 8) 2^-24."""
    seed = 0x123456789ABCDEF0
    u = ora.path_uniforms(seed, pixel=777, sample=3, frame=11, n=12)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    exp = []
    for j in range(3):
        exp += philox_generic([777, 3, 11, j], key, 32, M32, W32)
    exp = np.array([(w >> 8) * 2.0**-24 for w in exp], dtype=np.float32)
    assert np.array_equal(u, exp)


def test_uniforms_chi2(ora):
    from scipy import stats
    u = np.concatenate([ora.path_uniforms(99, p, 0, 0, 64) for p in range(2000)])
    assert u.min() >= 0.0 and u.max() <= 1.0 - 2.0**-24
    hist, _ = np.histogram(u, bins=64, range=(0, 1))
    chi2 = stats.chisquare(hist)
    assert chi2.pvalue > 1e-4


def _ulp_err(got, ref):
    got = got.astype(np.float64)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    ulp = np.maximum(ulp, np.float64(np.spacing(np.float32(1.1754944e-38))))
    return np.abs(got - ref) / ulp


def test_expf_within_3ulp(ora):
    x = np.linspace(-87.0, 88.5, 2_000_001).astype(np.float32)
    x = np.concatenate([x, np.float32([-5.5, -3.0, 0.0, -0.0, 1e-8, -1e-8, 0.5, 88.0])])
    y = ora.expf(x)
    ref = np.exp(x.astype(np.float64))
    assert _ulp_err(y, ref).max() <= 3.0
    assert ora.expf(np.float32([89.0]))[0] == np.inf
    assert ora.expf(np.float32([-88.0]))[0] == 0.0


def test_logf_within_3ulp_on_every_tracer_argument(ora):
    # The tracer only evaluates log(1 - u) with u = k 2^-24: every such argument.
    k = np.arange(0, 1 << 24, dtype=np.float64)
    x = (1.0 - k * 2.0**-24).astype(np.float32)
    y = ora.logf(x)
    ref = np.log(x.astype(np.float64))
    err = _ulp_err(y, ref)
    err[x == 1.0] = 0.0 if y[x == 1.0][0] == 0.0 else np.inf
    assert err.max() <= 3.0


def test_sincosf_within_3ulp_on_every_tracer_argument(ora):
    # phi = fl(2pi) * u for every u = k 2^-24.
    k = np.arange(0, 1 << 24, dtype=np.float64)
    u = (k * 2.0**-24).astype(np.float32)
    phi = np.float32(2.0 * math.pi) * u
    s, c = ora.sincosf(phi)
    p64 = phi.astype(np.float64)
    es = _ulp_err(s, np.sin(p64))
    ec = _ulp_err(c, np.cos(p64))
    # Absolute error bound as well, for results very close to zero.
    assert np.max(np.abs(s - np.sin(p64))) < 1.2e-7
    assert np.max(np.abs(c - np.cos(p64))) < 1.2e-7
    big_s, big_c = np.abs(np.sin(p64)) > 1e-3, np.abs(np.cos(p64)) > 1e-3
    assert es[big_s].max() <= 3.0 and ec[big_c].max() <= 3.0
