"""Pins of the oracle's random stream: Philox4x32-10 words, uniforms, Box-Muller
normals and uniform sphere directions (Sec. 2.3.2, eq. projected_chain_update:
zeta is a normalised standard Gaussian vector).

Known-answer vectors of Philox are not available here, so the generator is
pinned by the properties its published construction guarantees (bijectivity in
the counter, avalanche, equidistribution), and by a GPU-box test against the
ROCm library's own Philox4x32-10 (tests/test_gpu_rocrand_philox.py).
"""
import os

import numpy as np
import pytest
from scipy import stats


def _words(orc, n_blocks, key=(0, 0), field=0):
    out = np.zeros((n_blocks, 4), dtype=np.uint32)
    for i in range(n_blocks):
        ctr = [0, 0, 0, 0]
        ctr[field] = i
        out[i] = orc.philox(ctr, key)
    return out


def test_philox_deterministic_and_counter_sensitive(orc):
    a = orc.philox([1, 2, 3, 4], [5, 6])
    b = orc.philox([1, 2, 3, 4], [5, 6])
    assert np.array_equal(a, b)
    for f in range(4):
        c = [1, 2, 3, 4]
        c[f] += 1
        assert not np.array_equal(orc.philox(c, [5, 6]), a)
    assert not np.array_equal(orc.philox([1, 2, 3, 4], [5, 7]), a)
    assert not np.array_equal(orc.philox([1, 2, 3, 4], [6, 6]), a)


def test_philox_injective_over_counters(orc):
    # Philox is a bijection of the 128-bit counter for a fixed key.
    w = _words(orc, 20000, key=(123, 456))
    packed = {tuple(r) for r in w}
    assert len(packed) == 20000


def test_philox_word_equidistribution(orc):
    w = _words(orc, 16384).ravel()
    # top byte histogram: chi^2 with 255 dof
    hist = np.bincount(w >> 24, minlength=256)
    chi2 = ((hist - w.size / 256) ** 2 / (w.size / 256)).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    # every bit is set about half the time
    bits = ((w[:, None] >> np.arange(32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.02)


def test_philox_avalanche(orc):
    rng = np.random.default_rng(7)
    flips = []
    for _ in range(200):
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        base = orc.philox(ctr, key)
        bit = rng.integers(0, 128)
        c2 = ctr.copy()
        c2[bit // 32] ^= np.uint32(1 << (bit % 32))
        out = orc.philox(c2, key)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(base, out)))
    m = np.mean(flips)
    assert 60.0 < m < 68.0, m


def test_uniform_open_interval(orc):
    assert orc.uniform(0) == 0.5 * 2.0 ** -32
    assert orc.uniform(2 ** 32 - 1) == 1.0 - 0.5 * 2.0 ** -32
    assert 0.0 < orc.uniform(0) and orc.uniform(2 ** 32 - 1) < 1.0


def test_box_muller_pair(orc):
    # u0 = u1 = 1/2 -> radius sqrt(2 ln 2), angle pi
    x = 2 ** 31
    u = orc.uniform(x)
    g = orc.box_muller(x, x)
    rad = np.sqrt(-2.0 * np.log(u))
    assert g[0] == pytest.approx(rad * np.cos(2 * np.pi * u), rel=1e-15)
    assert g[1] == pytest.approx(rad * np.sin(2 * np.pi * u), abs=1e-15)


def test_normals_are_standard_gaussian(orc):
    g = np.concatenate([orc.normals(3, q, 0, k, 0, 8) for q in range(50) for k in range(200)])
    assert abs(g.mean()) < 0.015
    assert abs(g.var() - 1.0) < 0.02
    assert stats.kstest(g, "norm").pvalue > 1e-4
    # pairs are uncorrelated
    assert abs(np.corrcoef(g[0::2], g[1::2])[0, 1]) < 0.02


def test_substreams_are_independent(orc):
    a = np.concatenate([orc.normals(0, 1, w, 5, 0, 4) for w in range(4000)])
    b = np.concatenate([orc.normals(0, 1, w, 5, 1, 4) for w in range(4000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.03


@pytest.mark.parametrize("n", [2, 3, 10])
def test_sphere_direction_uniform(orc, n):
    z = np.array([orc.direction(11, 0, w, 0, 0, n) for w in range(6000)])
    assert np.max(np.abs(np.linalg.norm(z, axis=1) - 1.0)) < 1e-14
    if n == 2:
        ang = np.arctan2(z[:, 1], z[:, 0])
        assert stats.kstest(ang, stats.uniform(loc=-np.pi, scale=2 * np.pi).cdf).pvalue > 1e-4
    elif n == 3:
        # every coordinate of a uniform point on S^2 is uniform on [-1, 1]
        # (Archimedes), not only the one the sampler draws directly
        for i in range(3):
            assert stats.kstest(z[:, i], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-4, i
        # the azimuth about any axis is uniform: about x1 here
        ang = np.arctan2(z[:, 2], z[:, 1])
        assert stats.kstest(ang, stats.uniform(loc=-np.pi, scale=2 * np.pi).cdf).pvalue > 1e-4
    else:
        # x1^2 ~ Beta(1/2, (n-1)/2) on S^{n-1}
        assert stats.kstest(z[:, 0] ** 2, stats.beta(0.5, (n - 1) / 2).cdf).pvalue > 1e-4
    # rotation invariance: mean 0 and second moment I/n
    m2 = z.T @ z / len(z)
    assert np.max(np.abs(z.mean(0))) < 4.5 / np.sqrt(len(z))
    assert np.max(np.abs(m2 - np.eye(n) / n)) < 5.0 / np.sqrt(len(z)) / n


def test_direction_of_high_dimension_is_normalised_normals(orc):
    for n in (4, 7, 100):
        g = orc.normals(5, 1, 2, 3, 1, n)
        assert np.allclose(orc.direction(5, 1, 2, 3, 1, n), g / np.linalg.norm(g), rtol=0, atol=1e-15)


def test_direction_and_radius_words_are_independent(orc):
    # n <= 3: direction from words 0 (and 1), the Green radius from word 3
    for n in (2, 3):
        u = np.array([orc.radius_uniform(2, 0, w, 1, 1, n) for w in range(6000)])
        z = np.array([orc.direction(2, 0, w, 1, 1, n) for w in range(6000)])
        assert stats.kstest(u, stats.uniform().cdf).pvalue > 1e-4
        for i in range(n):
            assert abs(np.corrcoef(u, z[:, i])[0, 1]) < 0.05, (n, i)


def test_radius_uniform_word_position(orc):
    # The Green-sample radius uses word 3 of its sub-stream for n <= 3, word
    # 2*ceil(n/2) for n >= 4.
    for n, blk, word in [(2, 0, 3), (3, 0, 3), (4, 1, 0), (5, 1, 2), (100, 25, 0)]:
        u = orc.radius_uniform(9, 3, 4, 5, 1, n)
        x = orc.philox([3, 4, 5, (1 << 24) | blk], [9, 0])
        assert u == orc.uniform(x[word])


def _kat_vectors():
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = []
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(t, 16) for t in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors(orc):
    """The published Philox4x32-10 known-answer vectors (tests/golden)."""
    rows = _kat_vectors()
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = orc.philox(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))
        assert [int(x) for x in got] == out
