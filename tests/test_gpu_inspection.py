"""GPU checks of single steps through the inspection entry points: the device
Philox4x32-10 words, the device inverse of the radial Green law, and the
Newton closest-point solve on the implicit torus, each against the oracle;
plus the oracle's Philox against the ROCm library's own Philox4x32-10."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2606_21883_amd import inputs, mpwos
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def test_device_philox_matches_oracle_bitwise():
    announce("philox")
    for ctr, seed in [([0, 0, 0, 0], 0), ([5, 7, 11, (3 << 24) | 2], 0xDEADBEEF12345678), ([2 ** 32 - 9, 1, 2, 3], 1)]:
        dev = mpwos.debug_philox(ctr, seed, 64)
        for i in range(64):
            c = [(ctr[0] + i) % 2 ** 32, ctr[1], ctr[2], ctr[3]]
            ref = oracle.philox(c, [seed & 0xFFFFFFFF, seed >> 32])
            assert np.array_equal(dev[i], ref), (ctr, seed, i)


def test_device_philox_known_answer_vectors():
    """The published Philox4x32-10 known-answer vectors (tests/golden) on the device."""
    from tests.test_oracle_rng import _kat_vectors
    announce("philox kat")
    for ctr, key, out in _kat_vectors():
        dev = mpwos.debug_philox(ctr, key[0] | (key[1] << 32), 1)
        assert [int(x) for x in dev[0]] == out


def test_oracle_philox_matches_rocrand():
    """rocRAND's PHILOX4_32_10 generator with seed s emits, in order, the words
    of Philox4x32-10 blocks with key (s_lo, s_hi) and counters 0, 1, 2, ..."""
    import torch
    announce("rocrand philox")
    try:
        rr = ctypes.CDLL("librocrand.so")
    except OSError:
        rr = ctypes.CDLL("/opt/rocm/lib/librocrand.so")
    torch.cuda.init()
    for seed in (0, 0x123456789ABCDEF):
        gen = ctypes.c_void_p()
        assert rr.rocrand_create_generator(ctypes.byref(gen), 404) == 0
        assert rr.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
        out = torch.zeros(4096, dtype=torch.int32, device="cuda")
        assert rr.rocrand_generate(gen, ctypes.c_void_p(out.data_ptr()), ctypes.c_size_t(4096)) == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32).reshape(-1, 4)
        rr.rocrand_destroy_generator(gen)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        for j in range(1024):
            ref = oracle.philox([j, 0, 0, 0], key)
            assert np.array_equal(got[j], ref), (seed, j, got[j], ref)


@pytest.mark.parametrize("n", [2, 3, 10, 100, 1000, 11, 1001])
def test_device_radial_inverse_matches_oracle(n):
    announce(f"radial inverse n={n}")
    # n = 11, 1001: the dumbbell's X = sqrt(2(n-1)) r with r = 0.95 * 1.2 / (1 + 2.9294)
    X = {2: 0.57, 3: 0.806, 10: 0.57, 100: 0.57, 1000: 0.57, 11: 1.2975, 1001: 12.975}[n]
    rng = np.random.default_rng(n)
    u = np.concatenate([rng.uniform(size=200), [1e-9, 1e-6, 0.5, 1 - 1e-6, 1 - 2 ** -32]])
    s64 = mpwos.debug_radial_inv(n, X, u, "fp64")
    s32 = mpwos.debug_radial_inv(n, X, u, "fp32")
    ref = np.array([oracle.radial_inv(n, X, v) for v in u])
    # where F' is not small the roots agree closely; everywhere, the device
    # root solves F(s) = u to the rounding of F (the root itself is
    # ill-conditioned as u -> 1, where F' -> 0)
    ok = u < 0.99
    np.testing.assert_allclose(s64[ok], ref[ok], rtol=2e-14, atol=1e-15)
    res = np.array([oracle.radial_cdf(n, X, s) for s in s64]) - u
    assert np.max(np.abs(res)) <= 2e-15
    # the FP32 path takes u in binary32 (the walk's 23-bit uniforms are exact there)
    u32 = u.astype(np.float32).astype(np.float64)
    ref32 = np.array([oracle.radial_inv(n, X, v) if v < 1.0 else 1.0 for v in u32])
    np.testing.assert_allclose(s32, ref32, rtol=0, atol=2e-6)


def test_torus_newton_cp_matches_closed_form():
    announce("torus cp")
    prob = inputs.torus_problem()
    m = mpwos.Manifold(prob)
    rng = np.random.default_rng(1)
    base = inputs.torus_area_uniform(6000, seed=3)
    # points of the walk: on spheres of the walk radius around torus points
    # (half), and inside those balls (half) -- down to 0.037 from the core circle
    d = rng.standard_normal(base.shape)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = 0.95 * 1.2 / (1 + 1 / 0.3) * np.where(np.arange(len(base)) % 2 == 0, 1.0,
                                                 rng.uniform(0, 1, len(base)) ** (1 / 3))
    x = base + rad[:, None] * d
    ref = np.array([oracle.cp(prob, v) for v in x])
    y64 = mpwos.debug_cp(m, x, "fp64")
    y32 = mpwos.debug_cp(m, x, "fp32")
    np.testing.assert_allclose(y64, ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(y32, ref, rtol=0, atol=5e-7)
    m.close()


def test_sphere_cp():
    prob = inputs.hypersphere_problem(3)
    m = mpwos.Manifold(prob)
    x = np.random.default_rng(2).standard_normal((100, 3))
    y = mpwos.debug_cp(m, x, "fp64")
    np.testing.assert_allclose(y, x / np.linalg.norm(x, axis=1, keepdims=True), rtol=1e-15, atol=1e-16)
    m.close()
