"""Seeded MPPI perturbations (Sec. IV-A sampling): the oracle's generator
pinned to numpy's independent Philox4x64-10 and to the Box-Muller
transform's properties, and the library's host generator (vpm_sample_eps)
bit-identical to the oracle's. No GPU needed."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import sampling as S
from paper_2509_16079_amd import vpm as V

M64 = (1 << 64) - 1


def _numpy_block(counter, key):
    """numpy's Philox4x64-10 block at `counter` (numpy advances its counter
    before each block, so it starts one below)."""
    c = sum(int(v) << (64 * i) for i, v in enumerate(counter))
    k = int(key[0]) + (int(key[1]) << 64)
    g = np.random.Philox(counter=(c - 1) % (1 << 256), key=k)
    return [int(x) for x in g.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((0, 0, 0, 0), (0, 0)),
    ((5, 7, 9, 11), (123456789, 987654321)),
    ((M64, 3, 1 << 63, 17), (M64, M64 - 1)),
    ((0, 1, 0, 0), (42, 0)),
    ((12, 2047, 2, 0), (2**31 - 1, 0)),
])
def test_philox_block_matches_numpy(counter, key):
    assert S.philox4x64_10(counter, key) == _numpy_block(counter, key)


def test_uniform_ranges_at_the_extreme_words():
    assert S.uniform_open0(0) == 2.0 ** -53
    assert S.uniform_open0(M64) == 1.0
    assert S.uniform_open1(0) == 0.0
    assert S.uniform_open1(M64) == 1.0 - 2.0 ** -53
    # only the top 53 bits matter
    assert S.uniform_open1(0x7FF) == 0.0 and S.uniform_open1(0x800) == 2.0 ** -53


def test_box_muller_special_values():
    # u_a = 1 gives radius 0
    assert S.box_muller(M64, 12345) == (0.0, 0.0)
    # u_b = 1/4 gives the angle pi/2: all of the radius in the second normal
    wa = (1 << 63) - 1            # u_a = 2^-1 exactly
    wb = 1 << 62                  # u_b = 2^-2 exactly
    z0, z1 = S.box_muller(wa, wb)
    r = math.sqrt(-2.0 * math.log(0.5))
    assert z1 == r and abs(z0) < 1e-15 * r


def test_normals_are_standard_normal():
    z = np.array(S.eps(seed=2024, iteration=0, K=64, H=250, sigma=1.0)).ravel()
    n = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the pairs of one Box-Muller draw are uncorrelated
    zz = np.array(S.eps(seed=7, iteration=1, K=2000, H=2, sigma=1.0))
    assert abs(np.corrcoef(zz[:, 0], zz[:, 1])[0, 1]) < 4.0 / math.sqrt(2000)


def test_values_depend_on_seed_iteration_rollout_and_step_only():
    big = np.array(S.eps(seed=99, iteration=2, K=5, H=13, sigma=0.15))
    small = np.array(S.eps(seed=99, iteration=2, K=3, H=9, sigma=0.15))
    assert np.array_equal(big[:3, :9], small)
    other_iter = np.array(S.eps(seed=99, iteration=1, K=3, H=9, sigma=0.15))
    other_seed = np.array(S.eps(seed=98, iteration=2, K=3, H=9, sigma=0.15))
    assert not np.any(other_iter == small) and not np.any(other_seed == small)
    # sigma scales exactly
    unit = np.array(S.eps(seed=99, iteration=2, K=3, H=9, sigma=1.0))
    assert np.array_equal(small, 0.15 * unit)


@pytest.mark.parametrize("seed,iteration,K,H,sigma", [
    (0, 0, 4, 8, 0.15), (12345, 2, 7, 13, 0.15), (2**64 - 1, 5, 3, 1, 1.0),
    (2**40 + 17, 0, 2, 203, 0.3), (3, 63, 33, 6, 0.0)])
def test_library_generator_is_bit_identical_to_the_oracle(seed, iteration, K, H, sigma):
    lib = V.sample_eps(seed, iteration, K, H, sigma)
    ref = np.array(S.eps(seed, iteration, K, H, sigma))
    assert lib.shape == ref.shape
    assert np.array_equal(lib.view(np.uint64), ref.view(np.uint64))


def test_library_generator_rejects_bad_arguments():
    for args in ((1, -1, 2, 2, 0.1), (1, 0, 0, 2, 0.1), (1, 0, 2, 0, 0.1),
                 (1, 0, 2, 2, -0.1), (1, 0, 2, 2, float("nan"))):
        with pytest.raises(V.VpmError) as e:
            V.sample_eps(*args)
        assert e.value.code == V.EINVAL
