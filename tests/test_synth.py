"""Seeded input generators: published SplitMix64 values, cross-implementation
equality, and the statistics of each workload's inputs (CPU only)."""
import math

import numpy as np
import pytest

import synth

# First five outputs of SplitMix64 seeded with 1234567, as published with the
# generator's reference implementation (Vigna, prng.di.unimi.it/splitmix64.c).
SPLITMIX_1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                    4593380528125082431, 16408922859458223821]


def test_splitmix64_published_values():
    assert [synth.splitmix64_scalar(1234567, c) for c in range(5)] == SPLITMIX_1234567


def test_numpy_matches_scalar():
    c = np.arange(1000, dtype=np.uint64) * np.uint64(977) + np.uint64(3)
    got = synth.splitmix64_np(synth.BASE_SEED + 2, c)
    ref = [synth.splitmix64_scalar(synth.BASE_SEED + 2, int(v)) for v in c]
    assert [int(v) for v in got] == ref


def test_torch_matches_numpy():
    torch = pytest.importorskip("torch")
    a = synth.uniform_complex(synth.BASE_SEED + 1, 4096, 3, first=5)
    b = synth.uniform_complex_torch(synth.BASE_SEED + 1, 4096, 3, "cpu", first=5, chunk=5000)
    assert np.array_equal(a, b.numpy())


def test_uniform_values_exact_and_in_range():
    x = synth.uniform_complex(synth.BASE_SEED + 1, 4096, 64)
    f = x.view(np.float32)
    assert f.min() >= -1.0 and f.max() < 1.0
    # every value is k * 2^-23 - 1 for an integer k: exactly representable
    k = (f.astype(np.float64) + 1.0) * 2.0 ** 23
    assert np.array_equal(k, np.round(k))
    assert abs(f.mean()) < 2e-3 and abs(f.var() - 1 / 3) < 2e-3


def test_counter_layout_is_position_independent():
    # signal b of a batch equals the same signal generated alone
    whole = synth.uniform_complex(7, 256, 10)
    part = synth.uniform_complex(7, 256, 3, first=4)
    assert np.array_equal(whole[4:7], part)
    # a ragged batch of equal sizes is the uniform batch
    flat, offs = synth.uniform_ragged(7, [256] * 10)
    assert np.array_equal(flat.reshape(10, 256), whole)
    assert list(offs) == [256 * i for i in range(10)]


def test_smooth_sizes_table():
    s = synth.smooth_sizes()
    assert len(s) == 579 and s[0] == 64 and s[-1] == 65536
    for v in s:
        m = v
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        assert m == 1
    gaps = np.diff(np.log(s))
    assert gaps.max() < 0.1


def test_ragged_sizes_log_uniform():
    sizes = synth.ragged_sizes(synth.BASE_SEED + 5, 10000)
    table = set(synth.smooth_sizes())
    assert all(int(v) in table for v in sizes)
    lg = np.log(sizes.astype(np.float64))
    lo, hi = math.log(64), math.log(65536)
    # log-uniform: mean of log N at the midpoint, ~ uniform histogram in log space
    assert abs(lg.mean() - (lo + hi) / 2) < 0.05
    hist, _ = np.histogram(lg, bins=10, range=(lo, hi))
    assert hist.min() > 800 and hist.max() < 1200
    assert 9000 < sizes.mean() < 10100


def test_ragged_nearest_in_log_distance():
    table = np.array(synth.smooth_sizes(), dtype=np.float64)
    sizes = synth.ragged_sizes(99, 2000)
    z = synth.splitmix64_np(99, np.arange(2000, dtype=np.uint64))
    frac = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u = math.log(64) + frac * (math.log(65536) - math.log(64))
    d = np.abs(np.log(table)[None, :] - u[:, None])
    best = table[np.argmin(d, axis=1)]  # argmin takes the first (smaller) on ties
    assert np.array_equal(best.astype(np.int64), sizes)


def test_images_smooth_noise():
    img = synth.smooth_noise_image(synth.BASE_SEED + 3, 0, 256, 256)
    assert img.dtype == np.uint8 and img.shape == (256, 256)
    assert 60 < img.mean() < 190
    # smooth field + bounded noise: neighbour differences stay within the noise band
    d = np.abs(np.diff(img.astype(np.int32), axis=1))
    assert d.max() <= 48 + 8
    other = synth.smooth_noise_image(synth.BASE_SEED + 3, 1, 256, 256)
    assert not np.array_equal(img, other)
    c = synth.images_complex(synth.BASE_SEED + 3, 2, 256, 256)
    assert c.dtype == np.complex64 and np.all(c.imag == 0)
    assert np.array_equal(c[1].real.astype(np.uint8), other)


def test_workloads_sizes():
    w = synth.workloads()
    assert w["c1_n4096_b64"].n == 4096 and w["c1_n4096_b64"].batch == 64
    for k, v in w.items():
        if k.startswith("c2_"):
            assert v.n * v.batch == 1 << 27
        if k.startswith("c4_"):
            assert v.n == 1 << 16 and v.batch == 4096
