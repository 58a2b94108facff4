"""Pins of the oracle's delay generator."""
import math
from collections import Counter

from oracle import rng


def test_splitmix64_reference_outputs():
    """Outputs of the SplitMix64 reference generator (Steele, Lea & Flood 2014;
    the public splitmix64 reference code) for seed 0."""
    assert rng.splitmix64_stream(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_draw_is_the_stream_at_counter_positions():
    # draw(key, 0, f) is the (f + 1)-th output of the stream seeded with key
    for key in (0, 1, 12345):
        stream = rng.splitmix64_stream(key, 6)
        assert [rng.draw(key, 0, f) for f in range(6)] == stream


def test_thresholds_partition_exactly():
    for L in range(1, 10):
        thr = rng.thresholds(L)
        assert thr[-1] == 1 << 53
        assert all(thr[i] < thr[i + 1] for i in range(L - 1))
        assert rng.bin_delay(0, thr) == 0
        assert rng.bin_delay((1 << 53) - 1, thr) == L - 1
    # p = {0.6, 0.3, 0.1} (the example of Sec. 5.1) as integer weights
    thr = rng.thresholds(3, [6, 3, 1])
    assert thr == [(6 << 53) // 10, (9 << 53) // 10, 1 << 53]


def test_bin_frequencies_chi_square():
    """Sec. 5.1 example: L = 3, p = {0.6, 0.3, 0.1}. Chi-square with 2 dof below the
    0.999 quantile (13.8)."""
    thr = rng.thresholds(3, [6, 3, 1])
    n = 60000
    cnt = Counter(rng.raw_delay(7, i // 6, i % 6, thr) for i in range(n))
    exp = [0.6 * n, 0.3 * n, 0.1 * n]
    chi2 = sum((cnt[j] - exp[j]) ** 2 / exp[j] for j in range(3))
    assert chi2 < 13.8, (cnt, chi2)


def test_startup_clamp_never_reaches_before_t0():
    for T in (1, 2, 3, 4):
        for n in range(0, 12):
            for k in range(0, 8):
                kc = rng.clamp_startup(k, n, T)
                assert 0 <= kc <= k
                assert n - kc - (T - 1) >= 0 or kc == 0
                if n >= T - 1 + k:
                    assert kc == k


def test_ensemble_keys_distinct():
    keys = {rng.ensemble_key(3, i) for i in range(4096)}
    assert len(keys) == 4096
