"""Pins of the oracle's counter-based phase generator (Philox4x64-10)."""
import numpy as np

import oracle as O


def test_numpy_stream_matches_published_round_function():
    for seed, r, blocks in [(23, 0, 3), (23, 5, 2), (2 ** 63 + 11, 255, 2), (0, 1 << 40, 1)]:
        u32 = O.phase_uniforms_u32(8 * blocks, seed, r)
        for b in range(blocks):
            words = O.philox4x64_10((b, r, 0, 0), (seed, 0))
            for w in range(4):
                assert int(u32[8 * b + 2 * w]) == words[w] & 0xFFFFFFFF
                assert int(u32[8 * b + 2 * w + 1]) == words[w] >> 32


def test_counter_and_key_change_the_output():
    a = O.philox4x64_10((0, 0, 0, 0), (1, 0))
    assert a != O.philox4x64_10((1, 0, 0, 0), (1, 0))
    assert a != O.philox4x64_10((0, 1, 0, 0), (1, 0))
    assert a != O.philox4x64_10((0, 0, 0, 0), (2, 0))


def test_uniforms_range_and_moments():
    u = O.phase_uniforms(256, 23, 3)
    assert u.shape == (256, 256)
    assert u.min() >= 0.0 and u.max() < 1.0
    # 24-bit grid, exact in float32
    assert np.all(np.float32(u).astype(np.float64) == u)
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 0.002
    v = O.phase_uniforms(256, 23, 4)
    assert abs(np.corrcoef(u.ravel(), v.ravel())[0, 1]) < 0.02
