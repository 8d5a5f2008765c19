"""Pins of the oracle's channel (Section II: BPSK s = 1 - 2c; Section V: AWGN of
variance N0/2): the noise must be standard normal (moments and a
Kolmogorov-Smirnov test against the normal CDF), independent of the codeword
and of the stream, and the fixed-point inputs must be the clamped rounding of
the scaled value."""
import numpy as np
from scipy import stats

import oracle as O


def test_noise_is_standard_normal():
    N, F, sigma = 1000, 400, 0.7
    y, yd = O.channel(N, F, 0, None, 123, 0, sigma, want_double=True)
    g = ((yd - 1.0) / sigma).ravel()
    assert abs(g.mean()) < 5 / np.sqrt(g.size)
    assert abs(g.var() - 1.0) < 0.01
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # the sine and cosine members of each Box-Muller pair are uncorrelated
    gg = g.reshape(-1, 2)
    assert abs(np.corrcoef(gg[:, 0], gg[:, 1])[0, 1]) < 0.01
    assert np.array_equal(y, yd.astype(np.float32))


def test_codeword_and_stream_and_frame_offset():
    N = 64
    bits = np.zeros((2, N), np.uint8)
    bits[1, ::3] = 1
    pool = O.pack(bits)
    y, yd = O.channel(N, 4, 10, pool, 7, 2, 0.5, want_double=True)
    _, y0 = O.channel(N, 4, 10, None, 7, 2, 0.5, want_double=True)
    s = 1.0 - 2.0 * bits[np.arange(10, 14) % 2]
    # the same noise is added whatever the codeword
    assert np.allclose(yd - s, y0 - 1.0, atol=1e-12)
    # frames are addressed by absolute index: frame 12 generated alone is identical
    _, one = O.channel(N, 1, 12, pool, 7, 2, 0.5, want_double=True)
    assert np.array_equal(one[0], yd[2])
    _, other = O.channel(N, 4, 10, pool, 7, 3, 0.5, want_double=True)
    assert not np.allclose(other, yd)


def test_quantisation():
    N, F = 256, 64
    _, yd = O.channel(N, F, 0, None, 5, 0, 2.0, want_double=True)
    q8 = O.channel(N, F, 0, None, 5, 0, 2.0, scale=16.0, dtype=O.I8)
    q16 = O.channel(N, F, 0, None, 5, 0, 2.0, scale=256.0, dtype=O.I16)
    assert np.array_equal(q8, np.clip(np.rint(16 * yd), -127, 127).astype(np.int8))
    assert np.array_equal(q16, np.clip(np.rint(256 * yd), -32767, 32767).astype(np.int16))
    assert q8.min() == -127 and q8.max() == 127
