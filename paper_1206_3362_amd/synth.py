"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no decoder arithmetic: it only draws received frames for a
given set of transmitted codewords (BPSK over AWGN, Section II and Section V
of the paper) and a few structured test patterns, with numpy's PCG64
generator.  Both the HIP library and the CPU oracle consume what it returns.

Recipe (the paper's workloads: random-noise BPSK/AWGN frames of a fixed code):
  sigma^2 = N0/2 = 1 / (2 R 10^(EbN0/10)),  R = K/N;
  y = (1 - 2c) + sigma * g,  g ~ N(0, 1) i.i.d. (float64, then cast);
  int8 / int16 inputs: q = clamp(rint(A y), -qmax, qmax), A = 16 / 256,
  qmax = 127 / 32767 (symmetric, so |q| never overflows).
"""
from __future__ import annotations

import numpy as np

QMAX = {np.int8: 127, np.int16: 32767}
SCALE = {np.float32: 1.0, np.int8: 16.0, np.int16: 256.0}


def sigma_for(ebn0_db, rate):
    """Noise standard deviation for Eb/N0 in dB at code rate R (BPSK)."""
    return np.sqrt(1.0 / (2.0 * rate * 10.0 ** (np.asarray(ebn0_db, np.float64) / 10.0)))


def unpack_bits(packed, N):
    p = np.ascontiguousarray(packed, np.uint32)
    b = np.unpackbits(p.view(np.uint8).reshape(*p.shape[:-1], -1), axis=-1, bitorder="little")
    return b[..., :N]


def quantize(y64, dtype, scale=None):
    if dtype == np.float32:
        return y64.astype(np.float32)
    A = SCALE[dtype] if scale is None else scale
    q = np.rint(A * y64)
    qm = QMAX[dtype]
    return np.clip(q, -qm, qm).astype(dtype)


def awgn_frames(N, F, sigma, seed, codeword_bits=None, dtype=np.float32, scale=None):
    """F frames of N received values.

    codeword_bits: None (all-zero codeword) or uint8 [F, N] / [N] bits.
    sigma: scalar or [F] (one noise level per frame).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((F, N))
    s = np.ones((F, N))
    if codeword_bits is not None:
        s = 1.0 - 2.0 * np.broadcast_to(np.asarray(codeword_bits, np.float64), (F, N))
    sig = np.asarray(sigma, np.float64)
    if sig.ndim == 1:
        sig = sig[:, None]
    return quantize(s + sig * g, dtype, scale)


def uniform_frames(N, F, seed, lo, hi):
    """Per-frame values drawn uniformly in [lo, hi) (e.g. Eb/N0 in dB)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, F)


def error_pattern_frames(N, patterns, magnitude, dtype, codeword_bits=None):
    """Uniform-magnitude frames: every value is +-magnitude, sign flipped
    (a hard-decision error) at the listed positions of each pattern."""
    F = len(patterns)
    s = np.ones((F, N))
    if codeword_bits is not None:
        s = 1.0 - 2.0 * np.broadcast_to(np.asarray(codeword_bits, np.float64), (F, N))
    y = s * magnitude
    for f, pos in enumerate(patterns):
        y[f, list(pos)] *= -1.0
    return y.astype(dtype)


def tie_heavy_frames(N, F, seed, dtype, levels=3, zero_frac=0.05, flip_frac=0.06):
    """Frames whose magnitudes take only a few levels (many exact ties in the
    check minima and the metrics), with some exact zeros (and -0.0 for float)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if dtype == np.float32:
        mags = np.array([0.25, 0.5, 1.0, 1.5, 2.0][:levels], np.float64)
    else:
        mags = np.array([4, 8, 16, 24, 32][:levels], np.float64)
    y = mags[rng.integers(0, levels, (F, N))]
    y = np.where(rng.random((F, N)) < flip_frac, -y, y)
    zmask = rng.random((F, N)) < zero_frac
    y = np.where(zmask, 0.0, y)
    if dtype == np.float32:
        y = y.astype(np.float32)
        negz = zmask & (rng.random((F, N)) < 0.5)
        y[negz] = np.float32(-0.0)
        return y
    return y.astype(dtype)


def subnormal_frames(N, F, seed, flip_frac=0.08):
    """float32 frames whose magnitudes are subnormal numbers (checks that no
    flush-to-zero happens anywhere)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(1, 1 << 23, (F, N), dtype=np.uint32)
    sign = (rng.random((F, N)) < flip_frac).astype(np.uint32) << 31
    return (bits | sign).view(np.float32)


# --------------------------------------------------------------------------
# Type-I two-dimensional Euclidean-geometry cyclic codes (the codes of the
# paper's Section V).  The points of EG(2, 2^s) other than the origin are the
# nonzero elements alpha^e of GF(2^(2s)); the lines not through the origin
# are the cyclic shifts (multiplication by alpha^i) of one such line, and H
# lists their incidence vectors: an n x n circulant, n = 2^(2s) - 1, with
# row and column weight 2^s.  In the QC text this is Z = n, a 1 x 1 base and
# one block holding 2^s shifts (the exponents of the line's points).
# --------------------------------------------------------------------------
# primitive polynomials of degree 2s (bit i = coefficient of x^i)
EG_PRIMITIVE = {2: 0x13, 3: 0x43, 4: 0x11D, 5: 0x409}


def eg_line_exponents(s):
    """Exponents e (alpha^e) of the points of the line {1 + b alpha : b in GF(2^s)}."""
    m = 2 * s
    n = (1 << m) - 1
    exp = np.zeros(n, np.int64)
    x = 1
    for i in range(n):
        exp[i] = x
        x <<= 1
        if x >> m:
            x ^= EG_PRIMITIVE[s]
    log = {int(v): i for i, v in enumerate(exp)}
    if len(log) != n:
        raise ValueError("polynomial is not primitive")
    q = 1 << s
    # GF(2^s) inside GF(2^(2s)): 0 and the powers alpha^(k (q + 1))
    sub_logs = [k * (q + 1) % n for k in range(q - 1)]
    pts = [1] + [1 ^ int(exp[(lb + 1) % n]) for lb in sub_logs]
    return sorted(log[p] for p in pts)


def eg_code_text(s):
    """QC description of the (2^(2s) - 1)-bit EG code (s = 4: EG(255,175), s = 5: EG(1023,781))."""
    n = (1 << (2 * s)) - 1
    return (f"qc-ldpc v1\n# type-I 2-D Euclidean geometry code over GF(2^{s})\n"
            f"Z {n}\nbase 1 1\n" + ",".join(map(str, eg_line_exponents(s))) + "\n")
