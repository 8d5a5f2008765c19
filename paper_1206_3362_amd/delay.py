"""Clock-count model of the bit-choice delay of Section IV.

The paper's hardware reference: 2q basic decoding units compute 2q metrics
per clock, so all N metrics take N/(2q) clocks (N padded with "null" metrics
to a multiple of 2q, footnote 1); a pipelined comparator network of
log2(2q) stages (q comparators in the first) returns the maximum of 2q
values log2(2q) clocks after they enter, one group of 2q per clock.

  FWBF, eq. (3): every block of 2q metrics has its maximum after
      log2(2q) + N/(2q) clocks;
  MLP-WBF, eq. (2): the lambda largest metrics are found one after another,
      each needing the block maxima plus log2(N/(2q)) clocks for the
      maximum of the N/(2q) block maxima:
      lambda (log2(2q) + N/(2q) + log2(N/(2q))).

For EG(255,175) (N = 255 padded to 256, 2q = 16) this gives 20 clocks for
FWBF and 24 lambda for MLP-WBF, the figures of Section IV.  This is a model
of the paper's hypothetical decoder, not of the GPU kernels; bench.py sets
it beside the measured per-round cost of the cyclic kernel.
"""
from __future__ import annotations

import math


def _padded(N: int, two_q: int) -> int:
    if two_q < 2 or two_q & (two_q - 1):
        raise ValueError("2q must be a power of two >= 2")
    return -(-N // two_q) * two_q


def metric_clocks(N: int, two_q: int) -> int:
    """Clocks to compute all metrics with 2q basic decoding units."""
    return _padded(N, two_q) // two_q


def fwbf_delay(N: int, two_q: int) -> int:
    """Eq. (3): log2(2q) + N/(2q) clocks for the maxima of all 2q-blocks."""
    return int(math.log2(two_q)) + metric_clocks(N, two_q)


def mlp_wbf_delay(N: int, two_q: int, lam: int) -> int:
    """Eq. (2): lambda (log2(2q) + N/(2q) + log2(N/(2q))) clocks."""
    blocks = metric_clocks(N, two_q)
    return lam * (int(math.log2(two_q)) + blocks + math.ceil(math.log2(blocks)))


def decode_clocks(rounds: float, N: int, two_q: int, lam: int | None = None) -> float:
    """Bit-choice clocks of a whole decode: rounds x the per-round delay."""
    per = fwbf_delay(N, two_q) if lam is None else mlp_wbf_delay(N, two_q, lam)
    return rounds * per
