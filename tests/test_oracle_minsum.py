"""Pins of the oracle's min-sum BP decoder (the BP reference of Sections I
and V) against values the decoding rule fixes independently of the oracle:
maximum-likelihood decisions on a single-parity-check code (where one
min-sum iteration is exact), the normalised and offset closed forms on the
same code, the one-iteration correction of a single error on the EG codes,
noiseless input and codeword symmetry."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1206_3362_amd import synth


def spc(n):
    return O.Code.from_text(f"qc-ldpc v1\nZ 1\nbase 1 {n}\n" + " ".join(["0"] * n) + "\n")


def test_single_parity_check_is_maximum_likelihood():
    """One check over n bits, factor 1: the first iteration gives
    P_n = L_n + (product of the other signs) * (minimum of the other |L|),
    which flips exactly the least reliable bit when the parity fails: the ML
    codeword (maximum correlation over all even-weight words, enumerated)."""
    n = 7
    c = spc(n)
    words = np.array([w for w in itertools.product([0, 1], repeat=n) if sum(w) % 2 == 0], np.uint8)
    rng = np.random.default_rng(1)
    y = rng.normal(0.3, 1.0, size=(400, n)).astype(np.float32)
    z, it, ok = O.decode_minsum(c, y, c=1.0, max_iter=5)
    got = O.unpack(z, n)
    corr = y.astype(np.float64) @ (1.0 - 2.0 * words.T)
    ml = words[corr.argmax(1)]
    assert (got == ml).all() and (ok == 1).all()
    assert (it == np.where((y < 0).sum(1) % 2 == 0, 0, 1)).all()


@pytest.mark.parametrize("offset,cst", [(False, 0.75), (True, 0.2)])
def test_single_parity_check_closed_form(offset, cst):
    """Parity failing, least reliable bit k, next smallest magnitude m2:
    bit k flips iff r(m2) > |L_k|, where r(x) = c x (normalised) or
    max(x - c, 0) (offset); a bit n != k keeps its sign iff |L_n| > r(|L_k|)."""
    n = 6
    c = spc(n)
    rng = np.random.default_rng(2)
    y = rng.normal(0.2, 1.0, size=(500, n)).astype(np.float32)
    z, it, ok = O.decode_minsum(c, y, offset=offset, c=cst, max_iter=1)
    got = O.unpack(z, n)
    r = (lambda x: np.maximum(np.float32(x) - np.float32(cst), 0)) if offset else \
        (lambda x: np.float32(cst) * np.float32(x))
    for f in range(y.shape[0]):
        h = (y[f] < 0).astype(np.uint8)
        if h.sum() % 2 == 0:
            assert (got[f] == h).all() and it[f] == 0
            continue
        a = np.abs(y[f])
        k = int(np.argmin(a))
        m2 = np.sort(a)[1]
        want = h.copy()
        want[k] ^= int(r(m2) > a[k])
        for j in range(n):
            if j != k:
                want[j] ^= int(not (a[j] > r(a[k])))
        assert (got[f] == want).all(), f


@pytest.mark.parametrize("s", [4, 5])
def test_single_error_one_iteration_eg(s):
    """EG code, uniform magnitude A, one error e, normalised factor c with
    dv c > 2: after one iteration P_e = -A + dv c A > 0, a bit sharing a
    check with e has A + (dv - 2) c A > 0 and every other bit A + dv c A:
    one iteration for every position (RC constraint)."""
    c = O.Code.from_text(synth.eg_code_text(s))
    N = c.N
    pos = list(range(0, N, 7))
    y = synth.error_pattern_frames(N, [[e] for e in pos], 1.0, np.float32)
    z, it, ok = O.decode_minsum(c, y, c=0.75, max_iter=10)
    assert (O.unpack(z, N) == 0).all() and (it == 1).all() and (ok == 1).all()


def test_noiseless_and_codeword_symmetry():
    c = O.Code.from_seed(3, 6, 31, 1)
    cw = O.unpack(c.encode(3, 0, 64), c.N)
    x = (1.0 - 2.0 * cw).astype(np.float32)
    z, it, ok = O.decode_minsum(c, x, max_iter=10)
    assert (O.unpack(z, c.N) == cw).all() and (it == 0).all()
    y = synth.awgn_frames(c.N, 64, synth.sigma_for(2.5, 0.5), 4, None, np.float32)
    z0, it0, ok0 = O.decode_minsum(c, y, max_iter=15)
    z1, it1, ok1 = O.decode_minsum(c, y * x, max_iter=15)
    assert (O.unpack(z1, c.N) == (O.unpack(z0, c.N) ^ cw)).all()
    assert (it0 == it1).all() and (ok0 == ok1).all()
