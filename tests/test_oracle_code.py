"""Pins of the oracle's code construction against facts that do not depend on
it: published known-answer vectors of the generators, the RC constraint and
degrees checked by brute force on the materialised H, the rank bound of
full-circulant bases, and the null-space property H c = 0 (Section II)."""
import numpy as np
import pytest

import oracle as O
from conftest import CODES


def test_splitmix64_known_answers():
    # SplitMix64 reference outputs for seed 0 (Vigna's splitmix64.c)
    assert O.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert O.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert O.splitmix64(0, 2) == 0x06C45D188009454F


def test_philox4x32_10_known_answers():
    # Random123 known-answer vectors for philox4x32-10
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        assert list(O.philox4x32_10(ctr, key)) == want


def test_text_roundtrip_and_adjacency():
    txt = "qc-ldpc v1\nZ 5\nbase 2 3\n0 1 -1\n# comment\n2 -1 4\n"
    c = O.Code.from_text(txt)
    assert (c.N, c.M, c.Z, c.mb, c.nb) == (15, 10, 5, 2, 3)
    assert c.shifts.tolist() == [[0, 1, -1], [2, -1, 4]]
    H = c.dense()
    # block (1,2) has shift 4: row r of block row 1 has its one at column 2*5 + (r+4)%5
    for r in range(5):
        assert H[5 + r, 10 + (r + 4) % 5] == 1
        assert H[5 + r, 0 + (r + 2) % 5] == 1
        assert H[5 + r, 5:10].sum() == 0
    c2 = O.Code.from_text(c.to_text())
    assert (c2.shifts == c.shifts).all()


@pytest.mark.parametrize("bad", [
    "", "qc-ldpc v2\nZ 3\nbase 1 1\n0\n", "qc-ldpc v1\nZ 3\nbase 1 2\n0\n",
    "qc-ldpc v1\nZ 3\nbase 1 1\n3\n", "qc-ldpc v1\nZ 3\nbase 1 1\n-2\n",
    "qc-ldpc v1\nZ 0\nbase 1 1\n0\n", "qc-ldpc v1\nZ 3\nbase 1 1\n0 0\n",
    "qc-ldpc v1\nZ 3\nbase 1 1\nx\n",
])
def test_text_rejects_malformed(bad):
    with pytest.raises(O.OracleError, match="parse"):
        O.Code.from_text(bad)


@pytest.mark.parametrize("name", ["n186", "n1008", "n4032", "n8000"])
def test_rc_constraint_and_degrees_brute_force(ocodes, name):
    c = ocodes(name)
    mb, nb, Z, _ = CODES[name]
    H = c.dense().astype(np.float32)
    assert (H.sum(0) == mb).all() and (H.sum(1) == nb).all()
    # two rows sharing two columns <=> two columns sharing two rows (a 4-cycle)
    G = H @ H.T
    np.fill_diagonal(G, 0)
    assert G.max() <= 1
    assert not c.violates_rc()


def test_rc_check_detects_four_cycles():
    # Z=1 base with two columns sharing two rows
    c = O.Code.from_text("qc-ldpc v1\nZ 1\nbase 2 3\n0 0 -1\n0 0 0\n")
    assert c.violates_rc()
    # girth-4 draws are accepted as drawn; some of them must contain 4-cycles
    hits = sum(O.Code.from_seed(3, 6, 7, s, min_girth=4).violates_rc() for s in range(20))
    assert hits > 0
    for s in range(5):
        assert not O.Code.from_seed(3, 6, 7, s, min_girth=6).violates_rc()


def _gf2_rank(H):
    rows = [int("".join(map(str, r[::-1])), 2) for r in H]
    rank = 0
    while rows:
        piv = rows.pop()
        if piv == 0:
            continue
        rank += 1
        low = piv & -piv
        rows = [r ^ piv if r & low else r for r in rows]
    return rank


@pytest.mark.parametrize("name", ["n186", "n1008"])
def test_rank_matches_independent_elimination(ocodes, name):
    c = ocodes(name)
    mb = CODES[name][0]
    r, K = c.rank()
    assert r == _gf2_rank(c.dense())
    assert K == c.N - r
    # every block row of full circulant permutations sums to the all-ones row
    assert r <= c.M - mb + 1


@pytest.mark.parametrize("name", ["n186", "n1008", "n4032"])
def test_encoder_null_space_and_systematic(ocodes, name):
    c = ocodes(name)
    cw = O.unpack(c.encode(seed=5, first=0, count=64), c.N).astype(np.int64)
    H = c.dense().astype(np.int64)
    assert ((H @ cw.T) % 2 == 0).all()
    assert cw.sum() > 0
    info = c.info_positions()
    chunks = (c.K + 63) // 64
    for w in (0, 17, 63):
        bits = [(O.splitmix64(5, w * chunks + k // 64) >> (k % 64)) & 1 for k in range(c.K)]
        assert (cw[w, info] == np.array(bits)).all()
    # the pool is addressable: codeword 17 alone equals row 17 of the batch
    one = O.unpack(c.encode(seed=5, first=17, count=1), c.N)
    assert (one[0] == cw[17]).all()


def test_encoder_large_code_rank(ocodes):
    c = ocodes("n32400")
    r, K = c.rank()
    assert r <= c.M - 3 + 1 and K == c.N - r
    cw = O.unpack(c.encode(seed=9, first=0, count=2), c.N).astype(np.int64)
    rp, rb = c.rows()
    for f in range(2):
        par = np.add.reduceat(cw[f, rb], rp[:-1]) % 2
        assert (par == 0).all()


def _perm(Z, s):
    P = np.zeros((Z, Z), np.uint8)
    P[np.arange(Z), (np.arange(Z) + s) % Z] = 1
    return P


def test_multi_shift_blocks_are_sums_of_permutations():
    txt = "qc-ldpc v1\nZ 7\nbase 2 2\n0,1,3 2\n-1 4,6\n"
    c = O.Code.from_text(txt)
    Z = 7
    want = np.zeros((14, 14), np.uint8)
    want[:7, :7] = _perm(Z, 0) + _perm(Z, 1) + _perm(Z, 3)
    want[:7, 7:] = _perm(Z, 2)
    want[7:, 7:] = _perm(Z, 4) + _perm(Z, 6)
    assert (c.dense() == want).all()
    assert sorted(map(tuple, c.entries().tolist())) == [(0, 0, 0), (0, 0, 1), (0, 0, 3), (0, 1, 2),
                                                        (1, 1, 4), (1, 1, 6)]
    assert (O.Code.from_text(c.to_text()).dense() == want).all()
    # {0,1,3} is a perfect difference set mod 7: no difference repeats, so
    # the weight-3 circulant has no 4-cycle; {0,1,2} repeats the difference 1
    assert not O.Code.from_text("qc-ldpc v1\nZ 7\nbase 1 1\n0,1,3\n").violates_rc()
    assert O.Code.from_text("qc-ldpc v1\nZ 7\nbase 1 1\n0,1,2\n").violates_rc()


@pytest.mark.parametrize("bad", ["0,0", "0,7", "0,", ",1", "1,-1"])
def test_multi_shift_rejects_malformed(bad):
    with pytest.raises(O.OracleError, match="parse"):
        O.Code.from_text(f"qc-ldpc v1\nZ 7\nbase 1 1\n{bad}\n")


@pytest.mark.parametrize("s", [2, 3, 4, 5])
def test_euclidean_geometry_codes(s):
    """Type-I 2-D EG codes over GF(2^s) (the codes of Section V): length
    n = 4^s - 1, row and column weight 2^s, RC constraint (two lines meet in
    at most one point), cyclic H, and the closed-form rank n - k = 3^s - 1
    (Lin & Costello, Error Control Coding, 2nd ed., Ch. 17), which gives the
    (255,175) and (1023,781) codes named in the paper for s = 4 and 5."""
    from paper_1206_3362_amd import synth
    c = O.Code.from_text(synth.eg_code_text(s))
    n = 4 ** s - 1
    assert (c.N, c.M) == (n, n)
    assert c.K == n - (3 ** s - 1)
    if s == 4:
        assert c.K == 175
    if s == 5:
        assert c.K == 781
    H = c.dense()
    assert (H.sum(0) == 2 ** s).all() and (H.sum(1) == 2 ** s).all()
    for i in range(0, n, max(1, n // 17)):
        assert (H[i] == np.roll(H[0], i)).all()
    Hf = H.astype(np.float32)
    G = Hf @ Hf.T
    np.fill_diagonal(G, 0)
    assert G.max() <= 1
    assert not c.violates_rc()
    # the line's points lie outside the subfield line through the origin:
    # no point is zero, all 2^s exponents are distinct
    ex = synth.eg_line_exponents(s)
    assert len(set(ex)) == 2 ** s and ex[0] == 0
