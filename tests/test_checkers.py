"""The whole-launch property checker used by the full-size GPU tests, run on
the CPU over oracle outputs: it accepts them, and it rejects a planted flipped
bit, a planted flag and a failed frame that claims to have stopped early."""
import numpy as np
import pytest

import oracle as O
from conftest import CODES
from gpu_util import check_properties, torch
from paper_1206_3362_amd import synth


def _decoded(ebn0, F=64):
    oc = O.Code.from_seed(*CODES["n186"])
    pool = oc.encode(seed=5, first=0, count=F)
    cb = O.unpack(pool, oc.N)
    y = synth.awgn_frames(oc.N, F, synth.sigma_for(ebn0, 0.5), 3, cb, np.int8)
    z, it, ok = O.decode(oc, y, G=6, max_iter=30)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    return oc, t(z.view(np.int32)), t(it), t(ok)


def test_accepts_oracle_outputs():
    for eb in (1.0, 4.0, 8.0):
        oc, z, it, ok = _decoded(eb)
        check_properties(oc, z, it, ok, 30, f"{eb} dB")


def test_rejects_planted_mistakes():
    oc, z, it, ok = _decoded(3.0)
    okn, itn = ok.numpy(), it.numpy()
    assert okn.any() and (okn == 0).any(), "the sample needs decoded and failed frames"
    good = int(np.nonzero(okn)[0][0])
    bad = int(np.nonzero(okn == 0)[0][0])
    z1 = z.clone()
    z1[good, 0] ^= 1  # one bit of a valid codeword: one check of each column turns unsatisfied
    with pytest.raises(AssertionError, match="flag disagrees"):
        check_properties(oc, z1, it, ok, 30, "flipped bit")
    ok1 = ok.clone()
    ok1[bad] = 1
    with pytest.raises(AssertionError, match="flag disagrees"):
        check_properties(oc, z, it, ok1, 30, "planted flag")
    it1 = it.clone()
    it1[bad] = 29
    with pytest.raises(AssertionError, match="stopped before K_max"):
        check_properties(oc, z, it1, ok, 30, "short failure")
