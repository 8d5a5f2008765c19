"""Parity of the HIP min-sum BP decoder (fwbf_decode_minsum through the C
ABI) with the oracle's literal per-edge min-sum: hard decisions, iteration
counts and syndrome flags bit for bit, normalised and offset, on QC codes
(single shifts) and on the EG codes (multi-shift circulants)."""
import numpy as np
import pytest

import oracle as O
from conftest import CODES
from gpu_util import assert_same, need_gpu, torch
from paper_1206_3362_amd import synth

pytestmark = pytest.mark.gpu


def run(gcode, y, **kw):
    from paper_1206_3362_amd import fwbf
    yd = torch.from_numpy(np.ascontiguousarray(y)).to("cuda")
    z, it, ok = fwbf.decode_minsum(gcode, yd, **kw)
    torch.cuda.synchronize()
    return z.cpu().numpy().view(np.uint32), it.cpu().numpy(), ok.cpu().numpy()


def ocall(ocode, y, **kw):
    return O.decode_minsum(ocode, y, **kw)


CASES = [("n186", None, 2.0), ("n1008", None, 2.5), ("eg255", 4, 3.0), ("eg1023", 5, 3.5)]


@pytest.mark.parametrize("name,s,ebn0", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("offset,cst", [(False, 0.75), (True, 0.15)])
def test_minsum_parity(name, s, ebn0, offset, cst):
    need_gpu()
    from paper_1206_3362_amd import fwbf
    if s is None:
        g, o = fwbf.Code.from_seed(*CODES[name]), O.Code.from_seed(*CODES[name])
    else:
        t = synth.eg_code_text(s)
        g, o = fwbf.Code.from_text(t), O.Code.from_text(t)
    F = 256 if g.N > 1000 else 1024
    pool = o.encode(seed=8, first=0, count=32)
    cb = O.unpack(pool[np.arange(F) % 32], g.N)
    y = synth.awgn_frames(g.N, F, synth.sigma_for(ebn0, o.K / o.N), 40 + int(10 * ebn0), cb, np.float32)
    print(f"case minsum {name} offset={offset} c={cst}", flush=True)
    kw = dict(offset=offset, c=cst, max_iter=15)
    assert_same(run(g, y, **kw), ocall(o, y, **kw), f"minsum {name} {kw}")


def test_minsum_degenerate():
    need_gpu()
    from paper_1206_3362_amd import fwbf
    g, o = fwbf.Code.from_seed(*CODES["n186"]), O.Code.from_seed(*CODES["n186"])
    y = synth.awgn_frames(g.N, 64, synth.sigma_for(1.0, 0.5), 3, None, np.float32)
    for it_max in (0, 1):
        assert_same(run(g, y, max_iter=it_max), ocall(o, y, max_iter=it_max), f"max_iter={it_max}")
    # strided rows
    yd = torch.zeros((8, g.N + 10), dtype=torch.float32, device="cuda")
    yd[:, :g.N] = torch.from_numpy(y[:8]).to("cuda")
    z, it, ok = fwbf.decode_minsum(g, yd[:, :g.N], max_iter=10)
    torch.cuda.synchronize()
    assert_same((z.cpu().numpy().view(np.uint32), it.cpu().numpy(), ok.cpu().numpy()),
                ocall(o, y[:8], max_iter=10), "strided rows")
    z, it, ok = fwbf.decode_minsum(g, yd[:0, :g.N], max_iter=10)
    assert z.shape[0] == 0
    with pytest.raises(fwbf.FwbfError):
        fwbf.decode_minsum(g, yd[:, :g.N], max_iter=-1)
    with pytest.raises(fwbf.FwbfError):
        fwbf.decode_minsum(g, yd[:, :g.N], offset=True, c=float("nan"))
