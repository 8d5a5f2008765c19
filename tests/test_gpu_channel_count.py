"""Parity of the frame-generation (Philox4x32-10 + Box-Muller, BPSK/AWGN) and
error-accounting kernels with the oracle.  The channel kernel computes in
single precision with the device's logf/sqrtf/sincospif, the oracle in
double: float outputs must agree to a few ulp of the noise, and fixed-point
outputs exactly except where the oracle's value sits within that tolerance
of a rounding boundary.  Counting is integer and must be exact."""
import numpy as np
import pytest

import oracle as O
from gpu_util import need_gpu, torch
from paper_1206_3362_amd import fwbf

pytestmark = pytest.mark.gpu

# |y_gpu - y_oracle| bound: Box-Muller in float with ~1-2 ulp transcendental
# error on r = sqrt(-2 ln u) (r <= 5.7) times sigma <= 1.2, plus the final
# float rounding of y: 5.7 * 1.2 * 8 * 2^-24 ~ 3.3e-6; 1e-5 leaves margin.
TOL = 1e-5


@pytest.fixture(scope="module")
def code():
    need_gpu()
    return fwbf.Code.from_seed(3, 6, 168, 2), O.Code.from_seed(3, 6, 168, 2)


@pytest.mark.parametrize("f0", [0, 123456, (1 << 33) + 5])
def test_channel_float_matches_oracle(code, f0):
    g, o = code
    F, N = 512, g.N
    pool = o.encode(21, 0, 64)
    poold = torch.from_numpy(pool.view(np.int32)).cuda()
    sigma = 0.63
    y = fwbf.channel(N, F, f0, poold, seed=0x1234567890, stream_id=3, sigma=sigma)
    torch.cuda.synchronize()
    yo, yd = O.channel(N, F, f0, pool, 0x1234567890, 3, sigma, want_double=True)
    err = np.abs(y.cpu().numpy().astype(np.float64) - yd)
    assert err.max() < TOL, err.max()
    # the transmitted symbols are the codewords of the pool rows
    assert ((yd - 1.0 + 2.0 * O.unpack(pool[(np.arange(F) + f0) % 64], N)) ** 2).mean() < 0.5


@pytest.mark.parametrize("dtype,scale,qmax", [(torch.int8, 16.0, 127), (torch.int16, 256.0, 32767)])
def test_channel_fixed_point_matches_oracle(code, dtype, scale, qmax):
    g, o = code
    F, N = 1024, g.N
    y = fwbf.channel(N, F, 7, None, seed=99, stream_id=1, sigma=0.8, dtype=dtype, scale=scale)
    torch.cuda.synchronize()
    yq = y.cpu().numpy().astype(np.int64)
    _, yd = O.channel(N, F, 7, None, 99, 1, 0.8, want_double=True)
    want = np.clip(np.rint(scale * yd), -qmax, qmax).astype(np.int64)
    frac = np.abs(scale * yd - np.floor(scale * yd) - 0.5)
    near = frac < scale * TOL
    assert (yq[~near] == want[~near]).all()
    assert (np.abs(yq - want) <= 1).all()
    assert yq.min() >= -qmax and yq.max() <= qmax


def test_channel_per_frame_sigma_and_stride(code):
    g, o = code
    F, N = 64, g.N
    sig = np.linspace(0.4, 0.9, F).astype(np.float32)
    sigd = torch.from_numpy(sig).cuda()
    buf = torch.zeros((F, 1100), dtype=torch.float32, device="cuda")
    fwbf.channel_into(N, buf[:, :N], 0, None, 5, 0, 0.0, sigma_per_frame=sigd)
    torch.cuda.synchronize()
    b = buf.cpu().numpy()
    assert (b[:, N:] == 0).all()
    for f in (0, 31, 63):
        _, yd = O.channel(N, 1, f, None, 5, 0, float(sig[f]), want_double=True)
        assert np.abs(b[f, :N] - yd[0]).max() < TOL


def test_count_matches_oracle(code):
    g, o = code
    F, N = 4096, g.N
    pool = o.encode(3, 0, 32)
    rng = np.random.default_rng(1)
    cw = O.unpack(pool[np.arange(F) % 32], N)
    flips = rng.random((F, N)) < np.where(rng.random(F) < 0.7, 0.0, 0.01)[:, None]
    z = O.pack(cw ^ flips)
    it = rng.integers(0, 51, F).astype(np.int32)
    ok = (rng.random(F) < 0.5).astype(np.uint8)
    r = fwbf.count(N, torch.from_numpy(z.view(np.int32)).cuda(), torch.from_numpy(pool.view(np.int32)).cuda(),
                   0, torch.from_numpy(it).cuda(), torch.from_numpy(ok).cuda(), 50)
    ro = O.count(N, z, pool, 0, it, ok, 50)
    for k in ("bit_err", "frame_err", "undetected", "iter_sum", "frames"):
        assert r[k] == ro[k], k
    assert np.array_equal(r["hist"], ro["hist"])
    assert r["syn_ok"] == int(ok.sum())


def test_decode_of_generated_frames_matches_oracle(code):
    """Chain channel -> decode -> count on the GPU; the oracle decodes the same
    (copied) frames: decisions and counters are identical."""
    g, o = code
    F, N = 2048, g.N
    pool = o.encode(8, 0, 128)
    poold = torch.from_numpy(pool.view(np.int32)).cuda()
    y = fwbf.channel(N, F, 0, poold, 44, 0, 0.6, dtype=torch.int8, scale=16.0)
    z, it, ok = fwbf.decode(g, y, fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100))
    r = fwbf.count(N, z, poold, 0, it, ok, 100)
    yh = y.cpu().numpy()
    zo, ito, oko = O.decode(o, yh, G=8, max_iter=100)
    assert np.array_equal(z.cpu().numpy().view(np.uint32), zo) and np.array_equal(it.cpu().numpy(), ito)
    ro = O.count(N, zo, pool, 0, ito, oko, 100)
    for k in ("bit_err", "frame_err", "undetected", "iter_sum"):
        assert r[k] == ro[k], k


@pytest.mark.parametrize("N,F,f0,use_pool", [(186, 1001, 0, True), (1008, 777, 5, True), (2016, 333, 1 << 33, True),
                                              (4032, 129, 17, True), (1008, 65, 0, False)])
def test_count_layouts_match_oracle(N, F, f0, use_pool):
    """Frames of 6, 32, 63 and 126 words (several frames per wavefront pass,
    one, and a word loop), ragged frame counts, pool wrap-around at an offset,
    no pool, and round counts outside [0, K_max] (not histogrammed)."""
    need_gpu()
    rng = np.random.default_rng(N + F)
    max_iter = 40
    pool = O.pack(rng.random((37, N)) < 0.5) if use_pool else None
    base = O.unpack(pool[(f0 + np.arange(F)) % 37], N) if use_pool else np.zeros((F, N), np.uint8)
    flips = rng.random((F, N)) < np.where(rng.random(F) < 0.6, 0.0, 0.02)[:, None]
    z = O.pack(base ^ flips)
    it = rng.integers(-3, max_iter + 4, F).astype(np.int32)
    ok = (rng.random(F) < 0.5).astype(np.uint8)
    pd = torch.from_numpy(pool.view(np.int32)).cuda() if use_pool else None
    r = fwbf.count(N, torch.from_numpy(z.view(np.int32)).cuda(), pd, f0, torch.from_numpy(it).cuda(),
                   torch.from_numpy(ok).cuda(), max_iter)
    ro = O.count(N, z, pool, f0, it, ok, max_iter)
    for k in ("bit_err", "frame_err", "undetected", "iter_sum", "frames"):
        assert r[k] == ro[k], (k, r[k], ro[k])
    assert np.array_equal(r["hist"], ro["hist"])
    assert r["syn_ok"] == int(ok.sum())
