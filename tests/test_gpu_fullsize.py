"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times: the same codes, seeds, frame counts and
decoder parameters, one launch over every frame.  The oracle decodes a sample
of frames (the first, the last and seeded ones in between) from the very same
received values and must agree bit for bit; every frame is checked against
properties that hold at any size: the syndrome flag equals [H z = 0] (Section
III, Step 1) and a frame that ends with a nonzero syndrome reports K_max rounds
(the decoder stops only on a zero syndrome or at K_max)."""
import numpy as np
import pytest

import oracle as O
from conftest import CODES
from gpu_util import check_properties, need_gpu, oracle_decode, torch
from paper_1206_3362_amd import synth

pytestmark = pytest.mark.gpu

DT_OF = {torch.float32: np.float32, torch.int8: np.int8, torch.int16: np.int16}


def sample_rows(F, n, seed):
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(16, F - 16), size=max(0, n - 32), replace=False)
    return np.unique(np.concatenate([np.arange(16), np.arange(F - 16, F), mid]))


def check_sampled(ocode, y, z, it, ok, rows, what, **kw):
    idx = torch.from_numpy(rows).to(y.device)
    ys = y.index_select(0, idx).cpu().numpy()
    zg = z.index_select(0, idx).cpu().numpy().view(np.uint32)
    ig = it.index_select(0, idx).cpu().numpy()
    kg = ok.index_select(0, idx).cpu().numpy()
    print(f"{what}: oracle on {len(rows)} of {y.shape[0]} frames {kw}", flush=True)
    zo, io, ko = oracle_decode(ocode, ys, **kw)
    bad = np.nonzero((zg != zo).any(1) | (ig != io) | (kg != ko))[0]
    assert bad.size == 0, (f"{what}: {bad.size} sampled frames differ, first frames "
                           f"{rows[bad[:8]].tolist()}; gpu iters {ig[bad[:4]].tolist()} "
                           f"oracle {io[bad[:4]].tolist()}")


def test_headline_launch_n1008_int8():
    """(3,6) Z=168 code, 2^20 int8 frames (scale 16) of seeded codewords at
    4 dB, IMWBF alpha 1/5, G=8, K_max=100: the benchmark's timed launch."""
    need_gpu()
    from paper_1206_3362_amd import fwbf
    code = fwbf.Code.from_seed(3, 6, 168, 2)
    oc = O.Code.from_seed(*CODES["n1008"])
    N, F = code.N, 1 << 20
    pool = torch.from_numpy(code.encode(seed=1001, first=0, count=1024).view(np.int32)).cuda()
    y = torch.empty((F, N), dtype=torch.int8, device="cuda")
    fwbf.channel_into(N, y, 0, pool, seed=1100, stream_id=4, sigma=float(synth.sigma_for(4.0, code.rate)),
                      scale=16.0)
    p = fwbf.DecodeParams(dtype=fwbf.I8, weights=fwbf.IMWBF, select=fwbf.GROUPS, groups=8, max_iter=100,
                          alpha_num=1, alpha_den=5)
    z, it, ok = fwbf.decode(code, y, p)
    torch.cuda.synchronize()
    check_sampled(oc, y, z, it, ok, sample_rows(F, 512, 1), "n1008 i8 2^20", weights=2, groups=8,
                  max_iter=100, alpha_num=1, alpha_den=5)
    check_properties(oc, z, it, ok, 100, "n1008 i8 2^20")


def test_n186_wbf_all_frames():
    """(3,6) Z=31 code, all-zero codeword, 1000 float frames at 3 dB from the
    benchmark's channel seed, WBF, alpha 0.2, G=6, K_max=50, automatic launch
    width (the whole batch fits on the device, so the library widens it):
    every frame against the oracle."""
    need_gpu()
    from paper_1206_3362_amd import fwbf
    code = fwbf.Code.from_seed(3, 6, 31, 1)
    oc = O.Code.from_seed(*CODES["n186"])
    F = 1000
    y = fwbf.channel(code.N, F, 0, None, 2024, 0, float(synth.sigma_for(3.0, code.rate)))
    p = fwbf.DecodeParams(dtype=fwbf.F32, weights=fwbf.WBF, groups=6, max_iter=50, alpha=0.2)
    z, it, ok = fwbf.decode(code, y, p)
    torch.cuda.synchronize()
    check_sampled(oc, y, z, it, ok, np.arange(F), "n186 wbf 1000", weights=0, groups=6, max_iter=50, alpha=0.2)
    check_properties(oc, z, it, ok, 50, "n186 wbf 1000")


def test_mixed_batch_full_size():
    """N=1008/4032 (3,6) and N=8000 (4,20) codes with 2^18/2^16/2^15 float
    frames, Eb/N0 drawn per frame from U[3,6] dB, G=8/32/64, K_max=100, all
    in one persistent launch."""
    need_gpu()
    from paper_1206_3362_amd import fwbf
    specs = [("n1008", 1 << 18, 8), ("n4032", 1 << 16, 32), ("n8000", 1 << 15, 64)]
    jobs, ocs = [], []
    for i, (name, F, G) in enumerate(specs):
        code = fwbf.Code.from_seed(*CODES[name])
        pool = torch.from_numpy(code.encode(31 + i, 0, 256).view(np.int32)).cuda()
        eb = synth.uniform_frames(code.N, F, 77 + i, 3.0, 6.0)
        sig = torch.from_numpy(synth.sigma_for(eb, code.rate).astype(np.float32)).cuda()
        y = fwbf.channel(code.N, F, 0, pool, 500 + i, i, 0.0, sigma_per_frame=sig)
        jobs.append((code, y, fwbf.DecodeParams(dtype=fwbf.F32, groups=G, max_iter=100)))
        ocs.append(O.Code.from_seed(*CODES[name]))
    ws = torch.zeros(64, dtype=torch.int32, device="cuda")
    outs = fwbf.decode_batched(jobs, workspace=ws)
    torch.cuda.synchronize()
    for (name, F, G), (code, y, p), oc, (z, it, ok) in zip(specs, jobs, ocs, outs):
        check_sampled(oc, y, z, it, ok, sample_rows(F, 96, 2), f"batch {name} f32", groups=G, max_iter=100)
        check_properties(oc, z, it, ok, 100, f"batch {name} f32")


def test_mixed_batch_full_size_autotuned():
    """The mixed batch as the benchmark times it: the autotuner picks each
    code's G (under the frame-error constraint) and the launch shape with the
    benchmark's candidate lists, then the one launch at those settings is
    checked like the reference-G launch above."""
    need_gpu()
    import bench
    from paper_1206_3362_amd import autotune, fwbf
    jobs, ocs = [], []
    for i, (spec, F, G, _) in enumerate(bench.MIXED_JOBS):
        code = fwbf.Code.from_seed(*spec)
        pool = torch.from_numpy(code.encode(31 + i, 0, 256).view(np.int32)).cuda()
        eb = synth.uniform_frames(code.N, F, 77 + i, 3.0, 6.0)
        sig = torch.from_numpy(synth.sigma_for(eb, code.rate).astype(np.float32)).cuda()
        y = fwbf.channel(code.N, F, 0, pool, 500 + i, i, 0.0, sigma_per_frame=sig)
        jobs.append((code, y, pool, fwbf.DecodeParams(dtype=fwbf.F32, groups=G, max_iter=100)))
        ocs.append(O.Code.from_seed(*spec))
    tuned = autotune.tune_batch(jobs, [j[3] for j in bench.MIXED_JOBS], **bench.MIXED_TUNE)
    batch = [(code, y, p) for (code, y, _, _), p in zip(jobs, tuned["params"])]
    outs = fwbf.decode_batched(batch, threads_per_frame=tuned["threads_per_frame"],
                               blocks_per_cu=tuned["blocks_per_cu"])
    torch.cuda.synchronize()
    for (code, y, p), oc, (z, it, ok) in zip(batch, ocs, outs):
        what = f"tuned batch N={code.N} G={p.groups} f32"
        check_sampled(oc, y, z, it, ok, sample_rows(y.shape[0], 96, 3), what, groups=p.groups, max_iter=100)
        check_properties(oc, z, it, ok, 100, what)


def test_n32400_int16_full_size():
    """(3,30) Z=1080 rate-0.9 code, 2^18 int16 frames (scale 256) at 6 dB,
    G=64, K_max=100."""
    need_gpu()
    from paper_1206_3362_amd import fwbf
    code = fwbf.Code.from_seed(*CODES["n32400"])
    oc = O.Code.from_seed(*CODES["n32400"])
    N, F = code.N, 1 << 18
    pool = torch.from_numpy(code.encode(5, 0, 64).view(np.int32)).cuda()
    y = fwbf.channel(N, F, 0, pool, 900, 6, float(synth.sigma_for(6.0, code.rate)), dtype=torch.int16,
                     scale=256.0)
    p = fwbf.DecodeParams(dtype=fwbf.I16, groups=64, max_iter=100)
    z, it, ok = fwbf.decode(code, y, p)
    torch.cuda.synchronize()
    check_sampled(oc, y, z, it, ok, sample_rows(F, 64, 3), "n32400 i16 2^18", groups=64, max_iter=100)
    check_properties(oc, z, it, ok, 100, "n32400 i16 2^18")


@pytest.mark.parametrize("dt", [torch.float32, torch.int8])
def test_eg1023_full_size(dt):
    """EG(1023,781), 2^16 frames of seeded codewords at 4 dB, blocks of p=31
    bits (G=33), K_max=10: float with alpha 1.5, int8 (scale 16) with 3/2."""
    need_gpu()
    from paper_1206_3362_amd import fwbf
    text = synth.eg_code_text(5)
    code, oc = fwbf.Code.from_text(text), O.Code.from_text(text)
    N, F = code.N, 1 << 16
    pool = torch.from_numpy(code.encode(1023, 0, 1024).view(np.int32)).cuda()
    sigma = float(synth.sigma_for(4.0, code.rate))
    if dt == torch.float32:
        y = fwbf.channel(N, F, 0, pool, 1300, 2, sigma)
        p = fwbf.DecodeParams(dtype=fwbf.F32, weights=fwbf.IMWBF, groups=33, max_iter=10, alpha=1.5)
        kw = dict(weights=2, groups=33, max_iter=10, alpha=1.5)
    else:
        y = fwbf.channel(N, F, 0, pool, 1300, 2, sigma, dtype=torch.int8, scale=16.0)
        p = fwbf.DecodeParams(dtype=fwbf.I8, weights=fwbf.IMWBF, groups=33, max_iter=10, alpha_num=3,
                              alpha_den=2)
        kw = dict(weights=2, groups=33, max_iter=10, alpha_num=3, alpha_den=2)
    z, it, ok = fwbf.decode(code, y, p)
    torch.cuda.synchronize()
    check_sampled(oc, y, z, it, ok, sample_rows(F, 256, 4), f"eg1023 {DT_OF[dt].__name__} 2^16", **kw)
    check_properties(oc, z, it, ok, 10, f"eg1023 {DT_OF[dt].__name__} 2^16")


def test_sweep_graph_every_point_full_size():
    """The Eb/N0 sweep as the benchmark runs it: one HIP graph over the nine
    points 2.0 ... 6.0 dB of the N = 1008 int8 code, 2^20 frames per point,
    G = 8, K_max = 100.  After one replay every point's frames and outputs
    are read back: the oracle decodes 256 sampled frames per point, every
    frame is checked against the flag and K_max properties, and the graph's
    counters equal a recount of the outputs."""
    need_gpu()
    from paper_1206_3362_amd import fwbf
    code = fwbf.Code.from_seed(3, 6, 168, 2)
    oc = O.Code.from_seed(*CODES["n1008"])
    N, F = code.N, 1 << 20
    pool = torch.from_numpy(code.encode(1001, 0, 1024).view(np.int32)).cuda()
    ebs = np.arange(2.0, 6.01, 0.5)
    sw = fwbf.Sweep(code, fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100),
                    synth.sigma_for(ebs, code.rate), F, pool=pool, seed=1100, scale=16.0)
    sw.launch()
    c = sw.counters()
    for k, eb in enumerate(ebs):
        y, z, it, ok = sw.outputs(k)
        torch.cuda.synchronize()
        what = f"sweep point {eb:.1f} dB"
        check_sampled(oc, y, z, it, ok, sample_rows(F, 256, 100 + k), what, weights=2, groups=8,
                      max_iter=100, alpha_num=1, alpha_den=5)
        check_properties(oc, z, it, ok, 100, what)
        r = fwbf.count(N, z, pool, 0, it, ok, 100)
        assert (r["bit_err"], r["frame_err"], r["undetected"], r["iter_sum"], r["frames"]) == \
            tuple(int(v) for v in c[k, :5]), what
        del y, z, it, ok
    del sw
