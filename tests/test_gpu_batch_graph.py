"""Mixed-code persistent launch, HIP-graph Eb/N0 sweep and autotuner.

The batched launch must reproduce, frame for frame, what fwbf_decode gives on
each code alone (and the oracle on a sample); every replay of the captured
sweep must equal the same work launched eagerly (replays interleaved with
eager work); the autotuner's choice must satisfy its frame-error
constraint."""
import numpy as np
import pytest

import oracle as O
from gpu_util import assert_same, need_gpu, torch
from paper_1206_3362_amd import autotune, fwbf, synth

pytestmark = pytest.mark.gpu

CODES = [((3, 6, 168, 2), 2048, 8), ((3, 6, 672, 3), 512, 32), ((4, 20, 400, 4), 256, 64)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _frames(code, F, seed, dtype, scale):
    pool = torch.from_numpy(code.encode(seed, 0, 64).view(np.int32)).cuda()
    eb = synth.uniform_frames(code.N, F, seed, 3.0, 6.0)
    sig = torch.from_numpy(synth.sigma_for(eb, code.rate).astype(np.float32)).cuda()
    return fwbf.channel(code.N, F, 0, pool, seed, 2, 0.0, dtype=dtype, scale=scale, sigma_per_frame=sig)


@pytest.mark.parametrize("T", [0, 256])
def test_mixed_code_batch_equals_per_code_decoding(T):
    jobs, codes = [], []
    for i, (spec, F, G) in enumerate(CODES):
        code = fwbf.Code.from_seed(*spec)
        y = _frames(code, F, 10 + i, torch.float32, 1.0)
        jobs.append((code, y, fwbf.DecodeParams(dtype=fwbf.F32, groups=G, max_iter=100)))
        codes.append(spec)
    outs = fwbf.decode_batched(jobs, threads_per_frame=T)
    torch.cuda.synchronize()
    for (code, y, p), (z, it, ok), spec in zip(jobs, outs, codes):
        print(f"batch item N={code.N} F={y.shape[0]}", flush=True)
        zr, itr, okr = fwbf.decode(code, y, p)
        torch.cuda.synchronize()
        assert_same((z.cpu().numpy(), it.cpu().numpy(), ok.cpu().numpy()),
                    (zr.cpu().numpy(), itr.cpu().numpy(), okr.cpu().numpy()), f"batch N={code.N}")
        o = O.Code.from_seed(*spec)
        yh = y[:32].cpu().numpy()
        zo, ito, oko = O.decode(o, yh, G=p.groups, max_iter=100, alpha=0.2)
        assert_same((z[:32].cpu().numpy().view(np.uint32), it[:32].cpu().numpy(), ok[:32].cpu().numpy()),
                    (zo, ito, oko), f"oracle N={code.N}")


def test_batch_one_frame_per_wavefront_ragged_chunks():
    """Short frames decoded one per wavefront inside 256-thread workgroups
    (N = 186, EG(255) with strided blocks) next to frames that take the
    whole workgroup (N = 4032), with frame counts that leave partial
    chunks: equal to decoding each code alone."""
    eg = fwbf.Code.from_text(synth.eg_code_text(4))
    jobs = [(fwbf.Code.from_seed(3, 6, 31, 1), 1001, dict(groups=6)),
            (eg, 333, dict(select=fwbf.STRIDED, groups=16, alpha=1.0)),
            (fwbf.Code.from_seed(3, 6, 672, 3), 77, dict(groups=32))]
    batch = []
    for i, (code, F, kw) in enumerate(jobs):
        y = _frames(code, F, 30 + i, torch.float32, 1.0)
        batch.append((code, y, fwbf.DecodeParams(dtype=fwbf.F32, max_iter=60, **kw)))
    outs = fwbf.decode_batched(batch)
    torch.cuda.synchronize()
    for (code, y, p), (z, it, ok) in zip(batch, outs):
        print(f"batch item N={code.N} F={y.shape[0]}", flush=True)
        zr, itr, okr = fwbf.decode(code, y, p)
        torch.cuda.synchronize()
        assert_same((z.cpu().numpy(), it.cpu().numpy(), ok.cpu().numpy()),
                    (zr.cpu().numpy(), itr.cpu().numpy(), okr.cpu().numpy()), f"batch N={code.N}")


def test_int8_batch_equals_fast_kernel():
    jobs = []
    for i, (spec, F, G) in enumerate([((3, 6, 31, 1), 700, 6), ((3, 6, 168, 2), 1500, 8)]):
        code = fwbf.Code.from_seed(*spec)
        y = _frames(code, F, 20 + i, torch.int8, 16.0)
        jobs.append((code, y, fwbf.DecodeParams(dtype=fwbf.I8, groups=G, max_iter=80)))
    outs = fwbf.decode_batched(jobs, blocks_per_cu=4)
    for (code, y, p), (z, it, ok) in zip(jobs, outs):
        zr, itr, okr = fwbf.decode(code, y, p)
        torch.cuda.synchronize()
        assert_same((z.cpu().numpy(), it.cpu().numpy(), ok.cpu().numpy()),
                    (zr.cpu().numpy(), itr.cpu().numpy(), okr.cpu().numpy()), f"int8 batch N={code.N}")


def test_graph_sweep_replays_equal_eager_launches():
    code = fwbf.Code.from_seed(3, 6, 168, 2)
    pool = torch.from_numpy(code.encode(3, 0, 128).view(np.int32)).cuda()
    sig = synth.sigma_for(np.array([3.0, 4.0, 5.0, 6.0]), code.rate).astype(np.float32)
    p = fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100)
    F = 8192
    sw = fwbf.Sweep(code, p, sig, F, pool=pool, seed=77, scale=16.0)
    # the same work, launched eagerly
    eager = []
    for i, s in enumerate(sig):
        y = fwbf.channel(code.N, F, 0, pool, 77, i, float(s), dtype=torch.int8, scale=16.0)
        z, it, ok = fwbf.decode(code, y, p)
        r = fwbf.count(code.N, z, pool, 0, it, ok, 100)
        eager.append([r["bit_err"], r["frame_err"], r["undetected"], r["iter_sum"], r["frames"],
                      r["syn_ok"]] + list(r["hist"]))
    eager = np.array(eager)
    for rep in range(3):
        sw.launch()
        c = sw.counters()
        assert np.array_equal(c, eager), f"replay {rep}"
        # unrelated eager work between replays
        y = fwbf.channel(code.N, 1024, 5, pool, 9, 9, 0.7, dtype=torch.int8, scale=16.0)
        fwbf.decode(code, y, p)
        torch.cuda.synchronize()
    assert eager[:, 1].tolist() == sorted(eager[:, 1].tolist(), reverse=True)  # FER falls with Eb/N0


def test_autotuner_respects_fer_constraint(tmp_path):
    code = fwbf.Code.from_seed(3, 6, 168, 2)
    cache = str(tmp_path / "tune.json")
    r = autotune.tune(code, 6.0, G_ref=8, Gs=(8, 16, 32), widths=(0, 128), frames=8192,
                      cache=cache)
    assert r["admissible"]
    n = 8192
    for row in r["table"]:
        assert row["admissible"] == autotune.fer_admissible(round(row["fer"] * n), n,
                                                            round(r["fer_ref"] * n), n)
        if row["admissible"]:
            assert row["gbps"] <= r["gbps"] + 1e-9
    # cached
    r2 = autotune.tune(code, 6.0, G_ref=8, Gs=(8, 16, 32), widths=(0, 128), frames=8192,
                       cache=cache)
    assert r2 == r


def test_batch_autotuner_choices():
    """Each job's chosen G passes the frame-error test against its reference
    G on the tuning frames, the chosen launch shape is the fastest timed one,
    and the batch decoded with the chosen settings equals each code decoded
    alone with the same G."""
    jobs = []
    for i, (spec, F, G) in enumerate(CODES):
        code = fwbf.Code.from_seed(*spec)
        pool = torch.from_numpy(code.encode(40 + i, 0, 64).view(np.int32)).cuda()
        eb = synth.uniform_frames(code.N, F, 40 + i, 3.0, 6.0)
        sig = torch.from_numpy(synth.sigma_for(eb, code.rate).astype(np.float32)).cuda()
        y = fwbf.channel(code.N, F, 0, pool, 40 + i, 2, 0.0, sigma_per_frame=sig)
        jobs.append((code, y, pool, fwbf.DecodeParams(dtype=fwbf.F32, groups=G, max_iter=100)))
    cands = [(8, 16), (32, 64), (64, 128)]
    r = autotune.tune_batch(jobs, cands, tune_frames=256, widths=(0, 256), blocks=(0, 2), repeats=1)
    for (code, y, pool, p0), p, cand in zip(jobs, r["params"], cands):
        assert p.groups in cand or p.groups == p0.groups
        rows = [row for row in r["g_table"] if row["N"] == code.N]
        n = min(256, y.shape[0])
        for row in rows:
            assert row["admissible"] == autotune.fer_admissible(round(row["fer"] * n), n,
                                                                round(row["fer_ref"] * n), n)
        pick = [row for row in rows if row["G"] == p.groups]
        assert not pick or pick[0]["admissible"]
    assert r["ms"] == min(row["ms"] for row in r["shape_table"])
    batch = [(code, y, p) for (code, y, _, _), p in zip(jobs, r["params"])]
    outs = fwbf.decode_batched(batch, threads_per_frame=r["threads_per_frame"],
                               blocks_per_cu=r["blocks_per_cu"])
    for (code, y, p), (z, it, ok) in zip(batch, outs):
        z1, it1, ok1 = fwbf.decode(code, y, p)
        assert torch.equal(z, z1) and torch.equal(it, it1) and torch.equal(ok, ok1)
