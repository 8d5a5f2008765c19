"""Decoded throughput of plain FWBF on one MI355X.

Workload: the (3,6)-regular QC-LDPC code with Z=168 (N=1008, M=504, seeded
draw, seed 2), random codewords from the seeded systematic encoder, BPSK over
AWGN at Eb/N0 = 4 dB, y quantised to int8 (scale 16), IMWBF metric (eq. (1))
with alpha = 1/5, G = 8 blocks (p = 126), at most 100 flip rounds, 2^20
frames per batch.  Frames are generated on the GPU (Philox + Box-Muller)
before the timed region; a step decodes one resident batch and accumulates
its error counts.  Value = coded decoded Gb/s = frames * N / time.

Prints one JSON line (rank 0).  Only N=1 is supported: the decoder runs on a
single GPU (frames are independent: several GPUs would each decode their own
share of the frames and add up the error counters once at the end).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded Gb/s at fixed FER (N=1008, 4 dB), learned vs plain FWBF; % HBM peak"
HBM_PEAK_GBS = 8000.0
# 32-bit VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 39.3216
# mixed-code batch: (code (mb, nb, Z, seed), frames, reference G, G candidates)
MIXED_JOBS = [((3, 6, 168, 2), 1 << 18, 8, (2, 3, 4, 6, 8, 12, 16)),
              ((3, 6, 672, 3), 1 << 16, 32, (4, 8, 12, 16, 24, 32, 48)),
              ((4, 20, 400, 4), 1 << 15, 64, (4, 8, 12, 16, 24, 32, 48, 64, 96))]
MIXED_TUNE = dict(tune_frames=1 << 14, widths=(0, 128, 256), blocks=(0, 2, 4), repeats=3)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=1 << 20)
    ap.add_argument("--ebn0", type=float, default=4.0)
    ap.add_argument("--groups", type=int, default=8)
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--batches", type=int, default=2, help="distinct resident batches cycled")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--traffic", type=str, default=os.path.join(ROOT, "profiles", "traffic_decode_n1008_i8_4db.json"))
    ap.add_argument("--learned", type=int, default=1, help="also time the learned decoder (1/0)")
    ap.add_argument("--n32400", type=int, default=1,
                    help="also compare learned and plain FWBF on the N=32400 int16 code at 6 and 7 dB (1/0)")
    ap.add_argument("--fer-table", type=int, default=1,
                    help="also time plain FWBF at G = 1, 2, 4, 8 and SINGLE on the same frames (1/0)")
    ap.add_argument("--scorer", type=str,
                    default=os.path.join(ROOT, "paper_1206_3362_amd", "scorer_n1008_g32_t16.npz"))
    ap.add_argument("--workload", default="n1008_i8",
                    choices=["n1008_i8", "n186_f32_wbf", "mixed_f32", "n32400_i16", "sweep_n1008_i8",
                             "eg1023", "eg1023_tab1", "eg255_delay", "strided_n1008", "minsum_eg255"],
                    help="n1008_i8: the headline workload; the others are further configurations "
                         "measured with the same protocol (one JSON line each)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (scales the HBM counters)")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}))


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration()
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the FWBF decoder has no multi-GPU path "
              "(frames are independent: several GPUs would each decode their own share "
              "of the frames and add up the error counters at the end).",
              file=sys.stderr)
        sys.exit(2)
    if a.workload != "n1008_i8":
        other_workload(a)
        return
    import numpy as np
    import torch

    from paper_1206_3362_amd import fwbf, synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    code = fwbf.Code.from_seed(3, 6, 168, 2)
    N, K = code.N, code.K
    sigma = float(synth.sigma_for(a.ebn0, code.rate))
    pool_h = code.encode(seed=1001, first=0, count=1024)
    pool = torch.from_numpy(pool_h.view(np.int32)).to(dev)
    F = a.frames
    ys = []
    for b in range(a.batches):
        y = torch.empty((F, N), dtype=torch.int8, device=dev)
        fwbf.channel_into(N, y, b * F, pool, seed=1100, stream_id=4, sigma=sigma, scale=16.0)
        ys.append(y)
    params = fwbf.DecodeParams(dtype=fwbf.I8, weights=fwbf.IMWBF, select=fwbf.GROUPS,
                               groups=a.groups, max_iter=a.max_iter, alpha_num=1, alpha_den=5)
    z = torch.empty((F, (N + 31) // 32), dtype=torch.int32, device=dev)
    it = torch.empty(F, dtype=torch.int32, device=dev)
    ok = torch.empty(F, dtype=torch.uint8, device=dev)
    counters = torch.zeros(7 + a.max_iter, dtype=torch.int64, device=dev)

    def step(s, ev=None):
        b = s % a.batches
        if ev is not None:
            ev[0].record()
        fwbf.decode_into(code, ys[b], params, z, it, ok)
        if ev is not None:
            ev[1].record()
        fwbf.count_into(N, z, pool, b * F, it, ok, a.max_iter, counters)

    for s in range(a.warmup):
        step(s)
    torch.cuda.synchronize()
    counters.zero_()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(a.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for s in range(a.steps):
        step(s, evs[s])
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    dec_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    ms_step = total_ms / a.steps
    c = counters.cpu().numpy()
    frames = int(c[4])
    value = F * N / (ms_step * 1e-3) / 1e9
    dec_avg = float(np.mean(dec_ms))
    bytes_per_frame = N * 1 + 4 * ((N + 31) // 32) + 4 + 1
    achieved = F * bytes_per_frame / (dec_avg * 1e-3) / 1e9
    traffic = None
    if os.path.exists(a.traffic):
        tr = json.load(open(a.traffic))
        if tr.get("frames") == F and tr.get("kernel_source_sha") == kernel_sha():
            traffic = tr.get("bytes_per_launch")
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gb/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded codewords, GPU Philox AWGN, int8 x16)",
        "config": {
            "workload": "plain FWBF, (3,6) QC-LDPC Z=168 N=1008 M=504 K=%d, Eb/N0 %.1f dB, int8 y, "
                        "IMWBF alpha=1/5, G=%d, K_max=%d, %d frames" % (K, a.ebn0, a.groups,
                                                                      a.max_iter, F),
            "frames": F, "N": N, "K": K, "ebn0_db": a.ebn0, "groups": a.groups,
            "max_iter": a.max_iter, "input": "int8 (scale 16)", "parallelism": "single GPU",
        },
        "decode_kernel_ms": round(dec_avg, 4),
        "info_gbps": round(F * K / (ms_step * 1e-3) / 1e9, 3),
        "fer": c[1] / frames, "ber": c[0] / (frames * N), "undetected": int(c[2]),
        "mean_iters": c[3] / frames, "frames_counted": frames,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": traffic, "kernel": "fast_kernel<int8,3,6,16>",
                     "bytes_per_frame": bytes_per_frame},
        "wall_s": round(wall, 3),
    }
    # rounds the kernel actually runs (the repeated-state shortcut reports
    # K_max for frames whose state repeats): an untimed diagnostic decode
    pe = fwbf.DecodeParams(**{**params.__dict__, "flags": params.flags | fwbf.FLAG_EXECUTED_ROUNDS})
    fwbf.decode_into(code, ys[0], pe, z, it, ok)
    out["executed_rounds"] = round(float(it.double().mean().item()), 3)
    # the same kernel against its arithmetic ceiling: the paper's round
    # recomputes every metric (2E + 2N lane-ops: E = N dv edges), the
    # initialisation takes N + 4E (syndrome and check minima); the rounds
    # counted are the ones the kernel executes
    E = 3 * N
    ops = F * ((N + 4 * E) + out["executed_rounds"] * (2 * E + 2 * N))
    alu = ops / (dec_avg * 1e-3) / 1e12
    out["roofline_alu"] = {"bound": "alu", "achieved": round(alu, 3), "peak": ALU_PEAK_TOPS,
                           "unit": "T lane-ops/s", "frac": round(alu / ALU_PEAK_TOPS, 4),
                           "ops_per_frame": round(ops / F)}
    prof = valu_profile()
    if prof:
        issue = F * prof["valu_insts_per_frame"] * 4 / (1024 * 2.4e9) / (dec_avg * 1e-3)
        out["valu_issue_frac"] = round(issue, 3)
        out["valu_note"] = ("wave64 VALU instructions per frame from %s x frames x 4 cycles over "
                            "1024 SIMDs at 2.4 GHz, divided by the decode time" % prof["source"])
    if a.learned:
        out["learned"] = learned_leg(code, ys, pool, params, a, N, F, ms_step, c)
    if a.fer_table:
        out["fer_vs_gbps"] = fer_table(code, ys, pool, params, a, N, F, out)
    if a.n32400:
        # the high-rate code, where the retrained learned decoder is both
        # faster and better than plain FWBF (6 and 7 dB, 3 timed steps each)
        res, tuned, lp = n32400_compare(3, 1, (6.0, 7.0))
        out["n32400_i16"] = {"points": res, "plain_G_tuned": int(tuned["G"]),
                             "workload": "N=32400 (3,30) QC rate 0.9, int16 x256, K_max=100, 2^18 frames per point; "
                                         "learned FWBF (scorer_n32400_g512_t16.npz, plain fallback) vs plain FWBF "
                                         "at the autotuned G"}
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(code, ys[0], params, a, N)
    print(json.dumps(out), flush=True)


def learned_leg(code, ys, pool, params, a, N, F, plain_ms, plain_counts):
    """The learned decoder (checkpointed scorer, plain FWBF fallback) on the
    same resident batches, same timing protocol."""
    import numpy as np
    import torch

    from paper_1206_3362_amd import fwbf
    d = np.load(a.scorer, allow_pickle=False)
    cfg = dict((k, v) for k, v in d["config"])
    lp = fwbf.LearnedParams(int(cfg["rounds"]), int(cfg["groups"]), int(cfg["topk"]), 16.0)
    sc = torch.from_numpy(d["params"]).cuda()
    z = torch.empty((F, (N + 31) // 32), dtype=torch.int32, device="cuda")
    it = torch.empty(F, dtype=torch.int32, device="cuda")
    ok = torch.empty(F, dtype=torch.uint8, device="cuda")
    lok = torch.empty(F, dtype=torch.uint8, device="cuda")
    counters = torch.zeros(7 + a.max_iter + lp.rounds, dtype=torch.int64, device="cuda")
    for s in range(a.warmup):
        fwbf.decode_learned_into(code, ys[s % a.batches], params, lp, sc, z, it, ok, lok)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for s in range(a.steps):
        b = s % a.batches
        fwbf.decode_learned_into(code, ys[b], params, lp, sc, z, it, ok, lok)
        fwbf.count_into(N, z, pool, b * F, it, ok, a.max_iter + lp.rounds, counters)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / a.steps
    cc = counters.cpu().numpy()
    fer = cc[1] / cc[4]
    pfer = plain_counts[1] / plain_counts[4]
    gbps = F * N / (ms * 1e-3) / 1e9
    pg = F * N / (plain_ms * 1e-3) / 1e9
    return {"value": round(gbps, 3), "unit": "Gb/s", "ms_per_step": round(ms, 4), "fer": float(fer),
            "ber": float(cc[0] / (cc[4] * N)), "plain_fer": float(pfer),
            "goodput_gbps": round(gbps * (1 - fer), 3), "plain_goodput_gbps": round(pg * (1 - pfer), 3),
            "learned_pass_only": float(lok.float().mean().item()),
            "scorer": os.path.basename(a.scorer), "rounds": lp.rounds, "groups": lp.groups,
            "topk": lp.topk}


def fer_table(code, ys, pool, params, a, N, F, out):
    """Decoded Gb/s against FER on the same resident frames: plain FWBF with
    fewer, longer blocks (G = 1, 2, 4, 8) and the single-bit rule (SINGLE),
    beside the learned decoder, so that Gb/s can be read at a fixed FER.
    Each row: 3 timed steps after 1 warm-up, counts over the first batch."""
    import torch

    from paper_1206_3362_amd import fwbf
    rows = []
    z = torch.empty((F, (N + 31) // 32), dtype=torch.int32, device="cuda")
    it = torch.empty(F, dtype=torch.int32, device="cuda")
    ok = torch.empty(F, dtype=torch.uint8, device="cuda")
    cases = [(f"plain G={G}", dict(groups=G)) for G in (1, 2, 4, 8)] + [("plain SINGLE", dict(select=fwbf.SINGLE))]
    for name, kw in cases:
        p = fwbf.DecodeParams(**{**params.__dict__, **kw})
        ms = _timed(lambda: fwbf.decode_into(code, ys[0], p, z, it, ok), 3, 1)
        r = fwbf.count(N, z, pool, 0, it, ok, a.max_iter)
        pe = fwbf.DecodeParams(**{**p.__dict__, "flags": p.flags | fwbf.FLAG_EXECUTED_ROUNDS})
        fwbf.decode_into(code, ys[0], pe, z, it, ok)
        rows.append({"decoder": name, "fer": round(r["frame_err"] / F, 5),
                     "gbps": round(F * N / (ms * 1e-3) / 1e9, 3), "ms": round(ms, 4),
                     "mean_rounds": round(r["iter_sum"] / F, 3),
                     "executed_rounds": round(float(it.double().mean().item()), 3)})
    if "learned" in out:
        L = out["learned"]
        rows.append({"decoder": "learned + plain fallback", "fer": round(L["fer"], 5), "gbps": L["value"],
                     "ms": L["ms_per_step"]})
        fer_l = L["fer"]
        sd = 3.0 * (fer_l * (1 - fer_l) * 2.0 / F) ** 0.5
        reach = [r for r in rows[:-1] if r["fer"] <= fer_l + sd]
        rows.append({"at_learned_fer": {
            "learned_gbps": L["value"], "learned_fer": round(fer_l, 5),
            "fastest_plain_at_or_below": max(reach, key=lambda r: r["gbps"]) if reach else None,
            "note": ("no plain configuration in the table reaches the learned decoder's FER at this "
                     "Eb/N0" if not reach else "plain configurations within 3 sigma of the learned FER")}})
    return rows


def valu_profile():
    """VALU instructions per frame of the timed kernel from the committed
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_decode_n1008_i8_4db.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    if tr.get("kernel_source_sha") != kernel_sha() or "valu_insts_per_frame" not in tr:
        return None
    return {"valu_insts_per_frame": tr["valu_insts_per_frame"], "source": "profiles/" + os.path.basename(path)}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def other_workload(a):
    """Further configurations: same protocol (inputs resident, warm-up, events
    around exactly `steps` steps), one JSON line each."""
    import numpy as np
    import torch

    from paper_1206_3362_amd import fwbf, synth
    dev = "cuda"
    line = {"n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "data": "synthetic", "unit": "Gb/s"}
    if a.workload == "n186_f32_wbf":
        code = fwbf.Code.from_seed(3, 6, 31, 1)
        F = 1000
        y = fwbf.channel(code.N, F, 0, None, 2024, 0, float(synth.sigma_for(3.0, code.rate)))
        p = fwbf.DecodeParams(dtype=fwbf.F32, weights=fwbf.WBF, groups=6, max_iter=50, alpha=0.2)
        z, it, ok = fwbf.decode(code, y, p)
        ms = _timed(lambda: fwbf.decode_into(code, y, p, z, it, ok), a.steps, a.warmup)
        r = fwbf.count(code.N, z, None, 0, it, ok, 50)
        line.update(metric="decoded Gb/s, plain FWBF + WBF, N=186 (3,6) QC, 3 dB, float32, G=6",
                    value=round(F * code.N / (ms * 1e-3) / 1e9, 4), ms_per_step=round(ms, 4),
                    dtype="f32", fer=r["frame_err"] / F, mean_iters=r["iter_sum"] / F,
                    config={"workload": "N=186 (3,6) QC Z=31, all-zero codeword, 3 dB, f32, WBF, "
                                        "alpha 0.2, G=6, K_max=50, 1000 frames", "frames": F})
    elif a.workload == "mixed_f32":
        from paper_1206_3362_amd import autotune
        specs = MIXED_JOBS
        jobs, bits = [], 0
        for i, (spec, F, G, _) in enumerate(specs):
            code = fwbf.Code.from_seed(*spec)
            pool = torch.from_numpy(code.encode(31 + i, 0, 256).view(np.int32)).to(dev)
            eb = synth.uniform_frames(code.N, F, 77 + i, 3.0, 6.0)
            sig = torch.from_numpy(synth.sigma_for(eb, code.rate).astype(np.float32)).to(dev)
            y = fwbf.channel(code.N, F, 0, pool, 500 + i, i, 0.0, sigma_per_frame=sig)
            jobs.append((code, y, pool, fwbf.DecodeParams(dtype=fwbf.F32, groups=G, max_iter=100)))
            bits += F * code.N
        tuned = autotune.tune_batch(jobs, [s[3] for s in specs], **MIXED_TUNE)
        batch = [(code, y, p) for (code, y, _, _), p in zip(jobs, tuned["params"])]
        T, bpc = tuned["threads_per_frame"], tuned["blocks_per_cu"]
        ws = torch.zeros(64, dtype=torch.int32, device=dev)
        ms = _timed(lambda: fwbf.decode_batched(batch, threads_per_frame=T, blocks_per_cu=bpc, workspace=ws),
                    a.steps, a.warmup)
        ref = [(code, y, p0) for code, y, _, p0 in jobs]
        ms_ref = _timed(lambda: fwbf.decode_batched(ref, workspace=ws), a.steps, a.warmup)
        sep = _timed(lambda: [fwbf.decode(c, y, p) for c, y, p in batch], a.steps, a.warmup)
        outs = fwbf.decode_batched(batch, threads_per_frame=T, blocks_per_cu=bpc, workspace=ws)
        fer = [fwbf.count(code.N, z, pool, 0, it, ok, 100)["frame_err"] / y.shape[0]
               for (code, y, pool, _), (z, it, ok) in zip(jobs, outs)]
        line.update(metric="decoded Gb/s, mixed-code persistent batch (float32)",
                    value=round(bits / (ms * 1e-3) / 1e9, 3), ms_per_step=round(ms, 4), dtype="f32",
                    separate_launches_gbps=round(bits / (sep * 1e-3) / 1e9, 3),
                    reference_G_gbps=round(bits / (ms_ref * 1e-3) / 1e9, 3),
                    tuned={"G": [p.groups for p in tuned["params"]], "threads_per_frame": T,
                           "blocks_per_cu": bpc, "fer": [round(x, 5) for x in fer],
                           "g_table": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()}
                                       for r in tuned["g_table"]],
                           "shape_table": tuned["shape_table"]},
                    config={"workload": "N=1008/4032 (3,6) + N=8000 (4,20) QC, 2^18/2^16/2^15 frames, "
                                        "Eb/N0 U[3,6] dB per frame, f32, K_max=100, G and launch shape "
                                        "autotuned (reference G=8/32/64), one launch",
                            "frames": sum(s[1] for s in specs)})
    elif a.workload == "n32400_i16":
        n32400_i16(a, line)
    elif a.workload == "minsum_eg255":
        minsum_eg255(a, line)
    elif a.workload == "strided_n1008":
        strided_n1008(a, line)
    elif a.workload == "eg255_delay":
        eg255_delay(a, line)
    elif a.workload in ("eg1023", "eg1023_tab1"):
        eg1023_tab1(a, line, sweep=a.workload == "eg1023_tab1")
    else:  # sweep_n1008_i8
        code = fwbf.Code.from_seed(3, 6, 168, 2)
        pool = torch.from_numpy(code.encode(1001, 0, 1024).view(np.int32)).to(dev)
        ebs = np.arange(2.0, 6.01, 0.5)
        F = 1 << 20
        sw = fwbf.Sweep(code, fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100),
                        synth.sigma_for(ebs, code.rate), F, pool=pool, seed=1100, scale=16.0)
        ms = _timed(sw.launch, a.steps, a.warmup)
        c = sw.counters()
        line.update(metric="Eb/N0 sweep (channel+decode+count per point), one HIP graph, Gb/s",
                    value=round(len(ebs) * F * code.N / (ms * 1e-3) / 1e9, 3), ms_per_step=round(ms, 4),
                    dtype="int32",
                    fer={f"{e:.1f}": float(c[k, 1] / c[k, 4]) for k, e in enumerate(ebs)},
                    ber={f"{e:.1f}": float(c[k, 0] / (c[k, 4] * code.N)) for k, e in enumerate(ebs)},
                    config={"workload": "N=1008 int8 G=8, 9 points 2..6 dB, 2^20 frames per point",
                            "frames": int(len(ebs) * F)})
    print(json.dumps(line), flush=True)


def n32400_compare(steps, warmup, ebn0s):
    """The (3,30) rate-0.9 code, N = 32400, int16 frames (scale 256), 2^18
    frames per Eb/N0 point: plain FWBF at the autotuned G (FER-constrained
    against the reference G = 64 on frames with Eb/N0 uniform in [5, 7] dB)
    beside the learned decoder (checkpoint retrained on this code, plain
    fallback at the same G), same frames, same timing protocol.  Returns
    (points, tuning result, learned parameters)."""
    import numpy as np
    import torch

    from paper_1206_3362_amd import autotune, fwbf, synth
    code = fwbf.Code.from_seed(3, 30, 1080, 5)
    N, F = code.N, 1 << 18
    tuned = autotune.tune(code, (5.0, 7.0), G_ref=64, Gs=(4, 8, 16, 32, 64), widths=(0,), dtype=fwbf.I16,
                          frames=1 << 14, repeats=2)
    G = int(tuned["G"])
    plain = fwbf.DecodeParams(dtype=fwbf.I16, groups=G, max_iter=100)
    ck = np.load(os.path.join(ROOT, "paper_1206_3362_amd", "scorer_n32400_g512_t16.npz"), allow_pickle=False)
    cfg = dict((k, v) for k, v in ck["config"])
    lp = fwbf.LearnedParams(int(cfg["rounds"]), int(cfg["groups"]), int(cfg["topk"]), 256.0)
    sc = torch.from_numpy(ck["params"]).cuda()
    pool = torch.from_numpy(code.encode(5, 0, 64).view(np.int32)).cuda()
    z = torch.empty((F, (N + 31) // 32), dtype=torch.int32, device="cuda")
    it = torch.empty(F, dtype=torch.int32, device="cuda")
    ok = torch.empty(F, dtype=torch.uint8, device="cuda")
    lok = torch.empty(F, dtype=torch.uint8, device="cuda")
    res = {}
    for eb in ebn0s:
        y = fwbf.channel(N, F, 0, pool, 900, int(eb), float(synth.sigma_for(eb, code.rate)),
                         dtype=torch.int16, scale=256.0)
        ms_p = _timed(lambda: fwbf.decode_into(code, y, plain, z, it, ok), steps, warmup)
        rp = fwbf.count(N, z, pool, 0, it, ok, 100)
        ms_l = _timed(lambda: fwbf.decode_learned_into(code, y, plain, lp, sc, z, it, ok, lok), steps, warmup)
        rl = fwbf.count(N, z, pool, 0, it, ok, 100 + lp.rounds)
        fp, fl = rp["frame_err"] / F, rl["frame_err"] / F
        pooled = (rp["frame_err"] + rl["frame_err"]) / (2 * F)
        res[f"{eb:.0f}dB"] = dict(
            plain=dict(gbps=round(F * N / (ms_p * 1e-3) / 1e9, 3), ms=round(ms_p, 4), fer=fp,
                       ber=rp["bit_err"] / (F * N), mean_rounds=round(rp["iter_sum"] / F, 3)),
            learned=dict(gbps=round(F * N / (ms_l * 1e-3) / 1e9, 3), ms=round(ms_l, 4), fer=fl,
                         ber=rl["bit_err"] / (F * N), learned_pass_only=float(lok.float().mean().item())),
            learned_fer_at_or_below_plain=bool(fl <= fp + 3.0 * np.sqrt(pooled * (1 - pooled) * 2.0 / F)),
            learned_over_plain_gbps=round(ms_p / ms_l, 3))
        del y
    return res, tuned, lp


def n32400_i16(a, line):
    """Plain vs learned FWBF on the N = 32400 int16 code at 5, 6 and 7 dB."""
    res, tuned, lp = n32400_compare(a.steps, a.warmup, (5.0, 6.0, 7.0))
    line.update(metric="decoded Gb/s, N=32400 (3,30) QC rate 0.9, int16: learned FWBF vs plain FWBF (tuned G)",
                value=res["6dB"]["learned"]["gbps"], ms_per_step=res["6dB"]["learned"]["ms"], dtype="int32",
                points=res,
                tuned={"G": int(tuned["G"]), "G_ref": 64, "fer_ref": tuned["fer_ref"],
                       "table": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()}
                                 for r in tuned["table"]]},
                scorer={"file": "scorer_n32400_g512_t16.npz", "rounds": lp.rounds, "groups": lp.groups,
                        "topk": lp.topk},
                config={"workload": "N=32400 (3,30) QC Z=1080 K=29162, int16 x256, K_max=100, 2^18 frames per "
                                    "point, 5/6/7 dB; plain FWBF at the autotuned G and learned FWBF (plain "
                                    "fallback) on the same frames", "frames": 1 << 18})


# averaged rounds printed in Tab. 1 (K_max = 10, EG(1023,781), 3.0/3.5/4.0/4.5 dB)
TAB1 = {"MLP-WBF": [8.86, 6.20, 4.54, 3.83], "FWBF p=93": [9.29, 7.37, 6.06, 5.12],
        "FWBF p=31": [8.62, 5.60, 4.19, 3.64]}


def eg1023_tab1(a, line, sweep=True):
    """Tab. 1 of the paper on the EG(1023,781) code: averaged rounds of FWBF
    with blocks of p=93 (G=11) and p=31 (G=33) bits, K_max=10, float32
    BPSK/AWGN, IMWBF metric with alpha swept (the paper does not state it),
    plus the top-lambda choice (lambda=10) in the MLP-WBF row's place."""
    import numpy as np
    import torch

    from paper_1206_3362_amd import fwbf, synth
    code = fwbf.Code.from_text(synth.eg_code_text(5))
    N, F = code.N, 1 << 16
    pool = torch.from_numpy(code.encode(1023, 0, 1024).view(np.int32)).to("cuda")
    ebs = (3.0, 3.5, 4.0, 4.5)
    alphas = (0.0, 0.1, 0.2, 0.3, 0.5, 0.8, 1.0, 1.5, 2.0) if sweep else (1.5,)
    rows = {}
    timed = None
    for eb in (ebs if sweep else (4.0,)):
        k = ebs.index(eb)
        y = fwbf.channel(N, F, 0, pool, 1300, k, float(synth.sigma_for(eb, code.rate)))
        cases = [(f"FWBF p={-(-N // G)}", dict(groups=G), al) for G in ((11, 33) if sweep else (33,))
                 for al in alphas]
        if sweep:
            cases += [("top-lambda 10", dict(select=fwbf.TOPL, lam=10), al) for al in alphas]
        for name, sel, al in cases:
            p = fwbf.DecodeParams(dtype=fwbf.F32, weights=fwbf.IMWBF, max_iter=10, alpha=al, **sel)
            z, it, ok = fwbf.decode(code, y, p)
            r = fwbf.count(N, z, pool, 0, it, ok, 10)
            h = r["hist"]
            # syndrome evaluations (Step 1 passes): rounds + 1 for a frame
            # that stops on a zero syndrome before K_max, K_max otherwise
            passes = float(sum(h[i] * (i + 1) for i in range(10)) + h[10] * 10) / F
            rows.setdefault(name, {}).setdefault(f"{al:g}", []).append(
                dict(iters=round(r["iter_sum"] / F, 3), passes=round(passes, 3),
                     fer=round(r["frame_err"] / F, 5), ber=float(r["bit_err"] / (F * N))))
            if name == "FWBF p=31" and al == 1.5 and eb == 4.0:
                timed = (y, p, z, it, ok)
    y, p, z, it, ok = timed
    ms = _timed(lambda: fwbf.decode_into(code, y, p, z, it, ok), a.steps, a.warmup)
    # the same point with int8 inputs (scale 16, alpha 3/2)
    yq = fwbf.channel(N, F, 0, pool, 1300, 2, float(synth.sigma_for(4.0, code.rate)), dtype=torch.int8,
                      scale=16.0)
    pq = fwbf.DecodeParams(dtype=fwbf.I8, weights=fwbf.IMWBF, groups=33, max_iter=10, alpha_num=3, alpha_den=2)
    zq, iq, oq = fwbf.decode(code, yq, pq)
    ms8 = _timed(lambda: fwbf.decode_into(code, yq, pq, zq, iq, oq), a.steps, a.warmup)
    r8 = fwbf.count(N, zq, pool, 0, iq, oq, 10)
    best = {}
    for name, by_alpha in (rows.items() if sweep else ()):
        ref = TAB1["MLP-WBF" if name.startswith("top") else name]
        for count in ("iters", "passes"):
            err = {al: float(np.sqrt(np.mean([(v[count] - r) ** 2 for v, r in zip(vals, ref)])))
                   for al, vals in by_alpha.items()}
            al = min(err, key=err.get)
            best[f"{name} ({count})"] = dict(alpha=float(al), avg=[v[count] for v in by_alpha[al]],
                                             paper=ref, rms_diff=round(err[al], 3))
    line.update(metric="decoded Gb/s, FWBF on EG(1023,781), p=31, alpha 1.5, 4 dB, float32, K_max=10",
                value=round(F * N / (ms * 1e-3) / 1e9, 3), ms_per_step=round(ms, 4), dtype="f32",
                int8_gbps=round(F * N / (ms8 * 1e-3) / 1e9, 3), int8_ms=round(ms8, 4),
                int8_fer=r8["frame_err"] / F, int8_mean_rounds=r8["iter_sum"] / F,
                tab1_best_alpha=best or None, tab1_sweep=rows, ebn0=list(ebs) if sweep else [4.0],
                config={"workload": "EG(1023,781) type-I 2-D Euclidean geometry code, random "
                                    "codewords, BPSK/AWGN 3.0-4.5 dB, f32, IMWBF, K_max=10, "
                                    "2^16 frames per point", "frames": F})


def _ebn0_at(ebs, bers, target):
    """Eb/N0 where log10(BER) crosses the target (linear interpolation)."""
    import numpy as np
    lb = np.log10(np.maximum(np.asarray(bers, float), 1e-12))
    for i in range(len(ebs) - 1):
        if lb[i] >= np.log10(target) > lb[i + 1]:
            t = (lb[i] - np.log10(target)) / (lb[i] - lb[i + 1])
            return round(float(ebs[i] + t * (ebs[i + 1] - ebs[i])), 3)
    return None


def minsum_eg255(a, line):
    """BER of min-sum BP against FWBF on EG(255,175) (code 1 of Section V,
    where the paper puts BP 0.5 dB ahead of FWBF at BER 1e-4), float32,
    2^18 random codewords per point; the Eb/N0 at BER 1e-4 of each decoder,
    and both decoders' throughput at 4 dB."""
    import numpy as np
    import torch

    from paper_1206_3362_amd import fwbf, synth
    code = fwbf.Code.from_text(synth.eg_code_text(4))
    N, F = code.N, 1 << 18
    pool = torch.from_numpy(code.encode(255, 0, 4096).view(np.int32)).to("cuda")
    ebs = [3.0 + 0.25 * i for i in range(11)]
    decs = {f"min-sum c={c}": ("ms", dict(c=c, max_iter=50)) for c in (0.625, 0.75, 1.0)}
    decs.update({f"FWBF p={-(-N // G)} alpha={al}": ("fwbf", dict(groups=G, alpha=al))
                 for G in (5, 16) for al in (1.0, 2.0)})
    ber = {k: [] for k in decs}
    fer = {k: [] for k in decs}
    rounds = {k: [] for k in decs}
    timing = {}
    for k_eb, eb in enumerate(ebs):
        y = fwbf.channel(N, F, 0, pool, 2550, k_eb, float(synth.sigma_for(eb, code.rate)))
        for name, (kind, kw) in decs.items():
            if kind == "ms":
                run = lambda: fwbf.decode_minsum(code, y, **kw)
                K = kw["max_iter"]
            else:
                p = fwbf.DecodeParams(dtype=fwbf.F32, weights=fwbf.IMWBF, max_iter=10, **kw)
                run = lambda: fwbf.decode(code, y, p)
                K = 10
            z, it, ok = run()
            r = fwbf.count(N, z, pool, 0, it, ok, K)
            ber[name].append(r["bit_err"] / (F * N))
            fer[name].append(r["frame_err"] / F)
            rounds[name].append(round(r["iter_sum"] / F, 3))
            if eb == 4.0:
                ms = _timed(run, a.steps, a.warmup)
                timing[name] = round(F * N / (ms * 1e-3) / 1e9, 3)
    at = {k: _ebn0_at(ebs, v, 1e-4) for k, v in ber.items()}
    best_ms = min((v, k) for k, v in at.items() if k.startswith("min") and v is not None)
    best_fw = min((v, k) for k, v in at.items() if k.startswith("FWBF") and v is not None)
    line.update(metric="decoded Gb/s, min-sum BP (c=0.75, 50 iterations) on EG(255,175), 4 dB, float32",
                value=timing["min-sum c=0.75"], ms_per_step=None, dtype="f32", gbps_at_4db=timing,
                ebn0_at_ber_1e4=at, gap_db=round(best_fw[0] - best_ms[0], 3),
                best={"min-sum": best_ms[1], "FWBF": best_fw[1]}, paper_gap_db=0.5,
                ebn0=ebs, ber=ber, fer=fer, mean_iterations=rounds,
                config={"workload": "EG(255,175), random codewords, BPSK/AWGN 3.0-5.5 dB step 0.25, f32, "
                                    "FWBF IMWBF K_max=10, min-sum flooding 50 iterations, 2^18 frames per point",
                        "frames": F})


def strided_n1008(a, line):
    """Contiguous blocks (Section III) against strided blocks
    (g = n mod G, what an interleaver of depth G makes contiguous) on the
    N=1008 code, int8, at equal K_max: FER, mean rounds and decoded Gb/s per
    Eb/N0, for G = 8 and 32."""
    import numpy as np
    import torch

    from paper_1206_3362_amd import fwbf, synth
    code = fwbf.Code.from_seed(3, 6, 168, 2)
    N, F = code.N, 1 << 18
    pool = torch.from_numpy(code.encode(1001, 0, 1024).view(np.int32)).to("cuda")
    res = {}
    for eb in (3.0, 4.0, 5.0, 6.0):
        y = fwbf.channel(N, F, 0, pool, 1500, int(eb), float(synth.sigma_for(eb, code.rate)),
                         dtype=torch.int8, scale=16.0)
        for G in (8, 32):
            for sel, name in ((fwbf.GROUPS, "contiguous"), (fwbf.STRIDED, "strided")):
                p = fwbf.DecodeParams(dtype=fwbf.I8, select=sel, groups=G, max_iter=100)
                z, it, ok = fwbf.decode(code, y, p)
                ms = _timed(lambda: fwbf.decode_into(code, y, p, z, it, ok), a.steps, a.warmup)
                r = fwbf.count(N, z, pool, 0, it, ok, 100)
                fe = r["frame_err"]
                res.setdefault(f"{eb:.0f}dB", {})[f"G{G} {name}"] = dict(
                    fer=round(fe / F, 5), fer_3sigma=round(3 * np.sqrt(max(fe, 1) * (1 - fe / F)) / F, 5),
                    mean_rounds=round(r["iter_sum"] / F, 3), gbps=round(F * N / (ms * 1e-3) / 1e9, 2))
    v = res["4dB"]["G8 strided"]
    line.update(metric="decoded Gb/s, plain FWBF, strided blocks, N=1008 int8, 4 dB, G=8",
                value=v["gbps"], ms_per_step=None, dtype="int32", points=res,
                config={"workload": "N=1008 (3,6) QC int8 x16, K_max=100, 2^18 frames per point, "
                                    "contiguous vs strided blocks", "frames": F})


def eg255_delay(a, line):
    """Per-round cost of FWBF on EG(255,175) next to the clock model of
    Section IV (FWBF: 20 clocks per bit choice with 16 units; MLP-WBF: 24
    lambda).  At -6 dB, with the repeated-state exit switched off, frames run
    K rounds unless they land on some codeword; the time difference between
    K = 41 and K = 1, divided by the difference of the rounds actually run,
    is the cost of one round.  One frame alone gives the latency of a round
    (one wave, cycles at 2.4 GHz); 2^16 frames give its throughput."""
    import numpy as np
    import torch

    from paper_1206_3362_amd import delay, fwbf, synth
    code = fwbf.Code.from_text(synth.eg_code_text(4))
    N = code.N
    out = {}
    for F in (1, 1 << 16):
        y = fwbf.channel(N, F, 0, None, 77, 0, float(synth.sigma_for(-6.0, code.rate)))
        ms, rnd = {}, {}
        for K in (1, 41):
            p = fwbf.DecodeParams(dtype=fwbf.F32, weights=fwbf.IMWBF, groups=16, max_iter=K, alpha=1.0,
                                  flags=fwbf.FLAG_NO_CYCLE_EXIT)
            z, it, ok = fwbf.decode(code, y, p)
            reps = [_timed(lambda: fwbf.decode_into(code, y, p, z, it, ok), max(a.steps, 5), a.warmup)
                    for _ in range(3)]
            ms[K] = float(np.median(reps))
            rnd[K] = float(it.double().mean())
        per_round_ns = (ms[41] - ms[1]) * 1e6 / (rnd[41] - rnd[1])
        out[F] = dict(ms_k1=round(ms[1], 5), ms_k41=round(ms[41], 5), mean_rounds_k41=round(rnd[41], 3),
                      per_round_ns=round(per_round_ns, 2))
    lat_ns = out[1]["per_round_ns"]
    thr_ns = out[1 << 16]["per_round_ns"] / (1 << 16)
    line.update(metric="bit-choice round cost, FWBF on EG(255,175), float32, G=16 (p=16)",
                value=round(1e3 / thr_ns, 3), unit="M frame-rounds/s", higher_is_better=True,
                ms_per_step=out[1 << 16]["ms_k41"], dtype="f32",
                one_frame_round_ns=lat_ns, one_frame_round_cycles=round(lat_ns * 2.4, 1),
                chip_ns_per_frame_round=round(thr_ns, 5),
                model_clocks={"fwbf_eq3": delay.fwbf_delay(255, 16),
                              "mlp_wbf_eq2_lambda10": delay.mlp_wbf_delay(255, 16, 10),
                              "metric_units_16": delay.metric_clocks(255, 16)},
                raw=out,
                config={"workload": "EG(255,175), -2 dB (no frame decodes), repeated-state exit off, "
                                    "K = 1 and 41 rounds, 1 frame and 2^16 frames", "frames": 1 << 16})


def kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for name in ("decode_fast.hip", "frames.h"):
        with open(os.path.join(ROOT, "paper_1206_3362_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(code, y_dev, params, a, N):
    """The CPU oracle (unchanged) on a bounded sample of the same frames:
    once on the host's CPU share (every CPU this process may run on, at most
    16, the share of one GPU on the GPU hosts), once on one thread."""
    import numpy as np

    import oracle as O
    oc = O.Code.from_seed(3, 6, 168, 2)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(avail, 16))
    y = y_dev[:1 << 18].cpu().numpy()
    kw = dict(weights=O.IMWBF, select=O.GROUPS, G=params.groups, max_iter=params.max_iter,
              alpha_num=1, alpha_den=5)

    def rate(nthreads, seconds):
        n0 = 64 * nthreads
        t = time.perf_counter()
        O.decode(oc, y[:n0], threads=nthreads, **kw)
        dt = time.perf_counter() - t
        n = int(min(len(y), max(n0, n0 * seconds / max(dt, 1e-6))))
        t = time.perf_counter()
        O.decode(oc, y[:n], threads=nthreads, **kw)
        dt = time.perf_counter() - t
        return n, dt

    n, dt = rate(threads, a.cpu_seconds)
    n1, dt1 = rate(1, a.cpu_seconds / 2)
    return {"value": round(n * N / dt / 1e9, 6), "unit": "Gb/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {n} frames of the timed batch, literal oracle, {threads} threads, "
                      f"{dt:.1f} s; single thread: first {n1} frames, {dt1:.1f} s",
            "single_thread_gbps": round(n1 * N / dt1 / 1e9, 6),
            "cpus_available": avail, "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


if __name__ == "__main__":
    main()
