"""Autotuner for the block count G and the launch shape.

G changes the decoder's output (more blocks flip more bits per round), so it
is tuned under a frame-error constraint: a candidate is admissible only if
its frame error rate on the tuning frames is within three standard errors of
the reference G's (two-proportion test,
|p1 - p2| <= 3 sqrt(p (1 - p) (1/n1 + 1/n2)) with p the pooled rate) or
below it.  Among admissible candidates the one with the highest decoded
throughput (timed with HIP events on the same frames) wins.  Launch shapes
(threads per frame; for the mixed-code batch also the cap on workgroups per
compute unit, which sets how many frames a compute unit holds) do not change
outputs and are tuned for throughput only.  Single-code results can be cached
in a JSON file keyed by the code, dtype, noise levels and candidate lists.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import fwbf, synth


def _key(code, dtype, ebn0, Gs, widths, frames):
    h = hashlib.sha256(code.text().encode()).hexdigest()[:16]
    return json.dumps(dict(code=h, dtype=dtype, ebn0=list(map(float, np.atleast_1d(ebn0))),
                           Gs=list(Gs), widths=[int(w) for w in widths], frames=frames),
                      sort_keys=True)


def fer_admissible(err, n, err_ref, n_ref):
    p1, p2 = err / n, err_ref / n_ref
    if p1 <= p2:
        return True
    p = (err + err_ref) / (n + n_ref)
    return abs(p1 - p2) <= 3.0 * np.sqrt(max(p * (1 - p), 1e-300) * (1.0 / n + 1.0 / n_ref))


def _time_ms(fn, repeats):
    import torch
    ms = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms))


def tune(code, ebn0, G_ref=8, Gs=(8, 12, 16, 24, 32), widths=(0, 64, 128), dtype=fwbf.I8,
         frames=1 << 16, max_iter=100, seed=5, cache=None, repeats=3):
    """One code: G under the FER constraint and threads per frame (0 = the
    library's choice).  Returns dict(G, threads_per_frame, gbps, fer,
    admissible, fer_ref, G_ref, table)."""
    import torch
    key = _key(code, dtype, ebn0, Gs, widths, frames)
    if cache and os.path.exists(cache):
        db = json.load(open(cache))
        if key in db:
            return db[key]
    tdt = {fwbf.F32: torch.float32, fwbf.I8: torch.int8, fwbf.I16: torch.int16}[dtype]
    scale = {fwbf.F32: 1.0, fwbf.I8: 16.0, fwbf.I16: 256.0}[dtype]
    pool = torch.from_numpy(code.encode(seed, 0, 256).view(np.int32)).cuda()
    eb = np.atleast_1d(np.asarray(ebn0, np.float64))
    if eb.size == 2:  # per-frame Eb/N0 uniform in [lo, hi]
        sig = synth.sigma_for(synth.uniform_frames(code.N, frames, seed, eb[0], eb[1]), code.rate)
        sigd = torch.from_numpy(sig.astype(np.float32)).cuda()
        y = fwbf.channel(code.N, frames, 0, pool, seed, 0, 0.0, dtype=tdt, scale=scale,
                         sigma_per_frame=sigd)
    else:
        y = fwbf.channel(code.N, frames, 0, pool, seed, 0, float(synth.sigma_for(eb[0], code.rate)),
                         dtype=tdt, scale=scale)
    table = []

    def run(G, T):
        p = fwbf.DecodeParams(dtype=dtype, groups=G, max_iter=max_iter, threads_per_frame=T)
        z, it, ok = fwbf.decode(code, y, p)
        ms = _time_ms(lambda: fwbf.decode_into(code, y, p, z, it, ok), repeats)
        r = fwbf.count(code.N, z, pool, 0, it, ok, max_iter)
        return ms, r["frame_err"]

    ref_ms, ref_err = run(G_ref, 0)
    best = None
    for G in Gs:
        for T in widths:
            try:
                ms, err = run(G, T)
            except fwbf.FwbfError:
                continue
            gbps = frames * code.N / (ms * 1e-3) / 1e9
            ok = fer_admissible(err, frames, ref_err, frames)
            table.append(dict(G=G, threads_per_frame=T, gbps=gbps, fer=err / frames, admissible=bool(ok)))
            if ok and (best is None or gbps > best["gbps"]):
                best = table[-1]
    out = dict(best, fer_ref=ref_err / frames, G_ref=G_ref, table=table)
    if cache:
        db = json.load(open(cache)) if os.path.exists(cache) else {}
        db[key] = out
        with open(cache, "w") as f:
            json.dump(db, f, indent=1)
    return out


def tune_batch(jobs, Gs, tune_frames=1 << 14, widths=(0, 128, 256), blocks=(0, 2, 4), repeats=3):
    """Mixed-code batch.  jobs: list of (code, y, pool, params) with y on the
    device, frame f of job j sent from codeword pool[f mod len(pool)] and
    params.groups the job's reference G; Gs: candidate G values per job.

    Each job's G is chosen on its first `tune_frames` frames (the fastest
    admissible candidate, timed alone); then every (threads_per_frame,
    blocks_per_cu) pair is timed on the whole batch with those G and the
    fastest wins.  Returns dict(params=[DecodeParams per job],
    threads_per_frame, blocks_per_cu, ms, g_table, shape_table)."""
    import dataclasses

    chosen, g_table = [], []
    for (code, y, pool, params), cand in zip(jobs, Gs):
        n = min(tune_frames, y.shape[0])
        ys = y[:n]

        def run(G):
            p = dataclasses.replace(params, groups=G)
            z, it, ok = fwbf.decode(code, ys, p)
            ms = _time_ms(lambda: fwbf.decode_into(code, ys, p, z, it, ok), repeats)
            return ms, fwbf.count(code.N, z, pool, 0, it, ok, p.max_iter)["frame_err"]

        _, ref_err = run(params.groups)
        best = None
        for G in cand:
            try:
                ms, err = run(G)
            except fwbf.FwbfError:
                continue
            ok = fer_admissible(err, n, ref_err, n)
            row = dict(N=code.N, G=G, ms=ms, fer=err / n, fer_ref=ref_err / n, admissible=bool(ok))
            g_table.append(row)
            if ok and (best is None or ms < best["ms"]):
                best = row
        chosen.append(dataclasses.replace(params, groups=best["G"] if best else params.groups))

    batch = [(code, y, p) for (code, y, _, _), p in zip(jobs, chosen)]
    import torch
    ws = torch.zeros(64, dtype=torch.int32, device=jobs[0][1].device)
    shape_table, best = [], None
    for T in widths:
        for b in blocks:
            try:
                fwbf.decode_batched(batch, threads_per_frame=T, blocks_per_cu=b, workspace=ws)
            except fwbf.FwbfError:
                continue
            ms = _time_ms(lambda: fwbf.decode_batched(batch, threads_per_frame=T, blocks_per_cu=b,
                                                      workspace=ws), repeats)
            shape_table.append(dict(threads_per_frame=T, blocks_per_cu=b, ms=ms))
            if best is None or ms < best["ms"]:
                best = shape_table[-1]
    if best is None:
        raise fwbf.FwbfError(fwbf.E_UNSUPPORTED, "no candidate launch shape could decode this batch")
    return dict(params=chosen, threads_per_frame=best["threads_per_frame"],
                blocks_per_cu=best["blocks_per_cu"], ms=best["ms"], g_table=g_table,
                shape_table=shape_table)
