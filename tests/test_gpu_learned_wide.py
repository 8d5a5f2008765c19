"""The learned pass with one frame per workgroup: codes beyond one
wavefront's reach (the (3,30) rate-0.9 codes, int16 inputs, up to 512
proposals per round), checked against the float64 reference of the learned
pass plus the plain oracle fallback, against the one-frame-per-wavefront
kernel on the same frames, and through the scorers whose outcome is known
exactly (identity scorer = plain FWBF, zero scorer = fallback everywhere)."""
import os

import numpy as np
import pytest

import oracle as O
import oracle.mlp_ref as R
from gpu_util import need_gpu, torch
from paper_1206_3362_amd import fwbf, synth

pytestmark = pytest.mark.gpu

NP_DT = {fwbf.I8: np.int8, fwbf.I16: np.int16}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def random_params(T, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.5, R.n_params(T))
    p[-2 * T:-T] = rng.uniform(0.1, 0.4, T)   # alpha_t
    p[-T:] = rng.uniform(0.7, 1.3, T)         # beta_t
    return p.astype(np.float32)


def _frames(o, Fn, eb, seed, dt):
    cw = O.unpack(o.encode(seed, 0, Fn), o.N)
    return synth.awgn_frames(o.N, Fn, synth.sigma_for(eb, o.K / o.N), seed + 1, cw, NP_DT[dt])


def _reference(o, y, p, T, G, k, A, plain_G):
    """Float64 learned pass, then the plain oracle for the frames it leaves."""
    zr, rr, okr, tr = R.learned_decode_batch(o, y, p.astype(np.float64), T, G, k, A, 3)
    zf, itf, okf = zr.copy(), rr.copy(), okr.copy()
    fb = np.nonzero(~okr)[0]
    if fb.size:
        zp, itp, okp = O.decode(o, y[fb], G=plain_G, max_iter=100, alpha_num=1, alpha_den=5)
        zf[fb], itf[fb], okf[fb] = O.unpack(zp, o.N), rr[fb] + itp, okp.astype(bool)
    return zf, itf, okf, okr, tr


def _round0_matches(rg, tr, f):
    """Round-0 proposals (exact single-precision metrics, no scores
    involved): bit indices, S and labels against the reference trace."""
    cand = R.trace_of_frame(tr, f)
    if not cand:
        return int(rg[f, 0]["valid"].sum()) == 0
    c0 = cand[0][0].ravel()
    c0 = c0[c0 >= 0]
    v = rg[f, 0][rg[f, 0]["valid"] == 1]
    return np.array_equal(v["n"].astype(np.int64), c0)


# forward scores: |GPU - float64| <= SCORE_BOUND (1 + |score|) (the bound of
# the forward-score test of the one-wavefront kernel)
SCORE_BOUND = 2e-2


def _near_tie(scores):
    """Some block's decision can go either way within the forward bound: its
    best score is that close to 0, or its two best scores to each other."""
    for row in np.atleast_2d(scores):
        v = np.sort(row[~np.isnan(row)])[::-1]
        if v.size == 0:
            continue
        if abs(v[0]) <= SCORE_BOUND * (1 + abs(v[0])):
            return True
        if v.size > 1 and v[0] - v[1] <= 2 * SCORE_BOUND * (1 + abs(v[0])):
            return True
    return False


def _check_against_reference(name, g, o, y, p, dt, A, T, G, k, pG):
    """Decode y with the wide learned pass and compare frame by frame with
    the float64 reference (see the test below for the bar)."""
    Fn = y.shape[0]
    lp = fwbf.LearnedParams(T, G, k, A)
    plain = fwbf.DecodeParams(dtype=dt, groups=pG, max_iter=100, flags=fwbf.FLAG_GENERIC_KERNEL)
    rec = fwbf.record_buffer(Fn, T, G, k)
    print(f"wide learned pass {name}: N={g.N} frames={Fn}", flush=True)
    z, it, ok, lok = fwbf.decode_learned(g, torch.from_numpy(y).cuda(), plain, lp, torch.from_numpy(p).cuda(),
                                         records=rec)
    torch.cuda.synchronize()
    zg = O.unpack(z.cpu().numpy().view(np.uint32), o.N)
    itg, okg, lokg = it.cpu().numpy(), ok.cpu().numpy().astype(bool), lok.cpu().numpy().astype(bool)
    zf, itf, okf, okr, tr = _reference(o, y, p, T, G, k, A, pG)
    rg = fwbf.records_host(rec)
    for f in range(Fn):
        assert _round0_matches(rg, tr, f), (name, f)
    same = (zg == zf).all(1) & (itg == itf) & (okg == okf) & (lokg == okr)
    near = 0
    for f in range(Fn):
        # every round's proposals, up to the first round that a near-tie may
        # have decided differently
        rounds = R.trace_of_frame(tr, f)
        decide = len(rounds) - 1
        parted = False
        for t_, (cand, _) in enumerate(rounds):
            n_gpu = rg[f, t_]["n"][rg[f, t_]["valid"] == 1].astype(np.int64)
            if not np.array_equal(n_gpu, cand.ravel()[cand.ravel() >= 0]):
                decide, parted = t_ - 1, True
                break
        if parted or not same[f]:
            assert decide >= 0 and _near_tie(rounds[decide][1]), (name, f, decide)
            near += 1
    print(f"{name}: {int(same.sum())}/{Fn} frames identical, {near} near-tie differences, "
          f"learned-pass successes {int(lokg.sum())} (reference {int(okr.sum())})", flush=True)
    assert same.mean() >= 0.9


CASES = [
    # name, (mb, nb, Z, seed, min_girth), dtype, A, T, G, k, frames, Eb/N0, plain G
    ("n930_i16_g64", (3, 30, 31, 21, 4), fwbf.I16, 256.0, 6, 64, 1, 48, 6.0, 16),
    ("n930_i16_g16k4", (3, 30, 31, 22, 4), fwbf.I16, 256.0, 5, 16, 4, 48, 6.0, 8),
    ("n1008_i8_g64k2", (3, 6, 168, 2, 6), fwbf.I8, 16.0, 8, 64, 2, 48, 4.5, 8),
    ("n32400_i16_g512", (3, 30, 1080, 5, 6), fwbf.I16, 256.0, 6, 512, 1, 6, 6.0, 64),
]


@pytest.mark.parametrize("name,spec,dt,A,T,G,k,Fn,eb,pG", CASES, ids=[c[0] for c in CASES])
def test_wide_learned_pass_matches_reference(name, spec, dt, A, T, G, k, Fn, eb, pG):
    """Random scorers (alpha_t = 0.2, beta_t = 1: the plain metric, so that
    the learned pass decodes frames on its own) on noisy frames: z, rounds
    and flags frame by frame, and every round-0 proposal exactly.  MFMA
    sums may order near-ties differently from float64, so a frame may
    differ only where some block's best score is within the forward bound
    of 0 in the round where the two first part."""
    g = fwbf.Code.from_seed(*spec)
    o = O.Code.from_seed(*spec)
    p = random_params(T, 41)
    p[-2 * T:-T] = 0.2
    p[-T:] = 1.0
    y = _frames(o, Fn, eb, 5, dt)
    _check_against_reference(name, g, o, y, p, dt, A, T, G, k, pG)



@pytest.mark.parametrize("spec,k,G,pG", [((3, 30, 31, 21, 4), 1, 64, 16), ((3, 30, 31, 22, 4), 4, 16, 8)],
                         ids=["k1", "k4"])
def test_wide_saturated_magnitudes_match_reference(spec, k, G, pG):
    """int16 frames scaled up 12-fold (clipped to the documented +-32767):
    the slot words hold min(|y|, 4095), so frames with a magnitude at or
    above 4095 take the general scan, which reads those magnitudes from the
    frame itself; the rest of the batch (unscaled frames) keeps the
    one-proposal fast scan.  Same bar as the unscaled cases."""
    g = fwbf.Code.from_seed(*spec)
    o = O.Code.from_seed(*spec)
    T = 6
    p = random_params(T, 43)
    p[-2 * T:-T] = 0.2
    p[-T:] = 1.0
    y = _frames(o, 48, 6.0, 9, fwbf.I16).astype(np.int32)
    y[::2] = np.clip(y[::2] * 12, -32767, 32767)
    y = y.astype(np.int16)
    big = (np.abs(y[::2].astype(np.int32)) >= 4095).mean()
    assert big > 0.05 and (np.abs(y[1::2].astype(np.int32)) < 4095).all()
    print(f"saturated share of the scaled frames: {big:.3f}", flush=True)
    _check_against_reference(f"saturated_{k}", g, o, y, p, fwbf.I16, 256.0, T, G, k, pG)

def test_wide_kernel_equals_wave_kernel_on_checkpoint():
    """The committed N = 1008 scorer (T = 16, 32 blocks, k = 1) on 4096 int8
    frames at 4 dB: the one-frame-per-workgroup kernel (general fallback)
    and the one-frame-per-wavefront kernel (specialised fallback) compute
    the same scores in the same order, so every output and every record is
    identical."""
    g = fwbf.Code.from_seed(3, 6, 168, 2)
    ck = np.load(os.path.join(os.path.dirname(fwbf.__file__), "scorer_n1008_g32_t16.npz"), allow_pickle=False)
    pd = torch.from_numpy(ck["params"].astype(np.float32)).cuda()
    T, G, k, Fn = 16, 32, 1, 4096
    pool = torch.from_numpy(g.encode(19, 0, 256).view(np.int32)).cuda()
    y = fwbf.channel(g.N, Fn, 0, pool, 555, 1, float(synth.sigma_for(4.0, g.rate)), dtype=torch.int8, scale=16.0)
    lp = fwbf.LearnedParams(T, G, k, 16.0)
    outs = []
    for flags in (0, fwbf.FLAG_GENERIC_KERNEL):
        rec = fwbf.record_buffer(Fn, T, G, k)
        plain = fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100, flags=flags)
        z, it, ok, lok = fwbf.decode_learned(g, y, plain, lp, pd, records=rec, pool=pool)
        torch.cuda.synchronize()
        r = fwbf.records_host(rec)
        outs.append((z.cpu().numpy(), it.cpu().numpy(), ok.cpu().numpy(), lok.cpu().numpy(), r))
    (za, ia, oa, la, ra), (zb, ib, ob, lb, rb) = outs
    print(f"checkpoint: learned-pass successes {int(la.sum())}/{Fn}", flush=True)
    assert la.sum() > Fn // 4
    assert np.array_equal(za, zb) and np.array_equal(ia, ib) and np.array_equal(oa, ob) and np.array_equal(la, lb)
    va, vb = ra["valid"] == 1, rb["valid"] == 1
    assert np.array_equal(va, vb)
    for fld in ("S", "a", "n", "u", "label"):
        assert np.array_equal(ra[fld][va], rb[fld][vb]), fld


def _identity_params(T, alpha):
    W1 = np.zeros((32, 4)); W1[0, 1] = 1.0; W1[1, 1] = -1.0
    W2 = np.zeros((32, 32)); W2[0, 0] = 1.0; W2[1, 1] = 1.0
    W3 = np.zeros(32); W3[0] = 1.0; W3[1] = -1.0
    return np.concatenate([W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), W3, [0.0],
                           np.full(T, alpha), np.full(T, 1.0)]).astype(np.float32)


@pytest.mark.parametrize("spec,G", [((3, 30, 31, 23, 4), 30), ((3, 30, 31, 24, 4), 93)])
def test_wide_identity_scorer_equals_plain_int16(spec, G):
    """Score = ReLU(E/A) - ReLU(-E/A) = E/A, exact in bfloat16 on frames of
    two magnitudes (256 and 128 at scale 256): the learned pass flips in
    each block the bit of largest positive E, i.e. plain FWBF with G blocks
    and alpha = 1/4, so its decisions equal the plain oracle's wherever the
    learned pass decodes (rounds <= T) and the fallback takes the rest."""
    g = fwbf.Code.from_seed(*spec)
    o = O.Code.from_seed(*spec)
    T = 40
    p = _identity_params(T, 0.25)
    rng = np.random.default_rng(8)
    Fn = 512
    y = (np.where(rng.random((Fn, g.N)) < 0.5, 256, 128) *
         np.where(rng.random((Fn, g.N)) < 0.004, -1, 1)).astype(np.int16)
    plain = fwbf.DecodeParams(dtype=fwbf.I16, groups=G, max_iter=100, alpha_num=1, alpha_den=4)
    z, it, ok, lok = fwbf.decode_learned(g, torch.from_numpy(y).cuda(), plain, fwbf.LearnedParams(T, G, 1, 256.0),
                                         torch.from_numpy(p).cuda())
    zp, itp, okp = O.decode(o, y, G=G, max_iter=100, alpha_num=1, alpha_den=4)
    print(f"identity scorer N={g.N} G={G}: plain decodes {int(okp.sum())}/{Fn}", flush=True)
    assert np.array_equal(z.cpu().numpy().view(np.uint32), zp)
    assert np.array_equal(ok.cpu().numpy(), okp)
    assert lok.cpu().numpy().sum() == okp.sum()


def test_wide_zero_scorer_falls_back_everywhere_n32400():
    """A scorer that never scores above 0 flips nothing: every frame of the
    N = 32400 int16 code goes to the plain fallback from its original y, and
    the outputs equal plain FWBF's (general kernel) bit for bit."""
    g = fwbf.Code.from_seed(3, 30, 1080, 5)
    T = 4
    p = np.zeros(R.n_params(T), np.float32)
    p[1248] = -0.5
    p[-T:] = 1.0
    Fn = 96
    pool = torch.from_numpy(g.encode(3, 0, 16).view(np.int32)).cuda()
    y = fwbf.channel(g.N, Fn, 0, pool, 77, 2, float(synth.sigma_for(6.5, g.rate)), dtype=torch.int16, scale=256.0)
    plain = fwbf.DecodeParams(dtype=fwbf.I16, groups=64, max_iter=100)
    z, it, ok, lok = fwbf.decode_learned(g, y, plain, fwbf.LearnedParams(T, 512, 1, 256.0), torch.from_numpy(p).cuda())
    zp, itp, okp = fwbf.decode(g, y, plain)
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy(), zp.cpu().numpy())
    assert np.array_equal(it.cpu().numpy(), itp.cpu().numpy()) and np.array_equal(ok.cpu().numpy(), okp.cpu().numpy())
    # only frames with a zero syndrome from the start count as learned successes
    assert int(lok.sum()) == int(((itp == 0) & (okp == 1)).sum())


def test_checkpoint_n32400_frame_by_frame():
    """The committed N = 32400 scorer (T = 16, 512 blocks, k = 1, int16 at
    scale 256) on 24 frames at 6 dB, where its learned pass decides almost
    every frame: z, rounds and flags frame by frame against the float64
    learned pass plus the plain oracle fallback (G = 16); differences only
    at near-ties, as for the random scorers."""
    g = fwbf.Code.from_seed(3, 30, 1080, 5)
    o = O.Code.from_seed(3, 30, 1080, 5)
    ck = np.load(os.path.join(os.path.dirname(fwbf.__file__), "scorer_n32400_g512_t16.npz"), allow_pickle=False)
    p = ck["params"].astype(np.float32)
    T, G, k, Fn, pG = 16, 512, 1, 24, 16
    y = _frames(o, Fn, 6.0, 13, fwbf.I16)
    lp = fwbf.LearnedParams(T, G, k, 256.0)
    plain = fwbf.DecodeParams(dtype=fwbf.I16, groups=pG, max_iter=100)
    rec = fwbf.record_buffer(Fn, T, G, k)
    print(f"N=32400 checkpoint: {Fn} frames", flush=True)
    z, it, ok, lok = fwbf.decode_learned(g, torch.from_numpy(y).cuda(), plain, lp, torch.from_numpy(p).cuda(),
                                         records=rec)
    torch.cuda.synchronize()
    zg = O.unpack(z.cpu().numpy().view(np.uint32), o.N)
    itg, okg, lokg = it.cpu().numpy(), ok.cpu().numpy().astype(bool), lok.cpu().numpy().astype(bool)
    zf, itf, okf, okr, tr = _reference(o, y, p, T, G, k, 256.0, pG)
    rg = fwbf.records_host(rec)
    for f in range(Fn):
        assert _round0_matches(rg, tr, f), f
    same = (zg == zf).all(1) & (itg == itf) & (okg == okf) & (lokg == okr)
    for f in np.nonzero(~same)[0]:
        rounds = R.trace_of_frame(tr, f)
        decide = len(rounds) - 1
        for t_, (cand, _) in enumerate(rounds):
            n_gpu = rg[f, t_]["n"][rg[f, t_]["valid"] == 1].astype(np.int64)
            if not np.array_equal(n_gpu, cand.ravel()[cand.ravel() >= 0]):
                decide = t_ - 1
                break
        assert decide >= 0 and _near_tie(rounds[decide][1]), (f, decide)
    print(f"N=32400 checkpoint: {int(same.sum())}/{Fn} identical, learned pass decoded {int(lokg.sum())} "
          f"(reference {int(okr.sum())})", flush=True)
    assert okr.sum() >= Fn // 2
    assert same.mean() >= 0.9


def test_checkpoint_n32400_beats_plain_at_6db():
    """Ablation on 4096 fresh frames at 6 dB: the retrained learned decoder
    (with fallback) has a lower frame error rate than plain FWBF at G = 16
    (the autotuned G) by far more than three standard errors."""
    g = fwbf.Code.from_seed(3, 30, 1080, 5)
    ck = np.load(os.path.join(os.path.dirname(fwbf.__file__), "scorer_n32400_g512_t16.npz"), allow_pickle=False)
    sc = torch.from_numpy(ck["params"].astype(np.float32)).cuda()
    F = 4096
    pool = torch.from_numpy(g.encode(71, 0, 64).view(np.int32)).cuda()
    y = fwbf.channel(g.N, F, 0, pool, 8080, 6, float(synth.sigma_for(6.0, g.rate)), dtype=torch.int16, scale=256.0)
    plain = fwbf.DecodeParams(dtype=fwbf.I16, groups=16, max_iter=100)
    zl, itl, okl, lokl = fwbf.decode_learned(g, y, plain, fwbf.LearnedParams(16, 512, 1, 256.0), sc)
    zp, itp, okp = fwbf.decode(g, y, plain)
    rl = fwbf.count(g.N, zl, pool, 0, itl, okl, 116)["frame_err"] / F
    rp = fwbf.count(g.N, zp, pool, 0, itp, okp, 100)["frame_err"] / F
    print(f"N=32400 6 dB: FER learned {rl:.4f} plain {rp:.4f}", flush=True)
    pooled = (rl + rp) / 2
    assert rp - rl > 3 * np.sqrt(pooled * (1 - pooled) * 2 / F)
