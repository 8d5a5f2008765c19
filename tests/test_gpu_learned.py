"""The learned flip scorer on the GPU against the float64 reference: MFMA
forward scores, backward gradients (with the same bfloat16 rounding points),
the learned pass with its plain-FWBF fallback, the special cases that reduce
to plain FWBF (identity scorer, zero scorer), and an ablation: a scorer
trained on decoder-generated frames must not lose to the plain decoder."""
import numpy as np
import pytest

import oracle as O
from gpu_util import need_gpu, torch
from oracle import mlp_ref as R
from paper_1206_3362_amd import fwbf, synth

pytestmark = pytest.mark.gpu


def random_params(T, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.5 * scale, R.n_params(T))
    p[-2 * T:-T] = rng.uniform(0.1, 0.4, T)   # alpha_t
    p[-T:] = rng.uniform(0.7, 1.3, T)         # beta_t
    return p.astype(np.float32)


def random_records(n_tiles, T, seed):
    rng = np.random.default_rng(seed)
    rec = np.zeros((n_tiles, 32), fwbf.RECORD_DTYPE)
    rec["S"] = rng.integers(-381, 382, rec.shape)
    rec["a"] = rng.integers(0, 128, rec.shape)
    rec["u"] = rng.integers(0, 4, rec.shape)
    rec["label"] = rng.random(rec.shape) < 0.4
    rec["valid"] = rng.random(rec.shape) < 0.9
    rec["n"] = rng.integers(0, 1008, rec.shape)
    t = np.arange(n_tiles) % T
    return rec, t


def to_dev(rec):
    return torch.from_numpy(rec.view(np.uint8).reshape(rec.shape[0], 32, fwbf.RECORD_DTYPE.itemsize).copy()).cuda()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def test_forward_scores_match_reference():
    T = 4
    p = random_params(T, 1)
    rec, t = random_records(256, T, 2)
    lp = fwbf.LearnedParams(T, 32, 1, 16.0)
    scores = torch.zeros(256 * 32, dtype=torch.float32, device="cuda")
    fwbf.scorer_grad(to_dev(rec), 256, lp, torch.from_numpy(p).cuda(), 1.0, scores=scores)
    got = scores.cpu().numpy().reshape(256, 32)
    tt = np.broadcast_to(t[:, None], rec.shape)
    x = R.features(rec["a"].ravel(), rec["S"].ravel(), rec["u"].ravel(), tt.ravel(), T, 16.0, 3,
                   p[-2 * T:-T].astype(np.float64), p[-T:].astype(np.float64))
    want, _ = R.forward(x, p.astype(np.float64), T)
    want = want.reshape(256, 32)
    v = rec["valid"].astype(bool)
    err = np.abs(got - want)[v]
    scale = 1.0 + np.abs(want[v])
    # single-precision sums in a different order: isolated bfloat16 rounding
    # flips of h1 move a score by ~2^-8 of one hidden contribution
    assert np.median(err / scale) < 1e-5
    assert (err / scale < 2e-2).all(), (err / scale).max()
    assert (got[~v] == 0).all()


def test_gradients_match_reference():
    T = 4
    p = random_params(T, 3)
    rec, t = random_records(512, T, 4)
    lp = fwbf.LearnedParams(T, 32, 1, 16.0)
    P = R.n_params(T)
    out = torch.zeros(P + 2, dtype=torch.float32, device="cuda")
    fwbf.scorer_grad(to_dev(rec), 512, lp, torch.from_numpy(p).cuda(), 2.0, out=out)
    g = out.cpu().numpy().astype(np.float64)
    # the workgroup partials are summed in a fixed order: a second run is bit-identical
    out2 = torch.zeros_like(out)
    fwbf.scorer_grad(to_dev(rec), 512, lp, torch.from_numpy(p).cuda(), 2.0, out=out2)
    assert torch.equal(out, out2)
    v = rec["valid"].astype(bool)
    tt = np.broadcast_to(t[:, None], rec.shape)[v]
    a, S, u, lab = rec["a"][v], rec["S"][v], rec["u"][v], rec["label"][v].astype(np.float64)
    x = R.features(a, S, u, tt, T, 16.0, 3, p[-2 * T:-T].astype(np.float64), p[-T:].astype(np.float64))
    ref = R.backward(x, lab, tt, a, S, 16.0, p.astype(np.float64), T, 2.0, round_bf16=True)
    s, _ = R.forward(x, p.astype(np.float64), T)
    assert g[P + 1] == v.sum()
    assert abs(g[P] - R.loss(s, lab, 2.0)) < 1e-4 * abs(R.loss(s, lab, 2.0))
    bounds = [("W1", 0, 128), ("b1", 128, 160), ("W2", 160, 1184), ("b2", 1184, 1216),
              ("W3", 1216, 1248), ("b3", 1248, 1249), ("alpha", 1249, 1249 + T),
              ("beta", 1249 + T, 1249 + 2 * T)]
    for name, lo, hi in bounds:
        d = np.linalg.norm(g[lo:hi] - ref[lo:hi]) / max(np.linalg.norm(ref[lo:hi]), 1e-12)
        assert d < 1e-3, (name, d)


def _plain_oracle(ocode, y, G, alpha_den=5, max_iter=100):
    return O.decode(ocode, y, G=G, max_iter=max_iter, alpha_num=1, alpha_den=alpha_den)


def _learned_reference(ocode, y, p, T, G, k, plain_G, alpha_den=5, A=16.0):
    adj = R._adjacency(ocode)
    zs, its, oks, recs = [], [], [], []
    for f in range(y.shape[0]):
        z, rounds, ok, rc = R.learned_decode_frame(ocode, y[f], p.astype(np.float64), T, G, k, A, 3, adj)
        if not ok:
            zp, itp, okp = _plain_oracle(ocode, y[f:f + 1], plain_G, alpha_den)
            z, rounds, ok = O.unpack(zp, ocode.N)[0], rounds + int(itp[0]), bool(okp[0])
        zs.append(z), its.append(rounds), oks.append(ok), recs.append(rc)
    return np.array(zs), np.array(its), np.array(oks), recs


@pytest.mark.parametrize("name,mbnbZ,G,k,T,A", [("n186", (3, 6, 31, 1), 6, 4, 8, 16.0),
                                                ("n1008", (3, 6, 168, 2), 32, 1, 8, 16.0),
                                                ("n1008", (3, 6, 168, 2), 8, 4, 6, 16.0),
                                                ("n1008", (3, 6, 168, 2), 32, 1, 6, 12.0)])
def test_learned_pass_matches_reference(name, mbnbZ, G, k, T, A):
    """The learned pass plus fallback against the float64 reference; a scale
    A that is not a power of two takes the divided feature path, T = 6 the
    non-power-of-two round feature t / T."""
    g = fwbf.Code.from_seed(*mbnbZ)
    o = O.Code.from_seed(*mbnbZ)
    Fn = 96
    p = random_params(T, 11, scale=1.5)
    p[-2 * T:-T] = 0.2
    p[-T:] = 1.0
    y = synth.awgn_frames(g.N, Fn, synth.sigma_for(4.5, g.rate), 9, None, np.int8)
    lp = fwbf.LearnedParams(T, G, k, A)
    plain = fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100)
    rec = fwbf.record_buffer(Fn, T, G, k)
    z, it, ok, lok = fwbf.decode_learned(g, torch.from_numpy(y).cuda(), plain, lp,
                                         torch.from_numpy(p).cuda(), records=rec)
    torch.cuda.synchronize()
    zg = O.unpack(z.cpu().numpy().view(np.uint32), g.N)
    itg, okg = it.cpu().numpy(), ok.cpu().numpy().astype(bool)
    zr, itr, okr, recs = _learned_reference(o, y, p, T, G, k, 8, A=A)
    same = (zg == zr).all(1) & (itg == itr) & (okg == okr)
    print(f"{name} G={G} k={k} A={A}: {same.sum()}/{Fn} frames identical, "
          f"learned-pass successes {int(lok.sum())}", flush=True)
    assert same.mean() >= 0.95
    # round-0 proposals depend only on exact single-precision metrics
    rg = fwbf.records_host(rec)
    for f in range(Fn):
        r0 = [r for r in recs[f] if r[3] == 0]
        n_gpu = [int(x) for x in rg[f, 0, :len(r0)]["n"]]
        assert n_gpu == [r[4] for r in r0]
        assert [int(x) for x in rg[f, 0, :len(r0)]["S"]] == [r[1] for r in r0]
        assert [int(x) for x in rg[f, 0, :len(r0)]["label"]] == [r[5] for r in r0]


def test_identity_scorer_equals_plain():
    g = fwbf.Code.from_seed(3, 6, 31, 1)
    o = O.Code.from_seed(3, 6, 31, 1)
    T = 40
    W1 = np.zeros((32, 4)); W1[0, 1] = 1.0; W1[1, 1] = -1.0
    W2 = np.zeros((32, 32)); W2[0, 0] = 1.0; W2[1, 1] = 1.0
    W3 = np.zeros(32); W3[0] = 1.0; W3[1] = -1.0
    p = np.concatenate([W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), W3, [0.0],
                        np.full(T, 0.25), np.full(T, 1.0)]).astype(np.float32)
    rng = np.random.default_rng(5)
    Fn = 2000
    y = (np.where(rng.random((Fn, g.N)) < 0.5, 16, 8) *
         np.where(rng.random((Fn, g.N)) < 0.07, -1, 1)).astype(np.int8)
    plain = fwbf.DecodeParams(dtype=fwbf.I8, groups=6, max_iter=100, alpha_num=1, alpha_den=4)
    z, it, ok, lok = fwbf.decode_learned(g, torch.from_numpy(y).cuda(), plain,
                                         fwbf.LearnedParams(T, 6, 1, 16.0), torch.from_numpy(p).cuda())
    zp, itp, okp = O.decode(o, y, G=6, max_iter=100, alpha_num=1, alpha_den=4)
    assert np.array_equal(z.cpu().numpy().view(np.uint32), zp)
    assert np.array_equal(ok.cpu().numpy(), okp)
    assert lok.cpu().numpy().sum() == okp.sum()


def test_zero_scorer_falls_back_everywhere():
    g = fwbf.Code.from_seed(3, 6, 168, 2)
    o = O.Code.from_seed(3, 6, 168, 2)
    T = 8
    p = np.zeros(R.n_params(T), np.float32)
    p[1248] = -0.5
    p[-T:] = 1.0
    y = synth.awgn_frames(g.N, 1024, synth.sigma_for(5.0, g.rate), 3, None, np.int8)
    plain = fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100)
    z, it, ok, lok = fwbf.decode_learned(g, torch.from_numpy(y).cuda(), plain,
                                         fwbf.LearnedParams(T, 32, 1, 16.0), torch.from_numpy(p).cuda())
    zp, itp, okp = O.decode(o, y, G=8, max_iter=100)
    assert np.array_equal(z.cpu().numpy().view(np.uint32), zp)
    assert np.array_equal(it.cpu().numpy(), itp) and np.array_equal(ok.cpu().numpy(), okp)
    assert lok.cpu().numpy().sum() == 0


def test_training_gains_over_plain():
    """Ablation: after training on decoder-generated frames the learned
    decoder (with fallback) has a lower frame error rate than plain FWBF at
    4 dB, and the training loss went down."""
    from paper_1206_3362_amd import learned as L
    code = fwbf.Code.from_seed(3, 6, 168, 2)
    cfg = L.TrainConfig(rounds=16, groups=32, topk=1, batch=4096, steps=120, lr=3e-3)
    tr = L.Trainer(code, cfg).train(log_every=10)
    first, last = tr.history[0][1], tr.history[-1][1]
    print("loss", [round(h[1], 4) for h in tr.history], flush=True)
    assert last < first
    F = 8192
    pool = tr.pool
    y = fwbf.channel(code.N, F, 10 ** 9, pool, 4242, 1, float(synth.sigma_for(4.0, code.rate)),
                     dtype=torch.int8, scale=16.0)
    plain = fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100)
    zl, itl, okl, lokl = fwbf.decode_learned(code, y, plain, tr.lp, tr.params)
    zp, itp, okp = fwbf.decode(code, y, plain)
    rl = fwbf.count(code.N, zl, pool, 10 ** 9, itl, okl, 300)
    rp = fwbf.count(code.N, zp, pool, 10 ** 9, itp, okp, 100)
    print("FER learned", rl["frame_err"] / F, "plain", rp["frame_err"] / F, flush=True)
    assert rl["frame_err"] <= rp["frame_err"]


def test_adam_matches_reference():
    """fwbf_adam against the float64 Adam of Kingma & Ba over six steps with
    changing gradients: parameters and both moments element by element.
    The entry point takes its hyperparameters in single precision, so the
    reference runs with those same values (0.999 as a float is
    0.99900001...; with the decimal value (1 - beta2) alone would differ by
    1.3e-5).  Each step starts the reference from the state the kernel left,
    so the bound is that of one step in single precision: a few units of
    rounding (u = 2^-24) of the terms each result is formed from (a moment
    that cancels to near zero is judged against its terms, not itself)."""
    rng = np.random.default_rng(31)
    P = R.n_params(16)
    p = rng.normal(0, 1, P).astype(np.float32)
    lr, b1, b2, eps = (float(np.float32(x)) for x in (3e-3, 0.9, 0.999, 1e-8))
    u = 2.0 ** -24
    pd = torch.from_numpy(p).cuda()
    md = torch.zeros(P, dtype=torch.float32, device="cuda")
    vd = torch.zeros_like(md)
    for step in range(1, 7):
        g = (rng.normal(0, 1, P) * 10.0 ** rng.uniform(-5, 1, P)).astype(np.float32)
        p0 = pd.cpu().numpy().astype(np.float64)
        m0 = md.cpu().numpy().astype(np.float64)
        v0 = vd.cpu().numpy().astype(np.float64)
        fwbf.adam(pd, torch.from_numpy(g).cuda(), md, vd, step, lr, b1, b2, eps)
        pr, mr, vr = R.adam_step(p0, g.astype(np.float64), m0, v0, step, lr, b1, b2, eps)
        torch.cuda.synchronize()
        gg = g.astype(np.float64)
        m_sc = b1 * np.abs(m0) + (1 - b1) * np.abs(gg)
        v_sc = b2 * v0 + (1 - b2) * gg * gg
        upd = np.abs(p0 - pr)
        assert np.all(np.abs(md.cpu().numpy() - mr) <= 4 * u * m_sc), step
        assert np.all(np.abs(vd.cpu().numpy() - vr) <= 6 * u * v_sc), step
        assert np.all(np.abs(pd.cpu().numpy() - pr) <= 2 * u * np.abs(pr) + 32 * u * upd + 1e-30), step
        assert np.abs(pd.cpu().numpy() - p0).max() > 0  # the step moved the parameters


@pytest.mark.parametrize("mbnbZ,G,k", [((3, 6, 31, 1), 32, 1), ((3, 6, 168, 2), 8, 2),
                                        ((3, 6, 168, 2), 5, 4)])
def test_empty_record_slots_are_invalid(mbnbZ, G, k):
    """With fewer than 32 proposals per round (G' k < 32; N = 186 with 32
    blocks of 6 bits has only 31 blocks) the slots without a proposal are
    written with valid = 0 in every round run, whatever the buffer held
    before; the gradient over the records does not depend on it."""
    g = fwbf.Code.from_seed(*mbnbZ)
    T, Fn = 6, 256
    p = random_params(T, 13)
    p[-2 * T:-T] = 0.2
    p[-T:] = 1.0
    y = synth.awgn_frames(g.N, Fn, synth.sigma_for(4.0, g.rate), 5, None, np.int8)
    lp = fwbf.LearnedParams(T, G, k, 16.0)
    plain = fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100)
    pd = torch.from_numpy(p).cuda()
    P = R.n_params(T)
    grads, recs = [], []
    for fill in (0xFF, 0x00):
        rec = fwbf.record_buffer(Fn, T, G, k)
        rec.fill_(fill)
        fwbf.decode_learned(g, torch.from_numpy(y).cuda(), plain, lp, pd, records=rec)
        out = torch.zeros(P + 2, dtype=torch.float32, device="cuda")
        fwbf.scorer_grad(rec, Fn * T, lp, pd, 1.0, out=out)
        torch.cuda.synchronize()
        grads.append(out.cpu().numpy())
        recs.append(fwbf.records_host(rec))
    p_ = -(-g.N // G)
    nc = (-(-g.N // p_)) * k
    assert nc < 32
    for r in recs:
        assert (r["valid"] <= 1).all() and (r["label"][r["valid"] == 1] <= 1).all()
        assert (r["valid"][:, :, nc:] == 0).all()
    v = recs[0]["valid"] == 1
    assert np.array_equal(recs[0]["valid"], recs[1]["valid"]) and v.any()
    assert np.array_equal(recs[0][v], recs[1][v])
    assert np.array_equal(grads[0], grads[1])


def test_gradients_match_reference_many_tiles():
    """4133 tiles on the 1024-workgroup grid: every workgroup accumulates
    four or five tiles of mixed rounds before the fixed-order reduction, as
    a training step does (there: 131072 tiles).  Against the float64
    backward with the same bfloat16 rounding points."""
    T = 8
    p = random_params(T, 23)
    n_tiles = 4 * 1024 + 37
    rec, t = random_records(n_tiles, T, 24)
    lp = fwbf.LearnedParams(T, 32, 1, 16.0)
    P = R.n_params(T)
    out = torch.zeros(P + 2, dtype=torch.float32, device="cuda")
    fwbf.scorer_grad(to_dev(rec), n_tiles, lp, torch.from_numpy(p).cuda(), 1.5, out=out)
    g = out.cpu().numpy().astype(np.float64)
    v = rec["valid"].astype(bool)
    tt = np.broadcast_to(t[:, None], rec.shape)[v]
    a, S, u, lab = rec["a"][v], rec["S"][v], rec["u"][v], rec["label"][v].astype(np.float64)
    x = R.features(a, S, u, tt, T, 16.0, 3, p[-2 * T:-T].astype(np.float64), p[-T:].astype(np.float64))
    ref = R.backward(x, lab, tt, a, S, 16.0, p.astype(np.float64), T, 1.5, round_bf16=True)
    s, _ = R.forward(x, p.astype(np.float64), T)
    assert g[P + 1] == v.sum()
    assert abs(g[P] - R.loss(s, lab, 1.5)) < 1e-4 * abs(R.loss(s, lab, 1.5))
    bounds = [("W1", 0, 128), ("b1", 128, 160), ("W2", 160, 1184), ("b2", 1184, 1216),
              ("W3", 1216, 1248), ("b3", 1248, 1249), ("alpha", 1249, 1249 + T),
              ("beta", 1249 + T, 1249 + 2 * T)]
    for name, lo, hi in bounds:
        d = np.linalg.norm(g[lo:hi] - ref[lo:hi]) / max(np.linalg.norm(ref[lo:hi]), 1e-12)
        assert d < 1e-3, (name, d)


# forward scores: |GPU - float64| <= SCORE_BOUND (1 + |score|), the bound the
# forward test holds every score to (bfloat16 rounding of h1 can move by one
# unit where single-precision sums sit on a rounding boundary)
SCORE_BOUND = 2e-2


def test_checkpoint_learned_pass_frame_by_frame():
    """The committed checkpoint (T = 16, 32 blocks, k = 1) on 2048 frames of
    the N = 1008 code at 4 dB, int8: z, rounds and flags frame by frame
    against the float64 learned pass plus the plain oracle fallback.  Under
    this scorer the learned pass decides most frames itself.  A frame may
    differ only where the MFMA scores can decide differently from the
    float64 ones: at the first round whose proposals differ (or the last
    round, if none do), some block's best score lies within the forward
    bound of 0."""
    import os
    g = fwbf.Code.from_seed(3, 6, 168, 2)
    o = O.Code.from_seed(3, 6, 168, 2)
    ck = np.load(os.path.join(os.path.dirname(fwbf.__file__), "scorer_n1008_g32_t16.npz"),
                 allow_pickle=False)
    p = ck["params"].astype(np.float32)
    T, G, k, Fn = 16, 32, 1, 2048
    cw = O.unpack(o.encode(11, 0, Fn), o.N)
    y = synth.awgn_frames(o.N, Fn, synth.sigma_for(4.0, o.K / o.N), 77, cw, np.int8)
    lp = fwbf.LearnedParams(T, G, k, 16.0)
    plain = fwbf.DecodeParams(dtype=fwbf.I8, groups=8, max_iter=100)
    rec = fwbf.record_buffer(Fn, T, G, k)
    z, it, ok, lok = fwbf.decode_learned(g, torch.from_numpy(y).cuda(), plain, lp,
                                         torch.from_numpy(p).cuda(), records=rec)
    torch.cuda.synchronize()
    zg = O.unpack(z.cpu().numpy().view(np.uint32), o.N)
    itg, okg, lokg = it.cpu().numpy(), ok.cpu().numpy().astype(bool), lok.cpu().numpy().astype(bool)
    rg = fwbf.records_host(rec)
    zr, rr, okr, tr = R.learned_decode_batch(o, y, p.astype(np.float64), T, G, k, 16.0, 3)
    same_pass = (zg == zr).all(1) & (lokg == okr)
    # plain fallback for the frames the reference's learned pass leaves
    itr = rr.copy()
    zf, okf = zr.copy(), okr.copy()
    fb = np.nonzero(~okr)[0]
    zp, itp, okp = O.decode(o, y[fb], G=8, max_iter=100, alpha_num=1, alpha_den=5)
    zf[fb], itr[fb], okf[fb] = O.unpack(zp, o.N), rr[fb] + itp, okp.astype(bool)
    same = (zg == zf).all(1) & (itg == itr) & (okg == okf) & (lokg == okr)
    unexplained = []
    for f in np.nonzero(~same)[0]:
        rounds = R.trace_of_frame(tr, f)
        decide = len(rounds) - 1
        for t_, (cand, _) in enumerate(rounds):
            n_gpu = rg[f, t_]["n"][rg[f, t_]["valid"] == 1].astype(np.int64)
            if not np.array_equal(n_gpu, cand.ravel()[cand.ravel() >= 0]):
                decide = t_ - 1
                break
        if decide < 0:
            unexplained.append((int(f), "round-0 proposals differ"))
            continue
        sc = rounds[decide][1].max(1)
        margin = np.abs(sc) / (1.0 + np.abs(sc))
        if margin.min() > SCORE_BOUND:
            unexplained.append((int(f), decide, float(margin.min())))
    print(f"learned pass alone: GPU {lokg.mean():.4f} reference {okr.mean():.4f}; "
          f"frames identical {same.sum()}/{Fn} (learned pass {same_pass.sum()}); "
          f"near-tie frames {Fn - same.sum() - len(unexplained)}; unexplained {unexplained[:5]}",
          flush=True)
    assert okr.mean() > 0.5
    assert not unexplained
    assert same.mean() >= 0.98
