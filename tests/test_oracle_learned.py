"""Pins of the float64 scorer reference: analytic gradients against central
finite differences, the bfloat16 rounding helper against exact cases, and the
learned pass against the plain decoder in the special cases where the scorer
reproduces the bare metric test (identity score) or never flips (zero
weights, non-positive bias)."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp_ref as R


def test_bf16_rounding():
    vals = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -3.0, 0.0, 1e-40, 65504.0])
    got = R.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties to even -> 1
    assert got[0] == 1.0 and got[1] == 1.0
    # 1 + 1.5 * 2^-8 rounds up to 1 + 2^-7
    assert got[2] == 1.0078125 and got[3] == 1.0078125
    assert got[4] == -3.0 and got[5] == 0.0
    assert got[7] == 65536.0


def _records(rng, n, T):
    a = rng.integers(0, 128, n)
    S = rng.integers(-381, 382, n)
    u = rng.integers(0, 4, n)
    t = rng.integers(0, T, n)
    lab = (rng.random(n) < 0.4).astype(np.float64)
    return a, S, u, t, lab


def test_exact_gradients_match_finite_differences():
    T = 4
    rng = np.random.default_rng(0)
    P = R.n_params(T)
    p = rng.normal(0, 0.3, P)
    p[-2 * T:] = rng.uniform(0.5, 1.5, 2 * T)
    a, S, u, t, lab = _records(rng, 200, T)
    g = R.exact_backward(p, a, S, u, t, lab, 16.0, 3, T, 2.0)
    idx = rng.choice(P, 60, replace=False).tolist() + list(range(P - 2 * T, P))
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (R.loss_of_params(pp, a, S, u, t, lab, 16.0, 3, T, 2.0) -
              R.loss_of_params(pm, a, S, u, t, lab, 16.0, 3, T, 2.0)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_rounded_backward_equals_exact_when_values_are_bf16_exact():
    """With weights, features and backward operands all exactly
    representable in bfloat16, the rounded backward equals the exact one."""
    T = 2
    P = R.n_params(T)
    rng = np.random.default_rng(3)
    # weights in {-1, -1/2, 0, 1/2, 1}, biases in multiples of 1/8: every
    # pre-activation is a multiple of 1/16 below 8 in magnitude (7 bits)
    p = rng.integers(-2, 3, P) / 2.0
    W1, b1, W2, b2, W3, b3, al, be = R.unpack_params(p, T)
    o = 32 * 4
    p[o:o + 32] = rng.integers(-8, 9, 32) / 8.0
    p[-2 * T:] = 1.0
    a = rng.integers(0, 8, 50) * 2
    S = rng.integers(-8, 9, 50) * 2
    u = rng.integers(0, 4, 50)
    t = rng.integers(0, T, 50)
    lab = (rng.random(50) < 0.5).astype(np.float64)
    x = R.features(a, S, u, t, T, 16.0, 4, p[-2 * T:-T], p[-T:])
    g1 = R.backward(x, lab, t, a, S, 16.0, p, T, 1.0, round_bf16=False)
    g2 = R.exact_backward(p, a, S, u, t, lab, 16.0, 4, T, 1.0)
    assert np.allclose(g1, g2, rtol=1e-12, atol=1e-15)


def _identity_params(T, alpha, beta=1.0):
    """score = ReLU(E/A) - ReLU(-E/A) = E/A: hidden unit 0 = ReLU(x1),
    unit 1 = ReLU(-x1), passed through W2 = identity on units 0, 1."""
    W1 = np.zeros((32, 4)); W1[0, 1] = 1.0; W1[1, 1] = -1.0
    W2 = np.zeros((32, 32)); W2[0, 0] = 1.0; W2[1, 1] = 1.0
    W3 = np.zeros(32); W3[0] = 1.0; W3[1] = -1.0
    return np.concatenate([W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), W3, [0.0],
                           np.full(T, alpha), np.full(T, beta)])


def test_identity_scorer_reproduces_plain_blocks():
    """With the identity score, k = 1 and alpha = 1/4 the learned pass makes
    the plain FWBF choice every round (the metrics are bfloat16-exact on
    inputs +-16, +-8): same decisions while the learned pass runs."""
    code = O.Code.from_seed(3, 6, 31, 1)
    T = 40
    params = _identity_params(T, 0.25)
    rng = np.random.default_rng(5)
    n_same = 0
    for f in range(30):
        y = np.where(rng.random(code.N) < 0.5, 16, 8) * np.where(rng.random(code.N) < 0.07, -1, 1)
        y = y.astype(np.int8)
        tr = []
        z, rounds, ok, recs = R.learned_decode_frame(code, y, params, T, 6, 1, 16.0, 3, trace=tr)
        pt = O.decode_trace(code, y, G=6, max_iter=rounds, alpha_num=1, alpha_den=4)
        assert [list(map(int, f_)) for f_ in pt["flips"][:rounds]] == tr[:rounds]
        if ok:
            assert pt["ok"] and (O.unpack(pt["z"], code.N) == z).all()
        n_same += 1
    assert n_same == 30


def test_zero_scorer_never_flips():
    code = O.Code.from_seed(3, 6, 31, 1)
    T = 8
    params = np.zeros(R.n_params(T))
    params[R.n_params(T) - 2 * T - 1] = -0.5   # b3 < 0
    params[-T:] = 1.0
    y = np.where(np.arange(code.N) % 17 == 0, -16, 16).astype(np.int8)
    z, rounds, ok, recs = R.learned_decode_frame(code, y, params, T, 6, 2, 16.0, 3)
    assert rounds == 0 and not ok and (z == (y < 0)).all()
    assert len(recs) == 6 * 2


# ---- the Adam step (Kingma & Ba, Algorithm 1) against closed forms --------
def test_adam_first_step_closed_form():
    """From zero moments the bias-corrected moments of step 1 are g and g^2,
    so the first step moves every parameter by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(21)
    p0 = rng.normal(size=500)
    g = rng.normal(size=500) * 10.0 ** rng.uniform(-6, 2, 500)
    for lr, b1, b2, eps in [(1e-3, 0.9, 0.999, 1e-8), (0.3, 0.5, 0.25, 1e-3)]:
        p1, m1, v1 = R.adam_step(p0, g, np.zeros(500), np.zeros(500), 1, lr, b1, b2, eps)
        np.testing.assert_allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(m1, (1 - b1) * g, rtol=1e-15)
        np.testing.assert_allclose(v1, (1 - b2) * g * g, rtol=1e-15)


def test_adam_constant_gradient_and_zero_gradient():
    """A constant gradient keeps the corrected moments at g and g^2 in every
    step: after t steps p = p0 - t lr g / (|g| + eps).  A zero gradient
    never moves the parameters."""
    g = np.array([2.0, -0.5, 1e-4, -3e3])
    p = np.array([1.0, 2.0, -3.0, 0.5])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 21):
        p, m, v = R.adam_step(p, g, m, v, t, lr, 0.9, 0.999, eps)
        np.testing.assert_allclose(p, np.array([1.0, 2.0, -3.0, 0.5]) - t * lr * g / (np.abs(g) + eps),
                                   rtol=1e-11, atol=1e-13)
    q, _, _ = R.adam_step(np.ones(3), np.zeros(3), np.zeros(3), np.zeros(3), 1, 0.1)
    assert (q == 1.0).all()


def test_adam_two_steps_by_hand_and_eps_placement():
    """beta1 = beta2 = 1/2, lr = 0.3, eps = 0: gradient 1 then -1 from zero
    moments.  Step 1: m = 1/2, v = 1/2, corrected 1 and 1, p = -0.3.
    Step 2: m = -1/4, v = 3/4, corrected -1/3 and 1, p = -0.3 + 0.1 = -0.2.
    eps sits outside the square root: with g = eps = 1e-8 the first step is
    lr / 2 (inside the root it would be about lr 1e-4)."""
    p, m, v = R.adam_step([0.0], [1.0], [0.0], [0.0], 1, 0.3, 0.5, 0.5, 0.0)
    assert abs(p[0] + 0.3) < 1e-15 and m[0] == 0.5 and v[0] == 0.5
    p, m, v = R.adam_step(p, [-1.0], m, v, 2, 0.3, 0.5, 0.5, 0.0)
    assert abs(p[0] + 0.2) < 1e-15 and m[0] == -0.25 and v[0] == 0.75
    p, _, _ = R.adam_step([0.0], [1e-8], [0.0], [0.0], 1, 0.5, 0.9, 0.999, 1e-8)
    assert abs(p[0] + 0.25) < 1e-12


@pytest.mark.parametrize("mbnbZ,G,k,T", [((3, 6, 31, 1), 6, 4, 8), ((3, 6, 31, 1), 7, 1, 12),
                                          ((3, 6, 168, 2), 32, 1, 16)])
def test_batched_learned_pass_equals_per_frame(mbnbZ, G, k, T):
    """The frame-batched learned pass takes the same steps as the literal
    one-frame loop: identical bits, rounds, flags and candidate lists."""
    from paper_1206_3362_amd import synth
    code = O.Code.from_seed(*mbnbZ)
    rng = np.random.default_rng(G + k)
    p = rng.normal(0, 0.75, R.n_params(T))
    p[-2 * T:-T] = 0.2
    p[-T:] = 1.0
    y = synth.awgn_frames(code.N, 24, synth.sigma_for(4.5, 0.5), 17, None, np.int8)
    z, r, ok, tr = R.learned_decode_batch(code, y, p, T, G, k, 16.0, 3)
    adj = R._adjacency(code)
    for f in range(y.shape[0]):
        zf, rf, okf, recs = R.learned_decode_frame(code, y[f], p, T, G, k, 16.0, 3, adj)
        assert (z[f] == zf).all() and r[f] == rf and ok[f] == okf
        cands = [int(n) for c, _ in R.trace_of_frame(tr, f) for blk in c for n in blk if n >= 0]
        assert cands == [rc[4] for rc in recs]
