"""Float64 reference of the learned flip scorer -- test infrastructure only.

The learned variant of the decoder (a design extension, not in the paper;
it keeps the paper's per-block choice of Section III and replaces the bare
metric test by a small scorer) is defined here in plain numpy so that the
HIP kernels can be checked against it.  Only the test suite and bench.py's
CPU-baseline leg may import this module.

Definitions (int8 inputs, scale A; IMWBF check weights of eq. (1)):
  S_n = sum over M(n) of (2 s_m - 1) w_{n,m}      (integer)
  a_n = |y_n|,  u_n = sum over M(n) of s_m       (unsatisfied checks)
  round t (0-based, t < T rounds of the learned pass):
    E_n = fmaf(-alpha_t, a_n, beta_t * S_n)      (single precision)
    candidates: in each of G blocks (p = ceil(N/G), contiguous, as in
      Section III), the k bits with the largest E_n (ties: lower index)
    features x = [a/A, E/A, u/dv, t/T]  rounded to bfloat16
    h1 = relu(W1 x + b1) rounded to bfloat16  (W1, W2 rounded to bfloat16,
      products accumulated in single precision on the GPU, exactly here)
    h2 = relu(W2 h1 + b2);  score = W3 . h2 + b3
    in each block the candidate with the largest score (ties: lower index)
    is flipped iff its score > 0
  the learned pass stops on a zero syndrome (success), on a round without a
  flip, on a round repeating the previous round's flips, or after T rounds;
  frames that end with a nonzero syndrome are decoded again from the
  original y by plain FWBF, and their round count is T_learned + plain.

Parameter vector (float32, P = 1249 + 2T):
  W1[32][4], b1[32], W2[32][32], b2[32], W3[32], b3, alpha[T], beta[T].
"""
from __future__ import annotations

import numpy as np

H = 32
NF = 4


def n_params(T: int) -> int:
    return H * NF + H + H * H + H + H + 1 + 2 * T


def unpack_params(p, T):
    p = np.asarray(p, np.float64)
    o = 0

    def take(n, shape):
        nonlocal o
        v = p[o:o + n].reshape(shape)
        o += n
        return v
    W1 = take(H * NF, (H, NF))
    b1 = take(H, (H,))
    W2 = take(H * H, (H, H))
    b2 = take(H, (H,))
    W3 = take(H, (H,))
    b3 = take(1, ())
    al = take(T, (T,))
    be = take(T, (T,))
    assert o == p.size
    return W1, b1, W2, b2, W3, float(b3), al, be


def bf16(x):
    """Round to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def metric_t(a, S, alpha_t, beta_t):
    """E = fmaf(-alpha, a, beta * S) in single precision."""
    al = np.asarray(alpha_t, np.float32).astype(np.float64)
    be = np.asarray(beta_t, np.float32).astype(np.float64)
    prod = f32(be * np.asarray(S, np.float64))
    # the product of two floats is exact in double; one rounding to float
    return f32(-al * np.asarray(a, np.float64) + prod)


def features(a, S, u, t, T, A, dv, alpha, beta):
    """Feature rows [R][4] before rounding (float32 values)."""
    a = np.asarray(a, np.float64)
    t = np.broadcast_to(np.asarray(t), a.shape)
    E = metric_t(a, S, np.asarray(alpha)[t], np.asarray(beta)[t])
    x = np.stack([f32(a / A), f32(E / A), f32(np.asarray(u, np.float64) / dv),
                  f32(t.astype(np.float64) / T)], -1)
    return x


def forward(x, params, T):
    """x [R][4] -> (score [R], cache)."""
    W1, b1, W2, b2, W3, b3, _, _ = unpack_params(params, T)
    xb = bf16(x)
    W1b, W2b = bf16(W1), bf16(W2)
    pre1 = xb @ W1b.T + b1
    h1 = np.maximum(pre1, 0.0)
    h1b = bf16(h1)
    pre2 = h1b @ W2b.T + b2
    h2 = np.maximum(pre2, 0.0)
    s = h2 @ W3 + b3
    return s, dict(xb=xb, W1b=W1b, W2b=W2b, pre1=pre1, h1b=h1b, pre2=pre2, h2=h2)


def loss(score, label, pos_weight, R=None):
    R = len(score) if R is None else R
    sp = np.logaddexp(0.0, score)      # softplus(s)
    spn = np.logaddexp(0.0, -score)    # softplus(-s)
    return float(np.sum(pos_weight * label * spn + (1 - label) * sp) / R)


def backward(x, label, t_idx, a, S, A, params, T, pos_weight, round_bf16=True):
    """Gradients of loss() w.r.t. the parameter vector.

    The feature x1 = E/A depends on alpha_t and beta_t:
    dE/dalpha_t = -a, dE/dbeta_t = S.  Rounding to bfloat16 is treated as the
    identity in the backward pass (straight-through).  With round_bf16 the
    two contractions of the backward pass use bfloat16-rounded operands
    (dpre2 and W2), as the GPU does; without it everything is exact."""
    W1, b1, W2, b2, W3, b3, al, be = unpack_params(params, T)
    s, c = forward(x, params, T)
    R = len(s)
    # per-record derivative of the unnormalised sum; the mean's 1/R is
    # applied to the finished sums (after the bfloat16 rounding points), and
    # sigma(s) - 1 = -sigma(-s) is written without cancellation
    ds = -pos_weight * label / (1.0 + np.exp(s)) + (1 - label) / (1.0 + np.exp(-s))
    dW3 = c["h2"].T @ ds
    db3 = ds.sum()
    dpre2 = np.outer(ds, W3) * (c["pre2"] > 0)
    db2 = dpre2.sum(0)
    d2 = bf16(dpre2) if round_bf16 else dpre2
    dW2 = d2.T @ c["h1b"]
    W2u = c["W2b"] if round_bf16 else W2
    dh1 = d2 @ W2u
    dpre1 = dh1 * (c["pre1"] > 0)
    db1 = dpre1.sum(0)
    dW1 = dpre1.T @ c["xb"]
    W1u = c["W1b"] if round_bf16 else W1
    dx1 = dpre1 @ W1u[:, 1]
    dal = np.zeros(T)
    dbe = np.zeros(T)
    np.add.at(dal, t_idx, dx1 * (-np.asarray(a, np.float64) / A))
    np.add.at(dbe, t_idx, dx1 * (np.asarray(S, np.float64) / A))
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, [db3], dal, dbe]) / R


def loss_of_params(params, a, S, u, t_idx, label, A, dv, T, pos_weight):
    """Loss as a function of the parameters, with features recomputed from
    the records (for finite differences; no bfloat16 rounding)."""
    W1, b1, W2, b2, W3, b3, al, be = unpack_params(params, T)
    a = np.asarray(a, np.float64)
    E = be[t_idx] * np.asarray(S, np.float64) - al[t_idx] * a
    x = np.stack([a / A, E / A, np.asarray(u, np.float64) / dv, np.asarray(t_idx, np.float64) / T], -1)
    h1 = np.maximum(x @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    s = h2 @ W3 + b3
    return loss(s, label, pos_weight)


def exact_backward(params, a, S, u, t_idx, label, A, dv, T, pos_weight):
    """Analytic gradient of loss_of_params (float64, no rounding)."""
    W1, b1, W2, b2, W3, b3, al, be = unpack_params(params, T)
    a = np.asarray(a, np.float64)
    E = be[t_idx] * np.asarray(S, np.float64) - al[t_idx] * a
    x = np.stack([a / A, E / A, np.asarray(u, np.float64) / dv, np.asarray(t_idx, np.float64) / T], -1)
    pre1 = x @ W1.T + b1
    h1 = np.maximum(pre1, 0)
    pre2 = h1 @ W2.T + b2
    h2 = np.maximum(pre2, 0)
    s = h2 @ W3 + b3
    R = len(s)
    ds = (-pos_weight * label / (1.0 + np.exp(s)) + (1 - label) / (1.0 + np.exp(-s))) / R
    dW3 = h2.T @ ds
    db3 = ds.sum()
    dpre2 = np.outer(ds, W3) * (pre2 > 0)
    dW2 = dpre2.T @ h1
    db2 = dpre2.sum(0)
    dpre1 = (dpre2 @ W2) * (pre1 > 0)
    dW1 = dpre1.T @ x
    db1 = dpre1.sum(0)
    dx1 = dpre1 @ W1[:, 1]
    dal = np.zeros(T)
    dbe = np.zeros(T)
    np.add.at(dal, t_idx, -dx1 * a / A)
    np.add.at(dbe, t_idx, dx1 * np.asarray(S, np.float64) / A)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, [db3], dal, dbe])


# --------------------------------------------------------------------------
# optimizer
# --------------------------------------------------------------------------
def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam (Kingma & Ba, 2015, Algorithm 1), float64, written
    out as the published algorithm: biased moments, bias correction for step
    number `step` (1-based), then the update with eps added to the square
    root of the corrected second moment.  Returns new (params, m, v)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    p = np.asarray(params, np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v


# --------------------------------------------------------------------------
# learned decoding of one frame (literal, per round)
# --------------------------------------------------------------------------
def _adjacency(code):
    rp, rb = code.rows()
    M, N = code.M, code.N
    checks_of = [[] for _ in range(N)]
    for m in range(M):
        for n in rb[rp[m]:rp[m + 1]]:
            checks_of[n].append(m)
    return rp, rb, checks_of


def learned_decode_frame(code, y, params, T, G, k, A, dv, adj=None, trace=None):
    """One int8 frame through the learned pass.  Returns (z bits, rounds, ok,
    records): rounds counts the rounds whose flips were applied; records lists
    (a, S, u, t, n, z_n) of every candidate scored, in (round, block, rank)
    order.  The fallback is not applied here."""
    W1, b1, W2, b2, W3, b3, al, be = unpack_params(params, T)
    rp, rb, checks_of = adj or _adjacency(code)
    N, M = code.N, code.M
    y = np.asarray(y, np.int64)
    a = np.abs(y)
    z = (y < 0).astype(np.int64)
    # IMWBF weights per (check, member): minimum of |y| over the other members
    w = {}
    for m in range(M):
        bits = rb[rp[m]:rp[m + 1]]
        for n in bits:
            others = [a[i] for i in bits if i != n]
            w[(m, int(n))] = min(others) if others else 0
    p = -(-N // G)
    prev = None
    recs = []
    t = 0
    while True:
        s = np.array([z[rb[rp[m]:rp[m + 1]]].sum() % 2 for m in range(M)])
        if s.sum() == 0:
            return z, t, True, recs
        if t == T:
            return z, t, False, recs
        S = np.array([sum((w[(m, n)] if s[m] else -w[(m, n)]) for m in checks_of[n]) for n in range(N)])
        u = np.array([sum(s[m] for m in checks_of[n]) for n in range(N)])
        E = metric_t(a, S, al[t], be[t])
        flips = []
        for lo in range(0, N, p):
            hi = min(N, lo + p)
            idx = np.arange(lo, hi)
            order = sorted(idx, key=lambda n: (-E[n], n))[:k]
            cand = np.array(order)
            x = features(a[cand], S[cand], u[cand], t, T, A, dv, al, be)
            sc, _ = forward(x, params, T)
            for r_, n in enumerate(cand):
                recs.append((int(a[n]), int(S[n]), int(u[n]), t, int(n), int(z[n])))
            best = max(range(len(cand)), key=lambda j: (sc[j], -cand[j]))
            if sc[best] > 0:
                flips.append(int(cand[best]))
        if trace is not None:
            trace.append(list(flips))
        if not flips or (prev is not None and flips == prev):
            return z, t, False, recs
        for n in flips:
            z[n] ^= 1
        prev = flips
        t += 1


def learned_decode_batch(code, Y, params, T, G, k, A, dv):
    """The learned pass of learned_decode_frame over many frames at once (the
    frames are independent and all live frames are in the same round, so
    each step of a round is one array operation over the frames).  Returns
    (z bits [F][N], rounds [F], ok [F], trace): trace[t] = (frames, cand,
    score) for round t, with cand and score [frames][G'][k'] (G' blocks, k'
    candidates per block) for the frames that ran round t."""
    rp, rb = code.rows()
    N, M = code.N, code.M
    Y = np.asarray(Y, np.int64)
    if Y.ndim == 1:
        Y = Y[None]
    F = Y.shape[0]
    deg = np.diff(rp)
    dcm = int(deg.max())
    members = np.full((M, dcm), N, np.int64)           # column N: a zero pad
    for m in range(M):
        members[m, :deg[m]] = rb[rp[m]:rp[m + 1]]
    # the checks of every bit (ascending m) and the bit's place in each check
    chk_of = [[] for _ in range(N)]
    for m in range(M):
        for j in range(deg[m]):
            chk_of[members[m, j]].append((m, j))
    dvm = max(len(c) for c in chk_of)
    bm = np.full((N, dvm), M, np.int64)                # row M: a zero pad
    bj = np.zeros((N, dvm), np.int64)
    for n in range(N):
        for t_, (m, j) in enumerate(chk_of[n]):
            bm[n, t_], bj[n, t_] = m, j
    a = np.abs(Y)
    apad = np.concatenate([a, np.zeros((F, 1), np.int64)], 1)
    # IMWBF weight of edge (m, j): minimum of |y| over the other members of m
    am = apad[:, members]                               # [F][M][dcm]
    big = np.iinfo(np.int64).max
    w = np.zeros((F, M + 1, dcm), np.int64)
    for j in range(dcm):
        others = [i for i in range(dcm) if i != j]
        if others:
            vals = am[:, :, others].copy()
            pad = members[None, :, others] == N
            vals[np.broadcast_to(pad, vals.shape)] = big
            mn = vals.min(-1)
            w[:, :M, j] = np.where(mn == big, 0, mn)
    W1, b1, W2, b2, W3, b3, al, be = unpack_params(params, T)
    z = (Y < 0).astype(np.int64)
    rounds = np.zeros(F, np.int64)
    ok = np.zeros(F, bool)
    live = np.ones(F, bool)
    prev = [None] * F
    trace = []
    p = -(-N // G)
    blocks = [(lo, min(N, lo + p)) for lo in range(0, N, p)]
    t = 0
    fr = np.arange(F)
    while live.any():
        idx = fr[live]
        zp = np.concatenate([z[idx], np.zeros((idx.size, 1), np.int64)], 1)
        s = zp[:, members].sum(-1) % 2                  # syndrome [F'][M]
        zero = s.sum(1) == 0
        ok[idx[zero]] = True
        live[idx[zero]] = False
        if t == T:
            live[:] = False
            break
        idx = idx[~zero]
        if idx.size == 0:
            break
        s = np.concatenate([s[~zero], np.zeros((idx.size, 1), np.int64)], 1)
        sb = s[:, bm]                                    # [F'][N][dvm]
        wb = w[idx][:, bm, bj]                           # [F'][N][dvm]
        S = np.where(sb == 1, wb, -wb).sum(-1)
        u = sb.sum(-1)
        E = metric_t(a[idx], S, al[t], be[t])
        kmax = min(k, p)
        cand = np.full((idx.size, len(blocks), kmax), -1, np.int64)
        score = np.full((idx.size, len(blocks), kmax), np.nan)
        flip_n = np.full((idx.size, len(blocks)), -1, np.int64)
        for b, (lo, hi) in enumerate(blocks):
            kk = min(k, hi - lo)
            order = np.argsort(-E[:, lo:hi], axis=1, kind="stable")[:, :kk] + lo   # ties: lower index
            ai = np.take_along_axis(a[idx], order, 1)
            Si = np.take_along_axis(S, order, 1)
            ui = np.take_along_axis(u, order, 1)
            x = features(ai.ravel(), Si.ravel(), ui.ravel(), t, T, A, dv, al, be)
            sc, _ = forward(x, params, T)
            sc = sc.reshape(idx.size, kk)
            # the block's best score, ties to the lower bit index
            best = np.zeros(idx.size, np.int64)
            for j in range(1, kk):
                sb_, ob_ = sc[np.arange(idx.size), best], order[np.arange(idx.size), best]
                better = (sc[:, j] > sb_) | ((sc[:, j] == sb_) & (order[:, j] < ob_))
                best = np.where(better, j, best)
            bs = sc[np.arange(idx.size), best]
            flip_n[:, b] = np.where(bs > 0, order[np.arange(idx.size), best], -1)
            cand[:, b, :kk] = order
            score[:, b, :kk] = sc
        trace.append((idx.copy(), cand, score))
        for q, f in enumerate(idx):
            fl = flip_n[q][flip_n[q] >= 0]
            if fl.size == 0 or (prev[f] is not None and np.array_equal(fl, prev[f])):
                live[f] = False
                continue
            z[f, fl] ^= 1
            prev[f] = fl
            rounds[f] = t + 1
        t += 1
    return z, rounds, ok, trace


def trace_of_frame(trace, f):
    """Per round run by frame f: (candidates [G'][k'], scores [G'][k'])."""
    out = []
    for idx, cand, score in trace:
        q = np.nonzero(idx == f)[0]
        if q.size == 0:
            break
        out.append((cand[q[0]], score[q[0]]))
    return out
