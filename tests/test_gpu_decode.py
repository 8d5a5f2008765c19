"""Parity of the HIP decoder (fwbf_decode through the C ABI) with the CPU
oracle: every output (packed hard decisions, rounds, syndrome flag) must be
bit-exact, for integer and float inputs, every weight and selection variant,
exhaustive single and double error patterns, ties, subnormals, signed zeros,
degenerate calls and the sizes of the workloads."""
import numpy as np
import pytest

import oracle as O
from conftest import CODES
from gpu_util import assert_same, gpu_decode, need_gpu, oracle_decode, torch
from paper_1206_3362_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codes():
    need_gpu()
    from paper_1206_3362_amd import fwbf
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = (fwbf.Code.from_seed(*CODES[name]), O.Code.from_seed(*CODES[name]))
        return cache[name]
    return get


def run_both(codes, name, y, **kw):
    g, o = codes(name)
    print(f"case {name} dtype={y.dtype} F={y.shape[0]} {kw}", flush=True)
    return gpu_decode(g, y, **kw), oracle_decode(o, y, **kw)


def test_small_workload_wbf_f32(codes):
    """N=186 (3,6) code, all-zero codeword, 3 dB, float, WBF, alpha 0.2, G=6,
    50 rounds, 1000 frames."""
    g, o = codes("n186")
    y = synth.awgn_frames(g.N, 1000, synth.sigma_for(3.0, g.rate), 100, None, np.float32)
    a, b = run_both(codes, "n186", y, weights=0, groups=6, max_iter=50, alpha=0.2)
    assert_same(a, b, "n186 wbf f32")


@pytest.mark.parametrize("ebn0", [2.0, 4.0, 6.0])
def test_n1008_int8_codewords(codes, ebn0):
    g, o = codes("n1008")
    F = 4096
    pool = o.encode(seed=77, first=0, count=256)
    cb = O.unpack(pool[np.arange(F) % 256], g.N)
    y = synth.awgn_frames(g.N, F, synth.sigma_for(ebn0, g.rate), int(ebn0 * 10), cb, np.int8)
    a, b = run_both(codes, "n1008", y, weights=2, groups=8, max_iter=100, alpha_num=1, alpha_den=5)
    assert_same(a, b, f"n1008 i8 {ebn0}dB")


VARIANTS = [dict(weights=w, alpha=0.2, alpha_num=1, alpha_den=5) for w in (0, 1, 2)]
SELECTS = [dict(select=0, groups=1), dict(select=0, groups=8), dict(select=0, groups=126),
           dict(select=0, groups=1008), dict(select=1), dict(select=2, lam=1),
           dict(select=2, lam=10)]


@pytest.mark.parametrize("dt", [np.float32, np.int8, np.int16])
@pytest.mark.parametrize("sel", SELECTS, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_variants_n1008(codes, dt, sel):
    g, o = codes("n1008")
    F = 512
    y = synth.awgn_frames(g.N, F, synth.sigma_for(5.0, g.rate), 5, None, dt)
    for v in VARIANTS:
        a, b = run_both(codes, "n1008", y, max_iter=60, **v, **sel)
        assert_same(a, b, f"{dt} {sel} {v}")


@pytest.mark.parametrize("G", [1, 2, 6, 31, 186])
def test_exhaustive_single_and_double_errors_n186(codes, G):
    g, o = codes("n186")
    singles = [[e] for e in range(g.N)]
    doubles = [[a, b] for a in range(g.N) for b in range(a + 1, g.N)]
    for dt, A in ((np.int8, 16), (np.float32, 1.0)):
        y = synth.error_pattern_frames(g.N, singles + doubles, A, dt)
        for v in VARIANTS:
            a, b = run_both(codes, "n186", y, groups=G, max_iter=50, **v)
            assert_same(a, b, f"n186 patterns G={G} {dt} {v}")
        if G == 6:
            assert (a[1][:g.N] == 1).all() and (a[2][:g.N] == 1).all()


def test_exhaustive_single_errors_n1008(codes):
    g, o = codes("n1008")
    y = synth.error_pattern_frames(g.N, [[e] for e in range(g.N)], 16, np.int8)
    for G in (1, 8, 126, 1008):
        a, b = run_both(codes, "n1008", y, groups=G, max_iter=100)
        assert_same(a, b, f"n1008 singles G={G}")
        assert (a[1] == 1).all() and (a[0] == 0).all()


@pytest.mark.parametrize("kind", ["ties_f32", "ties_i8", "ties_i16", "subnormal"])
def test_ties_zeros_subnormals(codes, kind):
    g, o = codes("n1008")
    F = 512
    if kind == "subnormal":
        y = synth.subnormal_frames(g.N, F, 3)
    else:
        dt = {"ties_f32": np.float32, "ties_i8": np.int8, "ties_i16": np.int16}[kind]
        y = synth.tie_heavy_frames(g.N, F, 9, dt)
    for sel in (dict(select=0, groups=8), dict(select=1), dict(select=2, lam=5)):
        for v in VARIANTS:
            a, b = run_both(codes, "n1008", y, max_iter=40, **v, **sel)
            assert_same(a, b, f"{kind} {sel} {v}")


def test_cycle_exit_is_exact(codes):
    """Outputs with the repeated-state shortcut equal those of running every
    round (both on the GPU) and the oracle's."""
    g, o = codes("n1008")
    y = synth.awgn_frames(g.N, 2048, synth.sigma_for(3.0, g.rate), 31, None, np.int8)
    for sel in (dict(select=0, groups=8), dict(select=1), dict(select=2, lam=4)):
        fast = gpu_decode(g, y, max_iter=57, **sel)
        slow = gpu_decode(g, y, max_iter=57, flags=1, **sel)
        assert_same(fast, slow, f"shortcut {sel}")
        assert_same(fast, oracle_decode(o, y, max_iter=57, **sel), f"oracle {sel}")


@pytest.mark.parametrize("dt", [np.int8, np.int16])
def test_specialised_and_generic_kernels_agree(codes, dt):
    """The one-wave integer kernel (regular (3,6) codes) and the general
    kernel give identical outputs, equal to the oracle's."""
    g, o = codes("n1008")
    y = synth.awgn_frames(g.N, 2048, synth.sigma_for(4.5, g.rate), 41, None, dt)
    for sel in (dict(select=0, groups=1), dict(select=0, groups=8), dict(select=0, groups=63),
                dict(select=0, groups=126), dict(select=0, groups=1008), dict(select=1)):
        for v in VARIANTS:
            fast = gpu_decode(g, y, max_iter=80, **sel, **v)
            gen = gpu_decode(g, y, max_iter=80, flags=2, **sel, **v)
            assert_same(fast, gen, f"fast vs generic {sel} {v}")
            assert_same(fast, oracle_decode(o, y, max_iter=80, **sel, **v), f"oracle {sel} {v}")


RAGGED = {"n1008": (4.0, [5, 10, 11, 37, 50, 61]), "n186": (3.0, [4, 5, 7])}


@pytest.mark.parametrize("name", ["n1008", "n186"])
@pytest.mark.parametrize("dt", [np.int8, np.int16])
def test_specialised_kernel_ragged_blocks(codes, name, dt):
    """The one-wave kernel that the benchmark times, pinned with
    FLAG_SPECIALISED_ONLY, on block counts that do not divide N: a short
    last block (the null-metric padding of footnote 1), fewer blocks than G
    where ceil(N/p) < G (N = 1008: G = 37 gives 36 blocks of 28, G = 50 gives
    48 of 21), and strided classes of unequal size; every weight variant,
    against the oracle.  N = 186 adds every single-error pattern (one round
    for any blocks, by the closed form)."""
    g, o = codes(name)
    eb, Gs = RAGGED[name]
    F = 512
    y = synth.awgn_frames(g.N, F, synth.sigma_for(eb, g.rate), 61, None, dt)
    if name == "n186":
        A = 16 if dt == np.int8 else 256
        y = np.concatenate([y, synth.error_pattern_frames(g.N, [[e] for e in range(g.N)], A, dt)])
    for G in Gs:
        for sel in (0, 3):
            for v in VARIANTS:
                kw = dict(select=sel, groups=G, max_iter=60, **v)
                a = gpu_decode(g, y, flags=4, **kw)
                assert_same(a, oracle_decode(o, y, **kw), f"{name} {dt} G={G} select={sel} {v}")
                if name == "n186":
                    assert (a[1][F:] == 1).all() and (a[2][F:] == 1).all()


def test_specialised_only_flag_refuses_other_shapes(codes):
    """G = 100 on N = 1008 (92 blocks of 11) does not fit one wave's lanes:
    with FLAG_SPECIALISED_ONLY the call fails and enqueues nothing."""
    from paper_1206_3362_amd import fwbf
    g, o = codes("n1008")
    y = torch.zeros((4, g.N), dtype=torch.int8, device="cuda")
    with pytest.raises(fwbf.FwbfError, match="E_UNSUPPORTED"):
        fwbf.decode(g, y, fwbf.DecodeParams(dtype=fwbf.I8, groups=100, flags=4))
    with pytest.raises(fwbf.FwbfError, match="E_UNSUPPORTED"):
        fwbf.decode(g, y.float(), fwbf.DecodeParams(dtype=fwbf.F32, groups=8, flags=4))


def _executed_rounds(ocode, y, **kw):
    """Rounds run before the decoder's state repeats, from the oracle's
    literal trace: the first round with no flip or with the previous
    round's flips; a frame that never repeats runs all its rounds."""
    out = []
    for f in range(y.shape[0]):
        tr = O.decode_trace(ocode, y[f], **kw)
        fl = [sorted(x.tolist()) for x in tr["flips"]]
        ex = tr["iters"]
        for r in range(len(fl)):
            if not fl[r] or (r > 0 and fl[r] == fl[r - 1]):
                ex = r
                break
        out.append(ex)
    return np.array(out)


def test_executed_rounds_flag(codes, eg):
    """FLAG_EXECUTED_ROUNDS reports the rounds run before the state repeats
    (the work the repeated-state shortcut leaves) and changes nothing else:
    the specialised, general and cyclic kernels against the oracle's trace."""
    cases = [("n1008", np.int8, 4.0, dict(groups=8, max_iter=100), 0),
             ("n1008", np.int8, 4.0, dict(groups=8, max_iter=100), 2),
             ("n1008", np.int16, 3.0, dict(select=1, max_iter=70), 0),
             ("n186", np.float32, 3.0, dict(groups=6, max_iter=50, weights=0), 0)]
    for name, dt, eb, kw, extra in cases:
        g, o = codes(name)
        y = synth.awgn_frames(g.N, 192, synth.sigma_for(eb, g.rate), 71, None, dt)
        base = gpu_decode(g, y, flags=extra, **kw)
        ex = gpu_decode(g, y, flags=extra | 8, **kw)
        assert np.array_equal(base[0], ex[0]) and np.array_equal(base[2], ex[2])
        okm = base[2] == 1
        assert np.array_equal(base[1][okm], ex[1][okm])
        m = dict(kw)
        m["G"] = m.pop("groups", 8)
        want = _executed_rounds(o, y, **m)
        assert np.array_equal(ex[1], want), (name, dt, kw, extra)
        assert (ex[1] < base[1]).any()
    ge, oe = eg(4)
    y = synth.awgn_frames(ge.N, 128, synth.sigma_for(3.0, ge.rate), 72, None, np.float32)
    base = gpu_decode(ge, y, groups=16, max_iter=30, alpha=1.0)
    ex = gpu_decode(ge, y, groups=16, max_iter=30, alpha=1.0, flags=8)
    assert np.array_equal(base[0], ex[0]) and np.array_equal(base[2], ex[2])
    assert np.array_equal(ex[1], _executed_rounds(oe, y, G=16, max_iter=30, alpha=1.0))


def test_degenerate_calls(codes):
    from paper_1206_3362_amd import fwbf
    g, o = codes("n186")
    y = synth.awgn_frames(g.N, 64, 0.9, 2, None, np.int8)
    a, b = run_both(codes, "n186", y, groups=6, max_iter=0)
    assert_same(a, b, "max_iter 0")
    a, b = run_both(codes, "n186", y, groups=6, max_iter=1)
    assert_same(a, b, "max_iter 1")
    # strided frames: every other row of a wider buffer
    wide = np.zeros((64, 256), np.int8)
    wide[:, :g.N] = y
    yd = torch.from_numpy(wide).to("cuda")[:, :g.N]
    z, it, ok = fwbf.decode(g, yd, fwbf.DecodeParams(dtype=fwbf.I8, groups=6))
    zo, ito, oko = O.decode(o, y, G=6)
    assert np.array_equal(z.cpu().numpy().view(np.uint32), zo)
    assert np.array_equal(it.cpu().numpy(), ito)
    # F = 0 is a no-op
    z, it, ok = fwbf.decode(g, yd[:0], fwbf.DecodeParams(dtype=fwbf.I8, groups=6))
    assert z.shape[0] == 0
    # threads per frame does not change results
    for T in (64, 128, 256):
        a = gpu_decode(g, y, groups=6, threads_per_frame=T)
        assert_same(a, b if False else oracle_decode(o, y, groups=6), f"T={T}")


@pytest.mark.parametrize("name,dt,G,F,ebn0", [
    ("n4032", np.float32, 32, 256, 4.0),
    ("n8000", np.float32, 64, 128, 5.0),
    ("n32400", np.int16, 64, 32, 6.0),
])
def test_large_codes(codes, name, dt, G, F, ebn0):
    g, o = codes(name)
    pool = o.encode(seed=3, first=0, count=8)
    cb = O.unpack(pool[np.arange(F) % 8], g.N)
    y = synth.awgn_frames(g.N, F, synth.sigma_for(ebn0, g.rate), 17, cb, dt)
    for sel in (dict(select=0, groups=G), dict(select=0, groups=1)):
        a, b = run_both(codes, name, y, max_iter=100, **sel)
        assert_same(a, b, f"{name} {sel}")


@pytest.fixture(scope="module")
def eg():
    need_gpu()
    from paper_1206_3362_amd import fwbf
    cache = {}

    def get(s):
        if s not in cache:
            t = synth.eg_code_text(s)
            cache[s] = (fwbf.Code.from_text(t), O.Code.from_text(t))
        return cache[s]
    return get


EG_SELECTS = [dict(select=0, groups=11), dict(select=0, groups=33), dict(select=0, groups=1),
              dict(select=0, groups=1023), dict(select=1), dict(select=2, lam=10)]


@pytest.mark.parametrize("dt", [np.float32, np.int8, np.int16])
@pytest.mark.parametrize("sel", EG_SELECTS, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_eg1023_parity(eg, dt, sel):
    """EG(1023,781) (one 1023 x 1023 circulant of weight 32, Section V),
    random codewords at 3.0 and 4.5 dB, K_max = 10 as in Tab. 1, every
    weight variant: bit-exact with the oracle."""
    g, o = eg(5)
    F = 512
    pool = o.encode(seed=21, first=0, count=64)
    cb = O.unpack(pool[np.arange(F) % 64], g.N)
    for ebn0 in (3.0, 4.5):
        y = synth.awgn_frames(g.N, F, synth.sigma_for(ebn0, g.rate), int(ebn0 * 10) + 5, cb, dt)
        for w in (0, 1, 2):
            kw = dict(weights=w, alpha=0.4, alpha_num=2, alpha_den=5, max_iter=10, **sel)
            print(f"case eg1023 dtype={np.dtype(dt).name} ebn0={ebn0} {kw}", flush=True)
            assert_same(gpu_decode(g, y, **kw), oracle_decode(o, y, **kw), f"eg1023 {ebn0} {kw}")


@pytest.mark.parametrize("dt", [np.float32, np.int8])
def test_eg255_parity_and_error_patterns(eg, dt):
    """EG(255,175): noisy frames at 3.5 dB with up to 100 rounds, plus frames
    of up to 8 uniform-magnitude errors (decoded in max-errors-per-block
    rounds, a closed form the oracle is pinned to)."""
    g, o = eg(4)
    rng = np.random.default_rng(4)
    F = 1024
    y = synth.awgn_frames(g.N, F, synth.sigma_for(3.5, g.rate), 35, None, dt)
    pats = [sorted(rng.choice(g.N, size=1 + f % 8, replace=False).tolist()) for f in range(256)]
    ye = synth.error_pattern_frames(g.N, pats, 1.0 if dt == np.float32 else 16, dt)
    for G in (1, 5, 16, 255):
        for w in (0, 2):
            kw = dict(weights=w, groups=G, alpha=1.0, alpha_num=1, alpha_den=1, max_iter=100)
            print(f"case eg255 dtype={np.dtype(dt).name} {kw}", flush=True)
            assert_same(gpu_decode(g, y, **kw), oracle_decode(o, y, **kw), f"eg255 {kw}")
            a = gpu_decode(g, ye, **kw)
            assert_same(a, oracle_decode(o, ye, **kw), f"eg255 patterns {kw}")
            assert (a[2] == 1).all()


def _cyclic_text(N, W, seed):
    rng = np.random.default_rng(seed)
    sh = sorted(rng.choice(N, size=W, replace=False).tolist())
    return f"qc-ldpc v1\nZ {N}\nbase 1 1\n{','.join(map(str, sh))}\n"


@pytest.mark.parametrize("text", [synth.eg_code_text(2), synth.eg_code_text(3), _cyclic_text(2047, 9, 1),
                                  _cyclic_text(1500, 5, 2), _cyclic_text(130, 64, 3)],
                         ids=["eg15", "eg63", "cyc2047w9", "cyc1500w5", "cyc130w64"])
@pytest.mark.parametrize("dt", [np.float32, np.int8, np.int16])
def test_cyclic_kernel_shapes(text, dt):
    """Single-circulant codes of several lengths (1 to 32 windows of 64 bits,
    ragged last window) and weights 4 to 64: the cyclic kernel and the
    generic kernel both match the oracle bit for bit, for block counts 1, 7
    and N (one bit per block) and the single global choice."""
    need_gpu()
    from paper_1206_3362_amd import fwbf
    g, o = fwbf.Code.from_text(text), O.Code.from_text(text)
    F = 384
    rate = max(o.K, 1) / o.N
    y = synth.awgn_frames(g.N, F, synth.sigma_for(4.0, rate), g.N, None, dt)
    for sel in (dict(select=0, groups=1), dict(select=0, groups=7), dict(select=0, groups=g.N),
                dict(select=1)):
        for w in (0, 2):
            kw = dict(weights=w, alpha=0.6, alpha_num=3, alpha_den=5, max_iter=25, **sel)
            print(f"case N={g.N} W={g.dv_max} dtype={np.dtype(dt).name} {kw}", flush=True)
            want = oracle_decode(o, y, **kw)
            assert_same(gpu_decode(g, y, **kw), want, f"cyclic {kw}")
            assert_same(gpu_decode(g, y, flags=fwbf.FLAG_GENERIC_KERNEL, **kw), want, f"generic {kw}")


@pytest.mark.parametrize("dt", [np.float32, np.int8, np.int16])
@pytest.mark.parametrize("G", [7, 8, 126, 1008])
def test_strided_blocks_n1008(codes, dt, G):
    """Strided blocks (block g = {n : n mod G = g}): the specialised and the
    general kernel against the oracle, with G dividing N or not."""
    from paper_1206_3362_amd import fwbf
    g, o = codes("n1008")
    F = 1024
    pool = o.encode(seed=5, first=0, count=64)
    cb = O.unpack(pool[np.arange(F) % 64], g.N)
    y = synth.awgn_frames(g.N, F, synth.sigma_for(4.0, g.rate), G, cb, dt)
    kw = dict(select=fwbf.STRIDED, groups=G, weights=2, alpha=0.2, alpha_num=1, alpha_den=5, max_iter=100)
    print(f"case n1008 strided dtype={np.dtype(dt).name} G={G}", flush=True)
    want = oracle_decode(o, y, **kw)
    assert_same(gpu_decode(g, y, **kw), want, f"strided {kw}")
    assert_same(gpu_decode(g, y, flags=fwbf.FLAG_GENERIC_KERNEL, **kw), want, f"strided generic {kw}")


def test_strided_blocks_eg255(eg):
    from paper_1206_3362_amd import fwbf
    g, o = eg(4)
    y = synth.awgn_frames(g.N, 512, synth.sigma_for(3.5, g.rate), 12, None, np.float32)
    for G in (5, 16, 100):
        kw = dict(select=fwbf.STRIDED, groups=G, weights=2, alpha=1.0, max_iter=20)
        print(f"case eg255 strided G={G}", flush=True)
        assert_same(gpu_decode(g, y, **kw), oracle_decode(o, y, **kw), f"eg255 strided {kw}")


def _irregular_text(mb, nb, Z, seed):
    """A base with zero blocks and blocks of two shifts (every column and row
    keeps at least one and two entries): rows and columns of unequal degree."""
    rng = np.random.default_rng(seed)
    while True:
        cells = []
        for _ in range(mb * nb):
            u = rng.random()
            k = 0 if u < 0.25 else (2 if u > 0.85 else 1)
            cells.append(sorted(rng.choice(Z, size=k, replace=False).tolist()))
        cols = [sum(len(cells[i * nb + j]) for i in range(mb)) for j in range(nb)]
        rows = [sum(len(cells[i * nb + j]) for j in range(nb)) for i in range(mb)]
        if min(cols) >= 1 and min(rows) >= 2:
            break
    toks = [",".join(map(str, c)) if c else "-1" for c in cells]
    lines = [" ".join(toks[i * nb:(i + 1) * nb]) for i in range(mb)]
    return f"qc-ldpc v1\nZ {Z}\nbase {mb} {nb}\n" + "\n".join(lines) + "\n"


@pytest.mark.parametrize("dt", [np.float32, np.int8, np.int16])
@pytest.mark.parametrize("T", [64, 256])
def test_irregular_multishift_general_kernel(dt, T):
    """The general kernel on an irregular base (zero blocks, two-shift blocks,
    Z = 97 not a multiple of 64) at one and four wavefronts per frame: every
    weight rule and selection, bit-exact with the oracle. (At four wavefronts
    integer frames list every toggle and skip the claim pass, and blocks held
    by one wavefront flip within the choice phase.)"""
    need_gpu()
    from paper_1206_3362_amd import fwbf
    text = _irregular_text(4, 14, 97, 11)
    g, o = fwbf.Code.from_text(text), O.Code.from_text(text)
    assert "-1" in text and any("," in t for t in text.split())  # zero and two-shift blocks
    rate = max(o.K, 1) / o.N
    # 32 frames at 3 dB (most fail) and 32 at 6 dB (about 80% decode)
    y = np.concatenate([synth.awgn_frames(g.N, 32, synth.sigma_for(eb, rate), T + int(eb), None, dt)
                        for eb in (3.0, 6.0)])
    sels = [dict(select=fwbf.GROUPS, groups=1), dict(select=fwbf.GROUPS, groups=5),
            dict(select=fwbf.GROUPS, groups=97), dict(select=fwbf.SINGLE), dict(select=fwbf.TOPL, lam=4),
            dict(select=fwbf.STRIDED, groups=7)]
    for sel in sels:
        for w in (0, 1, 2):
            kw = dict(weights=w, alpha=0.3, alpha_num=1, alpha_den=3, max_iter=40, **sel)
            print(f"case irregular N={g.N} dtype={np.dtype(dt).name} T={T} {kw}", flush=True)
            assert_same(gpu_decode(g, y, threads_per_frame=T, **kw), oracle_decode(o, y, **kw), f"irregular T={T} {kw}")
