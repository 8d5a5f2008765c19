"""Host logic of the autotuner: the frame-error constraint (two-proportion
test) and the batch tuner's choices, with the decoder calls replaced by
tables."""
from paper_1206_3362_amd import autotune


def test_fer_constraint():
    # lower or equal error rate is always admissible
    assert autotune.fer_admissible(10, 1000, 50, 1000)
    assert autotune.fer_admissible(50, 1000, 50, 1000)
    # p1 = 0.06, p2 = 0.05, pooled 0.055: 3 sigma = 3*sqrt(.055*.945*2/1000) = 0.0306
    assert autotune.fer_admissible(60, 1000, 50, 1000)
    assert not autotune.fer_admissible(90, 1000, 50, 1000)
    # zero errors on both sides
    assert autotune.fer_admissible(0, 100, 0, 100)
    assert not autotune.fer_admissible(10, 100, 0, 100)


class _FakeCode:
    def __init__(self, N):
        self.N = N


def _fake_library(monkeypatch, errs, ms_of_G, shape_ms):
    """Replaces the decode calls the batch tuner makes: frame errors and
    times come from the tables given (keyed by (N, G) and by
    (threads_per_frame, blocks_per_cu); a shape missing from shape_ms is
    rejected by the library)."""
    import torch
    from paper_1206_3362_amd import fwbf
    cur = {}

    def decode(code, y, p):
        cur["key"] = (code.N, p.groups)
        return (torch.zeros(1), torch.zeros(1), torch.zeros(1))

    def decode_into(code, y, p, z, it, ok):
        cur["key"] = (code.N, p.groups)

    def count(N, z, pool, f0, it, ok, max_iter):
        return {"frame_err": errs[cur["key"]]}

    def decode_batched(batch, threads_per_frame=0, blocks_per_cu=0, workspace=None):
        key = (threads_per_frame, blocks_per_cu)
        if key not in shape_ms:
            raise fwbf.FwbfError(fwbf.E_UNSUPPORTED, "shape")
        cur["key"] = key

    monkeypatch.setattr(fwbf, "decode", decode)
    monkeypatch.setattr(fwbf, "decode_into", decode_into)
    monkeypatch.setattr(fwbf, "count", count)
    monkeypatch.setattr(fwbf, "decode_batched", decode_batched)

    def time_ms(fn, repeats):
        fn()
        return ms_of_G.get(cur["key"], shape_ms.get(cur["key"]))

    monkeypatch.setattr(autotune, "_time_ms", time_ms)


def test_batch_tuner_selection_rules(monkeypatch):
    import torch
    from paper_1206_3362_amd import fwbf
    n = 1000
    # job A (N=100, reference G=8): G=4 is fastest but fails the FER test, G=16 is
    # admissible and faster than the reference -> 16
    # job B (N=200, reference G=32): no candidate is admissible -> the reference G
    errs = {(100, 8): 50, (100, 4): 90, (100, 16): 55, (200, 32): 10, (200, 64): 80}
    ms_of_G = {(100, 8): 3.0, (100, 4): 1.0, (100, 16): 2.0, (200, 32): 5.0, (200, 64): 1.0}
    shape_ms = {(0, 0): 9.0, (0, 2): 7.0, (128, 0): 8.0}
    _fake_library(monkeypatch, errs, ms_of_G, shape_ms)
    jobs = [(_FakeCode(100), torch.zeros(n, 100), None, fwbf.DecodeParams(groups=8)),
            (_FakeCode(200), torch.zeros(n, 200), None, fwbf.DecodeParams(groups=32))]
    r = autotune.tune_batch(jobs, [(4, 16), (64,)], tune_frames=n, widths=(0, 128, 256), blocks=(0, 2))
    assert [p.groups for p in r["params"]] == [16, 32]
    assert (r["threads_per_frame"], r["blocks_per_cu"], r["ms"]) == (0, 2, 7.0)
    assert len(r["shape_table"]) == 3  # (128, 2), (256, 0), (256, 2) were rejected
    adm = {(row["N"], row["G"]): row["admissible"] for row in r["g_table"]}
    assert adm == {(100, 4): False, (100, 16): True, (200, 64): False}


def test_batch_tuner_no_shape_runs(monkeypatch):
    import pytest
    import torch
    from paper_1206_3362_amd import fwbf
    _fake_library(monkeypatch, {(100, 8): 1}, {(100, 8): 1.0}, {})
    jobs = [(_FakeCode(100), torch.zeros(10, 100), None, fwbf.DecodeParams(groups=8))]
    with pytest.raises(fwbf.FwbfError):
        autotune.tune_batch(jobs, [()], tune_frames=10, widths=(0,), blocks=(0,))
