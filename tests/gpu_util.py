"""Helpers shared by the GPU parity tests (no decoder arithmetic here)."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")

DT_NP = {0: np.float32, 1: np.int8, 2: np.int16}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def gpu_decode(code, y, **kw):
    from paper_1206_3362_amd import fwbf
    yd = torch.from_numpy(np.ascontiguousarray(y)).to("cuda")
    dt = {np.dtype(np.float32): fwbf.F32, np.dtype(np.int8): fwbf.I8,
          np.dtype(np.int16): fwbf.I16}[y.dtype]
    p = fwbf.DecodeParams(dtype=dt, **kw)
    z, it, ok = fwbf.decode(code, yd, p)
    torch.cuda.synchronize()
    return z.cpu().numpy().view(np.uint32), it.cpu().numpy(), ok.cpu().numpy()


def oracle_decode(ocode, y, **kw):
    m = dict(kw)
    if "groups" in m:
        m["G"] = m.pop("groups")
    if "lam" in m:
        pass
    m.pop("threads_per_frame", None)
    flags = m.pop("flags", 0)
    return O.decode(ocode, y, **m)


def assert_same(g, o, what=""):
    zg, ig, kg = g
    zo, io, ko = o
    bad = np.nonzero((zg != zo).any(1) | (ig != io) | (kg != ko))[0]
    assert bad.size == 0, (f"{what}: {bad.size} frames differ, first {bad[:8].tolist()}; "
                           f"gpu iters {ig[bad[:4]].tolist()} oracle {io[bad[:4]].tolist()}")
