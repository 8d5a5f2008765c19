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


def check_properties(ocode, z, it, ok, max_iter, what):
    """Syndrome flag == [H z = 0] and ok == 0 -> rounds == K_max, on every frame."""
    rp, rb = ocode.rows()
    M, N = ocode.M, ocode.N
    deg = np.diff(rp)
    members = np.full((M, int(deg.max())), N, np.int64)  # column N is a zero pad
    for m in range(M):
        members[m, :deg[m]] = rb[rp[m]:rp[m + 1]]
    mem = torch.from_numpy(members).to(z.device)
    F, W = z.shape
    sh = torch.arange(32, device=z.device, dtype=torch.int32)
    chunk = max(1, (1 << 28) // (M * members.shape[1]))
    zero_syn = torch.empty(F, dtype=torch.bool, device=z.device)
    for f0 in range(0, F, chunk):
        zc = z[f0:f0 + chunk]
        bits = ((zc.unsqueeze(-1) >> sh) & 1).to(torch.uint8).reshape(zc.shape[0], W * 32)[:, :N]
        bits = torch.cat([bits, torch.zeros_like(bits[:, :1])], 1)
        par = bits[:, mem].sum(-1, dtype=torch.int32) & 1
        zero_syn[f0:f0 + chunk] = par.sum(1) == 0
    okb = ok.bool()
    n_bad = int((okb != zero_syn).sum())
    assert n_bad == 0, f"{what}: {n_bad} frames whose flag disagrees with H z"
    n_short = int(((~okb) & (it != max_iter)).sum())
    assert n_short == 0, f"{what}: {n_short} failed frames stopped before K_max"
    assert int(((it < 0) | (it > max_iter)).sum()) == 0, f"{what}: rounds outside [0, K_max]"
