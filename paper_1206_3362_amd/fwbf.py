"""Thin ctypes binding of libfwbf.so (include/fwbf.h).

Argument marshalling only: device buffers are torch tensors on the current
HIP device, passed to the library as raw pointers together with
``torch.cuda.current_stream()``.  Every step of decoding runs in the
library's HIP kernels; this module never computes anything itself and raises
``FwbfError`` if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfwbf.so")

F32, I8, I16 = 0, 1, 2
WBF, MWBF, IMWBF = 0, 1, 2
GROUPS, SINGLE, TOPL, STRIDED = 0, 1, 2, 3
FLAG_NO_CYCLE_EXIT = 1
FLAG_GENERIC_KERNEL = 2
FLAG_SPECIALISED_ONLY = 4
FLAG_EXECUTED_ROUNDS = 8

OK, E_INVALID, E_PARSE, E_GIRTH, E_UNSUPPORTED, E_NOMEM, E_HIP = 0, -1, -2, -3, -4, -5, -6
_NAMES = {-1: "E_INVALID", -2: "E_PARSE", -3: "E_GIRTH", -4: "E_UNSUPPORTED", -5: "E_NOMEM",
          -6: "E_HIP"}

# every symbol include/fwbf.h declares
EXPORTS = [
    "fwbf_code_from_text", "fwbf_code_from_seed", "fwbf_code_to_text", "fwbf_code_dims",
    "fwbf_code_shifts", "fwbf_code_has_4cycle", "fwbf_code_free", "fwbf_code_info_positions",
    "fwbf_encode", "fwbf_channel", "fwbf_decode", "fwbf_count", "fwbf_last_error", "fwbf_version",
    "fwbf_scorer_size", "fwbf_decode_learned", "fwbf_scorer_grad", "fwbf_adam",
    "fwbf_decode_batched", "fwbf_sweep_create", "fwbf_sweep_launch", "fwbf_sweep_counters",
    "fwbf_sweep_free", "fwbf_decode_minsum", "fwbf_sweep_outputs", "fwbf_decode_batched_noalloc",
]


class FwbfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("weights", C.c_int32), ("select", C.c_int32),
                ("groups", C.c_int32), ("lambda_", C.c_int32), ("max_iter", C.c_int32),
                ("alpha", C.c_float), ("alpha_num", C.c_int32), ("alpha_den", C.c_int32),
                ("threads_per_frame", C.c_int32), ("flags", C.c_uint32)]


class MinsumParams(C.Structure):
    _fields_ = [("offset", C.c_int32), ("c", C.c_float), ("max_iter", C.c_int32),
                ("threads_per_frame", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("code", C.c_void_p), ("params", C.c_void_p), ("y_dev", C.c_void_p),
                ("F", C.c_int64), ("y_stride", C.c_int64), ("z_dev", C.c_void_p),
                ("iters_dev", C.c_void_p), ("ok_dev", C.c_void_p)]


class LearnedParams(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("groups", C.c_int32), ("topk", C.c_int32),
                ("scale", C.c_float)]


# fwbf_record (12 bytes)
RECORD_DTYPE = np.dtype([("S", "<i4"), ("a", "<u2"), ("n", "<u2"), ("u", "u1"), ("label", "u1"),
                         ("valid", "u1"), ("pad", "u1")])
assert RECORD_DTYPE.itemsize == 12


def record_slots(groups: int, topk: int) -> int:
    """Proposal slots per round in the record layout (FWBF_RECORD_SLOTS)."""
    return 32 * ((groups * topk + 31) // 32)


_lib = None


def lib():
    """Load libfwbf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FwbfError(E_INVALID, f"{LIB_PATH} not built (run __graft_entry__.build())")
        # torch owns the device: bring it up before the library (and its HIP
        # code objects) is loaded into the process
        torch = _torch()
        if torch.cuda.is_available():
            torch.cuda.init()
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int, C.c_int64, C.c_uint64
        L.fwbf_last_error.restype = C.c_char_p
        L.fwbf_version.restype = C.c_char_p
        L.fwbf_code_from_text.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.fwbf_code_from_seed.argtypes = [i32, i32, i32, u64, i32, C.POINTER(vp)]
        L.fwbf_code_to_text.argtypes = [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
        L.fwbf_code_dims.argtypes = [vp] + [C.POINTER(i32)] * 5
        L.fwbf_code_shifts.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), vp]
        L.fwbf_code_has_4cycle.argtypes = [vp]
        L.fwbf_code_free.argtypes = [vp]
        L.fwbf_code_free.restype = None
        L.fwbf_code_info_positions.argtypes = [vp, vp]
        L.fwbf_encode.argtypes = [vp, u64, i64, i64, vp]
        L.fwbf_channel.argtypes = [i32, i64, i64, vp, i64, u64, C.c_uint32, C.c_float, vp,
                                   C.c_float, i32, vp, i64, vp]
        L.fwbf_decode.argtypes = [vp, C.POINTER(Params), vp, i64, i64, vp, vp, vp, vp]
        L.fwbf_decode_minsum.argtypes = [vp, C.POINTER(MinsumParams), vp, i64, i64, vp, vp, vp, vp]
        L.fwbf_count.argtypes = [i32, i64, i64, vp, vp, i64, vp, vp, i32, vp, vp]
        L.fwbf_scorer_size.argtypes = [i32]
        L.fwbf_decode_learned.argtypes = [vp, C.POINTER(Params), C.POINTER(LearnedParams), vp, vp, i64,
                                          i64, vp, vp, vp, vp, vp, vp, i64, i64, vp]
        L.fwbf_scorer_grad.argtypes = [vp, i64, C.POINTER(LearnedParams), vp, C.c_float, vp, vp, vp,
                                       i64, vp]
        L.fwbf_adam.argtypes = [vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_float, C.c_float,
                                vp]
        L.fwbf_decode_batched.argtypes = [vp, i32, i32, i32, vp, C.c_size_t, vp]
        L.fwbf_decode_batched_noalloc.argtypes = [vp, i32, i32, i32, vp]
        L.fwbf_sweep_create.argtypes = [vp, C.POINTER(Params), vp, i32, i64, vp, i64, u64, C.c_float,
                                        C.POINTER(vp)]
        L.fwbf_sweep_launch.argtypes = [vp, vp]
        L.fwbf_sweep_counters.argtypes = [vp, vp, vp]
        L.fwbf_sweep_outputs.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.fwbf_sweep_free.argtypes = [vp]
        L.fwbf_sweep_free.restype = None
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise FwbfError(rc, lib().fwbf_last_error().decode())
    return rc


def version() -> str:
    return lib().fwbf_version().decode()


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Code:
    """A QC-LDPC code owned by the library (immutable)."""

    def __init__(self, handle: int):
        self._h = C.c_void_p(handle)
        d = [C.c_int() for _ in range(5)]
        _check(lib().fwbf_code_dims(self._h, C.byref(d[0]), C.byref(d[1]), None, C.byref(d[3]),
                                    C.byref(d[4])))
        self.N, self.M = d[0].value, d[1].value
        self.dv_max, self.dc_max = d[3].value, d[4].value
        self._K = None

    @classmethod
    def from_text(cls, text: str) -> "Code":
        h = C.c_void_p()
        _check(lib().fwbf_code_from_text(text.encode(), C.byref(h)))
        return cls(h.value)

    @classmethod
    def from_seed(cls, mb: int, nb: int, Z: int, seed: int, min_girth: int = 6) -> "Code":
        h = C.c_void_p()
        _check(lib().fwbf_code_from_seed(mb, nb, Z, seed, min_girth, C.byref(h)))
        return cls(h.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.fwbf_code_free(h)
            self._h = None

    @property
    def K(self) -> int:
        if self._K is None:
            k = C.c_int()
            _check(lib().fwbf_code_dims(self._h, None, None, C.byref(k), None, None))
            self._K = k.value
        return self._K

    @property
    def rate(self) -> float:
        return self.K / self.N

    def text(self) -> str:
        need = C.c_size_t()
        lib().fwbf_code_to_text(self._h, None, 0, C.byref(need))
        buf = C.create_string_buffer(need.value)
        _check(lib().fwbf_code_to_text(self._h, buf, need.value, None))
        return buf.value.decode()

    def shifts(self) -> np.ndarray:
        mb, nb, Z = C.c_int(), C.c_int(), C.c_int()
        _check(lib().fwbf_code_shifts(self._h, C.byref(mb), C.byref(nb), C.byref(Z), None))
        out = np.empty((mb.value, nb.value), np.int32)
        _check(lib().fwbf_code_shifts(self._h, None, None, None, _np_ptr(out)))
        self.Z = Z.value
        return out

    def has_4cycle(self) -> bool:
        return bool(_check_nonneg(lib().fwbf_code_has_4cycle(self._h)))

    def info_positions(self) -> np.ndarray:
        out = np.empty(self.K, np.int32)
        _check(lib().fwbf_code_info_positions(self._h, _np_ptr(out)))
        return out

    def encode(self, seed: int, first: int, count: int) -> np.ndarray:
        """Host-side seeded codeword pool, packed uint32 [count][ceil(N/32)]."""
        out = np.zeros((count, (self.N + 31) // 32), np.uint32)
        _check(lib().fwbf_encode(self._h, seed, first, count, _np_ptr(out) if count else None))
        return out


def _check_nonneg(rc):
    if rc < 0:
        raise FwbfError(rc, lib().fwbf_last_error().decode())
    return rc


@dataclass
class DecodeParams:
    dtype: int = I8
    weights: int = IMWBF
    select: int = GROUPS
    groups: int = 8
    lam: int = 1
    max_iter: int = 100
    alpha: float = 0.2
    alpha_num: int = 1
    alpha_den: int = 5
    threads_per_frame: int = 0
    flags: int = 0

    def c(self) -> Params:
        return Params(self.dtype, self.weights, self.select, self.groups, self.lam, self.max_iter,
                      self.alpha, self.alpha_num, self.alpha_den, self.threads_per_frame,
                      self.flags)


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    return {torch.float32: F32, torch.int8: I8, torch.int16: I16}[t.dtype]


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def decode_into(code: Code, y, params: DecodeParams, z, iters, ok):
    """Decode y[F][stride] (device tensor) into preallocated device outputs."""
    p = params.c()
    F = y.shape[0]
    stride = y.stride(0) if y.dim() == 2 else code.N
    _check(lib().fwbf_decode(code._h, C.byref(p), _ptr(y), F, stride, _ptr(z), _ptr(iters),
                             _ptr(ok), _stream()))


def decode(code: Code, y, params: DecodeParams | None = None, **kw):
    """Returns (z packed int32 [F][ceil(N/32)], iterations int32 [F], ok uint8 [F])."""
    torch = _torch()
    params = params or DecodeParams(dtype=_dtype_code(y), **kw)
    if params.dtype != _dtype_code(y):
        raise FwbfError(E_INVALID, "params.dtype does not match y")
    F = y.shape[0]
    dev = y.device
    z = torch.empty((F, (code.N + 31) // 32), dtype=torch.int32, device=dev)
    it = torch.empty(F, dtype=torch.int32, device=dev)
    ok = torch.empty(F, dtype=torch.uint8, device=dev)
    decode_into(code, y, params, z, it, ok)
    return z, it, ok


def decode_minsum_into(code: Code, y, z, iters, ok, *, offset: bool = False, c: float = 0.75,
                       max_iter: int = 20, threads_per_frame: int = 0):
    """Min-sum BP over float frames y[F][stride] into preallocated outputs."""
    p = MinsumParams(int(bool(offset)), c, max_iter, threads_per_frame)
    F = y.shape[0]
    stride = y.stride(0) if y.dim() == 2 else code.N
    _check(lib().fwbf_decode_minsum(code._h, C.byref(p), _ptr(y), F, stride, _ptr(z), _ptr(iters),
                                    _ptr(ok), _stream()))


def decode_minsum(code: Code, y, **kw):
    """Returns (z packed int32 [F][ceil(N/32)], iterations int32 [F], ok uint8 [F])."""
    torch = _torch()
    if y.dtype != torch.float32:
        raise FwbfError(E_INVALID, "min-sum takes float32 frames")
    F = y.shape[0]
    dev = y.device
    z = torch.empty((F, (code.N + 31) // 32), dtype=torch.int32, device=dev)
    it = torch.empty(F, dtype=torch.int32, device=dev)
    ok = torch.empty(F, dtype=torch.uint8, device=dev)
    decode_minsum_into(code, y, z, it, ok, **kw)
    return z, it, ok


def channel_into(code_N: int, y, f0: int, pool, seed: int, stream_id: int, sigma: float,
                 sigma_per_frame=None, scale: float = 1.0):
    F = y.shape[0]
    _check(lib().fwbf_channel(code_N, F, f0, _ptr(pool), 0 if pool is None else pool.shape[0],
                              seed, stream_id, sigma, _ptr(sigma_per_frame), scale,
                              _dtype_code(y), _ptr(y), y.stride(0), _stream()))


def channel(N: int, F: int, f0: int, pool, seed: int, stream_id: int, sigma: float,
            dtype=None, scale: float = 1.0, sigma_per_frame=None, device="cuda"):
    torch = _torch()
    dtype = dtype or torch.float32
    y = torch.empty((F, N), dtype=dtype, device=device)
    channel_into(N, y, f0, pool, seed, stream_id, sigma, sigma_per_frame, scale)
    return y


def count_into(N: int, z, pool, f0: int, iters, ok, max_iter: int, counters):
    F = z.shape[0]
    _check(lib().fwbf_count(N, F, f0, _ptr(z), _ptr(pool), 0 if pool is None else pool.shape[0],
                            _ptr(iters), _ptr(ok), max_iter, _ptr(counters), _stream()))


def count(N: int, z, pool, f0: int, iters, ok, max_iter: int):
    torch = _torch()
    counters = torch.zeros(7 + max_iter, dtype=torch.int64, device=z.device)
    count_into(N, z, pool, f0, iters, ok, max_iter, counters)
    c = counters.cpu().numpy()
    return dict(bit_err=int(c[0]), frame_err=int(c[1]), undetected=int(c[2]),
                iter_sum=int(c[3]), frames=int(c[4]), syn_ok=int(c[5]), hist=c[6:])


# ---- learned scorer -------------------------------------------------------

def scorer_size(rounds: int) -> int:
    return _check_nonneg(lib().fwbf_scorer_size(rounds))


def decode_learned_into(code: Code, y, plain: DecodeParams, lp: LearnedParams, scorer, z, iters, ok,
                        learned_ok=None, records=None, pool=None, f0: int = 0):
    """Learned pass then plain FWBF for the frames it leaves undecoded."""
    p = plain.c()
    F = y.shape[0]
    _check(lib().fwbf_decode_learned(code._h, C.byref(p), C.byref(lp), _ptr(scorer), _ptr(y), F,
                                     y.stride(0), _ptr(z), _ptr(iters), _ptr(ok), _ptr(learned_ok),
                                     _ptr(records), _ptr(pool),
                                     0 if pool is None else pool.shape[0], f0, _stream()))


def decode_learned(code: Code, y, plain: DecodeParams, lp: LearnedParams, scorer, records=None,
                   pool=None, f0: int = 0):
    torch = _torch()
    F = y.shape[0]
    dev = y.device
    z = torch.empty((F, (code.N + 31) // 32), dtype=torch.int32, device=dev)
    it = torch.empty(F, dtype=torch.int32, device=dev)
    ok = torch.empty(F, dtype=torch.uint8, device=dev)
    lok = torch.empty(F, dtype=torch.uint8, device=dev)
    decode_learned_into(code, y, plain, lp, scorer, z, it, ok, lok, records, pool, f0)
    return z, it, ok, lok


def record_buffer(F: int, rounds: int, groups: int = 32, topk: int = 1, device="cuda"):
    """Device buffer for F * rounds * record_slots(groups, topk) records (12
    bytes each), shaped [F][rounds][slots][12]."""
    torch = _torch()
    return torch.empty((F, rounds, record_slots(groups, topk), RECORD_DTYPE.itemsize), dtype=torch.uint8,
                       device=device)


def records_host(rec):
    """Records of a record_buffer copied to the host as a structured array
    [F][rounds][slots]."""
    return rec.cpu().numpy().view(RECORD_DTYPE)[..., 0]


def scorer_grad(records, n_tiles: int, lp: LearnedParams, scorer, pos_weight: float, out=None,
                scores=None, workspace=None):
    torch = _torch()
    P = scorer_size(lp.rounds)
    if workspace is None and out is not None:
        workspace = torch.empty(1024 * (P + 2), dtype=torch.float32, device=scorer.device)
    _check(lib().fwbf_scorer_grad(_ptr(records), n_tiles, C.byref(lp), _ptr(scorer), pos_weight,
                                  _ptr(out), _ptr(scores), _ptr(workspace),
                                  0 if workspace is None else workspace.numel(), _stream()))
    return out, scores


def adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().fwbf_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), step, lr,
                           beta1, beta2, eps, _stream()))


# ---- mixed-code batch, graph sweep -----------------------------------------

def decode_batched(jobs, threads_per_frame: int = 0, blocks_per_cu: int = 0, workspace=None):
    """jobs: list of (code, y, DecodeParams); returns [(z, iters, ok)] per job.
    One persistent launch claims frames of all jobs from a shared queue."""
    torch = _torch()
    keep, items, outs = [], [], []
    for code, y, params in jobs:
        F = y.shape[0]
        z = torch.empty((F, (code.N + 31) // 32), dtype=torch.int32, device=y.device)
        it = torch.empty(F, dtype=torch.int32, device=y.device)
        ok = torch.empty(F, dtype=torch.uint8, device=y.device)
        pc = params.c()
        keep.append(pc)
        items.append(BatchItem(code._h.value, C.addressof(pc), y.data_ptr(), F, y.stride(0),
                               z.data_ptr(), it.data_ptr(), ok.data_ptr()))
        outs.append((z, it, ok))
    arr = (BatchItem * len(items))(*items)
    if workspace is None:
        workspace = torch.zeros(64, dtype=torch.int32, device=jobs[0][1].device)
    _check(lib().fwbf_decode_batched(arr, len(items), threads_per_frame, blocks_per_cu,
                                     _ptr(workspace), workspace.numel() * 4, _stream()))
    return outs


def decode_batched_noalloc(jobs, threads_per_frame: int = 0, blocks_per_cu: int = 0):
    """jobs: list of (code, y, DecodeParams, z, iters, ok) with caller-made
    output tensors.  The library call allocates nothing (its ticket counter
    is a library-owned device array); each code must have been decoded on
    this device before."""
    keep, items = [], []
    for code, y, params, z, it, ok in jobs:
        pc = params.c()
        keep.append(pc)
        items.append(BatchItem(code._h.value, C.addressof(pc), y.data_ptr(), y.shape[0], y.stride(0),
                               z.data_ptr(), it.data_ptr(), ok.data_ptr()))
    arr = (BatchItem * len(items))(*items)
    _check(lib().fwbf_decode_batched_noalloc(arr, len(items), threads_per_frame, blocks_per_cu, _stream()))


class Sweep:
    """channel -> decode -> count for several noise levels, one HIP graph."""

    def __init__(self, code: Code, params: DecodeParams, sigmas, frames_per_point: int, pool=None,
                 seed: int = 1, scale: float = 1.0):
        self.code, self.params = code, params
        self.n_points = len(sigmas)
        self.frames_per_point = frames_per_point
        self._p = params.c()
        sig = np.ascontiguousarray(sigmas, np.float32)
        h = C.c_void_p()
        self._pool = pool
        _check(lib().fwbf_sweep_create(code._h, C.byref(self._p), _np_ptr(sig), self.n_points,
                                       frames_per_point, _ptr(pool),
                                       0 if pool is None else pool.shape[0], seed, scale,
                                       C.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().fwbf_sweep_launch(self._h, _stream()))

    def counters(self):
        out = np.zeros((self.n_points, 7 + self.params.max_iter), np.int64)
        _check(lib().fwbf_sweep_counters(self._h, _np_ptr(out), _stream()))
        return out

    def outputs(self, point: int):
        """Point `point`'s frames and the outputs of the last replay, copied
        into new device tensors: (y [F][N], z [F][ceil(N/32)], iters, ok)."""
        torch = _torch()
        F, N = self.frames_per_point, self.code.N
        dt = {F32: torch.float32, I8: torch.int8, I16: torch.int16}[self.params.dtype]
        y = torch.empty((F, N), dtype=dt, device="cuda")
        z = torch.empty((F, (N + 31) // 32), dtype=torch.int32, device="cuda")
        it = torch.empty(F, dtype=torch.int32, device="cuda")
        ok = torch.empty(F, dtype=torch.uint8, device="cuda")
        _check(lib().fwbf_sweep_outputs(self._h, point, _ptr(y), _ptr(z), _ptr(it), _ptr(ok), _stream()))
        return y, z, it, ok

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.fwbf_sweep_free(h)
            self._h = None
