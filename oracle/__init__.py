"""CPU oracle for FWBF decoding -- test infrastructure only.

This package is the reference the HIP library is checked against.  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product path never does.  It shares no code
with ``paper_1206_3362_amd`` (the seeded input generators in
``paper_1206_3362_amd.synth`` hold none of the decoder's arithmetic and are
the only thing both sides use).

``fwbf_oracle.c`` holds the literal algorithm (Section III of the paper);
this module only builds it with gcc and marshals numpy arrays through ctypes.
``mlp_ref.py`` holds the float64 reference of the learned flip scorer.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fwbf_oracle.c")
_LIB = os.path.join(_HERE, "_fwbf_oracle.so")

WBF, MWBF, IMWBF = 0, 1, 2
GROUPS, SINGLE, TOPL, STRIDED = 0, 1, 2, 3
F32, I8, I16 = 0, 1, 2
_NP = {F32: np.float32, I8: np.int8, I16: np.int16}

_ERRORS = {-1: "invalid argument", -2: "parse error", -3: "girth constraint not met",
           -4: "out of memory"}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-pthread", "-Wall",
                               "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        vp, i32, i64, u64 = C.c_void_p, C.c_int, C.c_int64, C.c_uint64
        L.or_code_from_text.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.or_code_from_seed.argtypes = [i32, i32, i32, u64, i32, C.POINTER(vp)]
        L.or_code_free.argtypes = [vp]
        L.or_code_free.restype = None
        L.or_code_dims.argtypes = [vp] + [C.POINTER(i32)] * 5
        L.or_code_dims.restype = None
        L.or_code_shifts.argtypes = [vp, vp]
        L.or_code_shifts.restype = None
        L.or_code_edges.argtypes = [vp]
        L.or_code_n_entries.argtypes = [vp]
        L.or_code_entries.argtypes = [vp, vp]
        L.or_code_entries.restype = None
        L.or_code_rows.argtypes = [vp, vp, vp]
        L.or_code_rows.restype = None
        L.or_code_violates_rc.argtypes = [vp]
        L.or_code_rank.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.or_code_info_positions.argtypes = [vp, vp]
        L.or_encode.argtypes = [vp, u64, i64, i64, vp]
        L.or_decode.argtypes = [vp, i32, i32, i32, i32, i32, C.c_float, i32, i32, i32, vp, i64,
                                i64, vp, vp, vp, i32]
        L.or_decode_trace.argtypes = [vp, i32, i32, i32, i32, i32, C.c_float, i32, i32, i32, vp,
                                      vp, vp, vp, vp, vp, vp]
        L.or_philox4x32_10.argtypes = [vp, vp, vp]
        L.or_philox4x32_10.restype = None
        L.or_splitmix64.argtypes = [u64, u64]
        L.or_splitmix64.restype = u64
        L.or_channel.argtypes = [i32, i64, i64, vp, i64, u64, C.c_uint32, C.c_double, C.c_double,
                                 i32, vp, vp]
        L.or_count.argtypes = [i32, i64, i64, vp, vp, i64, vp, vp, i32, vp, vp]
        L.or_decode_minsum.argtypes = [vp, i32, C.c_float, i32, vp, i64, i64, vp, vp, vp, i32]
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what}: {_ERRORS.get(rc, rc)}")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Code:
    """Materialised QC-LDPC code (Section II: H, M(n), N(m))."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)
        d = [C.c_int() for _ in range(5)]
        lib().or_code_dims(self._h, *[C.byref(x) for x in d])
        self.N, self.M, self.Z, self.mb, self.nb = (x.value for x in d)
        self._rank = None

    @classmethod
    def from_text(cls, text: str) -> "Code":
        h = C.c_void_p()
        _check(lib().or_code_from_text(text.encode(), C.byref(h)), "code_from_text")
        return cls(h.value)

    @classmethod
    def from_seed(cls, mb, nb, Z, seed, min_girth=6) -> "Code":
        h = C.c_void_p()
        _check(lib().or_code_from_seed(mb, nb, Z, seed, min_girth, C.byref(h)), "code_from_seed")
        return cls(h.value)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.or_code_free(self._h)
            self._h = None

    @property
    def shifts(self) -> np.ndarray:
        out = np.empty((self.mb, self.nb), np.int32)
        lib().or_code_shifts(self._h, _ptr(out))
        return out

    def entries(self) -> np.ndarray:
        """(block row, block column, shift) of every circulant permutation."""
        n = lib().or_code_n_entries(self._h)
        out = np.zeros((n, 3), np.int32)
        lib().or_code_entries(self._h, _ptr(out))
        return out

    def to_text(self) -> str:
        cells = [[[] for _ in range(self.nb)] for _ in range(self.mb)]
        for i, j, s in self.entries():
            cells[i][j].append(int(s))
        rows = "\n".join(" ".join(",".join(map(str, c)) if c else "-1" for c in r) for r in cells)
        return f"qc-ldpc v1\nZ {self.Z}\nbase {self.mb} {self.nb}\n{rows}\n"

    def rows(self):
        """(row_ptr, row_bits): N(m) for every check m, ascending bit index."""
        E = lib().or_code_edges(self._h)
        rp = np.empty(self.M + 1, np.int32)
        rb = np.empty(E, np.int32)
        lib().or_code_rows(self._h, _ptr(rp), _ptr(rb))
        return rp, rb

    def dense(self) -> np.ndarray:
        rp, rb = self.rows()
        H = np.zeros((self.M, self.N), np.uint8)
        for m in range(self.M):
            H[m, rb[rp[m]:rp[m + 1]]] = 1
        return H

    def violates_rc(self) -> bool:
        return bool(lib().or_code_violates_rc(self._h))

    def rank(self):
        if self._rank is None:
            r, k = C.c_int(), C.c_int()
            _check(lib().or_code_rank(self._h, C.byref(r), C.byref(k)), "rank")
            self._rank = (r.value, k.value)
        return self._rank

    @property
    def K(self) -> int:
        return self.rank()[1]

    def info_positions(self) -> np.ndarray:
        out = np.empty(self.K, np.int32)
        _check(lib().or_code_info_positions(self._h, _ptr(out)), "info_positions")
        return out

    def encode(self, seed: int, first: int, count: int) -> np.ndarray:
        """Packed codewords [count][ceil(N/32)] (bit n in word n/32, LSB first)."""
        out = np.zeros((count, (self.N + 31) // 32), np.uint32)
        _check(lib().or_encode(self._h, seed, first, count, _ptr(out)), "encode")
        return out


def unpack(z: np.ndarray, N: int) -> np.ndarray:
    """Packed LSB-first words -> uint8 bits [..., N]."""
    z = np.ascontiguousarray(z, dtype=np.uint32)
    b = np.unpackbits(z.view(np.uint8).reshape(*z.shape[:-1], -1), axis=-1, bitorder="little")
    return b[..., :N]


def pack(bits: np.ndarray) -> np.ndarray:
    bits = np.asarray(bits, np.uint8)
    N = bits.shape[-1]
    W = (N + 31) // 32
    pad = np.zeros(bits.shape[:-1] + (W * 32,), np.uint8)
    pad[..., :N] = bits
    return np.packbits(pad, axis=-1, bitorder="little").view(np.uint32).reshape(*bits.shape[:-1], W)


def _dtype_of(y):
    for k, v in _NP.items():
        if y.dtype == v:
            return k
    raise TypeError(f"unsupported y dtype {y.dtype}")


def decode(code: Code, y: np.ndarray, *, weights=IMWBF, select=GROUPS, G=8, lam=1, max_iter=100,
           alpha=0.2, alpha_num=1, alpha_den=5, threads=None):
    """Literal FWBF over frames y[F][N]; returns (z packed, iterations, ok)."""
    y = np.ascontiguousarray(y)
    if y.ndim == 1:
        y = y[None]
    F, N = y.shape
    assert N == code.N
    dt = _dtype_of(y)
    z = np.zeros((F, (N + 31) // 32), np.uint32)
    it = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    nt = threads or min(os.cpu_count() or 1, 16)
    _check(lib().or_decode(code._h, weights, select, G, lam, max_iter, alpha, alpha_num, alpha_den,
                           dt, _ptr(y), F, N, _ptr(z), _ptr(it), _ptr(ok), nt), "decode")
    return z, it, ok


def decode_minsum(code: Code, y: np.ndarray, *, offset=False, c=0.75, max_iter=20, threads=None):
    """Flooding min-sum BP over float frames y[F][N]: normalised (R = c*min)
    or offset (R = max(min - c, 0)); returns (z packed, iterations, ok)."""
    y = np.ascontiguousarray(y, dtype=np.float32)
    if y.ndim == 1:
        y = y[None]
    F, N = y.shape
    assert N == code.N
    z = np.zeros((F, (N + 31) // 32), np.uint32)
    it = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    nt = threads or min(os.cpu_count() or 1, 16)
    _check(lib().or_decode_minsum(code._h, int(bool(offset)), c, max_iter, _ptr(y), F, N, _ptr(z),
                                  _ptr(it), _ptr(ok), nt), "decode_minsum")
    return z, it, ok


def decode_trace(code: Code, y: np.ndarray, *, weights=IMWBF, select=GROUPS, G=8, lam=1,
                 max_iter=100, alpha=0.2, alpha_num=1, alpha_den=5):
    """One frame; returns dict(z, iters, ok, E0, flips=[list per round])."""
    y = np.ascontiguousarray(y).reshape(-1)
    N = code.N
    dt = _dtype_of(y)
    z = np.zeros((N + 31) // 32, np.uint32)
    it = np.zeros(1, np.int32)
    ok = np.zeros(1, np.uint8)
    E0 = np.full(N, np.nan)
    nfl = np.zeros(max(max_iter, 1), np.int32)
    fl = np.zeros((max(max_iter, 1), N), np.int32)
    _check(lib().or_decode_trace(code._h, weights, select, G, lam, max_iter, alpha, alpha_num,
                                 alpha_den, dt, _ptr(y), _ptr(z), _ptr(it), _ptr(ok), _ptr(E0),
                                 _ptr(nfl), _ptr(fl)), "decode_trace")
    k = int(it[0])
    return dict(z=z, iters=k, ok=bool(ok[0]), E0=E0,
                flips=[fl[r, :nfl[r]].copy() for r in range(k)])


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def splitmix64(seed: int, idx: int) -> int:
    return int(lib().or_splitmix64(seed, idx))


def channel(N, F, f0, pool, seed, stream, sigma, scale=1.0, dtype=F32, want_double=False):
    """Received frames (Section II BPSK, Section V AWGN); see or_channel."""
    out = np.zeros((F, N), _NP[dtype])
    yd = np.zeros((F, N), np.float64) if want_double else None
    pool_c = None if pool is None else np.ascontiguousarray(pool, np.uint32)
    pn = 0 if pool is None else pool_c.shape[0]
    _check(lib().or_channel(N, F, f0, _ptr(pool_c), pn, seed, stream, sigma, scale, dtype,
                            _ptr(out), _ptr(yd)), "channel")
    return (out, yd) if want_double else out


def count(N, z, pool, f0, iters, ok, max_iter):
    """Returns dict(bit_err, frame_err, undetected, iter_sum, frames, hist)."""
    z = np.ascontiguousarray(z, np.uint32)
    F = z.shape[0]
    counts = np.zeros(5, np.int64)
    hist = np.zeros(max_iter + 1, np.int64)
    pool_c = None if pool is None else np.ascontiguousarray(pool, np.uint32)
    pn = 0 if pool is None else pool_c.shape[0]
    _check(lib().or_count(N, F, f0, _ptr(z), _ptr(pool_c), pn,
                          _ptr(np.ascontiguousarray(iters, np.int32)),
                          _ptr(np.ascontiguousarray(ok, np.uint8)), max_iter, _ptr(counts),
                          _ptr(hist)), "count")
    return dict(bit_err=int(counts[0]), frame_err=int(counts[1]), undetected=int(counts[2]),
                iter_sum=int(counts[3]), frames=int(counts[4]), hist=hist)
