"""ctypes wrapper over the plain C oracle (TEST INFRASTRUCTURE ONLY).

Arguments and results are numpy arrays on the host.  ``build()`` compiles
``vbyte_oracle.c`` with gcc into ``liborc.so`` next to this file.
"""
import ctypes
import os
import subprocess

import numpy as np

OK, EINVAL, ECOUNT, ETRUNC, EMALFORMED = 0, 1, 2, 3, 4
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ECOUNT: "ECOUNT",
                ETRUNC: "ETRUNC", EMALFORMED: "EMALFORMED"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vbyte_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def lib_path():
    return _LIB


def build(src=_SRC, out=_LIB, extra_flags=()):
    """Compile the oracle (gcc -O2, no intrinsics, no vectorisation hints)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
           *extra_flags, "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _u8p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def load(path=None):
    """Load the oracle library (building it first when it is absent)."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _declare(lib):
    c = ctypes
    lib.orc_code_length.argtypes = [c.c_uint32]
    lib.orc_code_length.restype = c.c_int
    lib.orc_encode.argtypes = [c.POINTER(c.c_uint32), c.c_size_t, c.POINTER(c.c_uint8)]
    lib.orc_encode.restype = c.c_size_t
    lib.orc_encoded_size.argtypes = [c.POINTER(c.c_uint32), c.c_size_t]
    lib.orc_encoded_size.restype = c.c_size_t
    lib.orc_encode_delta.argtypes = [c.POINTER(c.c_uint32), c.c_size_t, c.c_uint32,
                                     c.POINTER(c.c_uint8)]
    lib.orc_encode_delta.restype = c.c_size_t
    lib.orc_count.argtypes = [c.POINTER(c.c_uint8), c.c_size_t]
    lib.orc_count.restype = c.c_uint64
    lib.orc_validate.argtypes = [c.POINTER(c.c_uint8), c.c_size_t, c.c_size_t]
    lib.orc_validate.restype = c.c_int
    lib.orc_decode.argtypes = [c.POINTER(c.c_uint8), c.c_size_t, c.POINTER(c.c_uint32),
                               c.c_size_t]
    lib.orc_decode.restype = c.c_int
    lib.orc_decode_delta.argtypes = [c.POINTER(c.c_uint8), c.c_size_t,
                                     c.POINTER(c.c_uint32), c.c_size_t, c.c_uint32]
    lib.orc_decode_delta.restype = c.c_int
    lib.orc_decode_delta_m1.argtypes = [c.POINTER(c.c_uint8), c.c_size_t,
                                        c.POINTER(c.c_uint32), c.c_size_t, c.c_uint32]
    lib.orc_decode_delta_m1.restype = c.c_int
    lib.orc_encode_delta_m1.argtypes = [c.POINTER(c.c_uint32), c.c_size_t, c.c_uint32,
                                        c.POINTER(c.c_uint8)]
    lib.orc_encode_delta_m1.restype = c.c_size_t
    lib.orc_decode_next.argtypes = [c.POINTER(c.c_uint8), c.c_size_t, c.c_size_t, c.c_size_t,
                                    c.c_uint32, c.c_int, c.POINTER(c.c_uint32),
                                    c.POINTER(c.c_size_t), c.POINTER(c.c_size_t),
                                    c.POINTER(c.c_uint32)]
    lib.orc_decode_next.restype = c.c_int
    lib.orc_decode_batch.argtypes = [c.POINTER(c.c_uint8), c.POINTER(c.c_int64),
                                     c.POINTER(c.c_uint32), c.POINTER(c.c_int64),
                                     c.c_size_t, c.POINTER(c.c_uint32), c.c_int,
                                     c.POINTER(c.c_int32)]
    lib.orc_decode_batch.restype = c.c_int
    lib.orc_decode_delta4.argtypes = [c.POINTER(c.c_uint8), c.c_size_t, c.POINTER(c.c_uint32),
                                      c.c_size_t, c.POINTER(c.c_uint32)]
    lib.orc_decode_delta4.restype = c.c_int
    lib.orc_encode_delta4.argtypes = [c.POINTER(c.c_uint32), c.c_size_t, c.POINTER(c.c_uint32),
                                      c.POINTER(c.c_uint8)]
    lib.orc_encode_delta4.restype = c.c_size_t
    u64p = c.POINTER(c.c_uint64)
    lib.orc_code_length64.argtypes = [c.c_uint64]
    lib.orc_code_length64.restype = c.c_int
    lib.orc_encode64.argtypes = [u64p, c.c_size_t, c.POINTER(c.c_uint8)]
    lib.orc_encode64.restype = c.c_size_t
    lib.orc_encoded_size64.argtypes = [u64p, c.c_size_t]
    lib.orc_encoded_size64.restype = c.c_size_t
    lib.orc_encode_delta64.argtypes = [u64p, c.c_size_t, c.c_uint64, c.POINTER(c.c_uint8)]
    lib.orc_encode_delta64.restype = c.c_size_t
    lib.orc_validate64.argtypes = [c.POINTER(c.c_uint8), c.c_size_t, c.c_size_t]
    lib.orc_validate64.restype = c.c_int
    lib.orc_decode64.argtypes = [c.POINTER(c.c_uint8), c.c_size_t, u64p, c.c_size_t]
    lib.orc_decode64.restype = c.c_int
    lib.orc_decode64_delta.argtypes = [c.POINTER(c.c_uint8), c.c_size_t, u64p, c.c_size_t,
                                       c.c_uint64]
    lib.orc_decode64_delta.restype = c.c_int
    return lib


def _as_u32(x):
    return np.ascontiguousarray(x, dtype=np.uint32)


def _as_u8(b):
    if isinstance(b, (bytes, bytearray)):
        return np.frombuffer(bytes(b), dtype=np.uint8).copy()
    return np.ascontiguousarray(b, dtype=np.uint8)


def code_length(x, lib=None):
    """L(x), section 1."""
    lib = lib or load()
    return lib.orc_code_length(int(x) & 0xFFFFFFFF)


def encoded_size(x, lib=None):
    lib = lib or load()
    x = _as_u32(x)
    return int(lib.orc_encoded_size(_u32p(x), x.size))


def encode(x, lib=None):
    """ENC of a uint32 sequence -> uint8 array (section 1, Table 1)."""
    lib = lib or load()
    x = _as_u32(x)
    out = np.empty(max(5 * x.size, 1), dtype=np.uint8)
    nb = lib.orc_encode(_u32p(x), x.size, _u8p(out))
    return out[:nb].copy()


def encode_delta(x, prev=0, lib=None):
    """ENC of the gaps x_i - x_{i-1} mod 2^32, x_0 = prev (section 1)."""
    lib = lib or load()
    x = _as_u32(x)
    out = np.empty(max(5 * x.size, 1), dtype=np.uint8)
    nb = lib.orc_encode_delta(_u32p(x), x.size, int(prev) & 0xFFFFFFFF, _u8p(out))
    return out[:nb].copy()


def count(b, lib=None):
    """Number of terminator bytes (top bit 0)."""
    lib = lib or load()
    b = _as_u8(b)
    return int(lib.orc_count(_u8p(b), b.size))


def validate(b, n, lib=None):
    lib = lib or load()
    b = _as_u8(b)
    return int(lib.orc_validate(_u8p(b), b.size, int(n)))


def decode(b, n, lib=None):
    """DEC (Algorithm 1 after validation).  Returns (status, uint32 array)."""
    lib = lib or load()
    b = _as_u8(b)
    y = np.zeros(max(int(n), 1), dtype=np.uint32)
    st = lib.orc_decode(_u8p(b), b.size, _u32p(y), int(n))
    return int(st), y[:int(n)]


def decode_delta(b, n, prev=0, lib=None):
    """DEC then inclusive prefix sum from prev, mod 2^32."""
    lib = lib or load()
    b = _as_u8(b)
    y = np.zeros(max(int(n), 1), dtype=np.uint32)
    st = lib.orc_decode_delta(_u8p(b), b.size, _u32p(y), int(n), int(prev) & 0xFFFFFFFF)
    return int(st), y[:int(n)]


def decode_delta_m1(b, n, prev=0, lib=None):
    """DEC then differences minus one: y_0 = prev + g_0, y_k = y_(k-1) + g_k + 1."""
    lib = lib or load()
    b = _as_u8(b)
    y = np.zeros(max(int(n), 1), dtype=np.uint32)
    st = lib.orc_decode_delta_m1(_u8p(b), b.size, _u32p(y), int(n), int(prev) & 0xFFFFFFFF)
    return int(st), y[:int(n)]


def encode_delta_m1(x, prev=0, lib=None):
    """ENC of the differences minus one (the first difference is x_0 - prev)."""
    lib = lib or load()
    x = _as_u32(x)
    out = np.zeros(max(5 * x.size, 1), dtype=np.uint8)
    m = lib.orc_encode_delta_m1(_u32p(x), x.size, int(prev) & 0xFFFFFFFF, _u8p(out))
    return out[:m].copy()


def decode_next(b, off, k, prev=0, delta=0, lib=None):
    """One resumable piece of at most k integers from byte off (reading R12).
    Returns (status, values, next_off, next_prev)."""
    lib = lib or load()
    b = _as_u8(b)
    y = np.zeros(max(int(k), 1), dtype=np.uint32)
    no, m, npv = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_uint32(0)
    st = lib.orc_decode_next(_u8p(b), b.size, int(off), int(k), int(prev) & 0xFFFFFFFF, int(delta),
                             _u32p(y), ctypes.byref(no), ctypes.byref(m), ctypes.byref(npv))
    return int(st), y[:m.value].copy(), int(no.value), int(npv.value)


def intersect_pieces(a, na, b_ids, piece, prev=0, lib=None):
    """List intersection by a bounded-buffer consumer (section 5 decodes long
    lists piece by piece into a small buffer; reading R15): the differential
    list a (na identifiers, from prev) is decoded in pieces of at most
    `piece` integers (decode_next, reading R12), and every identifier of a,
    in order, that occurs in the sorted array b_ids is kept (numpy isin).
    Status: the worst status of a piece (a failing piece leaves the cursor,
    so later pieces fail alike), else ETRUNC when fewer than na codes were
    found, else ECOUNT when bytes remain after the na-th code.
    Returns (status, matches)."""
    lib = lib or load()
    a = _as_u8(a)
    b_ids = np.asarray(b_ids, dtype=np.uint32)
    off, done, pv, worst = 0, 0, int(prev) & 0xFFFFFFFF, OK
    keep = []
    for _ in range((int(na) + piece - 1) // piece):
        st, y, noff, npv = decode_next(a, off, piece, pv, 1, lib=lib)
        if st != OK:
            worst = max(worst, st)
            continue
        take = y[:max(0, min(y.size, int(na) - done))]
        keep.append(take[np.isin(take, b_ids)])
        done += y.size
        off, pv = noff, npv
    out = np.concatenate(keep) if keep else np.zeros(0, np.uint32)
    if worst != OK:
        return worst, out
    if done < int(na):
        return ETRUNC, out
    if off < a.size or done > int(na):
        return ECOUNT, out
    return OK, out


def decode_batch(b, byte_off, out_off, prevs=None, delta=False, lib=None):
    """BATCH over CSR offsets (delta: 0/False plain, 1/True differences,
    2 differences minus one).  Returns (status, out, per-list status)."""
    lib = lib or load()
    b = _as_u8(b)
    byte_off = np.ascontiguousarray(byte_off, dtype=np.int64)
    out_off = np.ascontiguousarray(out_off, dtype=np.int64)
    nlists = byte_off.size - 1
    total = int(out_off[-1]) if nlists >= 0 and out_off.size else 0
    out = np.zeros(max(total, 1), dtype=np.uint32)
    st_list = np.zeros(max(nlists, 1), dtype=np.int32)
    pv = None
    if prevs is not None:
        pv = _as_u32(prevs)
    st = lib.orc_decode_batch(_u8p(b), _i64p(byte_off), _u32p(out), _i64p(out_off),
                              nlists, _u32p(pv) if pv is not None else None,
                              int(delta), _i32p(st_list))
    return int(st), out[:total], st_list[:nlists]


# ---------------------------------------------------------------- blocks of four (R14)
def _prev4(prev4):
    if prev4 is None:
        return None
    p = np.ascontiguousarray(np.asarray(prev4, dtype=np.uint64).astype(np.uint32))
    assert p.size == 4
    return p


def decode_delta4(b, n, prev4=None, lib=None):
    """DEC then y_i = g_i + y_(i-4) mod 2^32 from the four values prev4
    (zeros by default).  Returns (status, uint32 array)."""
    lib = lib or load()
    b = _as_u8(b)
    p = _prev4(prev4)
    y = np.zeros(max(int(n), 1), dtype=np.uint32)
    st = lib.orc_decode_delta4(_u8p(b), b.size, _u32p(y), int(n), None if p is None else _u32p(p))
    return int(st), y[:int(n)]


def encode_delta4(x, prev4=None, lib=None):
    """ENC of x_i - x_(i-4) mod 2^32 (x_(-4..-1) = prev4, zeros by default)."""
    lib = lib or load()
    x = _as_u32(x)
    p = _prev4(prev4)
    out = np.zeros(max(5 * x.size, 1), dtype=np.uint8)
    nb = lib.orc_encode_delta4(_u32p(x), x.size, None if p is None else _u32p(p), _u8p(out))
    return out[:nb].copy()


# ---------------------------------------------------------------- 64-bit (R13)
def _u64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _as_u64(x):
    return np.ascontiguousarray(x, dtype=np.uint64)


def code_length64(x, lib=None):
    lib = lib or load()
    return int(lib.orc_code_length64(int(x) & 0xFFFFFFFFFFFFFFFF))


def encoded_size64(x, lib=None):
    lib = lib or load()
    x = _as_u64(x)
    return int(lib.orc_encoded_size64(_u64p(x), x.size))


def encode64(x, lib=None):
    """ENC of uint64 values: up to ten 7-bit groups each."""
    lib = lib or load()
    x = _as_u64(x)
    out = np.zeros(max(10 * x.size, 1), dtype=np.uint8)
    nb = lib.orc_encode64(_u64p(x), x.size, _u8p(out))
    return out[:nb].copy()


def encode_delta64(x, prev=0, lib=None):
    """Gaps mod 2^64 from prev, then ENC."""
    lib = lib or load()
    x = _as_u64(x)
    out = np.zeros(max(10 * x.size, 1), dtype=np.uint8)
    nb = lib.orc_encode_delta64(_u64p(x), x.size, int(prev) & 0xFFFFFFFFFFFFFFFF, _u8p(out))
    return out[:nb].copy()


def validate64(b, n, lib=None):
    lib = lib or load()
    b = _as_u8(b)
    return int(lib.orc_validate64(_u8p(b), b.size, int(n)))


def decode64(b, n, lib=None):
    """Algorithm 1 widened to uint64 after validation (R13).  Returns
    (status, uint64 array)."""
    lib = lib or load()
    b = _as_u8(b)
    y = np.zeros(max(int(n), 1), dtype=np.uint64)
    st = lib.orc_decode64(_u8p(b), b.size, _u64p(y), int(n))
    return int(st), y[:int(n)]


def decode64_delta(b, n, prev=0, lib=None):
    """decode64, then the inclusive prefix sum from prev, mod 2^64."""
    lib = lib or load()
    b = _as_u8(b)
    y = np.zeros(max(int(n), 1), dtype=np.uint64)
    st = lib.orc_decode64_delta(_u8p(b), b.size, _u64p(y), int(n), int(prev) & 0xFFFFFFFFFFFFFFFF)
    return int(st), y[:int(n)]
