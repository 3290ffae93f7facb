"""Python binding of libvbyte (argument marshalling only).

Every function forwards torch tensors that live on the GPU to the C ABI of
``include/vbyte.h``; PyTorch only provides device memory and the current
stream.  All decoding, counting and encoding runs in the HIP kernels of
``csrc/``.  The library is loaded from this directory and must have been
built (``python -m paper_1503_07387_amd.build``); there is no fallback.

uint32 results are returned as ``torch.int32`` tensors holding the same bits.
"""
import contextlib
import ctypes
import functools
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvbyte.so")

OK, EINVAL, ECOUNT, ETRUNC, EMALFORMED, EHIP, ENOMEM, ESTALLED = range(8)
STATUS_NAMES = {OK: "VBYTE_OK", EINVAL: "VBYTE_EINVAL", ECOUNT: "VBYTE_ECOUNT",
                ETRUNC: "VBYTE_ETRUNC", EMALFORMED: "VBYTE_EMALFORMED",
                EHIP: "VBYTE_EHIP", ENOMEM: "VBYTE_ENOMEM", ESTALLED: "VBYTE_ESTALLED"}

EXPORTS = ["vbyte_decode", "vbyte_decode_delta", "vbyte_decode_async",
           "vbyte_decode_delta_async", "vbyte_decode_delta_m1", "vbyte_decode_delta_m1_async",
           "vbyte_encode_delta_m1_async", "vbyte_decode_next_async", "vbyte_decode_delta4",
           "vbyte_decode_delta4_async", "vbyte_intersect_async", "vbyte_decode64",
           "vbyte_decode64_delta", "vbyte_decode64_async", "vbyte_decode64_delta_async",
           "vbyte_count", "vbyte_decode_batch",
           "vbyte_decode_lists", "vbyte_encode_async", "vbyte_encode_delta_async",
           "vbyte_encode_batch", "vbyte_server_create", "vbyte_server_destroy",
           "vbyte_server_run", "vbyte_batch_graph_create", "vbyte_batch_graph_launch",
           "vbyte_batch_graph_destroy", "vbyte_autotune_decode", "vbyte_autotune_batch",
           "vbyte_set_chunk_tiles", "vbyte_get_chunk_tiles", "vbyte_set_flow_grid",
           "vbyte_decode_ex", "vbyte_tuning_default", "vbyte_decode_noalloc",
           "vbyte_set_spin_limit",
           "vbyte_workspace_size", "vbyte_set_tuning", "vbyte_get_tuning",
           "vbyte_status_str", "vbyte_last_error"]


class TunePoint(ctypes.Structure):
    _fields_ = [("segs_per_wave", ctypes.c_int), ("waves_per_block", ctypes.c_int),
                ("small_list_bytes", ctypes.c_int64), ("tiles_per_chunk", ctypes.c_int),
                ("ms", ctypes.c_double), ("status", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    """vbyte_tuning: the kernel tuning of one single-stream decode."""
    _fields_ = [("segs_per_wave", ctypes.c_int), ("waves_per_block", ctypes.c_int),
                ("schedule", ctypes.c_int), ("grid", ctypes.c_int), ("recompute", ctypes.c_int)]


SCHED_ONE_READ, SCHED_TWO_PASS, SCHED_LOOKBACK = -2, -1, 0


def make_tuning(segs_per_wave=None, waves_per_block=None, schedule=None, grid=None, recompute=0):
    """A Tuning from the process defaults, with the given fields replaced."""
    t = Tuning()
    _lib().vbyte_tuning_default(ctypes.byref(t))
    if segs_per_wave is not None:
        t.segs_per_wave = int(segs_per_wave)
    if waves_per_block is not None:
        t.waves_per_block = int(waves_per_block)
    if schedule is not None:
        t.schedule = int(schedule)
    if grid is not None:
        t.grid = int(grid)
    t.recompute = int(recompute)
    return t


class VByteError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = int(status)
        msg = STATUS_NAMES.get(self.status, str(status))
        if what:
            msg = f"{what}: {msg}"
        if self.status == EHIP:
            msg += " (" + _lib().vbyte_last_error().decode() + ")"
        super().__init__(msg)


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libvbyte.so is not built ({LIB_PATH}); run "
                               "python -m paper_1503_07387_amd.build")
        _L = _declare(ctypes.CDLL(LIB_PATH))
    return _L


def load(path=LIB_PATH):
    """Load a libvbyte build from `path` with its prototypes declared."""
    return _declare(ctypes.CDLL(path))


def _declare(lib):
    c = ctypes
    vp, sz, u32, i32, i64 = c.c_void_p, c.c_size_t, c.c_uint32, c.c_int, c.c_int64
    sig = {
        "vbyte_decode": [vp, sz, vp, sz],
        "vbyte_decode_delta": [vp, sz, vp, sz, u32],
        "vbyte_decode_async": [vp, sz, vp, sz, vp, vp],
        "vbyte_decode_delta_async": [vp, sz, vp, sz, u32, vp, vp],
        "vbyte_decode_delta_m1": [vp, sz, vp, sz, u32],
        "vbyte_decode_delta_m1_async": [vp, sz, vp, sz, u32, vp, vp],
        "vbyte_decode_next_async": [vp, sz, vp, sz, i32, vp, vp, vp, vp],
        "vbyte_decode_delta4": [vp, sz, vp, sz, c.POINTER(u32)],
        "vbyte_decode_delta4_async": [vp, sz, vp, sz, c.POINTER(u32), vp, vp],
        "vbyte_intersect_async": [vp, sz, sz, u32, vp, sz, sz, vp, sz, vp, vp, vp],
        "vbyte_decode64": [vp, sz, vp, sz],
        "vbyte_decode64_delta": [vp, sz, vp, sz, c.c_uint64],
        "vbyte_decode64_async": [vp, sz, vp, sz, vp, vp],
        "vbyte_decode64_delta_async": [vp, sz, vp, sz, c.c_uint64, vp, vp],
        "vbyte_encode_delta_m1_async": [vp, sz, u32, vp, sz, vp, vp],
        "vbyte_count": [vp, sz, vp, vp],
        "vbyte_decode_batch": [vp, sz, vp, vp, sz, vp, sz, vp, i32, vp, vp],
        "vbyte_decode_lists": [vp, sz, vp, sz, sz, vp, sz, vp, i32, vp, vp],
        "vbyte_encode_async": [vp, sz, vp, sz, vp, vp],
        "vbyte_encode_delta_async": [vp, sz, u32, vp, sz, vp, vp],
        "vbyte_encode_batch": [vp, sz, vp, sz, vp, sz, vp, vp, vp],
        "vbyte_set_tuning": [i32, i32, i64],
        "vbyte_set_chunk_tiles": [i32],
        "vbyte_set_flow_grid": [i32],
        "vbyte_set_spin_limit": [u32],
        "vbyte_decode_ex": [vp, sz, vp, sz, u32, i32, vp, vp, vp],
        "vbyte_decode_noalloc": [vp, sz, vp, sz, u32, i32, vp, vp],
        "vbyte_batch_graph_create": [vp, sz, vp, vp, sz, vp, sz, vp, i32, vp, c.POINTER(vp)],
        "vbyte_batch_graph_launch": [vp, vp],
        "vbyte_autotune_decode": [vp, sz, vp, sz, i32, i32, vp, c.POINTER(TunePoint), sz,
                                  c.POINTER(sz), vp],
        "vbyte_autotune_batch": [vp, sz, vp, vp, sz, vp, sz, i32, i32, vp, c.POINTER(TunePoint),
                                 sz, c.POINTER(sz), vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c.c_int
    lib.vbyte_tuning_default.argtypes = [vp]
    lib.vbyte_tuning_default.restype = None
    lib.vbyte_get_chunk_tiles.argtypes = []
    lib.vbyte_get_chunk_tiles.restype = c.c_int
    lib.vbyte_batch_graph_destroy.argtypes = [vp]
    lib.vbyte_batch_graph_destroy.restype = None
    lib.vbyte_workspace_size.argtypes = [sz]
    lib.vbyte_workspace_size.restype = sz
    lib.vbyte_get_tuning.argtypes = [c.POINTER(c.c_int), c.POINTER(c.c_int), c.POINTER(c.c_int64)]
    lib.vbyte_get_tuning.restype = None
    lib.vbyte_status_str.argtypes = [c.c_int]
    lib.vbyte_status_str.restype = c.c_char_p
    lib.vbyte_last_error.argtypes = []
    lib.vbyte_last_error.restype = c.c_char_p
    return lib


def _on_stream(fn):
    """Run the wrapped call with ``stream`` (when one is given) as torch's
    current stream: tensors the call allocates belong to that stream, and a
    status or count read back with ``.item()`` is copied on that stream, after
    the kernels that write it."""
    @functools.wraps(fn)
    def call(*args, stream=None, **kw):
        ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
        with ctx:
            return fn(*args, stream=stream, **kw)
    return call


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _check_call(st, what):
    if st != OK:
        raise VByteError(st, what)


def _dev_u8(data):
    if data.dtype != torch.uint8 or not data.is_cuda or not data.is_contiguous():
        raise ValueError("data must be a contiguous torch.uint8 CUDA tensor")
    return data


def _mode(delta, minus_one):
    if minus_one:
        return 2
    return 1 if delta else 0


@_on_stream
def decode(data, n, *, delta=False, minus_one=False, prev=0, out=None, status=None, stream=None,
           check=True, tuning=None):
    """Decode ``n`` uint32 from the VByte bytes ``data`` (uint8 CUDA tensor).
    ``delta``: inclusive prefix sum of the gaps from ``prev``; ``minus_one``:
    differences minus one (vbyte_decode_delta_m1).

    Returns the int32 tensor of results.  With ``check`` the call waits for
    the kernel and raises VByteError on a data error; otherwise the status is
    left in ``status`` (an int32 CUDA tensor of one element) for the caller.
    ``tuning``: a Tuning (make_tuning) for this call only (vbyte_decode_ex);
    None uses the process-wide defaults.
    """
    _dev_u8(data)
    n = int(n)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=data.device)
    elif out.dtype != torch.int32 or out.numel() < n or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor of at least n elements")
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=data.device)
    s = _stream(stream)
    L = _lib()
    if tuning is not None:
        st = L.vbyte_decode_ex(_ptr(data), data.numel(), _ptr(out), n, int(prev) & 0xFFFFFFFF,
                               _mode(delta, minus_one), ctypes.byref(tuning), _ptr(status), s)
    elif minus_one:
        st = L.vbyte_decode_delta_m1_async(_ptr(data), data.numel(), _ptr(out), n,
                                           int(prev) & 0xFFFFFFFF, _ptr(status), s)
    elif delta:
        st = L.vbyte_decode_delta_async(_ptr(data), data.numel(), _ptr(out), n,
                                        int(prev) & 0xFFFFFFFF, _ptr(status), s)
    else:
        st = L.vbyte_decode_async(_ptr(data), data.numel(), _ptr(out), n, _ptr(status), s)
    _check_call(st, "decode")
    if check:
        v = int(status.item())
        if v != OK:
            raise VByteError(v, "decode")
    return out[:n]


@_on_stream
def decode_noalloc(data, n, out, status, *, delta=False, minus_one=False, prev=0, stream=None):
    """vbyte_decode_noalloc: decode into the caller's `out` (int32, at least
    n elements) with the status in `status` (int32 CUDA tensor of one
    element), allocating nothing; asynchronous.  Raises VByteError for
    argument errors (a stream beyond the library's fixed scratch array)."""
    _dev_u8(data)
    n = int(n)
    if out.dtype != torch.int32 or out.numel() < n or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor of at least n elements")
    if status.dtype != torch.int32 or status.numel() < 1:
        raise ValueError("status must be an int32 tensor of one element")
    st = _lib().vbyte_decode_noalloc(_ptr(data), data.numel(), _ptr(out), n, int(prev) & 0xFFFFFFFF,
                                     _mode(delta, minus_one), _ptr(status), _stream(stream))
    _check_call(st, "decode_noalloc")
    return out[:n]


@_on_stream
def decode_delta4(data, n, *, prev4=None, out=None, status=None, stream=None, check=True):
    """Decode ``n`` uint32 coded as differences between blocks of four:
    out[i] = g_i + out[i-4] mod 2^32 from the four values ``prev4`` (zeros
    by default).  Returns the int32 tensor; ``check`` as in decode()."""
    _dev_u8(data)
    n = int(n)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=data.device)
    elif out.dtype != torch.int32 or out.numel() < n or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor of at least n elements")
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=data.device)
    p = None
    if prev4 is not None:
        vals = [int(v) & 0xFFFFFFFF for v in prev4]
        if len(vals) != 4:
            raise ValueError("prev4 must hold four values")
        p = (ctypes.c_uint32 * 4)(*vals)
    st = _lib().vbyte_decode_delta4_async(_ptr(data), data.numel(), _ptr(out), n, p, _ptr(status),
                                          _stream(stream))
    _check_call(st, "decode_delta4")
    if check:
        v = int(status.item())
        if v != OK:
            raise VByteError(v, "decode_delta4")
    return out[:n]


@_on_stream
def decode64(data, n, *, delta=False, prev=0, out=None, status=None, stream=None, check=True):
    """Decode ``n`` uint64 from the 64-bit VByte bytes ``data`` (uint8 CUDA
    tensor; codes of up to 10 bytes).  ``delta``: inclusive prefix sum from
    ``prev`` mod 2^64.  Returns an int64 tensor holding the uint64 bits;
    ``check`` as in decode()."""
    _dev_u8(data)
    n = int(n)
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=data.device)
    elif out.dtype != torch.int64 or out.numel() < n or not out.is_contiguous():
        raise ValueError("out must be a contiguous int64 tensor of at least n elements")
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=data.device)
    s = _stream(stream)
    L = _lib()
    if delta:
        st = L.vbyte_decode64_delta_async(_ptr(data), data.numel(), _ptr(out), n,
                                          int(prev) & 0xFFFFFFFFFFFFFFFF, _ptr(status), s)
    else:
        st = L.vbyte_decode64_async(_ptr(data), data.numel(), _ptr(out), n, _ptr(status), s)
    _check_call(st, "decode64")
    if check:
        v = int(status.item())
        if v != OK:
            raise VByteError(v, "decode64")
    return out[:n]


@_on_stream
def intersect(a, na, b_ids, *, prev=0, piece=1 << 16, out=None, count=None, status=None,
              stream=None, check=True):
    """Identifiers of the differential list ``a`` (VByte bytes, ``na``
    identifiers from ``prev``) that occur in the sorted ``b_ids`` (int32
    tensor of uint32 values), in list order (vbyte_intersect_async: each
    tile of ``a`` is decoded and tested in registers; the status is the one
    that decoding in pieces of ``piece`` integers gives).  Returns (matches
    tensor, count tensor); with ``check`` the call waits and raises
    VByteError on a data error, after which matches and count are
    unspecified."""
    _dev_u8(a)
    if b_ids.dtype != torch.int32 or not b_ids.is_cuda or not b_ids.is_contiguous():
        raise ValueError("b_ids must be a contiguous int32 CUDA tensor (uint32 bits)")
    na = int(na)
    if out is None:
        out = torch.empty(max(min(na, 1 << 28), 1), dtype=torch.int32, device=a.device)
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=a.device)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=a.device)
    st = _lib().vbyte_intersect_async(_ptr(a), a.numel(), na, int(prev) & 0xFFFFFFFF, _ptr(b_ids),
                                      b_ids.numel(), int(piece), _ptr(out), out.numel(), _ptr(count),
                                      _ptr(status), _stream(stream))
    _check_call(st, "intersect")
    if check:
        v = int(status.item())
        if v != OK:
            raise VByteError(v, "intersect")
        return out[: min(int(count.item()), out.numel())], count
    return out, count


def new_cursor(prev=0, device=None):
    """A device cursor (int64 tensor of 3: byte offset, decoded, prev) at
    the start of a stream."""
    return torch.tensor([0, 0, int(prev) & 0xFFFFFFFF], dtype=torch.int64,
                        device=device or torch.device("cuda"))


@_on_stream
def decode_next(data, k, out, cursor_in, cursor_out, *, delta=False, minus_one=False, status=None,
                stream=None):
    """Decode the next piece of at most k integers of ``data`` into out[0..k)
    from ``cursor_in`` and write the advanced cursor to ``cursor_out`` (both
    int64 CUDA tensors of 3, see new_cursor).  Does not wait; the data status
    goes to ``status`` (int32 CUDA tensor of one element)."""
    _dev_u8(data)
    if out.dtype != torch.int32 or not out.is_contiguous() or out.numel() < int(k):
        raise ValueError("out must be a contiguous int32 tensor of at least k elements")
    for c in (cursor_in, cursor_out):
        if c.dtype != torch.int64 or c.numel() != 3 or not c.is_cuda:
            raise ValueError("cursors must be int64 CUDA tensors of 3 elements")
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=data.device)
    st = _lib().vbyte_decode_next_async(_ptr(data), data.numel(), _ptr(out), int(k),
                                        _mode(delta, minus_one), _ptr(cursor_in), _ptr(cursor_out),
                                        _ptr(status), _stream(stream))
    _check_call(st, "decode_next")
    return status


@_on_stream
def count(data, *, stream=None, result=None):
    """Number of terminator bytes (codes) in ``data``; returns a Python int
    (or fills the uint64 slot of ``result``, an int64 CUDA tensor, without
    waiting when given).  A count whose look-back gave up (VBYTE_ESTALLED,
    see set_spin_limit) reads as -1 (2^64 - 1 as int64)."""
    _dev_u8(data)
    res = result if result is not None else torch.empty(1, dtype=torch.int64, device=data.device)
    _check_call(_lib().vbyte_count(_ptr(data), data.numel(), _ptr(res), _stream(stream)), "count")
    if result is not None:
        return result
    return int(res.item())


@_on_stream
def decode_batch(data, byte_off, out_off, *, delta=False, minus_one=False, prevs=None, out=None,
                 list_status=None, stream=None):
    """Batched CSR decode.  byte_off/out_off: int64 CUDA tensors of nlists+1.
    Returns (out int32 tensor, per-list int32 status tensor); no wait."""
    _dev_u8(data)
    nlists = byte_off.numel() - 1
    if out is None:
        total = int(out_off[-1].item()) if nlists > 0 else 0
        out = torch.empty(max(total, 0), dtype=torch.int32, device=data.device)
    if list_status is None:
        list_status = torch.empty(max(nlists, 0), dtype=torch.int32, device=data.device)
    st = _lib().vbyte_decode_batch(_ptr(data), data.numel(), _ptr(byte_off), _ptr(out), out.numel(),
                                   _ptr(out_off), max(nlists, 0), _ptr(prevs),
                                   _mode(delta, minus_one), _ptr(list_status), _stream(stream))
    _check_call(st, "decode_batch")
    return out, list_status


@_on_stream
def decode_lists(data, rows, list_bytes, out, *, delta=False, minus_one=False, prevs=None,
                 list_status=None, stream=None):
    """Gather-form batch: rows is an int64 CUDA tensor [nlists, 4] of
    (byte_begin, byte_end, out_begin, n).  Returns the per-list status."""
    _dev_u8(data)
    nlists = rows.shape[0] if rows.numel() else 0
    if list_status is None:
        list_status = torch.empty(nlists, dtype=torch.int32, device=data.device)
    st = _lib().vbyte_decode_lists(_ptr(data), data.numel(), _ptr(rows), nlists, int(list_bytes),
                                   _ptr(out), out.numel(), _ptr(prevs), _mode(delta, minus_one),
                                   _ptr(list_status), _stream(stream))
    _check_call(st, "decode_lists")
    return list_status


class BatchGraph:
    """A batched decode captured into a HIP graph (vbyte_batch_graph_*):
    the buffers are fixed at creation, their contents are read at each
    replay.  Replays of one graph must be ordered."""

    def __init__(self, data, byte_off, out_off, out, list_status, *, delta=False, minus_one=False,
                 prevs=None):
        _dev_u8(data)
        nlists = byte_off.numel() - 1
        self._keep = (data, byte_off, out_off, out, list_status, prevs)
        h = ctypes.c_void_p()
        st = _lib().vbyte_batch_graph_create(_ptr(data), data.numel(), _ptr(byte_off), _ptr(out),
                                             out.numel(), _ptr(out_off), max(nlists, 0),
                                             _ptr(prevs), _mode(delta, minus_one),
                                             _ptr(list_status), ctypes.byref(h))
        _check_call(st, "batch_graph_create")
        self.handle = h

    def launch(self, stream=None):
        _check_call(_lib().vbyte_batch_graph_launch(self.handle, _stream(stream)), "batch_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize()
            _lib().vbyte_batch_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _points(arr, n):
    return [{"segs_per_wave": p.segs_per_wave, "waves_per_block": p.waves_per_block,
             "small_list_bytes": p.small_list_bytes, "tiles_per_chunk": p.tiles_per_chunk,
             "ms": p.ms, "status": p.status}
            for p in arr[:n]]


@_on_stream
def autotune_decode(data, n, *, delta=False, out=None, reps=5, stream=None):
    """Run the library's autotuner on a single-stream decode of `data` and
    apply the fastest tiling; returns the timed candidates."""
    _dev_u8(data)
    n = int(n)
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.int32, device=data.device)
    status = torch.empty(1, dtype=torch.int32, device=data.device)
    arr = (TunePoint * 32)()
    cnt = ctypes.c_size_t()
    st = _lib().vbyte_autotune_decode(_ptr(data), data.numel(), _ptr(out), n, 1 if delta else 0,
                                      int(reps), _ptr(status), arr, 32, ctypes.byref(cnt),
                                      _stream(stream))
    _check_call(st, "autotune_decode")
    return _points(arr, cnt.value)


@_on_stream
def autotune_batch(data, byte_off, out_off, *, delta=False, out=None, reps=3, stream=None):
    """Run the library's autotuner on a batched CSR decode and apply the
    fastest tiling and small-list threshold; returns the timed candidates."""
    _dev_u8(data)
    nlists = byte_off.numel() - 1
    if out is None:
        total = int(out_off[-1].item()) if nlists > 0 else 0
        out = torch.empty(max(total, 1), dtype=torch.int32, device=data.device)
    status = torch.empty(max(nlists, 1), dtype=torch.int32, device=data.device)
    arr = (TunePoint * 32)()
    cnt = ctypes.c_size_t()
    st = _lib().vbyte_autotune_batch(_ptr(data), data.numel(), _ptr(byte_off), _ptr(out),
                                     out.numel(), _ptr(out_off), max(nlists, 0), 1 if delta else 0,
                                     int(reps), _ptr(status), arr, 32, ctypes.byref(cnt),
                                     _stream(stream))
    _check_call(st, "autotune_batch")
    return _points(arr, cnt.value)


@_on_stream
def encode(values, *, delta=False, minus_one=False, prev=0, out=None, nbytes=None, stream=None,
           trim=True):
    """Canonical VByte encoding on the GPU of an int32/uint32-bits CUDA tensor.
    Returns the uint8 tensor of codes (trimmed to the encoded size when
    ``trim``, which waits for the kernel)."""
    if values.dtype != torch.int32 or not values.is_cuda or not values.is_contiguous():
        raise ValueError("values must be a contiguous int32 CUDA tensor (uint32 bits)")
    n = values.numel()
    if out is None:
        out = torch.empty(max(5 * n, 1), dtype=torch.uint8, device=values.device)
    if nbytes is None:
        nbytes = torch.empty(1, dtype=torch.int64, device=values.device)
    s = _stream(stream)
    L = _lib()
    if minus_one:
        st = L.vbyte_encode_delta_m1_async(_ptr(values), n, int(prev) & 0xFFFFFFFF, _ptr(out),
                                           out.numel(), _ptr(nbytes), s)
    elif delta:
        st = L.vbyte_encode_delta_async(_ptr(values), n, int(prev) & 0xFFFFFFFF, _ptr(out),
                                        out.numel(), _ptr(nbytes), s)
    else:
        st = L.vbyte_encode_async(_ptr(values), n, _ptr(out), out.numel(), _ptr(nbytes), s)
    _check_call(st, "encode")
    if trim:
        return out[: int(nbytes.item())]
    return out, nbytes


@_on_stream
def encode_batch(values, vals_off, *, stream=None):
    """Batched CSR encoding on the GPU.  values: int32 CUDA tensor (uint32
    bits, all lists concatenated); vals_off: int64 CUDA tensor of nlists+1
    value offsets.  Returns (bytes uint8 tensor, byte_off int64 tensor);
    waits for the kernel to learn the encoded size."""
    if values.dtype != torch.int32 or not values.is_cuda or not values.is_contiguous():
        raise ValueError("values must be a contiguous int32 CUDA tensor (uint32 bits)")
    n = values.numel()
    nlists = vals_off.numel() - 1
    out = torch.empty(max(5 * n, 1), dtype=torch.uint8, device=values.device)
    byte_off = torch.empty(max(nlists + 1, 1), dtype=torch.int64, device=values.device)
    nbytes = torch.empty(1, dtype=torch.int64, device=values.device)
    st = _lib().vbyte_encode_batch(_ptr(values), n, _ptr(vals_off), max(nlists, 0), _ptr(out),
                                   out.numel(), _ptr(byte_off), _ptr(nbytes), _stream(stream))
    _check_call(st, "encode_batch")
    return out[: int(nbytes.item())], byte_off[: nlists + 1]


def set_tuning(segs_per_wave=0, waves_per_block=0, small_list_bytes=0, tiles_per_chunk=None):
    """Set the kernel tuning (0 keeps a value); tiles_per_chunk selects the
    single-stream kernel (-2: one read, -1: two passes, 0: per-tile
    look-back, k: chunks of k tiles)."""
    _check_call(_lib().vbyte_set_tuning(int(segs_per_wave), int(waves_per_block),
                                        int(small_list_bytes)), "set_tuning")
    if tiles_per_chunk is not None:
        _check_call(_lib().vbyte_set_chunk_tiles(int(tiles_per_chunk)), "set_chunk_tiles")


def set_spin_limit(rounds=0):
    """Look-back round trips before a waiting tile gives up (0: default)."""
    _check_call(_lib().vbyte_set_spin_limit(int(rounds)), "set_spin_limit")


def set_flow_grid(grid=0):
    """Default workgroups of the one-read schedule (0: 16 wavefronts per CU)."""
    _check_call(_lib().vbyte_set_flow_grid(int(grid)), "set_flow_grid")


def get_tuning():
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
    _lib().vbyte_get_tuning(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return {"segs_per_wave": a.value, "waves_per_block": b.value, "small_list_bytes": c.value,
            "tiles_per_chunk": int(_lib().vbyte_get_chunk_tiles())}


def workspace_size(nbytes):
    return int(_lib().vbyte_workspace_size(int(nbytes)))


def as_u32_numpy(t):
    """Host numpy uint32 view of an int32 result tensor."""
    return t.detach().cpu().numpy().view("uint32")
