"""Python binding of the serving loop (vbyte_server_* in include/vbyte.h).

Argument marshalling only: the loop itself (arrivals, admission by pool
memory, batching, stream overlap, completion tracking) runs in
``csrc/serve.cpp`` inside libvbyte.
"""
import ctypes

import numpy as np
import torch

from . import vbyte


class ServerConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_size_t), ("nstreams", ctypes.c_int),
                ("max_batch_requests", ctypes.c_int), ("batching", ctypes.c_int),
                ("delta", ctypes.c_int)]


class ServeStats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("integers", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("mean_batch_requests", ctypes.c_double), ("worst_status", ctypes.c_int32),
                ("rejected", ctypes.c_uint64)]


def _declare(lib):
    if getattr(lib, "_serve_declared", False):
        return lib
    c = ctypes
    lib.vbyte_server_create.argtypes = [c.c_void_p, c.c_size_t, c.c_void_p, c.c_void_p, c.c_size_t,
                                        c.POINTER(ServerConfig), c.POINTER(c.c_void_p)]
    lib.vbyte_server_create.restype = c.c_int
    lib.vbyte_server_destroy.argtypes = [c.c_void_p]
    lib.vbyte_server_destroy.restype = None
    lib.vbyte_server_run.argtypes = [c.c_void_p, c.c_size_t, c.c_void_p, c.c_void_p, c.c_void_p,
                                     c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p,
                                     c.POINTER(ServeStats)]
    lib.vbyte_server_run.restype = c.c_int
    lib._serve_declared = True
    return lib


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else ctypes.c_void_p(0)


class Server:
    """Continuous-batching decode server over an index resident in HBM.

    index: uint8 CUDA tensor holding every list's codes; byte_off: host int64
    array of nlists+1 list boundaries; counts: host int64 integers per list.
    """

    def __init__(self, index, byte_off, counts, *, pool_bytes=1 << 30, nstreams=4,
                 max_batch_requests=256, batching=True, delta=True):
        self.lib = _declare(vbyte._lib())
        self.index = index
        self.byte_off = np.ascontiguousarray(byte_off, dtype=np.int64)
        self.counts = np.ascontiguousarray(counts, dtype=np.int64)
        cfg = ServerConfig(int(pool_bytes), int(nstreams), int(max_batch_requests),
                           1 if batching else 0, 1 if delta else 0)
        h = ctypes.c_void_p()
        st = self.lib.vbyte_server_create(ctypes.c_void_p(index.data_ptr()), index.numel(),
                                          _np_ptr(self.byte_off), _np_ptr(self.counts),
                                          self.counts.size, ctypes.byref(cfg), ctypes.byref(h))
        if st != vbyte.OK:
            raise vbyte.VByteError(st, "server_create")
        self.handle = h

    def run(self, arrivals, terms, *, capture=False):
        """Run one open-loop workload.  arrivals: seconds (non-decreasing);
        terms: list of int64 arrays of list indices.  Returns (latencies in
        seconds, stats dict, results) where results is (uint32 CUDA tensor,
        offsets) when capture is set; stats["status"] holds every request's
        status (int32 array)."""
        torch.cuda.synchronize()
        arrivals = np.ascontiguousarray(arrivals, dtype=np.float64)
        nreq = arrivals.size
        term_off = np.zeros(nreq + 1, np.int64)
        term_off[1:] = np.cumsum([len(t) for t in terms])
        flat = np.ascontiguousarray(np.concatenate(terms) if nreq else np.zeros(0), dtype=np.int64)
        lat = np.zeros(nreq, np.float64)
        rst = np.zeros(nreq, np.int32)
        res = None
        res_off = None
        if capture:
            need = np.array([int(self.counts[t].sum()) for t in terms], np.int64)
            res_off = np.zeros(nreq + 1, np.int64)
            res_off[1:] = np.cumsum(need)
            res = torch.empty(max(int(res_off[-1]), 1), dtype=torch.int32, device=self.index.device)
        stats = ServeStats()
        st = self.lib.vbyte_server_run(self.handle, nreq, _np_ptr(arrivals), _np_ptr(term_off),
                                       _np_ptr(flat), _np_ptr(lat), _np_ptr(rst),
                                       ctypes.c_void_p(res.data_ptr()) if capture else ctypes.c_void_p(0),
                                       _np_ptr(res_off) if capture else ctypes.c_void_p(0),
                                       ctypes.byref(stats))
        if st != vbyte.OK:
            raise vbyte.VByteError(st, "server_run")
        out = {k: getattr(stats, k) for k, _ in ServeStats._fields_}
        out["status"] = rst
        return lat, out, ((res, res_off) if capture else None)

    def close(self):
        if self.handle:
            self.lib.vbyte_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
