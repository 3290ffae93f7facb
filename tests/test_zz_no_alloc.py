"""The allocation-free decode (vbyte_decode_noalloc) against the decode
with a workspace (vbyte_decode_ex, the same two-pass schedule and tiling),
through the C ABI: bit-exact outputs and equal statuses, on two calls in a
row, the second with a smaller input, in plain, differential and
differences-minus-one modes; the size limit is an argument error."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_util import mixed_values, u32
from paper_1503_07387_amd import vbyte

pytestmark = pytest.mark.gpu


def reference(d, n, mode, prev):
    T = vbyte.make_tuning(2, 8, vbyte.SCHED_TWO_PASS)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    y = vbyte.decode(d, n, delta=mode == 1, minus_one=mode == 2, prev=prev, status=st, check=False,
                     tuning=T)
    torch.cuda.synchronize()
    return int(st.item()), u32(y)


def noalloc(d, n, mode, prev, boff=0):
    full = torch.full((n + 8,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    vbyte.decode_noalloc(d, n, full, st, delta=mode == 1, minus_one=mode == 2, prev=prev)
    torch.cuda.synchronize()
    h = u32(full)
    assert (h[n:] == 0x5A5A5A5A).all(), "write past out[n-1]"
    return int(st.item()), h[:n]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_two_calls_second_smaller(mode):
    rng = np.random.default_rng(70 + mode)
    for n, boff in ((3_000_017, 5), (40_001, 11)):   # the second call is smaller
        x = mixed_values(rng, n)
        b = oracle.encode(x)
        host = np.zeros(b.size + 64, np.uint8)
        host[boff:boff + b.size] = b
        d = torch.from_numpy(host).cuda()[boff:boff + b.size]
        st, y = noalloc(d, n, mode, 123)
        sr, yr = reference(d, n, mode, 123)
        assert st == sr == vbyte.OK, (st, sr)
        assert np.array_equal(y, yr)
        if mode == 0:
            assert np.array_equal(y, x)


def test_statuses_match_the_workspace_decode():
    rng = np.random.default_rng(77)
    x = mixed_values(rng, 100_000)
    b = oracle.encode(x)
    bad = b.copy()
    bad[5000:5006] = 0x80
    for buf, n in ((b, x.size), (b[:-1], x.size), (b, x.size + 3), (b, x.size - 2), (bad, x.size)):
        d = torch.from_numpy(np.ascontiguousarray(buf)).cuda()
        st, _ = noalloc(d, n, 0, 0)
        sr, _ = reference(d, n, 0, 0)
        assert st == sr == oracle.validate(np.ascontiguousarray(buf), n)


def test_empty_and_size_limit():
    d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    st, _ = noalloc(d[:0], 0, 0, 0)
    assert st == vbyte.OK
    out = torch.empty(8, dtype=torch.int32, device="cuda")
    status = torch.empty(1, dtype=torch.int32, device="cuda")
    lib = vbyte._lib()
    # a stream of more than 4 GiB: rejected on the host before any launch
    # (the pointer is never dereferenced)
    big = (4 << 30) + 1
    r = lib.vbyte_decode_noalloc(ctypes.c_void_p(d.data_ptr()), big, ctypes.c_void_p(out.data_ptr()),
                                 1, 0, 0, ctypes.c_void_p(status.data_ptr()), None)
    assert r == vbyte.EINVAL
    assert b"scratch" in lib.vbyte_last_error()
