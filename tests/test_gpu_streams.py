"""Binding calls given a stream other than torch's current one: the outputs
they allocate belong to that stream, and with check=True the status (or
count, or encoded size) is read after the kernels on that stream, never from
the uninitialised word.  The side stream is kept busy first so that a read
ordered on the wrong stream would run before the decode."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import u32
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu


def busy(stream):
    # a few hundred microseconds of work queued on `stream`
    with torch.cuda.stream(stream):
        a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        for _ in range(8):
            a.mul_(1.0000001)
    return a


def test_decode_on_side_stream_valid_and_malformed():
    x, _ = workloads.uniform_lengths(n=1 << 22)
    b = oracle.encode(x)
    data = torch.from_numpy(b).cuda()
    side = torch.cuda.Stream()
    for rep in range(3):
        keep = busy(side)
        y = vbyte.decode(data, x.size, stream=side)   # check=True: reads the status
        side.synchronize()
        assert np.array_equal(u32(y), x), f"rep {rep}"
        del keep
    # malformed: six continuation bytes in the middle
    bad = b.copy()
    bad[1000:1006] = 0x80
    dbad = torch.from_numpy(bad).cuda()
    for rep in range(3):
        keep = busy(side)
        with pytest.raises(vbyte.VByteError) as ei:
            vbyte.decode(dbad, x.size, stream=side)
        assert ei.value.status == vbyte.EMALFORMED
        del keep
    side.synchronize()


def test_delta_decode_count_and_encode_on_side_stream():
    g = workloads.geometric_gaps(n=1 << 22, mean=300)
    b = oracle.encode(g)
    data = torch.from_numpy(b).cuda()
    side = torch.cuda.Stream()
    keep = busy(side)
    y = vbyte.decode(data, g.size, delta=True, prev=5, stream=side)
    side.synchronize()
    st, ref = oracle.decode_delta(b, g.size, 5)
    assert st == oracle.OK and np.array_equal(u32(y), ref)
    keep = busy(side)
    assert vbyte.count(data, stream=side) == g.size
    gd = torch.from_numpy(g.view(np.int32)).cuda()
    side.synchronize()
    keep = busy(side)
    enc = vbyte.encode(gd, stream=side)
    side.synchronize()
    assert np.array_equal(enc.cpu().numpy(), b)
    del keep
