"""GPU parity at the full sizes of the five synthetic configurations, in the
default launch configuration (the one bench.py times), bit-exact against the
CPU oracle on the same inputs."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import u32
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu


def _decode(b, n, delta=False, prev=0):
    d = torch.from_numpy(b).cuda()
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    out = vbyte.decode(d, n, delta=delta, prev=prev, status=st, check=False)
    torch.cuda.synchronize()
    s = int(st.item())
    h = u32(out)
    del d, out
    return s, h


def test_config1_uniform_lengths():
    x, L = workloads.uniform_lengths()
    b = oracle.encode(x)
    assert abs(b.size / x.size - 3.0) < 0.01
    st, y = _decode(b, x.size)
    sto, yo = oracle.decode(b, x.size)
    assert st == sto == vbyte.OK
    assert np.array_equal(y, yo) and np.array_equal(y, x)


@pytest.fixture
def chunked_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


@pytest.mark.parametrize("chunk", [0, 2, 8, -1, -2])
@pytest.mark.parametrize("mean", [8, 300])
def test_config2_differential_streams(mean, chunk, chunked_tuning):
    vbyte.set_tuning(tiles_per_chunk=chunk)
    g = workloads.geometric_gaps(mean=mean)
    b = oracle.encode(g)
    expect_bpi = {8: 1.0, 300: 1.6544}[mean]
    assert abs(b.size / g.size - expect_bpi) < 0.002
    st, y = _decode(b, g.size, delta=True)
    sto, yo = oracle.decode_delta(b, g.size, 0)
    assert st == sto == vbyte.OK
    assert np.array_equal(y, yo)


def test_config3_batched_lists():
    d = workloads.zipf_lists()
    gaps, out_off, lengths = d["gaps"], d["out_off"], d["lengths"]
    assert int(out_off[-1]) == 1 << 28
    b = oracle.encode(gaps)   # the concatenation of the lists' codes
    nb = np.empty(lengths.size, np.int64)
    for i in range(lengths.size):
        nb[i] = oracle.encoded_size(gaps[out_off[i]:out_off[i + 1]])
    byte_off = np.zeros(lengths.size + 1, np.int64)
    np.cumsum(nb, out=byte_off[1:])
    assert byte_off[-1] == b.size
    bits_per_int = 8 * b.size / gaps.size
    assert 8.0 <= bits_per_int < 16.0          # the paper's range (section 5)
    bd = torch.from_numpy(b).cuda()
    out, st = vbyte.decode_batch(bd, torch.from_numpy(byte_off).cuda(),
                                 torch.from_numpy(out_off).cuda(), delta=True)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == vbyte.OK).all()
    y = u32(out)
    sto, yo, lst = oracle.decode_batch(b, byte_off, out_off, None, True)
    assert sto == oracle.OK and (lst == oracle.OK).all()
    assert np.array_equal(y, yo)


@pytest.fixture(scope="module")
def mix():
    x = workloads.worst_case_mix()
    b = oracle.encode(x)
    return x, b


@pytest.mark.parametrize("chunk", [0, 16, -1, -2])
def test_config5_plain(mix, chunk, chunked_tuning):
    vbyte.set_tuning(tiles_per_chunk=chunk)
    x, b = mix
    assert abs(b.size / x.size - 1.675) < 0.002
    st, y = _decode(b, x.size)
    assert st == vbyte.OK
    assert np.array_equal(y, x)          # DEC(ENC(x)) = x, pinned for the oracle
    k = workloads.MIX_CHUNK
    cut = oracle.encoded_size(x[:3 * k])
    cut2 = cut + oracle.encoded_size(x[3 * k:4 * k])
    sto, yo = oracle.decode(b[cut:cut2], k)
    assert sto == oracle.OK and np.array_equal(y[3 * k:4 * k], yo)


@pytest.mark.parametrize("chunk", [0, -1, -2])
def test_config5_delta(mix, chunk, chunked_tuning):
    vbyte.set_tuning(tiles_per_chunk=chunk)
    x, b = mix
    st, y = _decode(b, x.size, delta=True, prev=12345)
    assert st == vbyte.OK
    sto, yo = oracle.decode_delta(b, x.size, 12345)
    assert sto == oracle.OK and np.array_equal(y, yo)
