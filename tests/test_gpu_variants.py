"""GPU parity of the differential variant "differences minus one" (section 1,
reading R11): the single-stream decode over tilings, alignments, one-byte
segments, ragged tails and count guards; the batched and graph forms; the
encoder; and the full-size 64Mi streams of the benchmark workload."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import SENTINEL, mixed_values, place_bytes, u32
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def decode_m1(b, n, prev=0, boff=0, ooff=0):
    _, data = place_bytes(b, boff)
    full = torch.full((ooff + n + 16,), SENTINEL, dtype=torch.int32, device="cuda")
    out = full[ooff:ooff + n]
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    vbyte.decode(data, n, minus_one=True, prev=prev, out=out, status=st, check=False)
    torch.cuda.synchronize()
    h = u32(full)
    assert (h[:ooff] == SENTINEL).all() and (h[ooff + n:] == SENTINEL).all()
    return int(st.item()), h[ooff:ooff + n]


def check(b, n, prev=0, boff=0, ooff=0):
    st, y = decode_m1(b, n, prev, boff, ooff)
    sto, yo = oracle.decode_delta_m1(b, n, prev)
    assert st == sto
    if sto == oracle.OK:
        assert np.array_equal(y, yo), f"first mismatch at {np.nonzero(y != yo)[0][:1]}"


@pytest.mark.parametrize("tiling", [(4, 8, 0), (1, 2, 0), (2, 4, 0), (4, 8, 4), (2, 4, 2), (2, 8, -1), (1, 2, -1),
                                    (2, 8, -2), (1, 2, -2)])
@pytest.mark.parametrize("kind", ["mixed", "ones", "gaps300"])
@pytest.mark.parametrize("n", [1, 777, 40_000, 300_001])
def test_stream_m1(tiling, kind, n):
    vbyte.set_tuning(tiling[0], tiling[1], 0, tiles_per_chunk=tiling[2])
    rng = np.random.default_rng(n + len(kind))
    if kind == "mixed":
        g = mixed_values(rng, n)
    elif kind == "ones":
        g = rng.integers(0, 128, n).astype(np.uint32)
    else:
        g = rng.geometric(1 / 300.0, n).astype(np.uint32)
    b = oracle.encode(g)
    check(b, n, prev=0)
    check(b, n, prev=0xFFFFFFFF, boff=5, ooff=3)


def test_stream_m1_counts_and_errors():
    rng = np.random.default_rng(5)
    g = mixed_values(rng, 50_000)
    b = oracle.encode(g)
    check(b, 49_000)            # more codes than n: ECOUNT, nothing past n
    check(b, 51_000)            # fewer: ETRUNC
    check(b[:-1], 50_000)       # truncated tail
    check(np.zeros(0, np.uint8), 0)


def test_stream_m1_resumes_with_prev_plus_one():
    rng = np.random.default_rng(6)
    ids = np.unique(rng.integers(0, 1 << 31, 100_000, dtype=np.uint64)).astype(np.uint32)
    b = oracle.encode_delta_m1(ids, 0)
    m = 41_234
    cut = int(oracle.encode_delta_m1(ids[:m], 0).size)
    st1, y1 = decode_m1(b[:cut], m, 0)
    st2, y2 = decode_m1(b[cut:], ids.size - m, int(y1[-1]) + 1)
    assert st1 == st2 == vbyte.OK
    assert np.array_equal(np.concatenate([y1, y2]), ids)


def test_encoder_m1_matches_oracle():
    rng = np.random.default_rng(7)
    ids = np.unique(rng.integers(0, 1 << 32, 200_000, dtype=np.uint64)).astype(np.uint32)
    for prev in (0, 17):
        d = torch.from_numpy(ids.view(np.int32)).cuda()
        enc = vbyte.encode(d, minus_one=True, prev=prev)
        assert np.array_equal(enc.cpu().numpy(), oracle.encode_delta_m1(ids, prev))
        y = vbyte.decode(enc, ids.size, minus_one=True, prev=prev)
        assert np.array_equal(u32(y), ids)


def lists(seed, nl=300):
    rng = np.random.default_rng(seed)
    lens = np.concatenate([rng.integers(0, 400, nl - 4), [60_000, 150_000, 9_000, 1]])
    rng.shuffle(lens)
    out_off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=out_off[1:])
    gaps = rng.geometric(1 / 50.0, int(out_off[-1])).astype(np.uint32)
    b = oracle.encode(gaps)
    byte_off = np.zeros(lens.size + 1, np.int64)
    for i in range(lens.size):
        byte_off[i + 1] = byte_off[i] + oracle.encoded_size(gaps[out_off[i]:out_off[i + 1]])
    return b, byte_off, out_off


@pytest.mark.parametrize("small", [0, 4096, 1 << 20])
def test_batch_and_graph_m1(small):
    if small:
        vbyte.set_tuning(0, 0, small)
    b, byte_off, out_off = lists(8)
    nl = byte_off.size - 1
    prevs = np.random.default_rng(9).integers(0, 1 << 32, nl, dtype=np.uint64).astype(np.uint32)
    pd = torch.from_numpy(prevs.view(np.int32)).cuda()
    bd, bo, oo = (torch.from_numpy(x).cuda() for x in (b, byte_off, out_off))
    out, st = vbyte.decode_batch(bd, bo, oo, minus_one=True, prevs=pd)
    torch.cuda.synchronize()
    sto, yo, _ = oracle.decode_batch(b, byte_off, out_off, prevs, 2)
    assert sto == oracle.OK and (st.cpu().numpy() == vbyte.OK).all()
    assert np.array_equal(u32(out), yo)
    gout = torch.empty_like(out)
    gst = torch.empty_like(st)
    g = vbyte.BatchGraph(bd, bo, oo, gout, gst, minus_one=True, prevs=pd)
    try:
        for _ in range(2):
            gout.fill_(0)
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(u32(gout), yo)
    finally:
        g.close()


@pytest.mark.parametrize("chunk", [0, 4, -1, -2])
@pytest.mark.parametrize("mean", [8, 300])
def test_full_size_stream_m1(mean, chunk):
    vbyte.set_tuning(tiles_per_chunk=chunk)
    g = workloads.geometric_gaps(mean=mean)
    b = oracle.encode(g)
    d = torch.from_numpy(b).cuda()
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    out = vbyte.decode(d, g.size, minus_one=True, prev=3, status=st, check=False)
    torch.cuda.synchronize()
    sto, yo = oracle.decode_delta_m1(b, g.size, 3)
    assert int(st.item()) == sto == vbyte.OK
    assert np.array_equal(u32(out), yo)
