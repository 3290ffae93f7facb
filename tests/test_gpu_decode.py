"""GPU parity of the single-stream decode, count and encode (bit-exact
against the CPU oracle), through the C ABI on cuda:0."""
import numpy as np
import pytest
import torch

import oracle
import pins
from gpu_util import check_against_oracle, dev, gpu_decode, mixed_values, place_bytes, u32
from paper_1503_07387_amd import vbyte

pytestmark = pytest.mark.gpu

DEFAULT_TUNING = None


@pytest.fixture(autouse=True, params=[0, 3, -1, -2],
                ids=["tile_lookback", "chunks_of_3", "two_pass", "one_read"])
def restore_tuning(request):
    """Every test runs with the four single-stream schedules: one look-back
    per tile, chunks of 3 tiles per workgroup, the three launches with no
    look-back (tile byte sums, scan, decode), and the one launch that reads
    every byte once (persistent rounds, aggregates published per tile)."""
    t = vbyte.get_tuning()
    vbyte.set_tuning(tiles_per_chunk=request.param)
    yield
    vbyte.set_tuning(**t)


def test_table1_and_fig1():
    for v, b in pins.read_table1():
        st, y = gpu_decode(np.frombuffer(b, np.uint8), 1)
        assert st == vbyte.OK and int(y[0]) == v
    buf, _, ints = pins.read_fig1()
    st, y = gpu_decode(np.frombuffer(buf, np.uint8), len(ints))
    assert st == vbyte.OK and y.tolist() == ints


def test_empty_and_single_codes_every_alignment():
    st, y = gpu_decode(np.zeros(0, np.uint8), 0)
    assert st == vbyte.OK and y.size == 0
    st, _ = gpu_decode(np.zeros(0, np.uint8), 3)
    assert st == vbyte.ETRUNC
    for v in pins.boundary_values():
        b = oracle.encode(np.array([v], np.uint32))
        for boff in range(16):
            st, y = gpu_decode(b, 1, boff=boff, ooff=boff % 4)
            assert st == vbyte.OK and int(y[0]) == v, (v, boff)


@pytest.mark.parametrize("fill,n_of", [(0x00, 1), (0x7F, 1)])
def test_uniform_bytes(fill, n_of):
    for nb in (1, 15, 16, 17, 1023, 1024, 1025, 4096, 4097, 65536 + 7):
        b = np.full(nb, fill, np.uint8)
        for delta in (False, True):
            check_against_oracle(b, nb, delta=delta, prev=0xFFFFFFFF)


def test_alternating_one_two_bytes():
    # the mix that defeats a branchy scalar decoder (section 2)
    x = np.tile(np.array([5, 300], np.uint32), 50000)
    b = oracle.encode(x)
    for boff in (0, 3):
        check_against_oracle(b, x.size, boff=boff)
        check_against_oracle(b, x.size, delta=True, prev=0xFFFFFFFF, boff=boff)


SIZES = [1, 2, 15, 16, 17, 63, 64, 65, 1000, 1023, 1024, 1025, 4095, 4096, 4097, 16389,
         100003, (1 << 20) + 3]


@pytest.mark.parametrize("n", SIZES)
def test_random_mixed_lengths(n):
    rng = np.random.default_rng(n)
    x = mixed_values(rng, n)
    b = oracle.encode(x)
    for boff, ooff in ((0, 0), (1, 1), (7, 2), (15, 3)):
        st, y = check_against_oracle(b, n, boff=boff, ooff=ooff)
        assert st == vbyte.OK and np.array_equal(y, x)
        st, y = check_against_oracle(b, n, delta=True, prev=123456789, boff=boff, ooff=ooff)
        assert st == vbyte.OK


@pytest.mark.parametrize("lengths", [(1,), (2,), (3,), (4,), (5,), (1, 2), (1, 5), (4, 5)])
def test_fixed_length_mixes(lengths):
    rng = np.random.default_rng(sum(lengths))
    x = mixed_values(rng, 70001, lengths)
    b = oracle.encode(x)
    check_against_oracle(b, x.size, boff=5)
    check_against_oracle(b, x.size, delta=True, prev=7, boff=9)


@pytest.mark.parametrize("segs", [1, 2, 4])
@pytest.mark.parametrize("wpb", [1, 4, 8])
def test_tile_straddle(segs, wpb):
    """A 5-byte (and a 3-byte) code placed at every phase across every lane,
    segment and tile boundary, for each tiling the tuner can pick."""
    vbyte.set_tuning(segs, wpb, 0)
    tb = segs * 1024
    rng = np.random.default_rng(segs * 10 + wpb)
    for long_len in (5, 3):
        vals = []
        pos = 0
        targets = sorted({k * 16 for k in range(1, 70)} | {k * 1024 for k in range(1, 6)} |
                         {k * tb for k in range(1, 5)})
        for tgt in targets:
            for phase in range(long_len + 1):
                start = tgt - phase
                while pos < start:      # 1-byte fillers up to the start
                    vals.append(int(rng.integers(0, 128)))
                    pos += 1
                if pos == start:
                    lo = 1 << (7 * (long_len - 1))
                    hi = min(1 << (7 * long_len), 1 << 32)
                    vals.append(int(rng.integers(lo, hi)))
                    pos += long_len
        x = np.array(vals, np.uint32)
        b = oracle.encode(x)
        for boff in (0, 1, 13):
            st, y = check_against_oracle(b, x.size, boff=boff)
            assert np.array_equal(y, x)
            check_against_oracle(b, x.size, delta=True, prev=99, boff=boff)


def test_status_readings_match_oracle():
    for buf, n, expect in pins.STATUS_CASES:
        b = np.frombuffer(buf, np.uint8)
        for boff in (0, 6):
            st, _ = gpu_decode(b, n, boff=boff)
            assert st == expect, (buf.hex(), n, st)
            st, _ = gpu_decode(b, n, delta=True, boff=boff)
            assert st == expect


@pytest.mark.parametrize("segs", [1, 4])
def test_status_in_long_streams(segs):
    vbyte.set_tuning(segs, 4, 0)
    tb = segs * 1024
    rng = np.random.default_rng(77)
    x = mixed_values(rng, 50000, (1, 2, 3))
    b = oracle.encode(x)
    n = x.size
    # well-formed, count mismatch both ways, truncated tail
    assert check_against_oracle(b, n)[0] == vbyte.OK
    assert check_against_oracle(b, n - 1)[0] == vbyte.ECOUNT
    assert check_against_oracle(b, n + 1)[0] == vbyte.ETRUNC
    assert check_against_oracle(b[:-1], n)[0] in (vbyte.ETRUNC, vbyte.ECOUNT)
    # a run of 5 continuation bytes across tile, segment and lane boundaries
    for at in (5, 16 * 7 - 2, 1024 - 3, tb - 4, tb, 3 * tb + 1, b.size - 6):
        bad = b.copy()
        bad[at:at + 5] = 0x80
        st, _ = check_against_oracle(bad, n)
        assert st == vbyte.EMALFORMED
        st, _ = check_against_oracle(bad, n, delta=True)
        assert st == vbyte.EMALFORMED
    # run of exactly 4 continuation bytes then a terminator: valid 5-byte code
    ok = oracle.encode(np.array([1] * 3000 + [0xFFFFFFFF] + [2] * 3000, np.uint32))
    assert check_against_oracle(ok, 6001)[0] == vbyte.OK


def test_fifth_byte_wrap_and_overlong():
    cases = [bytes([0x81, 0x82, 0x83, 0x84, e]) for e in (0x10, 0x1F, 0x7F)]
    cases += [b"\x80\x00", b"\xff\x80\x00", b"\x80\x80\x80\x80\x00"]
    for c in cases:
        b = np.frombuffer(c * 3000, np.uint8)
        check_against_oracle(b, 3000)
        check_against_oracle(b, 3000, delta=True, prev=5)


def test_resumable_delta():
    rng = np.random.default_rng(21)
    g = rng.geometric(1 / 300, 200000).astype(np.uint32)
    b = oracle.encode(g)
    st, full = gpu_decode(b, g.size, delta=True, prev=11)
    assert st == vbyte.OK
    m = 77777
    cut = oracle.encoded_size(g[:m])
    st1, y1 = gpu_decode(b[:cut], m, delta=True, prev=11)
    st2, y2 = gpu_decode(b[cut:], g.size - m, delta=True, prev=int(y1[-1]), boff=cut % 16)
    assert st1 == st2 == vbyte.OK
    assert np.array_equal(np.concatenate([y1, y2]), full)


def test_synchronous_calls():
    import ctypes
    rng = np.random.default_rng(4)
    x = mixed_values(rng, 30000)
    b = oracle.encode(x)
    _, data = place_bytes(b, 3)
    out = torch.empty(x.size, dtype=torch.int32, device=dev())
    L = vbyte._lib()
    torch.cuda.synchronize()
    st = L.vbyte_decode(ctypes.c_void_p(data.data_ptr()), b.size, ctypes.c_void_p(out.data_ptr()), x.size)
    assert st == vbyte.OK and np.array_equal(u32(out), x)
    st = L.vbyte_decode_delta(ctypes.c_void_p(data.data_ptr()), b.size, ctypes.c_void_p(out.data_ptr()),
                              x.size, 5)
    assert st == vbyte.OK
    assert np.array_equal(u32(out), oracle.decode_delta(b, x.size, 5)[1])
    st = L.vbyte_decode(ctypes.c_void_p(data.data_ptr()), b.size, ctypes.c_void_p(out.data_ptr()), x.size - 1)
    assert st == vbyte.ECOUNT
    # argument errors come back before any launch
    assert L.vbyte_decode(ctypes.c_void_p(data.data_ptr()), b.size, ctypes.c_void_p(out.data_ptr() + 2),
                          x.size) == vbyte.EINVAL
    assert L.vbyte_decode(None, 10, ctypes.c_void_p(out.data_ptr()), 1) == vbyte.EINVAL


@pytest.mark.parametrize("nb", [0, 1, 17, 1024, 4097, 1 << 20])
def test_count(nb):
    rng = np.random.default_rng(nb + 1)
    b = rng.integers(0, 256, nb, dtype=np.uint8)
    for boff in (0, 9):
        _, data = place_bytes(b, boff)
        assert vbyte.count(data) == oracle.count(b)


@pytest.mark.parametrize("n", [0, 1, 1023, 1024, 1025, 50001, 1 << 20])
def test_encode_matches_oracle(n):
    rng = np.random.default_rng(n + 3)
    x = mixed_values(rng, n)
    xt = torch.from_numpy(x.view(np.int32)).to(dev())
    for boff in (0, 3):
        full = torch.full((5 * n + 64,), 0xEE, dtype=torch.uint8, device=dev())
        out = full[boff:boff + 5 * n]
        nbytes = torch.empty(1, dtype=torch.int64, device=dev())
        vbyte.encode(xt, out=out, nbytes=nbytes, trim=False)
        torch.cuda.synchronize()
        ref = oracle.encode(x)
        nbw = int(nbytes.item())
        assert nbw == ref.size
        h = full.cpu().numpy()
        assert np.array_equal(h[boff:boff + nbw], ref)
        assert (h[:boff] == 0xEE).all() and (h[boff + nbw:] == 0xEE).all()
        prev = 1000
        enc = vbyte.encode(xt, delta=True, prev=prev)
        assert np.array_equal(enc.cpu().numpy(), oracle.encode_delta(x, prev))


def test_encode_capacity_overflow():
    x = np.full(5000, 0xFFFFFFFF, np.uint32)
    xt = torch.from_numpy(x.view(np.int32)).to(dev())
    full = torch.full((12000 + 64,), 0xEE, dtype=torch.uint8, device=dev())
    out = full[:12000]
    nbytes = torch.empty(1, dtype=torch.int64, device=dev())
    vbyte.encode(xt, out=out, nbytes=nbytes, trim=False)
    torch.cuda.synchronize()
    assert int(nbytes.item()) == 25000
    h = full.cpu().numpy()
    assert np.array_equal(h[:12000], oracle.encode(x)[:12000])
    assert (h[12000:] == 0xEE).all()


def test_gpu_encode_then_decode_roundtrip():
    rng = np.random.default_rng(8)
    x = mixed_values(rng, 300001)
    xt = torch.from_numpy(x.view(np.int32)).to(dev())
    enc = vbyte.encode(xt)
    y = vbyte.decode(enc, x.size)
    assert np.array_equal(u32(y), x)


@pytest.mark.parametrize("segs,wpb", [(4, 8), (2, 4), (1, 1)])
def test_dense_one_byte_segments(segs, wpb):
    """Segments made only of 1-byte codes take the dense path; rare 2-byte
    codes (some straddling a segment start), every output misalignment and a
    truncated count check that it joins the general path seamlessly."""
    vbyte.set_tuning(segs, wpb, 0)
    rng = np.random.default_rng(segs + 10 * wpb)
    n = 300_000
    x = rng.integers(0, 128, n).astype(np.uint32)
    # 2-byte codes at a few random positions and right before segment starts
    b = oracle.encode(x)
    pos = list(rng.integers(0, n - 1, 20))
    for k in range(1, 40):
        pos.append(1024 * k - 1)          # code bytes k*1024-1 and k*1024 straddle
    for p in pos:
        x[p] = 200
    b = oracle.encode(x)
    for ooff in range(4):
        for boff in (0, 7):
            st, y = check_against_oracle(b, n, boff=boff, ooff=ooff)
            assert np.array_equal(y, x)
            check_against_oracle(b, n, delta=True, prev=0xFFFFFFF0, boff=boff, ooff=ooff)
    # fewer outputs than codes: the dense store respects n
    st, _ = check_against_oracle(b, n - 777)
    assert st == vbyte.ECOUNT
    pure = rng.integers(0, 128, 70_000).astype(np.uint8)
    for ooff in range(4):
        check_against_oracle(pure, pure.size, ooff=ooff)
        check_against_oracle(pure, pure.size, delta=True, prev=3, ooff=ooff)


@pytest.mark.parametrize("lens", [[0, 1, 1023, 1024, 1, 0, 3000, 5], [7], [0, 0], [2048, 2048]])
def test_encode_batch_offsets(lens):
    rng = np.random.default_rng(len(lens) + sum(lens))
    x = mixed_values(rng, int(sum(lens)))
    vals_off = np.zeros(len(lens) + 1, np.int64)
    vals_off[1:] = np.cumsum(lens)
    xt = torch.from_numpy(x.view(np.int32)).to(dev())
    enc, byte_off = vbyte.encode_batch(xt, torch.from_numpy(vals_off).to(dev()))
    torch.cuda.synchronize()
    assert np.array_equal(enc.cpu().numpy(), oracle.encode(x))
    ref = np.array([oracle.encoded_size(x[:v]) for v in vals_off], np.int64)
    assert np.array_equal(byte_off.cpu().numpy(), ref)
