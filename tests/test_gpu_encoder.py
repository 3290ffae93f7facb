"""GPU parity of the encoder (vbyte_encode*_async, vbyte_encode_batch) with
the oracle's ENC, byte for byte: plain, differential and differences minus
one, at sizes that span several chunks and scan blocks with ragged tails, at
every alignment of the values (0..3 elements past a 16-byte boundary), the
full 64Mi-gap streams, the 2^28-integer batch of 100,000 lists with its
list byte offsets, and a capacity below the encoded size (nothing written
past it, the size needed reported)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import mixed_values
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu


def on_gpu(x, e0):
    """x as int32 CUDA tensor starting e0 elements past a 16-byte boundary."""
    buf = torch.zeros(x.size + 8, dtype=torch.int32, device="cuda")
    buf[e0:e0 + x.size] = torch.from_numpy(x.view(np.int32)).cuda()
    return buf[e0:e0 + x.size]


@pytest.mark.parametrize("n", [1, 3, 255, 256, 257, 1000, 65_537, 8192 * 256 + 5, 3_000_001])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_encode_matches_oracle(n, mode):
    rng = np.random.default_rng(n * 7 + mode)
    x = mixed_values(rng, n)
    if mode:
        x = np.sort(x)
    for e0 in (0, 1, 2, 3):
        xt = on_gpu(x, e0)
        prev = int(x[0]) - 3 if mode else 0
        got = vbyte.encode(xt, delta=mode == 1, minus_one=mode == 2, prev=prev).cpu().numpy()
        if mode == 0:
            ref = oracle.encode(x)
        elif mode == 1:
            ref = oracle.encode_delta(x, prev)
        else:
            ref = oracle.encode_delta_m1(x, prev)
        assert np.array_equal(got, ref), (n, mode, e0)


def test_encode_wrapping_differences():
    # unsorted values: the differences wrap mod 2^32
    x = np.random.default_rng(3).integers(0, 1 << 32, 100_003, dtype=np.uint64).astype(np.uint32)
    got = vbyte.encode(on_gpu(x, 1), delta=True, prev=0xFFFFFFF0).cpu().numpy()
    assert np.array_equal(got, oracle.encode_delta(x, 0xFFFFFFF0))


def test_capacity_below_size():
    x = mixed_values(np.random.default_rng(4), 50_000)
    ref = oracle.encode(x)
    for cap in (0, 1, 17, ref.size // 2 + 3, ref.size - 1):
        out = torch.full((cap + 64,), 0xAB, dtype=torch.uint8, device="cuda")
        nbytes = torch.empty(1, dtype=torch.int64, device="cuda")
        vbyte.encode(on_gpu(x, 2), out=out[:cap], nbytes=nbytes, trim=False)
        torch.cuda.synchronize()
        h = out.cpu().numpy()
        assert int(nbytes.item()) == ref.size
        assert np.array_equal(h[:cap], ref[:cap])
        assert (h[cap:] == 0xAB).all(), "write past capacity"


@pytest.mark.parametrize("kind", ["one_byte", "one_or_two"])
def test_short_code_chunks_at_every_output_offset(kind):
    """Chunks whose codes are all one byte, or all one or two bytes, are
    stored with no LDS staging: every misalignment of the output, a
    two-byte code in an otherwise one-byte chunk, a chunk with a five-byte
    code, and capacities that cut a chunk (nothing written past them)."""
    rng = np.random.default_rng(9 if kind == "one_byte" else 10)
    n = 256 * 40 + 77
    if kind == "one_byte":
        x = rng.integers(0, 128, n).astype(np.uint32)
        x[256 * 7 + 100] = 200
        x[256 * 20:256 * 21] = 5000
    else:
        x = np.where(rng.random(n) < 0.5, rng.integers(0, 128, n), rng.integers(128, 16384, n)).astype(np.uint32)
        x[256 * 9 + 31] = 1 << 30
    ref = oracle.encode(x)
    for shift in range(4):
        for cap in (ref.size, ref.size - 1, 256 * 3 + 1, 256 * 11 + 2, 3):
            buf = torch.full((ref.size + 64,), 0xAB, dtype=torch.uint8, device="cuda")
            nbytes = torch.empty(1, dtype=torch.int64, device="cuda")
            vbyte.encode(on_gpu(x, shift), out=buf[shift:shift + cap], nbytes=nbytes, trim=False)
            torch.cuda.synchronize()
            h = buf.cpu().numpy()
            assert int(nbytes.item()) == ref.size
            assert (h[:shift] == 0xAB).all()
            assert np.array_equal(h[shift:shift + cap], ref[:cap]), (shift, cap)
            assert (h[shift + cap:] == 0xAB).all(), "write past capacity"


@pytest.mark.parametrize("gap_hi", [100, 10000])
def test_short_differences_minus_one(gap_hi):
    """Differences minus one of increasing values whose gaps code in one
    byte (gaps < 129) or in one or two bytes: the chunks take the register
    paths, at every alignment of the values."""
    rng = np.random.default_rng(gap_hi)
    x = np.cumsum(rng.integers(1, gap_hi, 256 * 30 + 41), dtype=np.uint64).astype(np.uint32)
    for e0 in (0, 1, 2, 3):
        got = vbyte.encode(on_gpu(x, e0), minus_one=True, prev=int(x[0]) - 1).cpu().numpy()
        assert np.array_equal(got, oracle.encode_delta_m1(x, int(x[0]) - 1)), e0


@pytest.mark.parametrize("mean", [8, 300])
def test_full_gap_streams(mean):
    g = workloads.geometric_gaps(mean=mean)
    got = vbyte.encode(torch.from_numpy(g.view(np.int32)).cuda()).cpu().numpy()
    assert np.array_equal(got, oracle.encode(g))
    # the identifiers coded as differences give the same bytes
    ids = np.cumsum(g, dtype=np.uint32)
    got = vbyte.encode(torch.from_numpy(ids.view(np.int32)).cuda(), delta=True).cpu().numpy()
    assert np.array_equal(got, oracle.encode(g))


def test_batch_of_100k_lists():
    d = workloads.zipf_lists()
    gaps, out_off = d["gaps"], d["out_off"]
    enc, byte_off = vbyte.encode_batch(torch.from_numpy(gaps.view(np.int32)).cuda(),
                                       torch.from_numpy(out_off).cuda())
    ref = oracle.encode(gaps)
    assert np.array_equal(enc.cpu().numpy(), ref)
    bo = byte_off.cpu().numpy()
    nl = d["lengths"].size
    want = np.zeros(nl + 1, np.int64)
    for i in range(nl):
        want[i + 1] = want[i] + oracle.encoded_size(gaps[out_off[i]:out_off[i + 1]])
    assert np.array_equal(bo, want)
