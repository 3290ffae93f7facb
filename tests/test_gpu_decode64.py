"""GPU parity of the 64-bit decode (vbyte_decode64*, reading R13) with the
oracle's 64-bit codec: element by element, with guard words around the
output and misleading bytes around the input, over tilings, alignments,
1..10-byte codes straddling every lane, segment and unit boundary, the
status readings, and a full-size stream."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, place_bytes
from paper_1503_07387_amd import vbyte

pytestmark = pytest.mark.gpu

SENT64 = 0x5A5A5A5A5A5A5A5A
M64 = (1 << 64) - 1


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def gpu64(b, n, delta=False, prev=0, boff=0, ooff=0):
    _, data = place_bytes(b, boff)
    full = torch.full((ooff + n + 8,), SENT64 - (1 << 64) if SENT64 >= 1 << 63 else SENT64,
                      dtype=torch.int64, device=dev())
    out = full[ooff:ooff + n]
    st = torch.full((1,), -1, dtype=torch.int32, device=dev())
    vbyte.decode64(data, n, delta=delta, prev=prev, out=out, status=st, check=False)
    torch.cuda.synchronize()
    h = u64(full)
    assert (h[:ooff] == SENT64).all(), "write before out[0]"
    assert (h[ooff + n:] == SENT64).all(), "write past out[n-1]"
    return int(st.item()), h[ooff:ooff + n]


def check64(b, n, delta=False, prev=0, boff=0, ooff=0):
    st, y = gpu64(b, n, delta, prev, boff, ooff)
    sto, yo = oracle.decode64_delta(b, n, prev) if delta else oracle.decode64(b, n)
    assert st == sto, f"status gpu={st} oracle={sto} (n={n}, nbytes={len(b)}, boff={boff})"
    if sto == oracle.OK and not np.array_equal(y, yo):
        bad = np.nonzero(y != yo)[0]
        raise AssertionError(f"{bad.size} mismatches, first at {bad[0]}: gpu={y[bad[0]]} "
                             f"oracle={yo[bad[0]]} (n={n}, boff={boff}, delta={delta})")
    return st, y


def values64(rng, n, lengths=tuple(range(1, 11))):
    """uint64 values whose code lengths are drawn from `lengths`."""
    L = rng.choice(np.array(lengths), size=n)
    out = np.empty(n, np.uint64)
    for k in set(int(v) for v in L):
        sel = L == k
        lo = 0 if k == 1 else 1 << (7 * (k - 1))
        hi = min(1 << (7 * k), 1 << 64)
        r = rng.integers(0, 1 << 63, int(sel.sum()), dtype=np.uint64).astype(object)
        out[sel] = np.array([lo + int(v) * 2 % (hi - lo) for v in r], dtype=np.uint64)
    return out


TILINGS = [(1, 1), (1, 4), (2, 8), (2, 2)]


@pytest.mark.parametrize("tiling", TILINGS)
@pytest.mark.parametrize("n", [0, 1, 63, 1000, 40_000, 250_001])
def test_random_mixed_lengths(tiling, n):
    vbyte.set_tuning(tiling[0], tiling[1], 0)
    rng = np.random.default_rng(n + 7 * tiling[0] + tiling[1])
    x = values64(rng, n)
    b = oracle.encode64(x)
    st, y = check64(b, n, boff=n % 16, ooff=n % 3)
    assert st == vbyte.OK and np.array_equal(y, x)
    check64(b, n, delta=True, prev=M64 - 5, boff=(n + 5) % 16)


@pytest.mark.parametrize("lengths", [(1,), (1, 2), (9, 10), (5, 6, 7, 8), (1, 10)])
def test_fixed_length_mixes(lengths):
    vbyte.set_tuning(2, 4, 0)
    rng = np.random.default_rng(sum(lengths))
    x = values64(rng, 30_000, lengths)
    b = oracle.encode64(x)
    check64(b, x.size, boff=3)
    check64(b, x.size, delta=True, prev=12345, boff=11, ooff=1)


@pytest.mark.parametrize("tiling", TILINGS)
def test_unit_straddle(tiling):
    """A 10-byte (and a 6-byte) code at every phase across every lane,
    segment, group and unit boundary."""
    segs, wpb = tiling
    vbyte.set_tuning(segs, wpb, 0)
    group = segs * 1024            # bytes a wavefront loads at once
    unit = 8 * group               # bytes of one wavefront's unit (one slot)
    rng = np.random.default_rng(segs * 10 + wpb)
    for long_len in (10, 6):
        vals, pos = [], 0
        targets = sorted({k * 16 for k in range(1, 40)} | {k * 1024 for k in range(1, 6)} |
                         {k * group for k in range(1, 5)} | {k * unit for k in range(1, 4)})
        for tgt in targets:
            for phase in range(long_len + 1):
                start = tgt - phase
                while pos < start:
                    vals.append(int(rng.integers(0, 128)))
                    pos += 1
                if pos == start:
                    lo = 1 << (7 * (long_len - 1))
                    hi = min(1 << (7 * long_len), 1 << 64)
                    vals.append(lo + int(rng.integers(0, 1 << 62)) % (hi - lo))
                    pos += long_len
        x = np.array(vals, np.uint64)
        b = oracle.encode64(x)
        for boff in (0, 1, 13):
            st, y = check64(b, x.size, boff=boff)
            assert np.array_equal(y, x)
            check64(b, x.size, delta=True, prev=99, boff=boff)


def test_boundary_values_every_alignment():
    vals = [0, 1, M64, 1 << 63, (1 << 63) - 1]
    for k in range(1, 10):
        vals += [(1 << (7 * k)) - 1, 1 << (7 * k), (1 << (7 * k)) + 1]
    x = np.array(vals * 3, np.uint64)
    b = oracle.encode64(x)
    for boff in range(16):
        st, y = check64(b, x.size, boff=boff, ooff=boff % 2)
        assert np.array_equal(y, x)


def test_statuses_match_oracle():
    ten = bytes([0x80] * 9 + [0x01])
    cases = [
        (ten, 1), (ten + b"\x05", 2), (bytes([0x80] * 10 + [0x01]), 1), (ten + b"\x81", 2),
        (ten, 2), (ten + b"\x01", 1), (b"", 0), (b"", 1), (bytes([0x80] * 12), 0),
        (bytes([0x80] * 9 + [0x03]), 1), (bytes([0xFF] * 9 + [0x7E]), 1),
        (b"\x05" + bytes([0x81] * 10) + b"\x00", 2),
    ]
    for buf, n in cases:
        b = np.frombuffer(buf, np.uint8)
        for boff in (0, 7):
            check64(b, n, boff=boff)
            check64(b, n, delta=True, prev=3, boff=boff)


@pytest.mark.parametrize("segs", [1, 2])
def test_statuses_in_long_streams(segs):
    vbyte.set_tuning(segs, 4, 0)
    unit = 8 * segs * 1024
    rng = np.random.default_rng(78)
    x = values64(rng, 40_000, (1, 2, 3, 9))
    b = oracle.encode64(x)
    n = x.size
    assert check64(b, n)[0] == vbyte.OK
    assert check64(b, n - 1)[0] == vbyte.ECOUNT
    assert check64(b, n + 1)[0] == vbyte.ETRUNC
    assert check64(b[:-1], n)[0] in (vbyte.ETRUNC, vbyte.ECOUNT)
    # a run of 10 continuation bytes across lane, segment and unit boundaries
    for at in (5, 16 * 7 - 4, 1024 - 5, unit - 9, unit, 3 * unit + 1, b.size - 11):
        bad = b.copy()
        bad[at:at + 10] = 0x80
        assert check64(bad, n)[0] == vbyte.EMALFORMED
        assert check64(bad, n, delta=True)[0] == vbyte.EMALFORMED
    # nine continuation bytes then a terminator: a whole 10-byte code
    ok = oracle.encode64(np.array([1] * 3000 + [M64] + [2] * 3000, np.uint64))
    assert check64(ok, 6001)[0] == vbyte.OK


def test_synchronous_calls_and_args():
    rng = np.random.default_rng(5)
    x = values64(rng, 5000)
    b = oracle.encode64(x)
    d = torch.from_numpy(b).to(dev())
    out = torch.empty(x.size, dtype=torch.int64, device=dev())
    L = vbyte._lib()
    assert L.vbyte_decode64(d.data_ptr(), b.size, out.data_ptr(), x.size) == vbyte.OK
    assert np.array_equal(u64(out), x)
    assert L.vbyte_decode64_delta(d.data_ptr(), b.size, out.data_ptr(), x.size, 9) == vbyte.OK
    assert np.array_equal(u64(out), oracle.decode64_delta(b, x.size, 9)[1])
    assert L.vbyte_decode64(d.data_ptr(), b.size, out.data_ptr(), x.size + 1) == vbyte.ETRUNC
    # misaligned output is refused before any launch
    assert L.vbyte_decode64(d.data_ptr(), b.size, out.data_ptr() + 4, x.size - 1) == vbyte.EINVAL


@pytest.mark.parametrize("delta", [False, True])
def test_full_size_stream(delta):
    """16Mi values of 1..10-byte codes (≈80 MB of codes, 128 MiB out)."""
    vbyte.set_tuning(2, 8, 0)
    rng = np.random.default_rng(64)
    n = 1 << 24
    L = rng.integers(1, 11, n)
    hi_bits = np.minimum(7 * L, 64)
    lo_bits = np.where(L == 1, 0, 7 * (L - 1))
    r = rng.integers(0, 1 << 63, n, dtype=np.uint64) | (rng.integers(0, 2, n, dtype=np.uint64) << np.uint64(63))
    span = hi_bits - lo_bits
    mask = np.where(span >= 64, np.uint64(M64), (np.uint64(1) << span.astype(np.uint64)) - np.uint64(1))
    x = (r & mask) | np.where(L == 1, np.uint64(0), np.uint64(1) << lo_bits.astype(np.uint64))
    b = oracle.encode64(x)
    st, y = gpu64(b, n, delta=delta, prev=5)
    sto, yo = oracle.decode64_delta(b, n, 5) if delta else oracle.decode64(b, n)
    assert st == sto == vbyte.OK
    assert np.array_equal(y, yo)
