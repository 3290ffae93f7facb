"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.

Each ``pin_*`` takes a loaded oracle library (ctypes) and raises
AssertionError on a mismatch.  ``test_oracle_pins.py`` runs them on the real
oracle; ``test_oracle_mutants.py`` runs them on deliberately broken copies of
the oracle and expects at least one of them to fail for every planted mistake.

Independent sources used here:
  * Table 1 and Figure 1 of the paper (fixtures under tests/golden/);
  * Protocol Buffers' varint encoder and decoder, a third-party implementation
    of the same byte format (the paper names Protocol Buffers' Varint as the
    same format, section 1);
  * closed forms of the format (byte-length boundaries 2^(7k), the 4-bit top
    group of a 5-byte code) written out as byte literals;
  * brute-force enumeration of every canonical 1-, 2- and 3-byte code;
  * numpy's wrapping uint32 cumsum and Python big-integer sums mod 2^32 for
    the differential decode.
"""
import os

import numpy as np

import oracle
from oracle import OK, EINVAL, ECOUNT, ETRUNC, EMALFORMED

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
M32 = 0xFFFFFFFF


def _hex(s):
    return bytes(int(t, 16) for t in s.split())


def read_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v, b = line.split(":")
            rows.append((int(v), _hex(b)))
    return rows


def read_fig1():
    d = {}
    with open(os.path.join(GOLDEN, "fig1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":")
            d[k.strip()] = v.split()
    return (_hex(" ".join(d["bytes"])),
            [int(t) for t in d["continuation_mask"]],
            [int(t) for t in d["integers"]])


def pb_encode(values):
    from google.protobuf.internal import encoder
    return b"".join(encoder._VarintBytes(int(v)) for v in values)


def pb_decode(buf, n):
    from google.protobuf.internal import decoder
    out, pos = [], 0
    for _ in range(n):
        v, pos = decoder._DecodeVarint32(buf, pos)
        out.append(v)
    assert pos == len(buf)
    return out


def boundary_values():
    vals = {0, 1, M32, M32 - 1}
    for k in range(1, 5):
        for d in (-1, 0, 1):
            vals.add((1 << (7 * k)) + d)
    return sorted(vals)


# ---------------------------------------------------------------- Table 1 / Fig 1
def pin_table1(lib):
    rows = read_table1()
    for v, b in rows:
        got = oracle.encode(np.array([v]), lib=lib).tobytes()
        assert got == b, f"ENC({v}) = {got.hex()} expected {b.hex()} (Table 1)"
        st, y = oracle.decode(b, 1, lib=lib)
        assert st == OK and int(y[0]) == v, f"DEC({b.hex()}) = {st},{y} expected {v}"
    cat = b"".join(b for _, b in rows)
    st, y = oracle.decode(cat, len(rows), lib=lib)
    assert st == OK and [int(t) for t in y] == [v for v, _ in rows]
    assert oracle.encode(np.array([v for v, _ in rows]), lib=lib).tobytes() == cat


def pin_fig1(lib):
    buf, cmask, ints = read_fig1()
    st, y = oracle.decode(buf, len(ints), lib=lib)
    assert st == OK and [int(t) for t in y] == ints, (st, y)
    assert [1 if b >= 0x80 else 0 for b in buf] == cmask
    # one terminator (top bit 0) per integer: the complement of the mask
    assert oracle.count(buf, lib=lib) == len(ints) == cmask.count(0)
    assert oracle.encode(np.array(ints), lib=lib).tobytes() == buf


# ---------------------------------------------------------------- closed forms
def pin_closed_form_boundaries(lib):
    # 2^(7k)-1: k-1 bytes FF then 7F;  2^(7k): k bytes 80 then 01;
    # 2^(7k)+1: 81, then k-1 bytes 80, then 01 (section 1 byte ranges).
    for k in range(1, 5):
        cases = {
            (1 << (7 * k)) - 1: bytes([0xFF] * (k - 1) + [0x7F]),
            (1 << (7 * k)): bytes([0x80] * k + [0x01]),
            (1 << (7 * k)) + 1: bytes([0x81] + [0x80] * (k - 1) + [0x01]),
        }
        for v, b in cases.items():
            got = oracle.encode(np.array([v]), lib=lib).tobytes()
            assert got == b, f"ENC({v}) = {got.hex()} expected {b.hex()}"
            st, y = oracle.decode(b, 1, lib=lib)
            assert st == OK and int(y[0]) == v
    # 0 is the single byte 00 (reading R1); 2^32-1 is FF FF FF FF 0F: the top
    # group of a 5-byte code holds only 4 bits (section 4, 2-integer case).
    fixed = {0: b"\x00", M32: b"\xff\xff\xff\xff\x0f", 1 << 31: b"\x80\x80\x80\x80\x08",
             (1 << 28) | 0x7F: b"\xff\x80\x80\x80\x01"}
    for v, b in fixed.items():
        assert oracle.encode(np.array([v]), lib=lib).tobytes() == b
        st, y = oracle.decode(b, 1, lib=lib)
        assert st == OK and int(y[0]) == v


def pin_length_closed_form(lib):
    rng = np.random.default_rng(7)
    vals = boundary_values() + [int(v) for v in rng.integers(0, 1 << 32, 2000, dtype=np.uint64)]
    for v in vals:
        expect = max(1, -(-int(v).bit_length() // 7))
        got = oracle.code_length(v, lib=lib)
        assert got == expect, f"L({v}) = {got} expected {expect}"
    x = np.array(vals, dtype=np.uint32)
    assert oracle.encoded_size(x, lib=lib) == sum(max(1, -(-int(v).bit_length() // 7)) for v in vals)


def pin_five_byte_algebra(lib):
    # x = a + b 2^7 + c 2^14 + d 2^21 + e 2^28 with e < 16 (section 4).
    rng = np.random.default_rng(11)
    for _ in range(200):
        a, b, c, d = (int(t) for t in rng.integers(0, 128, 4))
        e = int(rng.integers(1, 16))
        x = a + (b << 7) + (c << 14) + (d << 21) + (e << 28)
        buf = bytes([a | 0x80, b | 0x80, c | 0x80, d | 0x80, e])
        assert oracle.encode(np.array([x]), lib=lib).tobytes() == buf
        st, y = oracle.decode(buf, 1, lib=lib)
        assert st == OK and int(y[0]) == x


# ---------------------------------------------------------------- third-party codec
def pin_protobuf_exhaustive_21(lib):
    x = np.arange(0, 1 << 21, dtype=np.uint32)
    ours = oracle.encode(x, lib=lib).tobytes()
    assert ours == pb_encode(range(1 << 21)), "ENC differs from protobuf varint on [0, 2^21)"
    st, y = oracle.decode(ours, x.size, lib=lib)
    assert st == OK and np.array_equal(y, x)


def pin_protobuf_random_wide(lib):
    rng = np.random.default_rng(3)
    L = rng.integers(1, 6, 20000)
    lo = np.where(L == 1, 0, 1 << (7 * (L - 1)))
    hi = np.minimum(1 << (7 * L), 1 << 32)
    x = (lo + (rng.random(L.size) * (hi - lo)).astype(np.int64)).astype(np.uint32)
    x = np.concatenate([x, np.array(boundary_values(), dtype=np.uint32)])
    ours = oracle.encode(x, lib=lib).tobytes()
    ref = pb_encode(x.tolist())
    assert ours == ref
    st, y = oracle.decode(ref, x.size, lib=lib)
    assert st == OK and y.tolist() == pb_decode(ref, x.size)


def pin_canonical_bijection(lib):
    # Every canonical 2-byte code (b0 in [80,FF], b1 in [01,7F]) and 3-byte
    # code (b0,b1 in [80,FF], b2 in [01,7F]) decodes to a distinct value and
    # together they cover exactly [2^7, 2^14) and [2^14, 2^21).
    b0 = np.arange(0x80, 0x100, dtype=np.uint8)
    b1 = np.arange(0x01, 0x80, dtype=np.uint8)
    two = np.stack(np.meshgrid(b0, b1, indexing="ij"), -1).reshape(-1, 2)
    st, y = oracle.decode(two.reshape(-1), two.shape[0], lib=lib)
    assert st == OK
    assert np.array_equal(np.sort(y), np.arange(1 << 7, 1 << 14, dtype=np.uint32))
    three = np.stack(np.meshgrid(b0, b0, b1, indexing="ij"), -1).reshape(-1, 3)
    st, y = oracle.decode(three.reshape(-1), three.shape[0], lib=lib)
    assert st == OK
    assert np.array_equal(np.sort(y), np.arange(1 << 14, 1 << 21, dtype=np.uint32))
    # ENC is the inverse on those codes
    assert np.array_equal(oracle.encode(y, lib=lib), three.reshape(-1))


def pin_random_wide_roundtrip(lib, n=2_000_000):
    rng = np.random.default_rng(5)
    x = rng.integers(1 << 21, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    b = oracle.encode(x, lib=lib)
    st, y = oracle.decode(b, n, lib=lib)
    assert st == OK and np.array_equal(x, y)
    assert oracle.count(b, lib=lib) == n


# ---------------------------------------------------------------- differential
def pin_delta_cumsum(lib):
    rng = np.random.default_rng(9)
    for prev in (0, 1, 12345, M32):
        g = rng.integers(0, 1 << 32, 5000, dtype=np.uint64).astype(np.uint32)
        g[:100] = rng.integers(0, 300, 100)
        b = oracle.encode(g, lib=lib)
        st, y = oracle.decode_delta(b, g.size, prev, lib=lib)
        assert st == OK
        ref = (np.cumsum(g, dtype=np.uint32) + np.uint32(prev)).astype(np.uint32)
        assert np.array_equal(y, ref)
        acc, big = prev, []
        for v in g[:300].tolist():
            acc = (acc + v) % (1 << 32)
            big.append(acc)
        assert y[:300].tolist() == big


def pin_delta_encode_roundtrip(lib):
    rng = np.random.default_rng(10)
    ids = np.sort(rng.integers(0, 1 << 32, 4000, dtype=np.uint64)).astype(np.uint32)
    shuffled = rng.integers(0, 1 << 32, 4000, dtype=np.uint64).astype(np.uint32)
    for x in (ids, shuffled):
        for prev in (0, 77):
            b = oracle.encode_delta(x, prev, lib=lib)
            gaps = (x.astype(np.int64) - np.concatenate([[prev], x[:-1]]).astype(np.int64)) % (1 << 32)
            assert np.array_equal(b, oracle.encode(gaps.astype(np.uint32), lib=lib))
            st, y = oracle.decode_delta(b, x.size, prev, lib=lib)
            assert st == OK and np.array_equal(y, x)


def pin_resumable(lib):
    rng = np.random.default_rng(12)
    g = rng.geometric(1 / 300, 3000).astype(np.uint32)
    b = oracle.encode(g, lib=lib)
    st, full = oracle.decode_delta(b, g.size, 5, lib=lib)
    assert st == OK
    m = 1234
    cut = oracle.encoded_size(g[:m], lib=lib)
    st1, y1 = oracle.decode_delta(b[:cut], m, 5, lib=lib)
    st2, y2 = oracle.decode_delta(b[cut:], g.size - m, int(y1[-1]), lib=lib)
    assert st1 == OK and st2 == OK
    assert np.array_equal(np.concatenate([y1, y2]), full)


def pin_delta_m1_closed_form(lib):
    # Reading R11: y_k = prev + sum_{j<=k} g_j + k (mod 2^32), in Python
    # integers; all-zero gaps give consecutive identifiers.
    rng = np.random.default_rng(21)
    for prev in (0, 9, M32):
        g = rng.integers(0, 1 << 32, 3000, dtype=np.uint64).astype(np.uint32)
        g[:500] = rng.integers(0, 40, 500)
        b = oracle.encode(g, lib=lib)
        st, y = oracle.decode_delta_m1(b, g.size, prev, lib=lib)
        assert st == OK
        tot, ref = prev, []
        for k, v in enumerate(g.tolist()):
            tot += v
            ref.append((tot + k) % (1 << 32))
        assert y.tolist() == ref
        z = oracle.encode(np.zeros(50, np.uint32), lib=lib)
        st, y = oracle.decode_delta_m1(z, 50, prev, lib=lib)
        assert st == OK and y.tolist() == [(prev + k) % (1 << 32) for k in range(50)]
        # against the plain differential decode of the same bytes: + k
        st2, yd = oracle.decode_delta(b, g.size, prev, lib=lib)
        st, y = oracle.decode_delta_m1(b, g.size, prev, lib=lib)
        assert st2 == OK and np.array_equal(y - yd, np.arange(g.size, dtype=np.uint32))


def pin_delta_m1_encode_roundtrip(lib):
    rng = np.random.default_rng(22)
    ids = np.unique(rng.integers(0, 1 << 32, 5000, dtype=np.uint64)).astype(np.uint32)
    for prev in (0, int(ids[0]) // 2):
        b = oracle.encode_delta_m1(ids, prev, lib=lib)
        gaps = np.diff(ids.astype(np.int64), prepend=prev) - (np.arange(ids.size) > 0)
        assert (gaps >= 0).all()
        assert np.array_equal(b, oracle.encode(gaps.astype(np.uint32), lib=lib))
        st, y = oracle.decode_delta_m1(b, ids.size, prev, lib=lib)
        assert st == OK and np.array_equal(y, ids)
    # consecutive identifiers cost one byte each
    run = np.arange(1000, 3000, dtype=np.uint32)
    assert oracle.encode_delta_m1(run, 1000, lib=lib).tolist() == [0] * run.size


def pin_resumable_pieces(lib):
    # Reading R12: pieces of k integers, each resumed from the previous
    # piece's cursor and prev, reproduce the whole-stream decodes, and each
    # cursor is the canonical size of the values decoded so far.
    rng = np.random.default_rng(23)
    x = rng.integers(0, 1 << 32, 3000, dtype=np.uint64).astype(np.uint32)
    x[rng.random(3000) < 0.5] %= 200
    b = oracle.encode(x, lib=lib)
    whole = {0: oracle.decode(b, x.size, lib=lib)[1],
             1: oracle.decode_delta(b, x.size, 11, lib=lib)[1],
             2: oracle.decode_delta_m1(b, x.size, 11, lib=lib)[1]}
    for delta in (0, 1, 2):
        for k in (1, 7, 1000, 2999, 3000, 5000):
            off, prev, got = 0, 11, []
            while True:
                st, y, nxt, prev = oracle.decode_next(b, off, k, prev, delta, lib=lib)
                assert st == OK
                got.append(y)
                assert nxt == oracle.encoded_size(x[:sum(len(g) for g in got)], lib=lib)
                if y.size < k:
                    break
                off = nxt
            assert nxt == b.size and y.size == (x.size % k if x.size % k else (0 if k <= x.size else x.size))
            assert np.array_equal(np.concatenate(got), whole[delta])
    # a prefix piece equals the head of the whole decode
    for k in (1, 2, 5, 64):
        st, y, nxt, _ = oracle.decode_next(b, 0, k, 0, 0, lib=lib)
        assert st == OK and np.array_equal(y, whole[0][:k])


def pin_resumable_errors(lib):
    b = oracle.encode(np.array([1, 300, 70000, 5], np.uint32), lib=lib)
    st, *_ = oracle.decode_next(b[:-1] if b[-1] < 128 else b, 0, 10, lib=lib)
    assert st == OK                                  # the buffer ends on a terminator
    cut = np.concatenate([b, [0x85, 0x81]]).astype(np.uint8)   # then an unfinished code
    st, y, nxt, _ = oracle.decode_next(cut, 0, 4, lib=lib)
    assert st == OK and y.size == 4 and nxt == b.size          # k codes found first
    st, *_ = oracle.decode_next(cut, 0, 5, lib=lib)
    assert st == ETRUNC
    bad = np.concatenate([b, [0x80] * 5, [0x01]]).astype(np.uint8)
    st, *_ = oracle.decode_next(bad, 0, 4, lib=lib)
    assert st == EMALFORMED                          # the run lies in the 5k-byte window
    st, y, nxt, _ = oracle.decode_next(bad, 0, 1, lib=lib)
    assert st == OK and y.tolist() == [1]            # window of 5 bytes: no run inside
    assert oracle.decode_next(b, 0, 0, lib=lib)[0] == EINVAL
    assert oracle.decode_next(b, b.size + 1, 3, lib=lib)[0] == EINVAL
    st, y, nxt, pv = oracle.decode_next(b, b.size, 3, 9, 1, lib=lib)
    assert st == OK and y.size == 0 and nxt == b.size and pv == 9


# ---------------------------------------------------------------- status readings
# (bytes, n, expected status); the expectations follow readings R3-R6.
STATUS_CASES = [
    (b"", 0, OK),
    (b"", 1, ETRUNC),
    (b"\x00", 0, ECOUNT),
    (b"\x80", 0, ETRUNC),
    (b"\x80", 1, ETRUNC),
    (b"\x01\x02", 1, ECOUNT),
    (b"\x01", 2, ETRUNC),
    (b"\x01\x80", 1, ETRUNC),
    (b"\x01\x80", 2, ETRUNC),
    (b"\x80\x80\x80\x80\x01", 1, OK),
    (b"\x80\x80\x80\x80\x80\x01", 1, EMALFORMED),
    (b"\x80\x80\x80\x80\x80", 1, EMALFORMED),
    (b"\x01\x80\x80\x80\x80\x80\x01\x02\x03", 1, EMALFORMED),
    (b"\x01\x02\x80\x80\x80\x80\x80", 9, EMALFORMED),
    (b"\x01\x80\x80\x80\x80", 5, ETRUNC),
    (b"\x01\x02\x03\x80", 2, ETRUNC),
]


def pin_status_readings(lib):
    for buf, n, expect in STATUS_CASES:
        got = oracle.validate(buf, n, lib=lib)
        assert got == expect, f"validate({buf.hex()}, {n}) = {got} expected {expect}"
        st, _ = oracle.decode(buf, n, lib=lib)
        assert st == expect
        assert oracle.count(buf, lib=lib) == sum(1 for c in buf if c < 0x80)


def pin_fifth_byte_wrap(lib):
    # Reading R4: a fifth byte e >= 16 keeps only its low 4 bits (2^28 weight
    # wraps mod 2^32), exactly like Algorithm 1 in 32-bit arithmetic.
    for e in (0x10, 0x1F, 0x7F, 0x55):
        for low in ((0, 0, 0, 0), (0x7F, 0x7F, 0x7F, 0x7F), (1, 2, 3, 4)):
            buf = bytes([low[0] | 0x80, low[1] | 0x80, low[2] | 0x80, low[3] | 0x80, e])
            expect = (low[0] + (low[1] << 7) + (low[2] << 14) + (low[3] << 21) + (e << 28)) % (1 << 32)
            st, y = oracle.decode(buf, 1, lib=lib)
            assert st == OK and int(y[0]) == expect


def pin_overlong(lib):
    # Reading R5: over-long codes decode to the sum of their 7-bit groups.
    cases = {b"\x80\x00": 0, b"\x81\x00": 1, b"\x80\x80\x00": 0, b"\xff\x80\x00": 127,
             b"\x80\x80\x80\x80\x00": 0}
    for buf, v in cases.items():
        st, y = oracle.decode(buf, 1, lib=lib)
        assert st == OK and int(y[0]) == v


# ---------------------------------------------------------------- batch
def pin_batch(lib):
    rng = np.random.default_rng(13)
    lens = [0, 1, 5, 0, 300, 2, 1000]
    lists = [rng.integers(0, 1 << 32, k, dtype=np.uint64).astype(np.uint32) for k in lens]
    lists[4][:] = rng.integers(0, 200, lens[4])
    enc = [oracle.encode(x, lib=lib) for x in lists]
    byte_off = np.concatenate([[0], np.cumsum([e.size for e in enc])]).astype(np.int64)
    out_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    bts = np.concatenate(enc) if enc else np.zeros(0, np.uint8)
    prevs = rng.integers(0, 1 << 32, len(lens), dtype=np.uint64).astype(np.uint32)
    st, out, sts = oracle.decode_batch(bts, byte_off, out_off, None, False, lib=lib)
    assert st == OK and (sts == OK).all()
    assert np.array_equal(out, np.concatenate(lists))
    st, out, sts = oracle.decode_batch(bts, byte_off, out_off, prevs, True, lib=lib)
    assert st == OK
    for i, x in enumerate(lists):
        a, b = out_off[i], out_off[i + 1]
        ref = (np.cumsum(x, dtype=np.uint32) + prevs[i]).astype(np.uint32)
        assert np.array_equal(out[a:b], ref)
    # a list whose count is wrong fails alone; the others still decode
    bad_out = out_off.copy()
    bad_out[5:] += 1                      # list 4 now expects one more integer
    st, out, sts = oracle.decode_batch(bts, byte_off, bad_out, None, False, lib=lib)
    assert sts[4] == ETRUNC and st == ETRUNC
    assert all(sts[i] == OK for i in range(len(lens)) if i != 4)
    st, out, sts = oracle.decode_batch(bts, byte_off, out_off, prevs, 2, lib=lib)
    assert st == OK
    for i, x in enumerate(lists):
        a, b = out_off[i], out_off[i + 1]
        ref = (np.cumsum(x, dtype=np.uint32) + prevs[i] + np.arange(len(x), dtype=np.uint32)).astype(np.uint32)
        assert np.array_equal(out[a:b], ref)
    dec = byte_off.copy()
    dec[2] = dec[3] + 1                   # byte offsets decrease from list 2 to 3
    st, _, _ = oracle.decode_batch(bts, dec, out_off, None, False, lib=lib)
    assert st == EINVAL
    dec = out_off.copy()
    dec[5] = dec[6] + 1
    st, _, _ = oracle.decode_batch(bts, byte_off, dec, None, False, lib=lib)
    assert st == EINVAL


# ---------------------------------------------------------------- blocks of four (R14)
def pin_delta4_example_and_closed_form(lib):
    # section 1's example: x_1..x_4 coded as themselves, then x_5 - x_1, ...
    x = np.array([5, 9, 2, 7, 6, 11, 3, 9, 100, 12], np.uint32)
    want = [5, 9, 2, 7, 1, 2, 1, 2, 94, 1]
    assert oracle.encode_delta4(x, lib=lib).tobytes() == oracle.encode(np.array(want, np.uint32), lib=lib).tobytes()
    st, y = oracle.decode_delta4(oracle.encode(np.array(want, np.uint32), lib=lib), len(want), lib=lib)
    assert st == OK and np.array_equal(y, x)
    # closed form: four interleaved wrapping prefix sums (numpy cumsum on a
    # 4-column view) plus prev4, for ragged lengths too
    rng = np.random.default_rng(44)
    for n in (1, 3, 4, 5, 999, 4096, 10001):
        g = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        g[rng.random(n) < 0.5] >>= 20
        prev4 = rng.integers(0, 1 << 32, 4, dtype=np.uint64).astype(np.uint32)
        pad = np.zeros(-n % 4, np.uint32)
        cols = np.concatenate([g, pad]).reshape(-1, 4)
        ref = (np.cumsum(cols, axis=0, dtype=np.uint32) + prev4).reshape(-1)[:n]
        st, y = oracle.decode_delta4(oracle.encode(g, lib=lib), n, prev4, lib=lib)
        assert st == OK and np.array_equal(y, ref), n
        # and Python integers mod 2^32
        back = [int(v) for v in prev4]
        for i in range(min(n, 300)):
            back[i % 4] = (back[i % 4] + int(g[i])) % (1 << 32)
            assert int(y[i]) == back[i % 4]


def pin_delta4_roundtrip_and_resume(lib):
    rng = np.random.default_rng(45)
    x = rng.integers(0, 1 << 32, 20000, dtype=np.uint64).astype(np.uint32)
    for prev4 in (None, [1, 2, 3, 0xFFFFFFFF]):
        b = oracle.encode_delta4(x, prev4, lib=lib)
        st, y = oracle.decode_delta4(b, x.size, prev4, lib=lib)
        assert st == OK and np.array_equal(y, x)
    # resuming after m values passes the last four of them
    b = oracle.encode_delta4(x, lib=lib)
    for m in (4, 5, 6, 7, 12345):
        cut = oracle.encoded_size(np.concatenate([x[:4], x[4:m] - x[:m - 4]]).astype(np.uint32), lib=lib)
        st1, y1 = oracle.decode_delta4(b[:cut], m, None, lib=lib)
        st2, y2 = oracle.decode_delta4(b[cut:], x.size - m, x[m - 4:m], lib=lib)
        assert st1 == st2 == OK and np.array_equal(np.concatenate([y1, y2]), x)
    # statuses come from the byte stream alone
    assert oracle.decode_delta4(b, x.size + 1, lib=lib)[0] == ETRUNC
    assert oracle.decode_delta4(b, x.size - 1, lib=lib)[0] == ECOUNT


# ---------------------------------------------------------------- intersection (R15)
def pin_intersect_brute_force(lib):
    rng = np.random.default_rng(46)
    for trial in range(60):
        na = int(rng.integers(0, 300))
        ids = np.sort(rng.choice(2000, size=na, replace=False)).astype(np.uint32)
        prev = int(rng.integers(0, 5))
        ids = ids + np.uint32(prev)
        bset = set(int(v) for v in rng.choice(2400, size=int(rng.integers(0, 400)), replace=False))
        b_ids = np.array(sorted(bset), np.uint32)
        a = oracle.encode_delta(ids, prev, lib=lib)
        piece = int(rng.choice([1, 2, 7, 64, 1000]))
        st, got = oracle.intersect_pieces(a, na, b_ids, piece, prev, lib=lib)
        want = [int(v) for v in ids if int(v) in bset]     # Python sets, in list order
        assert st == OK and [int(v) for v in got] == want, (trial, piece)
    # statuses: too few codes, codes left over, a malformed run
    ids = np.arange(10, 1010, 3, dtype=np.uint32)
    a = oracle.encode_delta(ids, 0, lib=lib)
    assert oracle.intersect_pieces(a, ids.size + 1, ids, 64, lib=lib)[0] == ETRUNC
    assert oracle.intersect_pieces(a, ids.size - 1, ids, 64, lib=lib)[0] == ECOUNT
    bad = a.copy()
    bad[100:105] = 0x80
    assert oracle.intersect_pieces(bad, ids.size, ids, 64, lib=lib)[0] == EMALFORMED


# ---------------------------------------------------------------- 64-bit (R13)
M64 = (1 << 64) - 1


def pb_decode64(buf, n):
    from google.protobuf.internal import decoder
    out, pos = [], 0
    for _ in range(n):
        v, pos = decoder._DecodeVarint(buf, pos)
        out.append(v)
    assert pos == len(buf)
    return out


def pin64_closed_form_boundaries(lib):
    # 2^(7k)-1: k-1 bytes FF then 7F; 2^(7k): k bytes 80 then 01;
    # 2^(7k)+1: 81, k-1 bytes 80, 01 -- for k up to 9 (section 1 byte ranges)
    for k in range(1, 10):
        cases = {
            (1 << (7 * k)) - 1: bytes([0xFF] * (k - 1) + [0x7F]),
            (1 << (7 * k)): bytes([0x80] * k + [0x01]),
            (1 << (7 * k)) + 1: bytes([0x81] + [0x80] * (k - 1) + [0x01]),
        }
        for v, b in cases.items():
            got = oracle.encode64(np.array([v], dtype=np.uint64), lib=lib).tobytes()
            assert got == b, f"ENC64({v}) = {got.hex()} expected {b.hex()}"
            assert oracle.code_length64(v, lib=lib) == len(b)
            st, y = oracle.decode64(b, 1, lib=lib)
            assert st == OK and int(y[0]) == v
        # ENC64's size of the three boundary values: the sum of their lengths
        assert oracle.encoded_size64(np.array(list(cases), dtype=np.uint64), lib=lib) == \
            sum(len(b) for b in cases.values())
    # the top group of a 10-byte code holds bit 63 only
    fixed = {0: b"\x00", M64: b"\xff" * 9 + b"\x01", 1 << 63: b"\x80" * 9 + b"\x01",
             (1 << 63) - 1: b"\xff" * 8 + b"\x7f", M32: b"\xff\xff\xff\xff\x0f"}
    for v, b in fixed.items():
        assert oracle.encode64(np.array([v], dtype=np.uint64), lib=lib).tobytes() == b
        st, y = oracle.decode64(b, 1, lib=lib)
        assert st == OK and int(y[0]) == v


def pin64_protobuf(lib):
    # Protocol Buffers' varint is this format for 64-bit integers (section 1
    # names it); its encoder and decoder are a codec written by others
    rng = np.random.default_rng(64)
    vals = [0, 1, M64, 1 << 63]
    for L in range(1, 11):
        lo = 0 if L == 1 else 1 << (7 * (L - 1))
        hi = min(1 << (7 * L), 1 << 64)
        vals += [lo + int(r) % (hi - lo) for r in rng.integers(0, 1 << 63, 300, dtype=np.uint64)]
        vals += [hi - 1]
    x = np.array(vals, dtype=np.uint64)
    ours = oracle.encode64(x, lib=lib).tobytes()
    assert ours == pb_encode(vals), "ENC64 differs from protobuf varint"
    # the size of the whole coded sequence, against protobuf's byte count
    assert oracle.encoded_size64(x, lib=lib) == len(pb_encode(vals))
    assert oracle.encoded_size64(x[1:], lib=lib) == len(pb_encode(vals[1:]))
    assert pb_decode64(ours, len(vals)) == vals
    st, y = oracle.decode64(ours, len(vals), lib=lib)
    assert st == OK and [int(t) for t in y] == vals


def pin64_delta_bigint(lib):
    # DEC64_DELTA against Python big integers reduced mod 2^64, and numpy's
    # wrapping uint64 cumsum; the sum wraps many times
    rng = np.random.default_rng(65)
    g = rng.integers(0, 1 << 64, 5000, dtype=np.uint64)
    g[rng.random(g.size) < 0.5] >>= np.uint64(40)
    b = oracle.encode64(g, lib=lib)
    prev = 0xFEDCBA9876543210
    st, y = oracle.decode64_delta(b, g.size, prev, lib=lib)
    acc, ref = prev, []
    for v in g:
        acc = (acc + int(v)) % (1 << 64)
        ref.append(acc)
    assert st == OK and [int(t) for t in y] == ref
    with np.errstate(over="ignore"):
        assert np.array_equal(y, np.cumsum(g, dtype=np.uint64) + np.uint64(prev))
    # the encoder of differences round-trips any sequence
    x = rng.integers(0, 1 << 64, 3000, dtype=np.uint64)
    st, y = oracle.decode64_delta(oracle.encode_delta64(x, 77, lib=lib), x.size, 77, lib=lib)
    assert st == OK and np.array_equal(y, x)


def pin64_statuses(lib):
    ten = bytes([0x80] * 9 + [0x01])
    # a 10-byte code is whole; ten continuation bytes are malformed (R13)
    assert oracle.validate64(ten, 1, lib=lib) == OK
    assert oracle.validate64(bytes([0x80] * 10 + [0x01]), 1, lib=lib) == EMALFORMED
    assert oracle.validate64(b"\x05" + bytes([0x81] * 10) + b"\x00", 2, lib=lib) == EMALFORMED
    # a tenth byte above 1: only its low bit counts, 2^63 wraps (R13)
    st, y = oracle.decode64(bytes([0x80] * 9 + [0x03]), 1, lib=lib)
    assert st == OK and int(y[0]) == 1 << 63
    st, y = oracle.decode64(bytes([0x80] * 9 + [0x7E]), 1, lib=lib)
    assert st == OK and int(y[0]) == 0
    # truncation, count, precedence (R6)
    assert oracle.validate64(ten + b"\x81", 2, lib=lib) == ETRUNC
    assert oracle.validate64(ten, 2, lib=lib) == ETRUNC
    assert oracle.validate64(ten + b"\x01", 1, lib=lib) == ECOUNT
    assert oracle.validate64(bytes([0x80] * 12), 0, lib=lib) == EMALFORMED
    assert oracle.validate64(b"", 0, lib=lib) == OK
    # codes of 5..9 bytes, valid for 64-bit, are malformed for 32-bit (R3)
    b = oracle.encode64(np.array([1 << 40, 1 << 56], dtype=np.uint64), lib=lib)
    assert oracle.validate64(b, 2, lib=lib) == OK and oracle.validate(b, 2, lib=lib) == EMALFORMED


def pin64_agrees_with_32(lib):
    # below 2^32 the two independently written codecs must agree byte for byte
    rng = np.random.default_rng(66)
    x = rng.integers(0, 1 << 32, 20000, dtype=np.uint64)
    x[rng.random(x.size) < 0.5] >>= np.uint64(20)
    b32 = oracle.encode(x.astype(np.uint32), lib=lib)
    assert np.array_equal(oracle.encode64(x, lib=lib), b32)
    st, y = oracle.decode64(b32, x.size, lib=lib)
    assert st == OK and np.array_equal(y, x)


ALL_PINS = [pin_table1, pin_fig1, pin_closed_form_boundaries, pin_length_closed_form,
            pin_five_byte_algebra, pin_protobuf_exhaustive_21, pin_protobuf_random_wide,
            pin_canonical_bijection, pin_random_wide_roundtrip, pin_delta_cumsum,
            pin_delta_encode_roundtrip, pin_resumable, pin_delta_m1_closed_form,
            pin_delta_m1_encode_roundtrip, pin_resumable_pieces, pin_resumable_errors,
            pin_status_readings,
            pin_fifth_byte_wrap, pin_overlong, pin_batch,
            pin64_closed_form_boundaries, pin64_protobuf, pin64_delta_bigint, pin64_statuses,
            pin64_agrees_with_32, pin_delta4_example_and_closed_form, pin_delta4_roundtrip_and_resume,
            pin_intersect_brute_force]
