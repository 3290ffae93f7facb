"""CPU check of the identity behind the blocks-of-four aggregate (k4_agg).

The aggregate never assembles a code: a group's summary (count, class sums
S[c] = sum of its codes of rank = c mod 4 from its first code) is taken as
byte sums.  The class of a byte is the rank mod 4 of the code that holds it,
i.e. B (the class of the code running into the lane) plus the code starts at
or before the byte; a byte at depth d (continuation bytes right before it)
weighs 2^(7d), expressed as dot products of the 7-bit groups with 0/1 byte
marks (the byte-sum identity of the 32-bit aggregate).  The bytes of the
code running into the group are then taken out of class 3 (rank -1) and the
bytes after the group of the code running out of it are added to that
code's class.

This file models those steps in Python, dword by dword as the kernel takes
them (per-byte prefix counts by a multiply, class masks by a byte lookup,
dot products), and compares the result with the direct definition (walk the
codes, sum by rank) on every interior group of mixed-width streams.  It
shares nothing with the HIP source; the streams come from the oracle's
encoder."""
import numpy as np

import oracle

M32 = 0xFFFFFFFF
SEG = 1024          # bytes per segment
GROUP = 2 * SEG     # two segments per wavefront
LEVEL_WEIGHTS = [1, 127, 16256, 2080768, 266338304]   # 2^(7q) - 2^(7(q-1))


def dword(b, i):
    v = 0
    for k in range(4):
        if 0 <= i + k < len(b):
            v |= int(b[i + k]) << (8 * k)
    return v


def alignbyte(hi, lo, s):
    return (((hi << 32) | lo) >> (8 * s)) & M32


def udot4(a, m):
    return sum(((a >> (8 * k)) & 0xFF) * ((m >> (8 * k)) & 0xFF) for k in range(4))


def byte_lookup(table, sel):
    """v_perm with selector bytes 0..3: byte k of the result is byte sel_k of table."""
    out = 0
    for k in range(4):
        s = (sel >> (8 * k)) & 0xFF
        assert s < 4
        out |= ((table >> (8 * s)) & 0xFF) << (8 * k)
    return out


def top4(x):
    return sum(((x >> (8 * k + 7)) & 1) << k for k in range(4))


def class_bytes(w, below, emit, B):
    """A lane's byte sums for classes 0..2 and for all bytes."""
    c = [(below >> 7) & 0x01010101] + [(w[k] >> 7) & 0x01010101 for k in range(4)]
    q = (B * 0x01010101) & M32
    t = [[0] * 5 for _ in range(4)]
    for k in range(4):
        g = w[k] & 0x7F7F7F7F
        m1 = alignbyte(c[k + 1], c[k], 3)
        m2 = m1 & alignbyte(c[k + 1], c[k], 2)
        m3 = m2 & alignbyte(c[k + 1], c[k], 1)
        m4 = m3 & c[k]
        marks = [0x01010101, m1, m2, m3, m4]
        starts = ((((emit >> (4 * k)) & 0xF) * 0x00204081) & M32) & 0x01010101
        p = (starts * 0x01010101 + q) & M32
        q = ((p >> 24) * 0x01010101) & M32
        cls = p & 0x03030303
        for lev in range(5):
            t[3][lev] += udot4(g, marks[lev])
            for cc in range(3):
                mk = byte_lookup(1 << (8 * cc), cls)
                t[cc][lev] += udot4(g, mk & marks[lev])
    return [sum(LEVEL_WEIGHTS[lev] * t[cc][lev] for lev in range(5)) & M32 for cc in range(4)]


def run_across(last4, after):
    """Byte-sum terms, past a boundary, of the code running across it
    (last4: the 4 bytes before; after: the bytes after).  Returns
    (ends_within, rest); ends_within is None when no code runs across."""
    cb = top4(last4)
    p0 = 0
    while p0 < 4 and (cb >> (3 - p0)) & 1:
        p0 += 1
    if p0 == 0:
        return None, 0
    rest = 0
    for j, byte in enumerate(after):
        sh = 7 * (p0 + j)
        if sh < 32:
            rest += (int(byte) & 0x7F) << sh
        if byte < 0x80:
            return True, rest & M32
    return False, rest & M32


def lane_emit(b, o):
    """Bytes of the lane at o that begin a code ending in the stream."""
    e = 0
    for j in range(16):
        if o + j >= len(b):
            break
        if o + j == 0 or b[o + j - 1] < 0x80:
            k = o + j
            while k < len(b) and b[k] >= 0x80:
                k += 1
            if k < len(b):
                e |= 1 << j
    return e


def group_by_byte_sums(b, wv):
    cnt, acc = 0, [0, 0, 0, 0]
    for s in range(GROUP // SEG):
        base = wv + s * SEG
        emits = [lane_emit(b, base + 16 * ln) for ln in range(64)]
        before = 0
        for ln in range(64):
            o = base + 16 * ln
            w = [dword(b, o + 4 * k) for k in range(4)]
            sums = class_bytes(w, dword(b, o - 4), emits[ln], (cnt + before - 1) & 3)
            acc = [(x + y) & M32 for x, y in zip(acc, sums)]
            before += bin(emits[ln]).count("1")
        cnt += before
    S = acc[:3] + [(acc[3] - acc[0] - acc[1] - acc[2]) & M32]
    ends, rest = run_across(dword(b, wv - 4), [int(x) for x in b[wv:wv + 8]])
    if ends is not None:
        S[3] = (S[3] - rest) & M32
    ends, rest = run_across(dword(b, wv + GROUP - 4), [int(x) for x in b[wv + GROUP:wv + GROUP + 4]])
    if ends:
        S[(cnt - 1) & 3] = (S[(cnt - 1) & 3] + rest) & M32
    return cnt, S


def group_direct(b, wv):
    """The codes that begin in [wv, wv + GROUP) and end in the stream, summed
    by rank mod 4."""
    vals, pos = [], 0
    while pos < len(b):
        k, v, sh = pos, 0, 0
        while k < len(b) and b[k] >= 0x80:
            v += (int(b[k]) & 0x7F) << sh
            sh += 7
            k += 1
        if k >= len(b):
            break
        v += (int(b[k]) & 0x7F) << sh
        if wv <= pos < wv + GROUP:
            vals.append(v & M32)
        pos = k + 1
    S = [0, 0, 0, 0]
    for r, v in enumerate(vals):
        S[r & 3] = (S[r & 3] + v) & M32
    return len(vals), S


def streams():
    rng = np.random.default_rng(2024)
    m = 5000
    yield rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)        # mostly 5-byte codes
    yield rng.geometric(1 / 300, m).astype(np.uint32)                           # 1-2 byte codes
    yield rng.integers(0, 128, m).astype(np.uint32)                             # all 1-byte codes
    x = rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)
    yield x >> rng.integers(0, 32, m).astype(np.uint32)                         # every width mixed


def test_group_summary_by_byte_sums_matches_direct():
    groups = 0
    for x in streams():
        b = oracle.encode(x)
        for wv in range(GROUP, len(b) - GROUP - 8, GROUP):
            assert group_by_byte_sums(b, wv) == group_direct(b, wv), wv
            groups += 1
    assert groups >= 6


def test_identity_rejects_a_dropped_correction():
    # without taking the incoming code's bytes out of class 3 the sums differ
    # on a group that a code runs into
    # one 1-byte code, then 2-byte codes: every group boundary falls inside a code
    x = np.concatenate([[5], np.full(2999, 300)]).astype(np.uint32)
    b = oracle.encode(x)
    seen = 0
    for wv in range(GROUP, len(b) - GROUP - 8, GROUP):
        if b[wv - 1] >= 0x80:
            cnt, S = group_by_byte_sums(b, wv)
            _, rest = run_across(dword(b, wv - 4), [int(v) for v in b[wv:wv + 8]])
            assert rest != 0
            S_wrong = S[:3] + [(S[3] + rest) & M32]
            assert (cnt, S_wrong) != group_direct(b, wv)
            seen += 1
    assert seen >= 1
