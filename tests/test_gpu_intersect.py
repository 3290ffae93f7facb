"""GPU parity of the list intersection (vbyte_intersect_async, reading R15:
decode and consumer fused per tile, the status of decoding in pieces) with
the oracle's piece-by-piece intersection: matches in list order, their
count, and the status, over piece sizes, list densities, duplicates,
identifiers that wrap mod 2^32 (windows of b too wide for LDS), a capacity
below the match count, and the error cases, fixed and drawn at random."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, u32
from paper_1503_07387_amd import vbyte

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def run(a, na, b_ids, piece, prev=0, cap=None):
    ad = torch.from_numpy(np.asarray(a, np.uint8)).to(dev())
    bd = torch.from_numpy(np.ascontiguousarray(b_ids, np.uint32).view(np.int32)).to(dev())
    cap = max(na, 1) if cap is None else cap
    out = torch.full((cap + 8,), -1, dtype=torch.int32, device=dev())
    cnt = torch.empty(1, dtype=torch.int64, device=dev())
    st = torch.empty(1, dtype=torch.int32, device=dev())
    vbyte.intersect(ad, na, bd, prev=prev, piece=piece, out=out[:cap], count=cnt, status=st,
                    check=False)
    torch.cuda.synchronize()
    h = u32(out)
    assert (h[cap:] == 0xFFFFFFFF).all(), "write past out_cap"
    return int(st.item()), int(cnt.item()), h[:cap]


def lists(seed, na, nb, universe, dup=False):
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(universe, size=na, replace=dup)).astype(np.uint32)
    b = np.sort(rng.choice(universe, size=nb, replace=dup)).astype(np.uint32)
    return ids, b


@pytest.mark.parametrize("piece", [1, 100, 1024, 65_536, 1 << 20])
@pytest.mark.parametrize("shape", [(200_000, 5_000, 1 << 24), (50_000, 50_000, 200_000),
                                   (3, 10, 50), (0, 10, 50)])
def test_matches_oracle(piece, shape):
    na, nb, universe = shape
    ids, b = lists(na + nb + piece, na, nb, universe)
    a = oracle.encode_delta(ids, 5)
    st, cnt, got = run(a, na, b, piece, prev=5)
    # the oracle's result does not depend on the piece size for a valid list
    # (pinned against brute force over piece sizes); for one integer per
    # piece on the long lists its pieces of 4096 keep the host loop short
    opiece = 4096 if (piece == 1 and na > 10_000) else piece
    sto, want = oracle.intersect_pieces(a, na, b, opiece, 5)
    assert st == sto == vbyte.OK
    assert cnt == want.size and np.array_equal(got[:cnt], want)


def test_duplicates_on_both_sides():
    rng = np.random.default_rng(9)
    ids = np.sort(rng.integers(0, 3000, 20_000)).astype(np.uint32)   # many repeats: gaps of 0
    b = np.sort(rng.integers(0, 3000, 2_000)).astype(np.uint32)
    a = oracle.encode_delta(ids, 0)
    for piece in (7, 4096):
        st, cnt, got = run(a, ids.size, b, piece)
        sto, want = oracle.intersect_pieces(a, ids.size, b, piece)
        assert st == sto == vbyte.OK and cnt == want.size and np.array_equal(got[:cnt], want)


def test_capacity_below_count():
    ids, b = lists(10, 100_000, 80_000, 150_000)
    a = oracle.encode_delta(ids, 0)
    sto, want = oracle.intersect_pieces(a, ids.size, b, 4096)
    cap = want.size // 3
    st, cnt, got = run(a, ids.size, b, 4096, cap=cap)
    assert st == vbyte.OK and cnt == want.size
    assert np.array_equal(got[:cap], want[:cap])


def test_statuses():
    ids = np.arange(10, 30_010, 3, dtype=np.uint32)
    a = oracle.encode_delta(ids, 0)
    bad = a.copy()
    bad[5000:5005] = 0x80
    for piece in (64, 5000):
        for buf, na in ((a, ids.size + 1), (a, ids.size - 1), (bad, ids.size), (a[:-1], ids.size)):
            st, cnt, got = run(buf, na, ids, piece)
            sto, want = oracle.intersect_pieces(buf, na, ids, piece)
            assert st == sto, (piece, na, st, sto)
            if st == vbyte.OK:
                assert np.array_equal(got[:cnt], want)
    st, cnt, _ = run(np.zeros(0, np.uint8), 0, ids, 64)
    assert st == vbyte.OK and cnt == 0
    st, cnt, _ = run(np.zeros(0, np.uint8), 5, ids, 64)
    assert st == vbyte.ETRUNC and cnt == 0


def test_long_list_against_whole_decode():
    """The 4Mi-identifier list in pieces of 256Ki against the same list
    decoded whole in one piece: identical matches."""
    vbyte.set_tuning(2, 8, 0)
    ids, b = lists(11, 1 << 22, 1 << 16, 1 << 28)
    a = oracle.encode_delta(ids, 0)
    s1, c1, g1 = run(a, ids.size, b, 1 << 18)
    s2, c2, g2 = run(a, ids.size, b, 1 << 22)
    want = ids[np.isin(ids, b)]
    assert s1 == s2 == vbyte.OK and c1 == c2 == want.size
    assert np.array_equal(g1[:c1], want) and np.array_equal(g2[:c2], want)


@pytest.mark.parametrize("nb", [300, 1152, 1153, 40_000])
def test_wrapping_identifiers(nb):
    """Gaps up to 2^30: the identifiers wrap mod 2^32 every few codes, so a
    wavefront's identifiers span the whole range and its window of b is all
    of b (held in LDS up to 1152 entries, searched in memory above)."""
    rng = np.random.default_rng(nb)
    g = rng.integers(1, 1 << 30, size=150_000, dtype=np.uint64)
    ids = ((np.cumsum(g) + 7) & 0xFFFFFFFF).astype(np.uint32)
    pick = rng.choice(ids, size=nb // 2)
    b = np.sort(np.concatenate([pick, rng.integers(0, 1 << 32, size=nb - nb // 2,
                                                    dtype=np.uint64).astype(np.uint32)]))
    a = oracle.encode_delta(ids, 7)
    st, cnt, got = run(a, ids.size, b, 4096, prev=7)
    sto, want = oracle.intersect_pieces(a, ids.size, b, 4096, 7)
    assert st == sto == vbyte.OK
    assert cnt == want.size and np.array_equal(got[:cnt], want)


def test_dense_short_list():
    """b denser than the list: windows of about 2000 entries (searched in
    memory) next to windows that fit LDS."""
    ids, b = lists(21, 300_000, 250_000, 400_000)
    a = oracle.encode_delta(ids, 0)
    st, cnt, got = run(a, ids.size, b, 1 << 16)
    sto, want = oracle.intersect_pieces(a, ids.size, b, 1 << 16)
    assert st == sto == vbyte.OK
    assert cnt == want.size and np.array_equal(got[:cnt], want)


def test_random_statuses():
    """Short lists with runs of continuation bytes, cut tails, trailing
    continuation bytes and counts off by a few, over piece sizes 1 .. 64:
    the status of decoding in pieces, from the stream's totals."""
    rng = np.random.default_rng(77)
    ids = np.arange(3, 3 + 40, dtype=np.uint32)
    b = ids[::3].copy()
    seen = set()
    for it in range(300):
        n = int(rng.integers(0, 40))
        L = rng.integers(1, 6, size=n)
        vals = np.array([int(rng.integers(1 << (7 * (l - 1)) if l > 1 else 0,
                                          min(1 << (7 * l), 1 << 32))) for l in L],
                        dtype=np.uint64).astype(np.uint32)
        buf = oracle.encode(vals).copy()
        r = rng.random()
        if r < 0.3 and buf.size:
            q, ln = int(rng.integers(0, buf.size)), int(rng.integers(1, 8))
            buf[q:q + ln] = 0x80 | rng.integers(0, 128, size=min(ln, buf.size - q)).astype(np.uint8)
        elif r < 0.45 and buf.size:
            buf = buf[:int(rng.integers(0, buf.size))]
        elif r < 0.55:
            buf = np.concatenate([buf, (0x80 | rng.integers(0, 128, size=int(rng.integers(1, 7))))
                                  .astype(np.uint8)])
        na = max(0, n + int(rng.integers(-3, 4)))
        piece = int(rng.choice([1, 2, 3, 4, 5, 7, 16, 64]))
        st, cnt, got = run(buf, na, b, piece)
        sto, want = oracle.intersect_pieces(buf, na, b, piece)
        assert st == sto, (it, list(buf), na, piece, st, sto)
        if st == vbyte.OK:
            assert cnt == want.size and np.array_equal(got[:cnt], want)
        seen.add(st)
    assert seen == {vbyte.OK, vbyte.ECOUNT, vbyte.ETRUNC, vbyte.EMALFORMED}


def test_runs_far_into_long_lists():
    """A run of five continuation bytes deep in a list of many tiles, near
    tile edges, with na such that the last piece's window does or does not
    reach the run, for several piece sizes."""
    ids = np.cumsum(np.random.default_rng(4).integers(1, 300, size=100_000)).astype(np.uint32)
    a = oracle.encode_delta(ids, 0)
    seen = set()
    for pos in (16384 * 5 - 3, 16384 * 9 + 1, a.size - 6):
        bad = a.copy()
        bad[pos:pos + 5] = 0x81
        before = int((bad[:pos] < 0x80).sum())   # codes that end before the run
        for na in (ids.size, before, before - 37, before - 3000):
            for piece in (64, 1000, 50_000):
                st, _, _ = run(bad, na, ids[::7], piece)
                sto, _ = oracle.intersect_pieces(bad, na, ids[::7], piece)
                assert st == sto, (pos, na, piece, st, sto)
                seen.add(st)
    assert seen == {vbyte.EMALFORMED, vbyte.ECOUNT}
