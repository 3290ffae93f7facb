"""GPU parity of the batched decode (CSR and gather forms) against the CPU
oracle's BATCH, bit-exact, including per-list statuses."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import SENTINEL, dev, mixed_values, u32
from paper_1503_07387_amd import vbyte

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def make_lists(rng, lens, lengths=(1, 2, 3, 4, 5)):
    lists = [mixed_values(rng, int(k), lengths) for k in lens]
    enc = [oracle.encode(x) for x in lists]
    byte_off = np.zeros(len(lens) + 1, np.int64)
    byte_off[1:] = np.cumsum([e.size for e in enc])
    out_off = np.zeros(len(lens) + 1, np.int64)
    out_off[1:] = np.cumsum(lens)
    b = np.concatenate(enc) if enc else np.zeros(0, np.uint8)
    return lists, b, byte_off, out_off


def run_batch(b, byte_off, out_off, prevs=None, delta=False, boff=0, nout=None):
    host = np.full(boff + b.size + 32, 0x80, np.uint8)
    host[boff:boff + b.size] = b
    d = torch.from_numpy(host).to(dev())
    data = d[boff:boff + b.size]
    nl = byte_off.size - 1
    total = int(out_off[-1]) if nout is None else nout
    full = torch.full((total + 16,), SENTINEL, dtype=torch.int32, device=dev())
    out = full[:total]
    status = torch.full((max(nl, 1),), -1, dtype=torch.int32, device=dev())
    bo = torch.from_numpy(byte_off).to(dev())
    oo = torch.from_numpy(out_off).to(dev())
    pv = torch.from_numpy(np.asarray(prevs, np.uint32).view(np.int32)).to(dev()) if prevs is not None else None
    vbyte.decode_batch(data, bo, oo, delta=delta, prevs=pv, out=out, list_status=status[:nl])
    torch.cuda.synchronize()
    h = u32(full)
    assert (h[total:] == SENTINEL).all(), "write past out"
    return h[:total], status[:nl].cpu().numpy()


def compare(b, byte_off, out_off, prevs=None, delta=False, boff=0):
    y, st = run_batch(b, byte_off, out_off, prevs, delta, boff)
    sto, yo, lst = oracle.decode_batch(b, byte_off, out_off, prevs, delta)
    assert np.array_equal(st, lst), f"status gpu={st[st != lst][:5]} oracle={lst[st != lst][:5]}"
    for i in np.nonzero(lst == oracle.OK)[0]:
        a, e = out_off[i], out_off[i + 1]
        if not np.array_equal(y[a:e], yo[a:e]):
            bad = np.nonzero(y[a:e] != yo[a:e])[0]
            raise AssertionError(f"list {i} ({e - a} ints): {bad.size} mismatches from {bad[0]}")
    return y, st


LEN_MIXES = {
    "tiny": [0, 1, 2, 3, 0, 5, 1, 1, 7],
    "mixed": [0, 1, 17, 300, 1000, 5000, 20000, 0, 1, 64, 65, 100000, 3, 250000, 40000],
    "large": [300000, 1, 700000, 5, 123457],
}


@pytest.mark.parametrize("mix", list(LEN_MIXES))
@pytest.mark.parametrize("small", [1, 2048, 16384, 1 << 30])
def test_csr_random_lists(mix, small):
    vbyte.set_tuning(0, 0, small)
    rng = np.random.default_rng(len(mix) + small)
    lens = LEN_MIXES[mix]
    _, b, byte_off, out_off = make_lists(rng, lens)
    prevs = rng.integers(0, 1 << 32, len(lens), dtype=np.uint64).astype(np.uint32)
    for boff in (0, 5):
        y, st = compare(b, byte_off, out_off, boff=boff)
        assert (st == vbyte.OK).all()
        compare(b, byte_off, out_off, prevs=prevs, delta=True, boff=boff)
        compare(b, byte_off, out_off, prevs=None, delta=True, boff=boff)


@pytest.mark.parametrize("segs,wpb", [(1, 1), (2, 4), (4, 8), (1, 8)])
def test_csr_tilings(segs, wpb):
    vbyte.set_tuning(segs, wpb, 4096)
    rng = np.random.default_rng(segs * 100 + wpb)
    lens = list(rng.integers(0, 3000, 200)) + [50000, 120000, 1, 0, 9999]
    _, b, byte_off, out_off = make_lists(rng, lens, (1, 2, 5))
    prevs = rng.integers(0, 1 << 32, len(lens), dtype=np.uint64).astype(np.uint32)
    compare(b, byte_off, out_off, boff=3)
    compare(b, byte_off, out_off, prevs=prevs, delta=True, boff=3)


def test_many_small_lists():
    rng = np.random.default_rng(5)
    lens = rng.integers(0, 40, 20000)
    _, b, byte_off, out_off = make_lists(rng, lens, (1, 2))
    compare(b, byte_off, out_off)
    compare(b, byte_off, out_off, prevs=rng.integers(0, 1000, lens.size).astype(np.uint32), delta=True)


def test_bad_lists_fail_alone():
    vbyte.set_tuning(0, 0, 4096)
    rng = np.random.default_rng(6)
    lens = [1000, 20000, 7, 30000, 500, 9000]
    lists, b, byte_off, out_off = make_lists(rng, lens, (1, 2, 3))
    bad = b.copy()
    # malformed run inside list 1 (large) and list 4 (small)
    s1 = byte_off[1] + 5000
    bad[s1:s1 + 5] = 0x80
    s4 = byte_off[4] + 100
    bad[s4:s4 + 6] = 0x81
    y, st = compare(bad, byte_off, out_off)
    assert st[1] == vbyte.EMALFORMED and st[4] == vbyte.EMALFORMED
    assert st[0] == st[2] == st[3] == st[5] == vbyte.OK
    # count mismatches: list 3 expects one more integer, list 5 one fewer
    oo = out_off.copy()
    oo[4:] += 1
    oo[6] -= 2
    y, st = compare(b, byte_off, oo)
    assert st[3] == vbyte.ETRUNC and st[5] == vbyte.ECOUNT


@pytest.mark.parametrize("segs", [1, 4])
def test_bad_one_piece_lists(segs):
    """Lists that fit one wavefront's piece go to the piece decode with no
    aggregation pass, which then alone finds their malformed runs (start,
    middle and end of a list, runs that cross list boundaries) and their
    truncation and count statuses."""
    vbyte.set_tuning(segs, 8, 1)   # every non-empty list takes the piece path
    rng = np.random.default_rng(60 + segs)
    lens = list(rng.integers(1, 400 * segs, 300))
    lists, b, byte_off, out_off = make_lists(rng, lens, (1, 2, 3))
    bad = b.copy()
    for i in range(0, len(lens), 7):
        a0, e0 = int(byte_off[i]), int(byte_off[i + 1])
        at = [a0, (a0 + e0) // 2, max(a0, e0 - 5), e0 - 2][i % 4]
        bad[at:at + 5] = 0x80 | (i & 0x7F)
    y, st = compare(bad, byte_off, out_off, boff=7)
    assert (st == vbyte.EMALFORMED).sum() > 0 and (st == vbyte.OK).sum() > 0
    oo = out_off.copy()
    oo[1:] += np.arange(1, len(lens) + 1) % 3 - 1   # one more, same, one fewer, ...
    oo[1:] = np.maximum.accumulate(np.maximum(oo[1:], 0))
    compare(b, byte_off, oo, delta=True)


@pytest.mark.parametrize("segs", [1, 2, 4])
def test_lists_around_one_piece(segs):
    """Lists whose bytes (with their start misalignment) end just below, at
    and just above one piece of segs KiB and of two pieces: the one-piece
    lists skip the aggregation pass, the others do not.  One-byte codes, so
    n equals the byte count."""
    vbyte.set_tuning(segs, 4, 1)
    ub = segs * 1024
    rng = np.random.default_rng(70 + segs)
    sizes = [ub + d for d in range(-24, 25)] + [2 * ub + d for d in range(-20, 21, 4)]
    lens = list(rng.permutation(np.array(sizes * 2)))
    lists, b, byte_off, out_off = make_lists(rng, lens, (1,))
    prevs = rng.integers(0, 1 << 32, len(lens), dtype=np.uint64).astype(np.uint32)
    for boff in (0, 9):
        y, st = compare(b, byte_off, out_off, boff=boff)
        assert (st == vbyte.OK).all()
        compare(b, byte_off, out_off, prevs=prevs, delta=True, boff=boff)
    # differences minus one: strictly increasing lists
    inc = [np.cumsum(rng.integers(1, 100, int(k)), dtype=np.uint64).astype(np.uint32) for k in lens]
    enc = [oracle.encode_delta_m1(x, 0) for x in inc]
    bo = np.zeros(len(lens) + 1, np.int64)
    bo[1:] = np.cumsum([e.size for e in enc])
    data = torch.from_numpy(np.concatenate(enc)).to(dev())
    out, st = vbyte.decode_batch(data, torch.from_numpy(bo).to(dev()), torch.from_numpy(out_off).to(dev()),
                                 delta=True, minus_one=True)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == vbyte.OK).all()
    assert np.array_equal(u32(out), np.concatenate(inc))


def test_more_pieces_than_the_grid_cap():
    """More large-list pieces than the piece kernels' capped grid holds
    (2^16 workgroups of one wavefront with 1 KiB pieces): the grid stride
    takes the rest."""
    vbyte.set_tuning(1, 1, 1)
    rng = np.random.default_rng(61)
    lens = rng.integers(700, 1400, 48000)
    _, b, byte_off, out_off = make_lists(rng, lens, (1, 2))
    pieces = int(((byte_off[1:] - byte_off[:-1] + 1023) // 1024).sum())   # at least
    assert pieces > (1 << 16)
    y, st = compare(b, byte_off, out_off, boff=3)
    assert (st == vbyte.OK).all()
    compare(b, byte_off, out_off, prevs=rng.integers(0, 1 << 32, lens.size, dtype=np.uint64).astype(np.uint32),
            delta=True, boff=3)


def test_invalid_offsets_are_rejected_per_list():
    rng = np.random.default_rng(7)
    lens = [100, 200, 300, 400]
    _, b, byte_off, out_off = make_lists(rng, lens)
    bo = byte_off.copy()
    bo[2] = bo[3] + 1          # list 2 now ends before it starts; list 1 overruns
    y, st = run_batch(b, bo, out_off)
    assert st[2] == vbyte.EINVAL
    assert st[1] == oracle.validate(b[bo[1]:bo[2]], lens[1])
    assert st[0] == vbyte.OK and st[3] == vbyte.OK
    bo = byte_off.copy()
    bo[-1] = b.size + 100      # last list reaches past the byte array
    y, st = run_batch(b, bo, out_off)
    assert st[3] == vbyte.EINVAL and (st[:3] == vbyte.OK).all()
    oo = out_off.copy()
    oo[-1] += 50               # last list would write past `out`
    y, st = run_batch(b, byte_off, oo, nout=int(out_off[-1]))
    assert st[3] == vbyte.EINVAL and (st[:3] == vbyte.OK).all()


def test_gather_rows_with_repeats():
    vbyte.set_tuning(0, 0, 8192)
    rng = np.random.default_rng(8)
    lens = [5000, 10, 80000, 0, 333]
    lists, b, byte_off, out_off = make_lists(rng, lens)
    pick = [2, 0, 2, 4, 1, 3, 0]
    rows, pos = [], 0
    for i in pick:
        rows.append([byte_off[i], byte_off[i + 1], pos, lens[i]])
        pos += lens[i]
    rows = np.array(rows, np.int64)
    d = torch.from_numpy(b).to(dev())
    out = torch.full((pos + 8,), SENTINEL, dtype=torch.int32, device=dev())
    prevs = rng.integers(0, 1 << 32, len(pick), dtype=np.uint64).astype(np.uint32)
    for delta in (False, True):
        st = vbyte.decode_lists(d, torch.from_numpy(rows).to(dev()),
                                int((rows[:, 1] - rows[:, 0]).sum()), out[:pos], delta=delta,
                                prevs=torch.from_numpy(prevs.view(np.int32)).to(dev()))
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == vbyte.OK).all()
        h = u32(out)
        assert (h[pos:] == SENTINEL).all()
        for k, i in enumerate(pick):
            a = rows[k, 2]
            ref = oracle.decode_delta(b[byte_off[i]:byte_off[i + 1]], lens[i], int(prevs[k]))[1] if delta \
                else lists[i]
            assert np.array_equal(h[a:a + lens[i]], ref)


def test_gather_capacity_too_small_fails_cleanly():
    rng = np.random.default_rng(9)
    lens = [50000, 60000]
    _, b, byte_off, _ = make_lists(rng, lens)
    rows = np.array([[byte_off[0], byte_off[1], 0, lens[0]]] * 40, np.int64)
    out = torch.empty(lens[0], dtype=torch.int32, device=dev())
    rows[:, 2] = 0
    d = torch.from_numpy(b).to(dev())
    st = vbyte.decode_lists(d, torch.from_numpy(rows).to(dev()), 1000, out)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == vbyte.EINVAL).all()
