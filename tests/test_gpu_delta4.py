"""GPU parity of the blocks-of-four differential decode (vbyte_decode_delta4,
reading R14) with the oracle: element by element with guard words, over
tilings, alignments, prev4 values, ragged lengths, codes straddling every
lane, segment, group and unit boundary, the status readings, resumption in
two parts, and a full-size stream."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import SENTINEL, dev, mixed_values, place_bytes, u32
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def gpu4(b, n, prev4=None, boff=0, ooff=0):
    _, data = place_bytes(b, boff)
    full = torch.full((ooff + n + 16,), SENTINEL, dtype=torch.int32, device=dev())
    out = full[ooff:ooff + n]
    st = torch.full((1,), -1, dtype=torch.int32, device=dev())
    vbyte.decode_delta4(data, n, prev4=prev4, out=out, status=st, check=False)
    torch.cuda.synchronize()
    h = u32(full)
    assert (h[:ooff] == SENTINEL).all() and (h[ooff + n:] == SENTINEL).all()
    return int(st.item()), h[ooff:ooff + n]


def check4(b, n, prev4=None, boff=0, ooff=0):
    st, y = gpu4(b, n, prev4, boff, ooff)
    sto, yo = oracle.decode_delta4(b, n, prev4)
    assert st == sto, f"status gpu={st} oracle={sto} (n={n}, boff={boff})"
    if sto == oracle.OK and not np.array_equal(y, yo):
        bad = np.nonzero(y != yo)[0]
        raise AssertionError(f"{bad.size} mismatches, first at {bad[0]}: gpu={y[bad[0]]} "
                             f"oracle={yo[bad[0]]} (n={n}, boff={boff})")
    return st, y


@pytest.mark.parametrize("tiling", [(1, 1), (1, 4), (2, 8), (2, 2)])
@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 777, 40_000, 300_003])
def test_random_streams(tiling, n):
    vbyte.set_tuning(tiling[0], tiling[1], 0)
    rng = np.random.default_rng(n + 10 * tiling[0] + tiling[1])
    x = np.sort(rng.integers(0, 1 << 32, n, dtype=np.uint64)).astype(np.uint32)
    b = oracle.encode_delta4(x)
    st, y = check4(b, n, boff=n % 16, ooff=n % 4)
    assert st == vbyte.OK and np.array_equal(y, x)
    g = mixed_values(rng, n)
    check4(oracle.encode(g), n, prev4=[1, 0xFFFFFFFF, 7, 1 << 31], boff=(n + 3) % 16)


@pytest.mark.parametrize("tiling", [(1, 2), (2, 4)])
def test_straddle_every_boundary(tiling):
    segs, wpb = tiling
    vbyte.set_tuning(segs, wpb, 0)
    group = segs * 1024
    unit = 8 * group
    rng = np.random.default_rng(segs + wpb)
    for long_len in (5, 3):
        vals, pos = [], 0
        targets = sorted({k * 16 for k in range(1, 70)} | {k * 1024 for k in range(1, 6)} |
                         {k * group for k in range(1, 5)} | {k * unit for k in range(1, 4)})
        for tgt in targets:
            for phase in range(long_len + 1):
                start = tgt - phase
                while pos < start:
                    vals.append(int(rng.integers(0, 128)))
                    pos += 1
                if pos == start:
                    lo = 1 << (7 * (long_len - 1))
                    hi = min(1 << (7 * long_len), 1 << 32)
                    vals.append(int(rng.integers(lo, hi)))
                    pos += long_len
        g = np.array(vals, np.uint32)
        b = oracle.encode(g)
        for boff in (0, 1, 13):
            check4(b, g.size, boff=boff)
            check4(b, g.size, prev4=[9, 8, 7, 6], boff=boff, ooff=1)


def test_statuses_and_counts():
    rng = np.random.default_rng(3)
    g = mixed_values(rng, 50_000, (1, 2, 3))
    b = oracle.encode(g)
    n = g.size
    assert check4(b, n)[0] == vbyte.OK
    assert check4(b, n - 1)[0] == vbyte.ECOUNT       # nothing written past n
    assert check4(b, n + 1)[0] == vbyte.ETRUNC
    assert check4(b[:-1], n)[0] in (vbyte.ETRUNC, vbyte.ECOUNT)
    for at in (5, 1023, 8 * 2048 - 2, b.size - 6):
        bad = b.copy()
        bad[at:at + 5] = 0x80
        assert check4(bad, n)[0] == vbyte.EMALFORMED
    assert check4(np.zeros(0, np.uint8), 0)[0] == vbyte.OK
    assert check4(np.zeros(0, np.uint8), 1)[0] == vbyte.ETRUNC


def test_resume_in_two_parts():
    rng = np.random.default_rng(4)
    x = np.sort(rng.integers(0, 1 << 31, 100_000, dtype=np.uint64)).astype(np.uint32)
    b = oracle.encode_delta4(x)
    m = 54_321
    gaps = np.concatenate([x[:4], x[4:] - x[:-4]]).astype(np.uint32)
    cut = oracle.encoded_size(gaps[:m])
    st1, y1 = gpu4(b[:cut], m)
    st2, y2 = gpu4(b[cut:], x.size - m, prev4=[int(v) for v in x[m - 4:m]])
    assert st1 == st2 == vbyte.OK
    assert np.array_equal(np.concatenate([y1, y2]), x)


def test_synchronous_call():
    rng = np.random.default_rng(6)
    x = np.sort(rng.integers(0, 1 << 32, 9_999, dtype=np.uint64)).astype(np.uint32)
    b = oracle.encode_delta4(x)
    d = torch.from_numpy(b).to(dev())
    out = torch.empty(x.size, dtype=torch.int32, device=dev())
    L = vbyte._lib()
    assert L.vbyte_decode_delta4(d.data_ptr(), b.size, out.data_ptr(), x.size, None) == vbyte.OK
    assert np.array_equal(u32(out), x)
    assert L.vbyte_decode_delta4(d.data_ptr(), b.size, out.data_ptr(), x.size + 1, None) == vbyte.ETRUNC


def test_full_size_stream():
    """64Mi identifiers with gaps of mean 300, coded as differences of four."""
    vbyte.set_tuning(2, 8, 0)
    g = workloads.geometric_gaps(mean=300)
    with np.errstate(over="ignore"):
        x = np.cumsum(g, dtype=np.uint32)
    b = oracle.encode_delta4(x)
    st, y = gpu4(b, x.size)
    assert st == vbyte.OK and np.array_equal(y, x)
