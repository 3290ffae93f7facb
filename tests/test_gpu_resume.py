"""GPU parity of the resumable decode in pieces (vbyte_decode_next_async,
reading R12): every piece, cursor and carried prev against the oracle's
pieces, chains of pieces without host synchronisation against the
whole-stream decode, and the error cases (the cursor stays)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import mixed_values, u32
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def cursor_h(c):
    v = c.cpu().numpy()
    return int(v[0]), int(v[1]), int(v[2]) & 0xFFFFFFFF


def run_pieces(b, k, delta, prev=0, boff=0):
    """Decode b in pieces of k on the GPU, checking each piece against the
    oracle's piece from the same cursor; returns the concatenated values."""
    host = np.full(boff + b.size, 0x80, np.uint8)
    host[boff:] = b
    buf = torch.from_numpy(host).cuda()[boff:]
    out = torch.full((k + 8,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    cin, cout = vbyte.new_cursor(prev), vbyte.new_cursor(prev)
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    got = []
    ndone = 0
    off, oprev = 0, prev
    while True:
        vbyte.decode_next(buf, k, out, cin, cout, delta=delta == 1, minus_one=delta == 2, status=st)
        torch.cuda.synchronize()
        sto, yo, noff, nprev = oracle.decode_next(b, off, k, oprev, delta)
        assert int(st.item()) == sto == oracle.OK
        c_off, c_done, c_prev = cursor_h(cout)
        assert (c_off, c_prev) == (noff, nprev)
        assert c_done == ndone + yo.size
        ndone += yo.size
        y = u32(out)
        assert np.array_equal(y[:yo.size], yo)
        assert (y[k:] == 0x5A5A5A5A).all()
        got.append(yo)
        if yo.size < k:
            break
        off, oprev = noff, nprev
        cin, cout = cout, cin
    return np.concatenate(got) if got else np.zeros(0, np.uint32)


@pytest.mark.parametrize("delta", [0, 1, 2])
@pytest.mark.parametrize("k", [1, 100, 4096, 70_000, 300_000])
def test_pieces_match_oracle(delta, k):
    rng = np.random.default_rng(k + delta)
    x = mixed_values(rng, min(250_000, 40 * k + 17))   # at most ~40 pieces
    x[rng.random(x.size) < 0.6] %= 128
    b = oracle.encode(x)
    y = run_pieces(b, k, delta, prev=7, boff=(k % 13))
    whole = {0: oracle.decode(b, x.size), 1: oracle.decode_delta(b, x.size, 7),
             2: oracle.decode_delta_m1(b, x.size, 7)}[delta][1]
    assert np.array_equal(y, whole)


@pytest.mark.parametrize("tiling", [(4, 8), (1, 2)])
def test_chain_without_sync_matches_whole(tiling):
    vbyte.set_tuning(tiling[0], tiling[1], 0)
    g = workloads.geometric_gaps(n=3_000_000, mean=300)
    b = oracle.encode(g)
    buf = torch.from_numpy(b).cuda()
    k = 1 << 18
    npieces = (g.size + k - 1) // k
    pieces = torch.empty((npieces, k), dtype=torch.int32, device="cuda")
    curs = [vbyte.new_cursor(0) for _ in range(npieces + 1)]
    sts = torch.empty(npieces, dtype=torch.int32, device="cuda")
    for i in range(npieces):
        vbyte.decode_next(buf, k, pieces[i], curs[i], curs[i + 1], delta=True, status=sts[i:i + 1])
    torch.cuda.synchronize()
    assert (sts.cpu().numpy() == vbyte.OK).all()
    st, whole = oracle.decode_delta(b, g.size, 0)
    y = u32(pieces).reshape(-1)[:g.size]
    assert np.array_equal(y, whole)
    assert cursor_h(curs[-1])[:2] == (b.size, g.size)


def test_piece_errors_keep_cursor():
    b = oracle.encode(np.array([1, 300, 70000, 5], np.uint32))
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    cases = [
        (np.concatenate([b, [0x85, 0x81]]), 5, vbyte.ETRUNC),
        (np.concatenate([b, [0x80] * 5, [0x01]]), 4, vbyte.EMALFORMED),
        (np.concatenate([b, [0x85, 0x81]]), 4, vbyte.OK),
        (np.concatenate([b, [0x80] * 5, [0x01]]), 1, vbyte.OK),
    ]
    for buf, k, expect in cases:
        d = torch.from_numpy(buf.astype(np.uint8)).cuda()
        cin = torch.tensor([0, 3, 9], dtype=torch.int64, device="cuda")
        cout = torch.full((3,), -1, dtype=torch.int64, device="cuda")
        vbyte.decode_next(d, k, out, cin, cout, status=st)
        torch.cuda.synchronize()
        sto, yo, noff, _ = oracle.decode_next(buf.astype(np.uint8), 0, k, 9, 0)
        assert int(st.item()) == sto == expect
        if expect != vbyte.OK:
            assert cursor_h(cout) == (0, 3, 9)
        else:
            assert cursor_h(cout)[:2] == (noff, 3 + yo.size)
            assert np.array_equal(u32(out)[:yo.size], yo)
    # a cursor past the end of the data
    d = torch.from_numpy(b).cuda()
    cin = torch.tensor([b.size + 1, 0, 0], dtype=torch.int64, device="cuda")
    cout = torch.full((3,), -1, dtype=torch.int64, device="cuda")
    vbyte.decode_next(d, 2, out, cin, cout, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == vbyte.EINVAL and cursor_h(cout) == (b.size + 1, 0, 0)
    # at the end: nothing left, OK
    cin = torch.tensor([b.size, 4, 5], dtype=torch.int64, device="cuda")
    vbyte.decode_next(d, 2, out, cin, cout, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == vbyte.OK and cursor_h(cout) == (b.size, 4, 5)
