"""GPU tests of the graph-captured batched decode and of the autotuner.

The graph form is replayed several times with eager work and
synchronisations between replays, and every replay is checked against the
eager batched decode and the CPU oracle.  The autotuner must time every
candidate on the caller's workload, apply the fastest, leave results
bit-exact, refuse a workload that does not decode, and its JSON cache must
return the stored tiling without timing again."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import u32
from paper_1503_07387_amd import autotune, vbyte

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def csr_lists(seed, nlists=400):
    rng = np.random.default_rng(seed)
    lens = np.concatenate([rng.integers(1, 300, nlists - 6), [40000, 90000, 200000, 5000, 17000, 1]])
    rng.shuffle(lens)
    out_off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=out_off[1:])
    gaps = rng.geometric(1 / 60.0, int(out_off[-1])).astype(np.uint32)
    b = oracle.encode(gaps)
    byte_off = np.zeros(lens.size + 1, np.int64)
    for i in range(lens.size):
        byte_off[i + 1] = byte_off[i] + oracle.encoded_size(gaps[out_off[i]:out_off[i + 1]])
    return b, byte_off, out_off


@pytest.mark.parametrize("delta", [False, True])
def test_batch_graph_replays_match_eager(delta):
    b, byte_off, out_off = csr_lists(11)
    nl = byte_off.size - 1
    prevs = torch.from_numpy(np.arange(nl, dtype=np.uint32).view(np.int32) * 3).cuda() if delta else None
    bd = torch.from_numpy(b).cuda()
    bo = torch.from_numpy(byte_off).cuda()
    oo = torch.from_numpy(out_off).cuda()
    eager, est = vbyte.decode_batch(bd, bo, oo, delta=delta, prevs=prevs)
    torch.cuda.synchronize()
    assert (est.cpu().numpy() == vbyte.OK).all()
    ref = u32(eager)
    pv = None if prevs is None else prevs.cpu().numpy().view(np.uint32)
    sto, yo, _ = oracle.decode_batch(b, byte_off, out_off, pv, delta)
    assert sto == oracle.OK and np.array_equal(ref, yo)

    out = torch.empty(int(out_off[-1]), dtype=torch.int32, device="cuda")
    lst = torch.empty(nl, dtype=torch.int32, device="cuda")
    g = vbyte.BatchGraph(bd, bo, oo, out, lst, delta=delta, prevs=prevs)
    try:
        for rep in range(4):
            out.fill_(-1)
            lst.fill_(-1)
            g.launch()
            torch.cuda.synchronize()
            assert (lst.cpu().numpy() == vbyte.OK).all(), rep
            assert np.array_equal(u32(out), ref), rep
            # eager work between replays
            e2, _ = vbyte.decode_batch(bd, bo, oo, delta=not delta)
            torch.cuda.synchronize()
            del e2
    finally:
        g.close()


def test_batch_graph_reads_current_contents():
    b, byte_off, out_off = csr_lists(12, nlists=50)
    bd = torch.from_numpy(b).cuda()
    bo = torch.from_numpy(byte_off).cuda()
    oo = torch.from_numpy(out_off).cuda()
    out = torch.empty(int(out_off[-1]), dtype=torch.int32, device="cuda")
    lst = torch.empty(byte_off.size - 1, dtype=torch.int32, device="cuda")
    g = vbyte.BatchGraph(bd, bo, oo, out, lst)
    try:
        g.launch()
        torch.cuda.synchronize()
        first = u32(out).copy()
        # same layout, new contents: raise every 1-byte code by one (stays < 0x80 unless 0x7F)
        b2 = b.copy()
        one = (b2 < 0x7F) & np.concatenate([[True], b2[:-1] < 0x80])
        b2[one] += 1
        bd.copy_(torch.from_numpy(b2))
        g.launch()
        torch.cuda.synchronize()
        assert (lst.cpu().numpy() == vbyte.OK).all()
        st, yo, _ = oracle.decode_batch(b2, byte_off, out_off, None, False)
        assert st == oracle.OK
        assert np.array_equal(u32(out), yo)
        assert not np.array_equal(first, yo)
    finally:
        g.close()


def test_autotune_decode_applies_fastest():
    rng = np.random.default_rng(13)
    g = rng.geometric(1 / 200.0, 1_500_000).astype(np.uint32)
    b = oracle.encode(g)
    bd = torch.from_numpy(b).cuda()
    pts = vbyte.autotune_decode(bd, g.size, delta=True, reps=2)
    assert len(pts) == 24
    assert {p["tiles_per_chunk"] for p in pts} == {-1, 0, 2, 4, 8, 16}
    assert all(p["status"] == vbyte.OK and p["ms"] > 0 for p in pts)
    best = min(pts, key=lambda p: p["ms"])
    t = vbyte.get_tuning()
    keys = ("segs_per_wave", "waves_per_block", "tiles_per_chunk")
    assert {k: t[k] for k in keys} == {k: best[k] for k in keys}
    out = vbyte.decode(bd, g.size, delta=True)
    st, yo = oracle.decode_delta(b, g.size, 0)
    assert st == oracle.OK and np.array_equal(u32(out), yo)


def test_autotune_batch_applies_fastest():
    b, byte_off, out_off = csr_lists(14, nlists=300)
    bd = torch.from_numpy(b).cuda()
    bo = torch.from_numpy(byte_off).cuda()
    oo = torch.from_numpy(out_off).cuda()
    pts = vbyte.autotune_batch(bd, bo, oo, delta=True, reps=1)
    assert len(pts) == 16
    assert all(p["status"] == vbyte.OK for p in pts)
    best = min(pts, key=lambda p: p["ms"])
    t = vbyte.get_tuning()
    keys = ("segs_per_wave", "waves_per_block", "small_list_bytes")
    assert {k: t[k] for k in keys} == {k: best[k] for k in keys}
    out, st = vbyte.decode_batch(bd, bo, oo, delta=True)
    torch.cuda.synchronize()
    sto, yo, _ = oracle.decode_batch(b, byte_off, out_off, None, True)
    assert (st.cpu().numpy() == vbyte.OK).all() and np.array_equal(u32(out), yo)


def test_autotune_refuses_bad_stream_and_restores():
    before = vbyte.get_tuning()
    bad = np.array([0x80] * 6 + [0x01] * 100, np.uint8)   # a 7-byte code
    bd = torch.from_numpy(bad).cuda()
    with pytest.raises(vbyte.VByteError) as ei:
        vbyte.autotune_decode(bd, 101, reps=1)
    assert ei.value.status == vbyte.EMALFORMED
    assert vbyte.get_tuning() == before


def test_autotune_cache_roundtrip(tmp_path):
    rng = np.random.default_rng(15)
    g = rng.geometric(1 / 8.0, 400_000).astype(np.uint32)
    bd = torch.from_numpy(oracle.encode(g)).cuda()
    path = str(tmp_path / "tune.json")
    e1, pts = autotune.tune_stream(bd, g.size, delta=True, path=path, reps=1)
    assert pts is not None and len(pts) == 24
    vbyte.set_tuning(1, 2, 4096, tiles_per_chunk=0)
    e2, pts2 = autotune.tune_stream(bd, g.size, delta=True, path=path)
    assert pts2 is None and e2 == e1
    t = vbyte.get_tuning()
    keys = ("segs_per_wave", "waves_per_block", "tiles_per_chunk")
    assert {k: t[k] for k in keys} == {k: e1[k] for k in keys}
