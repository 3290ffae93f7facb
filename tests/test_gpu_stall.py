"""The bounded look-back wait: with a spin limit of one round trip, tiles
whose predecessors have not published yet give up instead of waiting; every
launch still ends normally, and the call reports VBYTE_ESTALLED (or VBYTE_OK
when no tile had to wait; a count of 2^64 - 1 for vbyte_count).  Only that
bound is forced; afterwards, with the default limit, the same workspaces
decode correctly.  No kernel faults or hangs: a tile that gives up keeps
every store inside its output."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import u32
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore():
    t = vbyte.get_tuning()
    yield
    vbyte.set_spin_limit(0)
    vbyte.set_tuning(**t)


def test_lookback_gives_up_and_recovers():
    g = workloads.geometric_gaps(n=1 << 24, mean=300)
    b = oracle.encode(g)
    d = torch.from_numpy(b).cuda()
    out = torch.empty(g.size, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    _, ref = oracle.decode_delta(b, g.size, 0)
    seen = set()
    for chunk, (sg, wv) in ((0, (1, 1)), (0, (1, 2)), (2, (1, 1))):
        vbyte.set_tuning(sg, wv, 0, tiles_per_chunk=chunk)
        vbyte.set_spin_limit(1)
        for _ in range(4):
            vbyte.decode(d, g.size, delta=True, out=out, status=st, check=False)
            torch.cuda.synchronize()
            s = int(st.item())
            assert s in (vbyte.OK, vbyte.ESTALLED), s
            seen.add(s)
        c = vbyte.count(d)
        assert c in (g.size, -1)   # 2^64 - 1 read back as int64
        vbyte.set_spin_limit(0)
        vbyte.decode(d, g.size, delta=True, out=out, status=st, check=False)
        torch.cuda.synchronize()
        assert int(st.item()) == vbyte.OK and np.array_equal(u32(out), ref)
        assert vbyte.count(d) == g.size
    assert vbyte.ESTALLED in seen, "no tile ever gave up with a limit of one round trip"


def test_batched_lists_give_up_and_recover():
    rng = np.random.default_rng(5)
    lens = rng.integers(1, 300_000, 64)
    gaps = [workloads.geometric_gaps(n=int(n), mean=100, seed=int(i)) for i, n in enumerate(lens)]
    enc = [oracle.encode(x) for x in gaps]
    byte_off = np.concatenate([[0], np.cumsum([e.size for e in enc])]).astype(np.int64)
    out_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    b = np.concatenate(enc)
    d = torch.from_numpy(b).cuda()
    bo, oo = torch.from_numpy(byte_off).cuda(), torch.from_numpy(out_off).cuda()
    vbyte.set_tuning(1, 1, 1024, tiles_per_chunk=0)
    vbyte.set_spin_limit(1)
    for _ in range(3):
        out, ls = vbyte.decode_batch(d, bo, oo, delta=True)
        torch.cuda.synchronize()
        assert set(ls.cpu().numpy().tolist()) <= {vbyte.OK, vbyte.ESTALLED}
    vbyte.set_spin_limit(0)
    out, ls = vbyte.decode_batch(d, bo, oo, delta=True)
    torch.cuda.synchronize()
    assert (ls.cpu().numpy() == vbyte.OK).all()
    sto, yo, _ = oracle.decode_batch(b, byte_off, out_off, None, True)
    assert sto == oracle.OK and np.array_equal(u32(out), yo)
