"""GPU parity of the single-workgroup scans over many rounds.

The scans of the two-pass decodes (tiles of the 32-bit decode, units of the
64-bit decode, workgroups of the blocks-of-four decode) take up to 1024 x 8
slots per round.  The benchmark streams at the default tiling fit one
round, so these cases pick 1 KiB segments and small workgroups to reach
several rounds with a partial last one, and compare every output with the
oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import mixed_values, place_bytes, u32
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu

ROUND = 1024 * 8   # slots per full round of a scan


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def decode32(b, n, delta, prev, boff):
    _, data = place_bytes(b, boff)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    y = vbyte.decode(data, n, delta=delta, prev=prev, status=st, check=False)
    torch.cuda.synchronize()
    return int(st.item()), u32(y)


@pytest.mark.parametrize("delta", [False, True])
def test_tile_scan_three_rounds(delta):
    # 1 KiB tiles (one segment, one wavefront): about 2.3 rounds of tiles
    vbyte.set_tuning(1, 1, 0, tiles_per_chunk=-1)
    rng = np.random.default_rng(31 + delta)
    x = mixed_values(rng, 9_000_000, (1, 2, 3))
    b = oracle.encode(x)
    ntiles = (b.size + 5 + 1023) // 1024
    assert 2 * ROUND < ntiles < 3 * ROUND
    st, y = decode32(b, x.size, delta, 11, boff=5)
    sto, yo = oracle.decode_delta(b, x.size, 11) if delta else oracle.decode(b, x.size)
    assert st == sto == vbyte.OK
    assert np.array_equal(y, yo)
    # a malformed run in the last round and a count mismatch still classify
    bad = b.copy()
    bad[b.size - 4000:b.size - 3995] = 0x80
    assert decode32(bad, x.size, delta, 0, 0)[0] == vbyte.EMALFORMED
    assert decode32(b, x.size + 1, delta, 0, 0)[0] == vbyte.ETRUNC


def test_unit_scan_two_rounds_64():
    # 8 KiB units (8 groups of one segment): the 111 MB stream has ~13.5K
    vbyte.set_tuning(1, 2, 0)
    g = workloads.geometric_gaps(mean=300)
    b = oracle.encode(g)
    assert ROUND < (b.size + 8191) // 8192 < 2 * ROUND
    n = g.size
    _, data = place_bytes(b, 0)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    out = vbyte.decode64(data, n, delta=True, prev=1 << 40, status=st, check=False)
    torch.cuda.synchronize()
    sto, yo = oracle.decode64_delta(b, n, 1 << 40)
    assert int(st.item()) == sto == vbyte.OK
    assert np.array_equal(out.cpu().numpy().view(np.uint64), yo)


def test_block_scan_two_rounds_delta4():
    # one-wavefront workgroups of 8 KiB units: ~13.5K blocks of the 111 MB stream
    vbyte.set_tuning(1, 1, 0)
    g = workloads.geometric_gaps(mean=300)
    b = oracle.encode(g)
    assert ROUND < (b.size + 8191) // 8192 < 2 * ROUND
    n = g.size
    _, data = place_bytes(b, 3)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    prev4 = [5, 0xFFFFFFFF, 1 << 31, 7]
    out = vbyte.decode_delta4(data, n, prev4=prev4, status=st, check=False)
    torch.cuda.synchronize()
    sto, yo = oracle.decode_delta4(b, n, prev4)
    assert int(st.item()) == sto == vbyte.OK
    assert np.array_equal(u32(out), yo)
