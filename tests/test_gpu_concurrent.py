"""Decodes on two HIP streams at once: every single-stream kernel (look-back
per tile, chunks, two passes), the batched decode and the encoder, each run
concurrently with a second call of its kind, must give the oracle's
results.  Tiles of look-back launches are numbered by ticket, so a tile
never waits for one whose workgroup has not started, whatever else the
device runs."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import u32
from paper_1503_07387_amd import vbyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_tuning():
    t = vbyte.get_tuning()
    yield
    vbyte.set_tuning(**t)


def two_streams(calls, reps=4):
    """Run calls[0] and calls[1] on two streams, started together, reps times."""
    main = torch.cuda.current_stream()
    side = [torch.cuda.Stream(), torch.cuda.Stream()]
    for _ in range(reps):
        ev = torch.cuda.Event()
        ev.record(main)
        ends = []
        for i in range(2):
            side[i].wait_event(ev)
            with torch.cuda.stream(side[i]):
                calls[i]()
            en = torch.cuda.Event()
            en.record(side[i])
            ends.append(en)
        for en in ends:
            main.wait_event(en)
    torch.cuda.synchronize()


@pytest.mark.parametrize("tiling", [(4, 8, 0), (1, 2, 0), (4, 8, 4), (2, 8, -1), (2, 8, -2), (1, 2, -2)])
def test_two_single_stream_decodes(tiling):
    vbyte.set_tuning(tiling[0], tiling[1], 0, tiles_per_chunk=tiling[2])
    ins = []
    for mean in (8, 300):
        g = workloads.geometric_gaps(n=1 << 24, mean=mean)
        b = oracle.encode(g)
        ins.append((g, torch.from_numpy(b).cuda(), torch.empty(g.size, dtype=torch.int32, device="cuda"),
                    torch.empty(1, dtype=torch.int32, device="cuda")))

    def call(i):
        g, d, out, st = ins[i]
        return lambda: vbyte.decode(d, g.size, delta=True, out=out, status=st, check=False)

    two_streams([call(0), call(1)])
    for g, d, out, st in ins:
        sto, yo = oracle.decode_delta(d.cpu().numpy(), g.size, 0)
        assert int(st.item()) == sto == vbyte.OK
        assert np.array_equal(u32(out), yo)


def test_two_batched_decodes():
    vbyte.set_tuning(4, 8, 4096)
    sets = []
    for seed in (1, 2):
        rng = np.random.default_rng(seed)
        lens = np.concatenate([rng.integers(0, 500, 3000), [300_000, 1_000_000]])
        out_off = np.zeros(lens.size + 1, np.int64)
        np.cumsum(lens, out=out_off[1:])
        gaps = rng.geometric(1 / 40.0, int(out_off[-1])).astype(np.uint32)
        b = oracle.encode(gaps)
        byte_off = np.zeros(lens.size + 1, np.int64)
        for i in range(lens.size):
            byte_off[i + 1] = byte_off[i] + oracle.encoded_size(gaps[out_off[i]:out_off[i + 1]])
        t = [torch.from_numpy(x).cuda() for x in (b, byte_off, out_off)]
        out = torch.empty(int(out_off[-1]), dtype=torch.int32, device="cuda")
        st = torch.empty(lens.size, dtype=torch.int32, device="cuda")
        sets.append((b, byte_off, out_off, t, out, st))

    def call(i):
        b, bo, oo, t, out, st = sets[i]
        return lambda: vbyte.decode_batch(t[0], t[1], t[2], delta=True, out=out, list_status=st)

    two_streams([call(0), call(1)])
    for b, bo, oo, t, out, st in sets:
        sto, yo, _ = oracle.decode_batch(b, bo, oo, None, True)
        assert sto == oracle.OK and (st.cpu().numpy() == vbyte.OK).all()
        assert np.array_equal(u32(out), yo)


def test_two_encodes():
    rng = np.random.default_rng(3)
    xs = [rng.integers(0, 1 << 32, 5_000_000, dtype=np.uint64).astype(np.uint32) for _ in range(2)]
    ds = [torch.from_numpy(x.view(np.int32)).cuda() for x in xs]
    outs = [torch.empty(5 * x.size, dtype=torch.uint8, device="cuda") for x in xs]
    nbs = [torch.empty(1, dtype=torch.int64, device="cuda") for _ in xs]
    L = vbyte._lib()

    def call(i):
        def f():
            s = torch.cuda.current_stream().cuda_stream
            assert L.vbyte_encode_async(ds[i].data_ptr(), xs[i].size, outs[i].data_ptr(),
                                        outs[i].numel(), nbs[i].data_ptr(), s) == vbyte.OK
        return f

    two_streams([call(0), call(1)], reps=2)
    for x, o, nb in zip(xs, outs, nbs):
        want = oracle.encode(x)
        assert int(nb.item()) == want.size
        assert np.array_equal(o[:want.size].cpu().numpy(), want)


@pytest.mark.parametrize("pair", [((4, 8, 0), (1, 2, -1)), ((2, 8, -1), (1, 4, 3)),
                                  ((2, 7, -2), (4, 4, 0))])
def test_per_call_tilings_on_two_streams(pair):
    """vbyte_decode_ex with a different tiling and schedule on each of two
    streams at once: each result bit-exact against the oracle, and the
    process-wide defaults untouched."""
    before = vbyte.get_tuning()
    ins = []
    for mean, (sg, wv, sch) in zip((8, 300), pair):
        g = workloads.geometric_gaps(n=1 << 23, mean=mean)
        b = oracle.encode(g)
        ins.append((g, torch.from_numpy(b).cuda(), torch.empty(g.size, dtype=torch.int32, device="cuda"),
                    torch.empty(1, dtype=torch.int32, device="cuda"), vbyte.make_tuning(sg, wv, sch)))

    def call(i):
        g, d, out, st, T = ins[i]
        return lambda: vbyte.decode(d, g.size, delta=True, prev=i, out=out, status=st, check=False,
                                    tuning=T)

    two_streams([call(0), call(1)])
    for i, (g, d, out, st, T) in enumerate(ins):
        sto, ref = oracle.decode_delta(d.cpu().numpy(), g.size, i)
        assert int(st.item()) == sto == oracle.OK
        assert np.array_equal(u32(out), ref)
    assert vbyte.get_tuning() == before


def test_host_threads_share_one_stream():
    """Four host threads decode on one stream at once, each with its own size
    (so the stream's workspace grows while others use it), checked decodes
    that read their status back, and asynchronous encodes in between."""
    from concurrent.futures import ThreadPoolExecutor
    st = torch.cuda.Stream()
    sizes = [(1 << 14) + 3, (1 << 18) + 77, (1 << 21) + 5, (1 << 22) + 1001]
    ins = []
    for k, n in enumerate(sizes):
        g = workloads.geometric_gaps(n=n, mean=8 if k % 2 else 300)
        ins.append((g, torch.from_numpy(oracle.encode(g)).cuda(),
                    torch.from_numpy(g.view(np.int32)).cuda()))
    torch.cuda.synchronize()

    def work(k):
        g, d, gv = ins[k]
        res = []
        for _ in range(6):
            y = vbyte.decode(d, g.size, delta=True, stream=st)
            b = vbyte.encode(gv, stream=st)
            res.append((u32(y), b.cpu().numpy()))
        return res

    with ThreadPoolExecutor(4) as ex:
        outs = list(ex.map(work, range(4)))
    torch.cuda.synchronize()
    for (g, d, gv), res in zip(ins, outs):
        want = np.cumsum(g, dtype=np.uint64).astype(np.uint32)
        want_b = oracle.encode(g)
        for y, b in res:
            assert np.array_equal(y, want)
            assert np.array_equal(b, want_b)
