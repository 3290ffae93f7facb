"""GPU tests of the serving loop: every served result equals the oracle's
decode of the request's lists, a request's result is byte-identical alone and
in a mix at high load, admission respects the output pool, and the per-list
baseline mode gives the same results."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import u32
from paper_1503_07387_amd import serve, vbyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def index():
    rng = np.random.default_rng(41)
    nl = 3000
    lens = np.minimum(np.maximum((4e5 / np.arange(1, nl + 1) ** 1.1).astype(np.int64), 1), 200_000)
    rng.shuffle(lens)
    out_off = np.zeros(nl + 1, np.int64)
    np.cumsum(lens, out=out_off[1:])
    gaps = np.empty(int(out_off[-1]), np.uint32)
    for i in range(nl):
        gaps[out_off[i]:out_off[i + 1]] = rng.geometric(min(1.0, lens[i] / 2 ** 25), int(lens[i]))
    b = oracle.encode(gaps)
    byte_off = np.zeros(nl + 1, np.int64)
    for i in range(nl):
        byte_off[i + 1] = byte_off[i] + oracle.encoded_size(gaps[out_off[i]:out_off[i + 1]])
    return {"bytes": b, "byte_off": byte_off, "counts": lens, "dev": torch.from_numpy(b).cuda()}


def expected(index, terms, delta=True):
    parts = []
    for t in terms:
        bb = index["bytes"][index["byte_off"][t]:index["byte_off"][t + 1]]
        n = int(index["counts"][t])
        st, y = oracle.decode_delta(bb, n, 0) if delta else oracle.decode(bb, n)
        assert st == oracle.OK
        parts.append(y)
    return np.concatenate(parts) if parts else np.zeros(0, np.uint32)


def queries(nq, qps, nl, seed):
    arr, ranks = workloads.query_stream(nq, qps, nlists=nl, seed=seed)
    return arr, ranks   # ranks used directly as list indices here


@pytest.mark.parametrize("batching", [True, False])
def test_served_results_match_oracle(index, batching):
    arr, terms = queries(300, 200_000.0, index["counts"].size, 7)
    srv = serve.Server(index["dev"], index["byte_off"], index["counts"], pool_bytes=64 << 20,
                       nstreams=4, batching=batching)
    lat, stats, (res, off) = srv.run(arr, terms, capture=True)
    srv.close()
    assert stats["worst_status"] == vbyte.OK and stats["rejected"] == 0
    assert (lat > 0).all()
    h = u32(res)
    for r in range(len(terms)):
        assert np.array_equal(h[off[r]:off[r + 1]], expected(index, terms[r])), r
    if batching:
        assert stats["mean_batch_requests"] > 1.0      # requests were batched together


def test_alone_equals_in_mix(index):
    arr, terms = queries(400, 500_000.0, index["counts"].size, 8)
    srv = serve.Server(index["dev"], index["byte_off"], index["counts"], pool_bytes=48 << 20,
                       nstreams=4)
    _, _, (mix, moff) = srv.run(arr, terms, capture=True)
    hm = u32(mix)
    for r in (0, 1, 57, 199, 399):
        _, _, (alone, aoff) = srv.run(np.zeros(1), [terms[r]], capture=True)
        ha = u32(alone)
        assert np.array_equal(ha[:aoff[1]], hm[moff[r]:moff[r + 1]]), r
    srv.close()


def test_admission_waits_for_pool_memory(index):
    arr, terms = queries(150, 1e7, index["counts"].size, 9)
    need = np.array([int(index["counts"][t].sum()) for t in terms])
    pool = int(need.max()) * 4 + 4096          # room for about one large request
    srv = serve.Server(index["dev"], index["byte_off"], index["counts"], pool_bytes=pool,
                       nstreams=3, delta=False)
    lat, stats, (res, off) = srv.run(arr, terms, capture=True)
    assert stats["rejected"] == 0 and stats["worst_status"] == vbyte.OK
    h = u32(res)
    for r in range(0, len(terms), 7):
        assert np.array_equal(h[off[r]:off[r + 1]], expected(index, terms[r], delta=False))
    # a request larger than the whole pool is rejected, the rest still served
    big = [np.argsort(index["counts"])[::-1][:60].astype(np.int64)]
    assert int(index["counts"][big[0]].sum()) * 4 > pool
    lat2, stats2, _ = srv.run(np.zeros(2), big + [terms[0]], capture=False)
    srv.close()
    assert stats2["rejected"] == 1 and lat2[0] == -1.0 and lat2[1] > 0


@pytest.fixture(scope="module")
def config3():
    """The batched workload's index: 100,000 Zipf-length lists (2^28
    integers, the longest 4Mi), coded by the oracle."""
    d = workloads.zipf_lists()
    gaps, out_off = d["gaps"], d["out_off"]
    b = oracle.encode(gaps)
    nl = d["lengths"].size
    byte_off = np.zeros(nl + 1, np.int64)
    for i in range(nl):
        byte_off[i + 1] = byte_off[i] + oracle.encoded_size(gaps[out_off[i]:out_off[i + 1]])
    assert byte_off[-1] == b.size
    return {"bytes": b, "byte_off": byte_off, "counts": d["lengths"].astype(np.int64),
            "rank_of": d["rank_of"], "dev": torch.from_numpy(b).cuda()}


def test_config3_alone_equals_in_mix(config3):
    """Queries of 2-8 Zipf(1.0) terms over the config-3 index, rank r the
    r-th longest list (so a quarter of the terms hit the 4Mi lists), served
    at a rate above saturation: a request's result is the same alone and in
    the mix, and equals the oracle's decode of its lists."""
    nl = config3["counts"].size
    pos_of_rank = np.argsort(config3["rank_of"])
    arr, ranks = workloads.query_stream(240, 1e6, nlists=nl, seed=12)
    terms = [pos_of_rank[r] for r in ranks]
    assert sum(int((config3["counts"][t] == 1 << 22).any()) for t in terms) > 20
    srv = serve.Server(config3["dev"], config3["byte_off"], config3["counts"], pool_bytes=3 << 30,
                       nstreams=4, max_batch_requests=64)
    _, stats, (mix, moff) = srv.run(arr, terms, capture=True)
    assert stats["worst_status"] == vbyte.OK and stats["rejected"] == 0
    assert stats["mean_batch_requests"] > 1.0
    hm = u32(mix)
    for r in (0, 3, 50, 121, 239):
        _, _, (alone, aoff) = srv.run(np.zeros(1), [terms[r]], capture=True)
        assert np.array_equal(u32(alone)[:aoff[1]], hm[moff[r]:moff[r + 1]]), r
        assert np.array_equal(hm[moff[r]:moff[r + 1]], expected(config3, terms[r])), r
    srv.close()


def test_small_request_does_not_wait_for_the_largest_in_its_batch():
    """Two requests admitted together into one batch: one asks for four
    32Mi-integer lists, the other for two 100-integer lists.  The small
    request completes when its own lists are decoded (the batch's requests
    are decoded in groups, smallest first, each followed by an event), well
    before the batch ends; both results equal the oracle's."""
    rng = np.random.default_rng(77)
    lens = np.array([1 << 25, 1 << 25, 1 << 25, 1 << 25, 100, 100, 5], np.int64)
    gaps = [rng.geometric(1 / 50, int(n)).astype(np.uint32) for n in lens]
    enc = [oracle.encode(g) for g in gaps]
    byte_off = np.concatenate([[0], np.cumsum([e.size for e in enc])]).astype(np.int64)
    b = np.concatenate(enc)
    idx = {"bytes": b, "byte_off": byte_off, "counts": lens, "dev": torch.from_numpy(b).cuda()}
    terms = [np.array([0, 1, 2, 3], np.int64), np.array([4, 5], np.int64)]
    srv = serve.Server(idx["dev"], byte_off, lens, pool_bytes=1 << 30, nstreams=1,
                       max_batch_requests=8)
    want = [expected(idx, terms[r]) for r in range(2)]
    worst_ratio = 0.0
    for rep in range(4):
        lat, stats, (res, off) = srv.run(np.zeros(2), terms, capture=True)
        assert stats["batches"] == 1 and stats["worst_status"] == vbyte.OK
        assert (stats["status"] == vbyte.OK).all()
        h = u32(res)
        for r in range(2):
            assert np.array_equal(h[off[r]:off[r + 1]], want[r]), r
        if rep:
            worst_ratio = max(worst_ratio, lat[1] / lat[0])
    srv.close()
    assert worst_ratio < 0.5, f"the small request took {worst_ratio:.2f} of the large one's latency"


def test_request_status_reports_a_bad_list():
    rng = np.random.default_rng(78)
    lens = np.array([1000, 2000, 3000], np.int64)
    gaps = [rng.geometric(1 / 50, int(n)).astype(np.uint32) for n in lens]
    enc = [oracle.encode(g) for g in gaps]
    enc[1][100:106] = 0x80          # list 1 malformed
    byte_off = np.concatenate([[0], np.cumsum([e.size for e in enc])]).astype(np.int64)
    b = np.concatenate(enc)
    srv = serve.Server(torch.from_numpy(b).cuda(), byte_off, lens, pool_bytes=1 << 24, nstreams=2)
    terms = [np.array([0], np.int64), np.array([0, 1], np.int64), np.array([2], np.int64)]
    lat, stats, _ = srv.run(np.zeros(3), terms)
    srv.close()
    assert stats["status"].tolist() == [vbyte.OK, vbyte.EMALFORMED, vbyte.OK]
    assert stats["worst_status"] == vbyte.EMALFORMED and (lat > 0).all()
