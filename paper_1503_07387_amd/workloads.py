"""Seeded synthetic workloads for VByte decoding of uint32.

This module draws the integers that get VByte-coded: plain values, gaps of
sorted document identifiers, posting-list lengths and query streams.  It holds
none of the coding arithmetic (no encoding, no decoding, no prefix sums); the
encoders live in the GPU library and, separately, in the CPU oracle used by
the tests.  Everything is drawn from numpy's PCG64 with fixed seeds.

The shapes follow the paper's workload (section 5): posting lists of
URL-sorted document identifiers from ClueWeb09, coded as gaps, lists grouped
by length, 8 to 16 bits per integer, shorter lists less compressible.  The
dataset is not available, so these synthetic streams stand in for it:

* ``uniform_lengths``  n values, code length L uniform in {1..5}, value uniform
  in [2^(7(L-1)), min(2^(7L), 2^32)).  For L = 1 the range is [1, 128).
* ``geometric_gaps``   gaps of a sorted stream, Geometric(p = 1/mean) on
  {1, 2, ...}.  Mean 8 gives almost only 1-byte codes, mean 300 a 35/65 mix of
  1- and 2-byte codes; the identifiers they encode wrap mod 2^32 for mean 300.
* ``zipf_lists``       100,000 posting lists with rank-Zipf(1.2) lengths,
  clipped to [1, 4Mi], scaled so that the lengths add up to about 2^28; the
  list order is shuffled; gaps per list are Geometric(p = len / 2^25), i.e. a
  universe of 2^25 documents.
* ``query_stream``     queries of 2..8 distinct terms drawn Zipf(1.0) over the
  list ranks (rank r = the r-th longest list), with Poisson arrival times.
* ``worst_case_mix``   values: 5 % uniform in [2^28, 2^32) (5-byte codes),
  else 50/50 uniform in [1,128) or [128, 2^14).  Drawn in fixed-size chunks,
  each from its own child seed, so a 2^30-value stream is reproducible chunk
  by chunk without holding every intermediate array.
"""
import numpy as np

SEED_UNIFORM = 1501
SEED_GAPS_MEAN8 = 1502
SEED_GAPS_MEAN300 = 15022
SEED_LISTS = 1503
SEED_QUERIES = 1504
SEED_MIX = 1505

MIX_CHUNK = 1 << 24


def _rng(seed):
    return np.random.default_rng(seed)


def uniform_lengths(n=1 << 20, seed=SEED_UNIFORM):
    """Values whose code length is uniform in {1..5}; returns (values, lengths)."""
    rng = _rng(seed)
    L = rng.integers(1, 6, size=n, dtype=np.int64)
    lo = np.where(L == 1, 1, np.left_shift(1, 7 * (L - 1)))
    hi = np.minimum(np.left_shift(1, 7 * L), 1 << 32)
    vals = lo + np.floor(rng.random(n) * (hi - lo)).astype(np.int64)
    vals = np.minimum(vals, hi - 1)
    return vals.astype(np.uint32), L.astype(np.uint8)


def geometric_gaps(n=1 << 26, mean=8, seed=None):
    """Gaps on {1, 2, ...} with the given mean (p = 1/mean)."""
    if seed is None:
        seed = SEED_GAPS_MEAN8 if mean == 8 else SEED_GAPS_MEAN300
    rng = _rng(seed)
    g = rng.geometric(1.0 / mean, size=n)
    return g.astype(np.uint32)


def zipf_list_lengths(nlists=100_000, total=1 << 28, s=1.2, max_len=1 << 22):
    """Rank-Zipf lengths clip(round(C r^-s), 1, max_len) with C chosen by
    bisection so the lengths add up to ``total`` as closely as rounding allows.
    Returned longest first (rank order)."""
    r = np.arange(1, nlists + 1, dtype=np.float64)
    w = r ** (-s)

    def lengths(C):
        return np.clip(np.rint(C * w), 1, max_len).astype(np.int64)

    lo, hi = 1.0, float(total) * 10
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if lengths(mid).sum() < total:
            lo = mid
        else:
            hi = mid
    a, b = lengths(lo), lengths(hi)
    return a if abs(int(a.sum()) - total) <= abs(int(b.sum()) - total) else b


def zipf_lists(nlists=100_000, total=1 << 28, universe=1 << 25, seed=SEED_LISTS):
    """Posting lists as gaps.

    Returns dict with ``lengths`` (int64, in storage order), ``rank_of``
    (int64: storage position -> length rank, 0 = longest), ``gaps`` (uint32,
    all lists concatenated in storage order) and ``out_off`` (int64 CSR output
    offsets).
    """
    rng = _rng(seed)
    by_rank = zipf_list_lengths(nlists, total)
    order = rng.permutation(nlists)          # storage position -> rank
    lengths = by_rank[order]
    out_off = np.zeros(nlists + 1, dtype=np.int64)
    np.cumsum(lengths, out=out_off[1:])
    gaps = np.empty(int(out_off[-1]), dtype=np.uint32)
    p = lengths.astype(np.float64) / float(universe)
    for i in range(nlists):
        a, b = int(out_off[i]), int(out_off[i + 1])
        gaps[a:b] = rng.geometric(p[i], size=b - a)
    return {"lengths": lengths, "rank_of": order.astype(np.int64),
            "gaps": gaps, "out_off": out_off}


def query_stream(nqueries, qps, nlists=100_000, seed=SEED_QUERIES, kmin=2, kmax=8):
    """Open-loop query stream.

    Returns (arrival_s float64[nq], terms list of int64 arrays of length ranks,
    0 = longest list).  Arrivals are a Poisson process of rate ``qps``; each
    query has k ~ U{kmin..kmax} distinct ranks drawn with P(r) proportional to
    1/r."""
    rng = _rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / qps, size=nqueries))
    cdf = np.cumsum(1.0 / np.arange(1, nlists + 1, dtype=np.float64))
    cdf /= cdf[-1]
    terms = []
    for _ in range(nqueries):
        k = int(rng.integers(kmin, kmax + 1))
        chosen = []
        while len(chosen) < k:
            r = int(np.searchsorted(cdf, rng.random(), side="right"))
            r = min(r, nlists - 1)
            if r not in chosen:
                chosen.append(r)
        terms.append(np.array(chosen, dtype=np.int64))
    return arrivals, terms


def worst_case_mix_chunk(chunk_index, chunk=MIX_CHUNK, seed=SEED_MIX):
    """One chunk of the 1/2/5-byte mix (values uint32)."""
    ss = np.random.SeedSequence([seed, chunk_index])
    rng = np.random.default_rng(ss)
    u = rng.random(chunk)
    v = rng.random(chunk)
    five = u < 0.05
    one = (~five) & (v < 0.5)
    vals = np.empty(chunk, dtype=np.uint32)
    nf = int(five.sum())
    no = int(one.sum())
    nt = chunk - nf - no
    vals[five] = rng.integers(1 << 28, 1 << 32, size=nf, dtype=np.uint64).astype(np.uint32)
    vals[one] = rng.integers(1, 128, size=no, dtype=np.uint32)
    vals[~five & ~one] = rng.integers(128, 1 << 14, size=nt, dtype=np.uint32)
    return vals


def worst_case_mix(n=1 << 30, seed=SEED_MIX, workers=8):
    """The full mix as one uint32 array (chunked draws, see module doc).
    Chunks are drawn by `workers` threads (numpy releases the GIL while it
    draws); the result does not depend on their number."""
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty(n, dtype=np.uint32)
    nchunks = (n + MIX_CHUNK - 1) // MIX_CHUNK

    def fill(c):
        a = c * MIX_CHUNK
        b = min(n, a + MIX_CHUNK)
        out[a:b] = worst_case_mix_chunk(c, seed=seed)[: b - a]

    with ThreadPoolExecutor(max(1, int(workers))) as ex:
        list(ex.map(fill, range(nchunks)))
    return out
