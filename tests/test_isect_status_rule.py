"""CPU check of the rule by which the fused intersection (k_isect_status)
gives the status of decoding a list in pieces of k integers (reading R15)
without decoding piece by piece.

The rule, from the stream's totals: C terminators; q0, the first byte of the
first run of five continuation bytes, if any; the last byte; P = ceil(na / k)
pieces.  A piece starts at the end of code p k and looks at the next 5k bytes,
so with a run the first piece whose window holds it is p = T / k + 1 for T the
terminators before byte q0 + 4 - 5k (p = 0 when that byte precedes the
stream): malformed if p < P, else the pieces stop short of the run (count).
Without a run: truncated when the last byte continues and the piece holding
the last code (C / k) is among the P; else the pieces decode min(P k, C)
codes, too few for na (truncated) or leaving codes or bytes behind (count).

This file restates that rule in Python and compares it with the oracle's
piece-by-piece intersection status (oracle.intersect_pieces, which calls
the oracle's resumable decode per piece) on random short lists with runs,
cut tails, trailing continuation bytes and counts off by a few, at piece
sizes 1 .. 64.  It shares nothing with the HIP source."""
import numpy as np

import oracle


def rule_status(a, na, k):
    a = np.asarray(a, np.uint8)
    cont = a >= 0x80
    C = int((~cont).sum())
    P = (na + k - 1) // k
    q0 = None
    for p in range(a.size - 4):
        if cont[p:p + 5].all():
            q0 = p
            break
    if q0 is not None:
        X = q0 + 5 - 5 * k
        pm = 0 if X <= 0 else int((~cont[:X - 1]).sum()) // k + 1
        return oracle.EMALFORMED if pm < P else oracle.ECOUNT
    if a.size and cont[-1]:
        return oracle.ETRUNC if C // k < P else oracle.ECOUNT
    done = min(P * k, C)
    if done < na:
        return oracle.ETRUNC
    if done < C or done > na:
        return oracle.ECOUNT
    return oracle.OK


def random_case(rng):
    n = int(rng.integers(0, 40))
    L = rng.integers(1, 6, size=n)
    vals = np.array([int(rng.integers(1 << (7 * (l - 1)) if l > 1 else 0, min(1 << (7 * l), 1 << 32)))
                     for l in L], dtype=np.uint64).astype(np.uint32)
    b = oracle.encode(vals).copy()
    r = rng.random()
    if r < 0.3 and b.size:
        q, ln = int(rng.integers(0, b.size)), int(rng.integers(1, 8))
        b[q:q + ln] = 0x80 | rng.integers(0, 128, size=min(ln, b.size - q)).astype(np.uint8)
    elif r < 0.45 and b.size:
        b = b[:int(rng.integers(0, b.size))]
    elif r < 0.55:
        b = np.concatenate([b, (0x80 | rng.integers(0, 128, size=int(rng.integers(1, 7))))
                            .astype(np.uint8)])
    na = max(0, n + int(rng.integers(-3, 4)))
    return b, na


def test_rule_matches_piecewise_status():
    rng = np.random.default_rng(1503)
    seen = {}
    for _ in range(4000):
        b, na = random_case(rng)
        k = int(rng.choice([1, 2, 3, 4, 5, 7, 16, 64]))
        st, _ = oracle.intersect_pieces(b, na, np.zeros(0, np.uint32), k)
        assert rule_status(b, na, k) == st, (list(b), na, k, st)
        seen[st] = seen.get(st, 0) + 1
    assert set(seen) == {oracle.OK, oracle.ECOUNT, oracle.ETRUNC, oracle.EMALFORMED}


def test_rule_edge_cases():
    """Exact counts, one code too many or too few, empty lists and a stream
    of continuation bytes only: the rule, the oracle and the expected code."""
    ok = oracle.encode(np.arange(1, 30, dtype=np.uint32))
    cases = []
    for k in (1, 4, 29, 100):
        cases += [(ok, 29, k, oracle.OK), (ok, 28, k, oracle.ECOUNT), (ok, 30, k, oracle.ETRUNC)]
    cases += [(np.zeros(0, np.uint8), 0, 8, oracle.OK), (np.zeros(0, np.uint8), 3, 8, oracle.ETRUNC),
              (np.full(3, 0x80, np.uint8), 0, 8, oracle.ECOUNT)]
    for b, na, k, want in cases:
        st, _ = oracle.intersect_pieces(b, na, np.zeros(0, np.uint32), k)
        assert st == want and rule_status(b, na, k) == want, (na, k, st)
