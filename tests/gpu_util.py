"""Helpers of the GPU parity tests: run the HIP path through the C ABI with
guard bytes around every buffer, and compare it with the CPU oracle."""
import numpy as np
import torch

import oracle
from paper_1503_07387_amd import vbyte

SENTINEL = 0x5A5A5A5A


def dev():
    return torch.device("cuda:0")


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def place_bytes(b, boff=0, pre=0x80, post=0x00):
    """Upload b so that it starts `boff` bytes past a 256-byte boundary, with
    `pre` bytes before it and `post` bytes after it.  A decoder that used any
    byte outside the stream would see continuation bytes before it and extra
    terminators after it.  Returns (device buffer, stream view)."""
    b = np.asarray(b, dtype=np.uint8)
    host = np.empty(boff + b.size + 48, dtype=np.uint8)
    host[:boff] = pre
    host[boff:boff + b.size] = b
    host[boff + b.size:] = post
    d = torch.from_numpy(host).to(dev())
    return d, d[boff:boff + b.size]


def gpu_decode(b, n, delta=False, prev=0, boff=0, ooff=0, pre=0x80, post=0x00):
    """Decode through vbyte_decode(_delta)_async; check the guard words
    around out[0..n) and return (status, uint32 result)."""
    _, data = place_bytes(b, boff, pre, post)
    full = torch.full((ooff + n + 16,), SENTINEL, dtype=torch.int32, device=dev())
    out = full[ooff:ooff + n]
    status = torch.full((1,), -1, dtype=torch.int32, device=dev())
    vbyte.decode(data, n, delta=delta, prev=prev, out=out, status=status, check=False)
    torch.cuda.synchronize()
    h = u32(full)
    assert (h[:ooff] == SENTINEL).all(), "write before out[0]"
    assert (h[ooff + n:] == SENTINEL).all(), "write past out[n-1]"
    return int(status.item()), h[ooff:ooff + n]


def check_against_oracle(b, n, delta=False, prev=0, boff=0, ooff=0):
    st, y = gpu_decode(b, n, delta, prev, boff, ooff)
    if delta:
        sto, yo = oracle.decode_delta(b, n, prev)
    else:
        sto, yo = oracle.decode(b, n)
    assert st == sto, f"status gpu={st} oracle={sto} (n={n}, nbytes={len(b)}, boff={boff})"
    if sto == oracle.OK:
        if not np.array_equal(y, yo):
            bad = np.nonzero(y != yo)[0]
            raise AssertionError(f"{bad.size} mismatches, first at {bad[0]}: gpu={y[bad[0]]} "
                                 f"oracle={yo[bad[0]]} (n={n}, boff={boff}, delta={delta})")
    return st, y


def mixed_values(rng, n, lengths=(1, 2, 3, 4, 5)):
    """Values whose code lengths are drawn from `lengths`."""
    L = rng.choice(np.array(lengths), size=n)
    lo = np.where(L == 1, 0, np.left_shift(1, 7 * (L - 1)))
    hi = np.minimum(np.left_shift(1, 7 * L), 1 << 32)
    v = lo + np.floor(rng.random(n) * (hi - lo)).astype(np.int64)
    return np.minimum(v, hi - 1).astype(np.uint32)
