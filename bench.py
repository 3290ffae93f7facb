"""Benchmark of the VByte decode hot path on one MI355X.

A step is one pass of the hot path over the headline workload: the plain
single-stream decode (VByte bytes -> uint32) of 2^30 values, 5 % 5-byte codes
and otherwise a 50/50 mix of 1- and 2-byte codes (1.80 GB in, 4 GiB out),
drawn with a fixed seed, VByte-encoded on the GPU and resident in HBM before
timing starts.  Beside it (side lines, each its own entry in the JSON): the
differential decode of the same bytes, the 2^20-value uniform-length stream
(the small case), the differential decode of two 64Mi-gap streams (gap means
8 and 300), the one-read schedule, 64-bit and blocks-of-four decodes, the
intersection consumer, the encoder, the batched decode of 100,000 lists and
the serving loop over them.

Printed: one JSON line with throughput (Gints/s), the HBM roofline of the
decode (algorithmic bytes in + 4n out per call over the call's HIP-event
time), and the scalar CPU oracle timed on the host, on one core and on all
cores, as a baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gints/s + HBM GB/s (% peak), batched vs plain per-list; p50/p99 query latency"
HBM_PEAK_GBPS = 8000.0
N_STREAM = 1 << 26
N_MIX = 1 << 30               # the headline stream: 2^30 values of the 1/2/5-byte mix
N_UNIFORM = 1 << 20           # the small case: uniform code lengths 1..5
COPY_ELEMS = 1 << 26          # calibration copy: 256 MiB read + 256 MiB written
FLUSH_BYTES = 1 << 30         # written before a "flushed" call: four times the 256 MB MALL
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "decode_plain_1Gi_mix_counters.json")
PROFILE_TRACE = os.path.join(ROOT, "profiles", "decode_plain_1Gi_mix_kernel_trace.md")
# the library's default single-stream schedule, named explicitly per call
HEADLINE_TUNING = {"segs_per_wave": 2, "waves_per_block": 8, "schedule": -1}
KERNEL_SRC = os.path.join(ROOT, "paper_1503_07387_amd", "csrc", "kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 prefix of the kernel source with comments and blank space
    removed, so that only changes to the code itself retire the counters."""
    import re
    with open(KERNEL_SRC) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def measured_traffic(bytes_per_launch_alg):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None
    when the kernel source changed since the counters were taken."""
    try:
        with open(PROFILE_COUNTERS) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return prof.get("hbm_bytes_per_launch")


def make_streams(torch, vbyte, workloads):
    """The two gap streams, encoded on the GPU.  Returns a list of dicts."""
    out = []
    for mean in (8, 300):
        t0 = time.time()
        g = workloads.geometric_gaps(n=N_STREAM, mean=mean)
        gd = torch.from_numpy(g.view("int32")).cuda()
        enc = vbyte.encode(gd)
        torch.cuda.synchronize()
        log(f"stream mean {mean}: {N_STREAM} gaps -> {enc.numel()} bytes "
            f"({enc.numel() / N_STREAM:.4f} B/int), prepared in {time.time() - t0:.1f}s")
        out.append({"mean": mean, "gaps": g, "gaps_dev": gd, "bytes": enc,
                    "out": torch.empty(N_STREAM, dtype=torch.int32, device="cuda"),
                    "status": torch.empty(1, dtype=torch.int32, device="cuda")})
    return out


def verify(torch, streams):
    for s in streams:
        if int(s["status"].item()) != 0:
            raise RuntimeError(f"decode status {int(s['status'].item())} on stream mean {s['mean']}")
        ref = torch.cumsum(s["gaps_dev"].to(torch.int64) & 0xFFFFFFFF, 0) & 0xFFFFFFFF
        got = s["out"].to(torch.int64) & 0xFFFFFFFF
        if not torch.equal(ref, got):
            raise RuntimeError(f"decoded identifiers differ from the gap prefix sum (mean {s['mean']})")


def shard_starts(b, parts):
    """Byte offsets that cut the VByte stream b into `parts` shards at code
    boundaries: each cut moves forward from i * len / parts to the byte after
    the next terminator (host logic of the multi-core baseline)."""
    import numpy as np
    cuts = [0]
    nb = b.size
    for i in range(1, parts):
        x = max(i * nb // parts, cuts[-1])
        while x < nb and b[x] >= 0x80:
            x += 1
        x = min(x + 1, nb)
        cuts.append(x)
    cuts.append(nb)
    return np.array(cuts, dtype=np.int64)


def cpu_baseline(b, x, reps=5):
    """The scalar oracle (plain C: validation then Algorithm 1) decoding the
    headline stream on the host: on one core, and on every core available
    to this process with the stream cut into one shard per core at code
    boundaries, a counting pass per shard (its integers, hence the shard's
    output offset) and then a decode pass per shard, both timed.  Median of
    `reps` runs each; the output is allocated and touched before timing."""
    import ctypes
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    lib = oracle.oracle.load()
    n = x.size
    y = np.empty(n, dtype=np.uint32)
    y.fill(0)
    bp = b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    yp = y.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    one = []
    for _ in range(reps):
        t0 = time.perf_counter()
        st = lib.orc_decode(bp, b.size, yp, n)
        one.append(time.perf_counter() - t0)
        if st != oracle.OK:
            raise RuntimeError("oracle failed on the benchmark stream")
    if not np.array_equal(y, x):
        raise RuntimeError("oracle output differs from the drawn values")
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cuts = shard_starts(b, cores)
    base = b.ctypes.data
    ybase = y.ctypes.data

    def count(k):
        p = ctypes.cast(base + int(cuts[k]), ctypes.POINTER(ctypes.c_uint8))
        return int(lib.orc_count(p, int(cuts[k + 1] - cuts[k])))

    def dec(args):
        k, off, m = args
        p = ctypes.cast(base + int(cuts[k]), ctypes.POINTER(ctypes.c_uint8))
        q = ctypes.cast(ybase + 4 * off, ctypes.POINTER(ctypes.c_uint32))
        return lib.orc_decode(p, int(cuts[k + 1] - cuts[k]), q, m)

    y.fill(0)
    allc = []
    with ThreadPoolExecutor(cores) as ex:
        for _ in range(reps):
            t0 = time.perf_counter()
            counts = list(ex.map(count, range(cores)))
            offs = np.concatenate([[0], np.cumsum(counts)])
            sts = list(ex.map(dec, [(k, int(offs[k]), counts[k]) for k in range(cores)]))
            allc.append(time.perf_counter() - t0)
            if any(st != oracle.OK for st in sts) or int(offs[-1]) != n:
                raise RuntimeError("sharded oracle decode failed")
    if not np.array_equal(y, x):
        raise RuntimeError("sharded oracle output differs from the drawn values")
    med1 = sorted(one)[reps // 2]
    medn = sorted(allc)[reps // 2]
    alg = b.size + 4 * n
    return {"value": round(n / medn / 1e9, 4), "unit": "Gints/s", "cores": cores, "kind": "oracle",
            "one_core_gints_per_s": round(n / med1 / 1e9, 4),
            "one_core_alg_gbps": round(alg / med1 / 1e9, 2),
            "all_cores_alg_gbps": round(alg / medn / 1e9, 2),
            "sample": f"the whole headline stream ({n} values, {b.size} bytes), plain decode by the "
                      f"scalar C oracle (validation pass then Algorithm 1), median of {reps} runs: "
                      f"1 core {med1:.2f} s; {cores} cores (one shard per core cut at code "
                      f"boundaries, a counting pass and a decode pass, both timed) {medn:.2f} s"}


# Kernels of one single-stream decode call: the look-back kernel alone, the
# chunked kernel alone, or the two-pass sequence (tile sums, scan, decode);
# a call ends with its last kernel.
DECODE_KERNELS = ("k_stream<", "k_chunks<", "k_tile_agg<", "k_tile_block", "k_known<")
CALL_END_KERNELS = ("k_stream<", "k_chunks<", "k_known<")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def short_kernel(name):
    return name.replace("vb::(anonymous namespace)::", "").split("(")[0]


def group_calls(rows, value):
    """Decode-call totals of value(row) over dispatch-ordered rows: every
    decode kernel adds to the current call, a call-ending kernel closes it."""
    calls, cur = [], 0.0
    for r in rows:
        name = r["Kernel_Name"]
        if not any(k in name for k in DECODE_KERNELS):
            continue
        cur += value(r)
        if any(k in name for k in CALL_END_KERNELS):
            calls.append(cur)
            cur = 0.0
    return calls


def describe_tuning(t):
    c = t.get("tiles_per_chunk", 0)
    mode = ("two-pass: k_tile_agg + k_tile_block_sums + k_tile_block_scan + k_known" if c == -1 else
            "one read: k_flow" if c == -2 else
            "look-back: k_stream" if c == 0 else f"chunks of {c} tiles: k_chunks")
    return f"{mode} (segs {t['segs_per_wave']}, waves {t['waves_per_block']})"


HEADLINE_KINDS = ("plain decode of the 2^30-value mix",)


def summarize_pmc(fetch_csv, write_csv, out_json, out_md, command_lines, kinds=HEADLINE_KINDS):
    """Turn two rocprofv3 --pmc runs of `bench.py --calibrate-copy` (one with
    FETCH_SIZE, one with WRITE_SIZE; values in KiB per dispatch) into HBM
    bytes per decode call.  Each counter is scaled by what it reads for the
    256 MiB calibration copy (known bytes / counted bytes).  Decode calls
    cycle through `kinds` in dispatch order (one kind: every call alike)."""
    import csv

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    known = COPY_ELEMS * 4
    res = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = load(path, name)
        copies = [float(r["Counter_Value"]) * 1024 for r in rows if COPY_KERNEL in r["Kernel_Name"]]
        copy = max(copies)
        factor = known / copy
        dec = group_calls(rows, lambda r: float(r["Counter_Value"]) * 1024 * factor)
        res[name] = {"copy_counted_bytes": copy, "factor": factor, "decode_bytes": dec}
    f, w = res["FETCH_SIZE"]["decode_bytes"], res["WRITE_SIZE"]["decode_bytes"]
    per = []
    nk = len(kinds)
    for k in range(nk):
        fk = f[k::nk]
        wk = w[k::nk]
        per.append({"kind": kinds[k], "calls": len(fk), "fetch_bytes": sum(fk) / len(fk),
                    "write_bytes": sum(wk) / len(wk),
                    "hbm_bytes": sum(fk) / len(fk) + sum(wk) / len(wk)})
    out = {"kernels": "all kernels of one decode call (" + ", ".join(DECODE_KERNELS) + ")",
           "kernel_source_sha256_16": kernel_source_hash(),
           "fetch_factor": res["FETCH_SIZE"]["factor"], "write_factor": res["WRITE_SIZE"]["factor"],
           "copy_counted_bytes": {"FETCH_SIZE": res["FETCH_SIZE"]["copy_counted_bytes"],
                                  "WRITE_SIZE": res["WRITE_SIZE"]["copy_counted_bytes"]},
           "per_stream": per,
           "hbm_bytes_per_launch": sum(p["hbm_bytes"] for p in per) / len(per),
           "commands": command_lines}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
    with open(out_md, "w") as fh:
        fh.write("# HBM traffic per decode call: " + "; ".join(kinds) + "\n\n")
        fh.write("Counters from two rocprofv3 runs (one counter each), scaled by the same counter\n"
                 "read for a plain 256 MiB device copy in the same process, summed over the\n"
                 "kernels of one decode call.\n\n")
        for c in command_lines:
            fh.write(f"    {c}\n")
        fh.write(f"\nFETCH_SIZE factor {out['fetch_factor']:.4f}, WRITE_SIZE factor {out['write_factor']:.4f}\n\n")
        fh.write("| call | calls | fetch MB | write MB | HBM MB |\n|---|---|---|---|---|\n")
        for p in per:
            fh.write(f"| {p['kind']} | {p['calls']} | {p['fetch_bytes'] / 1e6:.1f} | "
                     f"{p['write_bytes'] / 1e6:.1f} | {p['hbm_bytes'] / 1e6:.1f} |\n")
        fh.write(f"\nkernel source sha256[:16] (comments and blank space removed) = "
                 f"{out['kernel_source_sha256_16']}\n")
    return out


def bench_decode64(torch, vbyte, streams, reps=10):
    """64-bit differential decode (vbyte_decode64_delta) of the
    gap-mean-300 stream.  Codes of values below 2^32 are the same bytes in
    both widths, so the stream is a valid 64-bit code stream; decoding it from
    prev = 2^40 gives 64-bit identifiers.  Checked against a 64-bit cumsum."""
    s = streams[1]
    n = N_STREAM
    prev = 1 << 40
    vbyte.set_tuning(2, 8, 0)
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    vbyte.decode64(s["bytes"], n, delta=True, prev=prev, out=out, status=st, check=True)
    ref = torch.cumsum(s["gaps_dev"].to(torch.int64) & 0xFFFFFFFF, 0) + prev
    if not torch.equal(ref, out):
        raise RuntimeError("64-bit decode differs from the 64-bit prefix sum")
    del ref
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(reps):
        e0.record()
        vbyte.decode64(s["bytes"], n, delta=True, prev=prev, out=out, status=st, check=False)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    if int(st.item()) != 0:
        raise RuntimeError("64-bit decode status")
    avg = sum(ms) / len(ms)
    alg = s["bytes"].numel() + 8 * n
    return {"workload": "64-bit differential decode of the 64Mi-gap stream (gap mean 300) from "
                        "prev 2^40: uint64 identifiers, 8-byte outputs",
            "n": n, "bytes_in": int(s["bytes"].numel()), "tuning": "segs 2, waves 8",
            "kernels": "k64_agg + k64_scan + k64_known", "ms": round(avg, 4),
            "gints_per_s": round(n / (avg / 1e3) / 1e9, 2),
            "alg_gbps": round(alg / (avg / 1e3) / 1e9, 1),
            "pct_hbm_peak": round(100 * alg / (avg / 1e3) / 1e9 / HBM_PEAK_GBPS, 1)}


def bench_delta4(torch, vbyte, streams, reps=10):
    """Blocks-of-four differential decode (vbyte_decode_delta4)
    of the gap-mean-300 stream's bytes: out[i] = g_i + out[i-4], checked
    against four interleaved cumsums of the gaps."""
    s = streams[1]
    n = N_STREAM
    vbyte.set_tuning(2, 8, 0)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    vbyte.decode_delta4(s["bytes"], n, out=out, status=st, check=True)
    g = s["gaps_dev"].to(torch.int64) & 0xFFFFFFFF
    ref = (torch.cumsum(g.view(-1, 4), 0) & 0xFFFFFFFF).view(-1)
    if not torch.equal(ref, out.to(torch.int64) & 0xFFFFFFFF):
        raise RuntimeError("blocks-of-four decode differs from the interleaved cumsums")
    del ref, g
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(reps):
        e0.record()
        vbyte.decode_delta4(s["bytes"], n, out=out, status=st, check=False)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    if int(st.item()) != 0:
        raise RuntimeError("blocks-of-four decode status")
    avg = sum(ms) / len(ms)
    alg = s["bytes"].numel() + 4 * n
    return {"workload": "differences between blocks of four (y_i = g_i + y_(i-4)) over the "
                        "64Mi-gap stream (gap mean 300)",
            "n": n, "bytes_in": int(s["bytes"].numel()), "tuning": "segs 2, waves 8",
            "kernels": "k4_agg + k4_scan + k4_known", "ms": round(avg, 4),
            "gints_per_s": round(n / (avg / 1e3) / 1e9, 2),
            "alg_gbps": round(alg / (avg / 1e3) / 1e9, 1),
            "pct_hbm_peak": round(100 * alg / (avg / 1e3) / 1e9 / HBM_PEAK_GBPS, 1)}


def bench_intersect(torch, vbyte, streams, reps=5):
    """List intersection with the decode fused into the consumer
    (vbyte_intersect_async): the gap-mean-8 stream (64Mi identifiers)
    against a sorted list of 1Mi identifiers (half drawn from the long
    list), at several piece sizes (the piece size changes only the status of
    a bad list), beside decode-then-consume (the whole list decoded to HBM by
    vbyte_decode_delta, then torch.isin and a masked select).  Checked
    against torch.isin."""
    s = streams[0]
    n = N_STREAM
    ids = torch.cumsum(s["gaps_dev"].to(torch.int64) & 0xFFFFFFFF, 0)   # no wrap at gap mean 8
    g = torch.Generator(device="cuda").manual_seed(1503)
    pick = ids[torch.randint(0, n, (1 << 19,), device="cuda", generator=g)]
    other = torch.randint(0, int(ids[-1].item()) + 1, (1 << 19,), device="cuda", generator=g)
    b = torch.sort(torch.cat([pick, other]))[0]
    want = ids[torch.isin(ids, b)]
    b32 = b.to(torch.int32)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    nbytes = s["bytes"].numel()
    rows = []
    for piece in (1 << 18, 1 << 20, 1 << 22, n):
        vbyte.intersect(s["bytes"], n, b32, piece=piece, out=out, count=cnt, status=st, check=False)
        torch.cuda.synchronize()
        c = int(cnt.item())
        if int(st.item()) != 0 or c != want.numel() or \
                not torch.equal(out[:c].to(torch.int64) & 0xFFFFFFFF, want):
            raise RuntimeError(f"intersection differs from torch.isin (piece {piece})")
        ms = timed(lambda: vbyte.intersect(s["bytes"], n, b32, piece=piece, out=out, count=cnt,
                                           status=st, check=False))
        alg = nbytes + 4 * c   # list bytes read once, matches written
        rows.append({"piece": piece, "ms": round(ms, 4), "gints_per_s": round(n / (ms / 1e3) / 1e9, 2),
                     "alg_gbps": round(alg / (ms / 1e3) / 1e9, 1)})
    dec = torch.empty(n, dtype=torch.int32, device="cuda")
    bl = b.to(torch.int64)

    def decode_then_consume():
        vbyte.decode(s["bytes"], n, delta=True, out=dec, status=st, check=False)
        x = dec.to(torch.int64) & 0xFFFFFFFF
        return x[torch.isin(x, bl)]

    got = decode_then_consume()
    if not torch.equal(got, want):
        raise RuntimeError("decode-then-consume differs from torch.isin")
    base_ms = timed(decode_then_consume)
    return {"workload": "64Mi-identifier list (gap mean 8) intersected with 1Mi sorted identifiers",
            "kernels": "k_tile_agg + block scans + k_isect_tiles (count) + k_isect_status + "
                       "block scans + k_isect_tiles (store)",
            "matches": int(want.numel()), "points": rows,
            "workspace_bytes": 32 * ((nbytes + 16383) // 16384),
            "decode_then_torch_isin_ms": round(base_ms, 4)}


def build_index(torch, vbyte, workloads):
    """Config 3: 100,000 Zipf-length lists of gaps, VByte-encoded on the GPU
    with per-list byte offsets."""
    t0 = time.time()
    d = workloads.zipf_lists()
    gaps = torch.from_numpy(d["gaps"].view("int32")).cuda()
    vals_off = torch.from_numpy(d["out_off"]).cuda()
    enc, byte_off = vbyte.encode_batch(gaps, vals_off)
    torch.cuda.synchronize()
    log(f"config 3: {d['lengths'].size} lists, {int(d['out_off'][-1])} integers, {enc.numel()} bytes "
        f"({8 * enc.numel() / int(d['out_off'][-1]):.2f} bits/int), prepared in {time.time() - t0:.1f}s")
    return {"lists": d, "gaps": gaps, "bytes": enc, "byte_off": byte_off, "out_off": vals_off}


def bench_batched(torch, vbyte, serve, idx, reps=10):
    """Batched CSR decode of config 3 in one persistent launch (eager and as
    a graph replay, with the autotuned tiling), against one single-stream
    launch per list (both issued from native host loops); also the batched
    rate per list-length group [2^K, 2^(K+1))."""
    import numpy as np
    d = idx["lists"]
    nl = d["lengths"].size
    total = int(d["out_off"][-1])
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    st = torch.empty(nl, dtype=torch.int32, device="cuda")
    tune_points = vbyte.autotune_batch(idx["bytes"], idx["byte_off"], idx["out_off"], delta=True,
                                       out=out, reps=2)
    # per-list launches (below, and in the serving comparison) decode each
    # list with the single-launch look-back kernel, the fewest launches per list
    vbyte.set_tuning(tiles_per_chunk=0)
    tuned = vbyte.get_tuning()
    log(f"batch tuning: {tuned}")

    def once():
        vbyte.decode_batch(idx["bytes"], idx["byte_off"], idx["out_off"], delta=True, out=out,
                           list_status=st)

    once()
    torch.cuda.synchronize()
    if int(st.max().item()) != 0:
        raise RuntimeError("batched decode reported a bad list")
    # spot-check a few lists against the gaps' prefix sums
    for i in (0, 1, nl // 2, nl - 1, int(d["lengths"].argmax())):
        a, b = int(d["out_off"][i]), int(d["out_off"][i + 1])
        ref = torch.cumsum(idx["gaps"][a:b].to(torch.int64) & 0xFFFFFFFF, 0) & 0xFFFFFFFF
        if not torch.equal(ref, out[a:b].to(torch.int64) & 0xFFFFFFFF):
            raise RuntimeError(f"batched decode differs on list {i}")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / reps
    in_bytes = idx["bytes"].numel()
    # the same batch captured into a HIP graph and replayed
    gout = torch.empty_like(out)
    gst = torch.empty_like(st)
    g = vbyte.BatchGraph(idx["bytes"], idx["byte_off"], idx["out_off"], gout, gst, delta=True)
    g.launch()
    torch.cuda.synchronize()
    if not torch.equal(gout, out) or int(gst.max().item()) != 0:
        raise RuntimeError("graph replay differs from the eager batch")
    e0.record()
    for _ in range(reps):
        g.launch()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / reps
    g.close()
    del gout, gst
    # per list-length group: the group's lists as one gather batch
    lens = d["lengths"]
    bo_h = idx["byte_off"].cpu().numpy()
    oo_h = d["out_off"]
    groups = []
    for k in range(int(np.log2(lens.max())) + 1):
        sel = np.nonzero((lens >= (1 << k)) & (lens < (2 << k)))[0]
        if sel.size == 0:
            continue
        rows = np.stack([bo_h[sel], bo_h[sel + 1], oo_h[sel], lens[sel]], axis=1).astype(np.int64)
        rows_d = torch.from_numpy(np.ascontiguousarray(rows)).cuda()
        gbytes = int((bo_h[sel + 1] - bo_h[sel]).sum())
        gints = int(lens[sel].sum())
        gs = torch.empty(sel.size, dtype=torch.int32, device="cuda")
        vbyte.decode_lists(idx["bytes"], rows_d, gbytes, out, delta=True, list_status=gs)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            vbyte.decode_lists(idx["bytes"], rows_d, gbytes, out, delta=True, list_status=gs)
        e1.record()
        torch.cuda.synchronize()
        if int(gs.max().item()) != 0:
            raise RuntimeError(f"length group 2^{k} reported a bad list")
        ms = e0.elapsed_time(e1) / reps
        groups.append({"len_lo": 1 << k, "len_hi": (2 << k) - 1, "lists": int(sel.size),
                       "integers": gints, "bytes_in": gbytes, "ms": round(ms, 4),
                       "gints_per_s": round(gints / (ms / 1e3) / 1e9, 2),
                       "alg_gbps": round((gbytes + 4 * gints) / (ms / 1e3) / 1e9, 1)})
    # the batch tuning stays in force for the server runs below
    # per-list launches and the server's single gather launch, same lists
    bo = idx["byte_off"].cpu().numpy()
    counts = d["lengths"].astype("int64")
    res = {}
    for batching in (True, False):
        srv = serve.Server(idx["bytes"], bo, counts, pool_bytes=(total + 1024) * 4, nstreams=1,
                           max_batch_requests=1, batching=batching, delta=True)
        lat, stt, _ = srv.run(np.zeros(1), [np.arange(nl, dtype=np.int64)])
        lat, stt, _ = srv.run(np.zeros(1), [np.arange(nl, dtype=np.int64)])
        srv.close()
        if stt["worst_status"] != 0:
            raise RuntimeError("server decode reported a bad list")
        res[batching] = (float(lat[0]) * 1e3, int(stt["launches"]))
    return {"workload": "100,000 differential lists, Zipf(1.2) lengths clipped to [1, 4Mi], 2^28 "
                        "integers, gaps Geometric(len/2^25)",
            "bytes_in": int(in_bytes), "integers": total,
            "tuning": tuned, "tuned_candidates": len(tune_points),
            "batched_csr_ms": round(batched_ms, 4),
            "batched_gints_per_s": round(total / (batched_ms / 1e3) / 1e9, 2),
            "batched_alg_gbps": round((in_bytes + 4 * total) / (batched_ms / 1e3) / 1e9, 1),
            "graph_replay_ms": round(graph_ms, 4),
            "graph_replay_gints_per_s": round(total / (graph_ms / 1e3) / 1e9, 2),
            "per_length_group": groups,
            "gather_one_launch_ms": round(res[True][0], 3),
            "per_list_launches_ms": round(res[False][0], 3),
            "per_list_launches": res[False][1],
            # like for like: both sides through the server, host clock from
            # submission to completion
            "speedup_batched_vs_per_list": round(res[False][0] / res[True][0], 1),
            # the per-list server time against the GPU-event time of one
            # eager batched call or graph replay (two different clocks)
            "per_list_server_ms_over_batched_event_ms": round(res[False][0] / batched_ms, 1),
            "per_list_server_ms_over_graph_event_ms": round(res[False][0] / graph_ms, 1)}


def bench_serving(torch, vbyte, serve, workloads, idx, nq=10000, warm=1000):
    """Config 4: Poisson queries of 2-8 Zipf(1.0) terms over the config-3
    index; p50/p99 latency (per request: until its own lists are decoded)
    and throughput at fractions of saturation QPS, each point nq measured
    queries after `warm` warm-up ones; a sample of served results checked
    against the batched decode of the whole index."""
    import numpy as np
    d = idx["lists"]
    pos_of_rank = np.argsort(d["rank_of"])
    bo = idx["byte_off"].cpu().numpy()
    counts = d["lengths"].astype("int64")
    nl = counts.size
    # served results against the batched decode of every list
    full, lst = vbyte.decode_batch(idx["bytes"], idx["byte_off"], idx["out_off"], delta=True)
    torch.cuda.synchronize()
    if int(lst.max().item()) != 0:
        raise RuntimeError("batched decode of the index reported a bad list")
    oo = d["out_off"]
    arr, ranks = workloads.query_stream(300, 1e6, nlists=nl, seed=workloads.SEED_QUERIES + 7)
    terms = [pos_of_rank[r] for r in ranks]
    srv = serve.Server(idx["bytes"], bo, counts, pool_bytes=6 << 30, nstreams=4,
                       max_batch_requests=64, batching=True, delta=True)
    _, stt, (res, roff) = srv.run(arr, terms, capture=True)
    srv.close()
    if stt["worst_status"] != 0 or (stt["status"] != 0).any():
        raise RuntimeError("served requests reported a bad status")
    for r in range(0, len(terms), 7):
        want = torch.cat([full[int(oo[t]):int(oo[t + 1])] for t in terms[r]])
        if not torch.equal(res[int(roff[r]):int(roff[r + 1])], want):
            raise RuntimeError(f"served result {r} differs from the batched decode")
    checked = len(range(0, len(terms), 7))
    del full, res

    def make(qps, n, seed):
        arr, ranks = workloads.query_stream(n, qps, nlists=nl, seed=seed)
        return arr, [pos_of_rank[r] for r in ranks]

    def run(srv, arr, terms):
        lat, stt, _ = srv.run(arr, terms)
        if stt["worst_status"] != 0 or stt["rejected"] or (stt["status"] != 0).any():
            raise RuntimeError("serving run reported a bad list or a rejected query")
        lat = lat[warm:] if lat.size > warm else lat
        return lat, stt

    srv = serve.Server(idx["bytes"], bo, counts, pool_bytes=6 << 30, nstreams=4,
                       max_batch_requests=64, batching=True, delta=True)
    # saturation: every query queued at time 0 (closed loop)
    arr, terms = make(1.0, nq, workloads.SEED_QUERIES)
    _, stt = run(srv, np.zeros(nq), terms)
    sat_qps = nq / stt["wall_s"]
    ints_per_query = stt["integers"] / nq
    points = []
    for frac in (0.25, 0.5, 0.75, 0.9):
        qps = frac * sat_qps
        arr, terms = make(qps, nq + warm, workloads.SEED_QUERIES + int(frac * 100))
        lat, stt = run(srv, arr, terms)
        points.append({"qps": round(qps, 1), "frac_of_saturation": frac,
                       "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
                       "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
                       "gints_per_s": round(stt["integers"] / stt["wall_s"] / 1e9, 2),
                       "mean_batch_requests": round(stt["mean_batch_requests"], 2)})
    srv.close()
    # the same load at half saturation with one launch per list and no batching
    srv = serve.Server(idx["bytes"], bo, counts, pool_bytes=6 << 30, nstreams=4,
                       max_batch_requests=1, batching=False, delta=True)
    arr, terms = make(0.5 * sat_qps, nq + warm, workloads.SEED_QUERIES + 50)
    lat, stt = run(srv, arr, terms)
    srv.close()
    per_list = {"qps": round(0.5 * sat_qps, 1),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
                "gints_per_s": round(stt["integers"] / stt["wall_s"] / 1e9, 2)}
    return {"workload": "queries of 2-8 distinct Zipf(1.0) terms over the config-3 index (rank r = "
                        "r-th longest list), Poisson arrivals, differential decode into a 6 GiB "
                        "output pool, 4 streams",
            "queries_per_point": nq, "warmup_queries": warm,
            "results_checked": f"{checked} of 300 requests served at 1M QPS equal the batched decode",
            "saturation_qps": round(sat_qps, 1), "integers_per_query": round(ints_per_query, 1),
            "points": points, "per_list_launches_at_half_saturation": per_list}


def summarize_trace(trace_csv, stats_csv, out_md, command_line, kinds=HEADLINE_KINDS):
    """Turn a rocprofv3 --kernel-trace --stats run of bench.py (with a fixed
    --tuning, so that every decode call runs the same kernels) into the
    per-call duration table of profiles/decode_plain_1Gi_mix_kernel_trace.md:
    per decode call, the sum of its kernels' durations and its span from
    the first kernel's start to the last kernel's end (what the HIP events
    around the call in bench.py measure), and per kernel."""
    import csv
    rows = [r for r in csv.DictReader(open(trace_csv))
            if any(k in r["Kernel_Name"] for k in DECODE_KERNELS)]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    calls, cur = [], []
    for r in rows:
        cur.append(r)
        if any(k in r["Kernel_Name"] for k in CALL_END_KERNELS):
            calls.append(cur)
            cur = []
    names = []
    for r in rows:
        if short_kernel(r["Kernel_Name"]) not in names:
            names.append(short_kernel(r["Kernel_Name"]))

    def dur(r):
        return (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3

    nk = len(kinds)
    with open(out_md, "w") as fh:
        fh.write("# Kernel trace: " + "; ".join(kinds) + " (bench.py)\n\n")
        fh.write("Command (run from the repository root on one MI355X):\n\n")
        fh.write(f"    {command_line}\n\n")
        fh.write("Kernels of one decode call: " + ", ".join(f"`{n}`" for n in names) + ".\n")
        fh.write("Calls in dispatch order (first the warm-up steps, then the timed ones)"
                 + (", cycling through the kinds above" if nk > 1 else "") + ".\n\n")
        fh.write("| call | calls | kernel sum avg us | span avg us | span min us | span max us |\n"
                 "|---|---|---|---|---|---|\n")
        for k, name in enumerate(kinds):
            cs = calls[k::nk]
            if not cs:
                continue
            ksum = [sum(dur(r) for r in c) for c in cs]
            span = [(int(c[-1]["End_Timestamp"]) - int(c[0]["Start_Timestamp"])) / 1e3 for c in cs]
            fh.write(f"| {name} | {len(cs)} | {sum(ksum) / len(ksum):.1f} | {sum(span) / len(span):.1f} | "
                     f"{min(span):.1f} | {max(span):.1f} |\n")
        fh.write("\nPer kernel (average us per call):\n\n| call | " + " | ".join(names) + " |\n|---|"
                 + "---|" * len(names) + "\n")
        for k, name in enumerate(kinds):
            cs = calls[k::nk]
            if not cs:
                continue
            cells = []
            for n in names:
                d = [dur(r) for c in cs for r in c if short_kernel(r["Kernel_Name"]) == n]
                cells.append(f"{sum(d) / len(cs):.1f}")
            fh.write(f"| {name} | " + " | ".join(cells) + " |\n")
        fh.write("\nrocprofv3 --stats summary (the ten kernels with the most total time):\n\n")
        st = list(csv.DictReader(open(stats_csv)))
        st.sort(key=lambda r: -float(r.get("TotalDurationNs", 0) or 0))
        fh.write("| kernel | calls | avg ns | min ns | max ns |\n|---|---|---|---|---|\n")
        for r in st[:10]:
            fh.write(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                     f"{float(r['MinNs']):.0f} | {float(r['MaxNs']):.0f} |\n")
    return {"calls": len(calls), "kernels": names}


# the other bench lines whose kernels get a trace summary: (kernels, the
# call's last kernel, summary file, title)
SIDE_TRACES = {
    "decode64": (("k64_agg<", "k64_scan", "k64_known<"), "k64_known<",
                 os.path.join(ROOT, "profiles", "decode64_delta_64Mi_kernel_trace.md"),
                 "64-bit differential decode of the 64Mi-gap stream (gap mean 300)"),
    "delta4": (("k4_agg<", "k4_scan", "k4_known<"), "k4_known<",
               os.path.join(ROOT, "profiles", "decode_delta4_64Mi_kernel_trace.md"),
               "blocks-of-four differential decode of the 64Mi-gap stream (gap mean 300)"),
}


def summarize_side_trace(which, trace_csv, command_line):
    """Per-call durations of one side line's kernels (the decode64 or delta4
    entry of bench.py) from a rocprofv3 --kernel-trace run."""
    import csv
    kernels, last, out_md, title = SIDE_TRACES[which]
    rows = [r for r in csv.DictReader(open(trace_csv))
            if any(k in r["Kernel_Name"] for k in kernels)]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    calls, cur = [], []
    for r in rows:
        cur.append(r)
        if last in r["Kernel_Name"]:
            calls.append(cur)
            cur = []

    def dur(r):
        return (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3

    names = []
    for r in rows:
        if short_kernel(r["Kernel_Name"]) not in names:
            names.append(short_kernel(r["Kernel_Name"]))
    with open(out_md, "w") as fh:
        fh.write(f"# Kernel trace: {title}\n\n")
        fh.write("Command (run from the repository root on one MI355X):\n\n")
        fh.write(f"    {command_line}\n\n")
        span = [(int(c[-1]["End_Timestamp"]) - int(c[0]["Start_Timestamp"])) / 1e3 for c in calls]
        ksum = [sum(dur(r) for r in c) for c in calls]
        fh.write("| calls | kernel sum avg us | span avg us | span min us | span max us |\n"
                 "|---|---|---|---|---|\n")
        if calls:
            fh.write(f"| {len(calls)} | {sum(ksum) / len(ksum):.1f} | {sum(span) / len(span):.1f} | "
                     f"{min(span):.1f} | {max(span):.1f} |\n")
        fh.write("\nPer kernel (average us per call): " + ", ".join(
            f"`{n}` {sum(dur(r) for c in calls for r in c if short_kernel(r['Kernel_Name']) == n) / max(len(calls), 1):.1f}"
            for n in names) + "\n")
    return {"calls": len(calls), "kernels": names}


def device_info(torch):
    """Name, architecture and CU count of the GPU, ROCm and HIP versions,
    host cores."""
    p = torch.cuda.get_device_properties(0)
    rocm = None
    try:
        with open("/opt/rocm/.info/version") as fh:
            rocm = fh.read().strip()
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"gpu": p.name, "arch": getattr(p, "gcnArchName", None), "cus": p.multi_processor_count,
            "hbm_gib": round(p.total_memory / 2 ** 30, 1), "rocm": rocm, "hip": torch.version.hip,
            "torch": torch.__version__, "host_cores": cores}


def make_mix(torch, vbyte, workloads):
    """The headline stream: 2^30 values of the 1/2/5-byte mix, encoded on the
    GPU."""
    import numpy as np
    t0 = time.time()
    x = workloads.worst_case_mix(N_MIX, workers=16)
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    enc = vbyte.encode(xd)
    torch.cuda.synchronize()
    log(f"mix: {N_MIX} values -> {enc.numel()} bytes ({enc.numel() / N_MIX:.4f} B/int), "
        f"prepared in {time.time() - t0:.1f}s")
    return {"x": x, "x_dev": xd, "bytes": enc}


class Flusher:
    """Writes FLUSH_BYTES before a call so that its input is not served by
    the 256 MB Infinity Cache (MALL) from an earlier call."""

    def __init__(self, torch):
        self.buf = torch.empty(FLUSH_BYTES, dtype=torch.uint8, device="cuda")

    def __call__(self):
        self.buf.zero_()


def event_times(torch, fn, reps, before=None):
    """HIP-event time (ms) of each of `reps` calls of fn on the current
    stream; `before` runs ahead of each call, outside the events."""
    stream = torch.cuda.current_stream()
    ms = []
    for _ in range(reps):
        if before is not None:
            before()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return ms


def line(n, bytes_in, ms, out_bytes_per_int=4):
    """Throughput fields of a decode that took `ms` per call."""
    alg = bytes_in + out_bytes_per_int * n
    return {"ms": round(ms, 4), "gints_per_s": round(n / (ms / 1e3) / 1e9, 2),
            "alg_gbps": round(alg / (ms / 1e3) / 1e9, 1),
            "pct_hbm_peak": round(100 * alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 1)}


def median(v):
    v = sorted(v)
    return v[len(v) // 2]


def bench_mix_delta(torch, vbyte, mix, flush, tuning, reps=10):
    """Differential decode (wrapping prefix sum from prev 0) of the headline
    stream's bytes, checked against a cumsum of the drawn values."""
    n = N_MIX
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")

    def call():
        vbyte.decode(mix["bytes"], n, delta=True, out=out, status=st, check=False, tuning=tuning)

    call()
    torch.cuda.synchronize()
    ref = (torch.cumsum(mix["x_dev"].to(torch.int64) & 0xFFFFFFFF, 0) & 0xFFFFFFFF).to(torch.int32)
    if int(st.item()) != 0 or not torch.equal(ref, out):
        raise RuntimeError("differential decode of the mix differs from the cumsum")
    del ref
    warm = median(event_times(torch, call, reps))
    cold = median(event_times(torch, call, reps, before=flush))
    r = {"workload": "differential decode (wrapping uint32 prefix sum) of the 2^30-value 1/2/5-byte "
                     "mix, the headline stream's bytes", "n": n, "bytes_in": int(mix["bytes"].numel()),
         "tuning": dict(HEADLINE_TUNING), "back_to_back": line(n, mix["bytes"].numel(), warm),
         "mall_flushed": line(n, mix["bytes"].numel(), cold)}
    del out
    return r


def bench_one_read(torch, vbyte, mix, flush, reps=10):
    """The one-read schedule (one persistent launch) on the headline
    stream, plain and differential, against the same check."""
    n = N_MIX
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    T = vbyte.make_tuning(2, 7, vbyte.SCHED_ONE_READ)
    res = {"workload": "plain and differential decode of the 2^30-value mix with the one-read "
                       "schedule (k_flow, segs 2, 7 decode wavefronts + 1 control)"}
    for delta in (False, True):
        def call():
            vbyte.decode(mix["bytes"], n, delta=delta, out=out, status=st, check=False, tuning=T)
        call()
        torch.cuda.synchronize()
        if delta:
            ok = torch.equal((torch.cumsum(mix["x_dev"].to(torch.int64) & 0xFFFFFFFF, 0)
                              & 0xFFFFFFFF).to(torch.int32), out)
        else:
            ok = torch.equal(mix["x_dev"], out)
        if int(st.item()) != 0 or not ok:
            raise RuntimeError("one-read decode differs")
        res["delta" if delta else "plain"] = {
            "back_to_back": line(n, mix["bytes"].numel(), median(event_times(torch, call, reps))),
            "mall_flushed": line(n, mix["bytes"].numel(),
                                 median(event_times(torch, call, reps, before=flush)))}
    del out
    return res


def bench_uniform(torch, vbyte, workloads, flush, tuning, reps=30):
    """The small case: plain decode of 2^20 values with uniform code
    lengths 1..5 (3.1 MB in, 4.2 MB out), with the MALL flushed before each
    call and back to back (input and output then in the MALL)."""
    import numpy as np
    x, _ = workloads.uniform_lengths(n=N_UNIFORM)
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    enc = vbyte.encode(xd)
    out = torch.empty(x.size, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")

    def call():
        vbyte.decode(enc, x.size, out=out, status=st, check=False, tuning=tuning)

    call()
    torch.cuda.synchronize()
    if int(st.item()) != 0 or not torch.equal(out, xd):
        raise RuntimeError("uniform-length decode differs from the drawn values")
    cold = event_times(torch, call, reps, before=flush)
    warm = event_times(torch, call, reps)
    return {"workload": "plain decode of 2^20 values, code length uniform in 1..5",
            "n": int(x.size), "bytes_in": int(enc.numel()), "tuning": dict(HEADLINE_TUNING),
            "mall_flushed": line(x.size, enc.numel(), median(cold)),
            "mall_flushed_min_ms": round(min(cold), 4),
            "back_to_back": line(x.size, enc.numel(), median(warm))}


def bench_encoder(torch, vbyte, streams, flush, reps=10):
    """The GPU encoder on both 64Mi-gap streams (values -> canonical codes),
    checked against the bytes the decode lines use; algorithmic bytes are
    4n in + the encoded bytes out."""
    rows = []
    for s in streams:
        n = s["gaps"].size
        out = torch.empty(5 * n, dtype=torch.uint8, device="cuda")
        nb = torch.empty(1, dtype=torch.int64, device="cuda")

        def call():
            vbyte.encode(s["gaps_dev"], out=out, nbytes=nb, trim=False)

        call()
        torch.cuda.synchronize()
        m = int(nb.item())
        if m != s["bytes"].numel() or not torch.equal(out[:m], s["bytes"]):
            raise RuntimeError("encoder output differs")
        for label, before in (("back_to_back", None), ("mall_flushed", flush)):
            ms = median(event_times(torch, call, reps, before=before))
            alg = 4 * n + m
            rows.append({"gap_mean": s["mean"], "timing": label, "n": n, "bytes_out": m,
                         "ms": round(ms, 4), "gints_per_s": round(n / (ms / 1e3) / 1e9, 2),
                         "alg_gbps": round(alg / (ms / 1e3) / 1e9, 1),
                         "pct_hbm_peak": round(100 * alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 1)})
        del out
    return {"workload": "VByte encoding of the two 64Mi-gap streams (k_enc_len, k_enc_bscan, "
                        "k_enc_write)", "rows": rows}


def bench_config2(torch, vbyte, streams, flush, tuning, reps=10):
    """Differential decode of the two 64Mi-gap streams (gap means 8 and 300),
    each call timed alone, back to back and with the MALL flushed."""
    rows = []
    for s in streams:
        def call():
            vbyte.decode(s["bytes"], N_STREAM, delta=True, prev=0, out=s["out"], status=s["status"],
                         check=False, tuning=tuning)
        call()
        torch.cuda.synchronize()
        verify(torch, [s])
        warm = median(event_times(torch, call, reps))
        cold = median(event_times(torch, call, reps, before=flush))
        rows.append({"gap_mean": s["mean"], "n": N_STREAM, "bytes_in": int(s["bytes"].numel()),
                     "back_to_back": line(N_STREAM, s["bytes"].numel(), warm),
                     "mall_flushed": line(N_STREAM, s["bytes"].numel(), cold)})
    return {"workload": "differential decode of two single streams of 64Mi uint32 gaps "
                        "(geometric, means 8 and 300)", "tuning": dict(HEADLINE_TUNING),
            "streams": rows}


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-trace":
        o = summarize_trace(sys.argv[2], sys.argv[3], PROFILE_TRACE, sys.argv[4])
        print(json.dumps(o))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-side-trace":
        print(json.dumps(summarize_side_trace(sys.argv[2], sys.argv[3], sys.argv[4])))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-pmc":
        fetch_csv, write_csv = sys.argv[2], sys.argv[3]
        cmds = sys.argv[4:]
        o = summarize_pmc(fetch_csv, write_csv, PROFILE_COUNTERS,
                          PROFILE_COUNTERS.replace(".json", ".md"), cmds)
        print(json.dumps(o))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline decode only (profiling runs): no side lines, no "
                         "CPU baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the config-3 batched comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the config-4 serving run")
    ap.add_argument("--no-decode64", action="store_true", help="skip the 64-bit decode line")
    ap.add_argument("--no-delta4", action="store_true", help="skip the blocks-of-four decode line")
    ap.add_argument("--no-intersect", action="store_true", help="skip the intersection line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain device copy of 256 MiB (int32 tensor copy) before the "
                         "steps, as the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (a stream "
              "would shard by byte ranges with one exchange of per-range counts and sums)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1503_07387_amd import vbyte, workloads
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    vbyte._lib()
    info = device_info(torch)
    log(f"device: {info}")
    mix = make_mix(torch, vbyte, workloads)
    n = N_MIX
    nbytes = int(mix["bytes"].numel())
    alg = nbytes + 4 * n
    tuning = vbyte.make_tuning(**HEADLINE_TUNING)
    stream = torch.cuda.current_stream()
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    status = torch.empty(1, dtype=torch.int32, device="cuda")

    def call():
        vbyte.decode(mix["bytes"], n, out=out, status=status, check=False, tuning=tuning)

    def verify_mix():
        if int(status.item()) != 0:
            raise RuntimeError(f"decode status {int(status.item())}")
        if not torch.equal(out, mix["x_dev"]):
            raise RuntimeError("decoded values differ from the drawn values")

    if args.calibrate_copy:
        a = torch.arange(COPY_ELEMS, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    verify_mix()
    out.fill_(0)
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        call()
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    verify_mix()

    kernel_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    avg_ms = sum(kernel_ms) / len(kernel_ms)
    ms_per_step = wall * 1e3 / args.steps
    value = n / (ms_per_step / 1e3) / 1e9
    achieved = alg / (avg_ms / 1e3) / 1e9
    traffic = measured_traffic([alg])
    if traffic is not None:
        traffic = round(traffic)
    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "plain single-stream VByte decode of 2^30 uint32 values, 5 % 5-byte "
                               "codes >= 2^28, else 50/50 1-byte and 2-byte codes (1.80 GB in, "
                               "4 GiB out)",
                   "n": n, "bytes_in": nbytes, "tuning": dict(HEADLINE_TUNING)},
        "device": info,
        "kernel_ms": {"avg": round(avg_ms, 4), "min": round(min(kernel_ms), 4),
                      "max": round(max(kernel_ms), 4)},
        "hbm_gbps": round(achieved, 1),
        "pct_hbm_peak": round(100 * achieved / HBM_PEAK_GBPS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "kernel": "the whole decode call, all its launches: " + describe_tuning(
                         {"tiles_per_chunk": HEADLINE_TUNING["schedule"],
                          "segs_per_wave": HEADLINE_TUNING["segs_per_wave"],
                          "waves_per_block": HEADLINE_TUNING["waves_per_block"]}),
                     "alg_bytes_per_launch": alg},
    }
    if args.only_headline:
        print(json.dumps(res), flush=True)
        return
    flush = Flusher(torch)
    cold = event_times(torch, call, 10, before=flush)
    res["headline_mall_flushed"] = line(n, nbytes, median(cold))
    del out
    log("differential decode of the mix ...")
    res["config5_delta"] = bench_mix_delta(torch, vbyte, mix, flush, tuning)
    log("one-read schedule ...")
    res["one_read"] = bench_one_read(torch, vbyte, mix, flush)
    log("uniform-length stream ...")
    res["config1_plain"] = bench_uniform(torch, vbyte, workloads, flush, tuning)
    mix_host = (mix["bytes"].cpu().numpy(), mix["x"])
    del mix
    torch.cuda.empty_cache()
    streams = make_streams(torch, vbyte, workloads)
    log("64Mi-gap streams ...")
    res["config2_delta"] = bench_config2(torch, vbyte, streams, flush, tuning)
    log("encoder ...")
    res["encoder"] = bench_encoder(torch, vbyte, streams, flush)
    if not args.no_decode64:
        log("64-bit decode ...")
        res["decode64"] = bench_decode64(torch, vbyte, streams)
    if not args.no_delta4:
        log("blocks-of-four decode ...")
        res["delta4"] = bench_delta4(torch, vbyte, streams)
    if not args.no_intersect:
        log("intersection ...")
        res["intersect"] = bench_intersect(torch, vbyte, streams)
    del streams
    torch.cuda.empty_cache()
    if not (args.no_batched and args.no_serving):
        from paper_1503_07387_amd import serve
        idx = build_index(torch, vbyte, workloads)
        if not args.no_batched:
            log("batched vs per-list launches (config 3) ...")
            res["batched"] = bench_batched(torch, vbyte, serve, idx)
        if not args.no_serving:
            log("serving (config 4) ...")
            res["serving"] = bench_serving(torch, vbyte, serve, workloads, idx)
        del idx
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        res["cpu_baseline"] = cpu_baseline(*mix_host)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
