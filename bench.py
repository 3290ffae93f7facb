"""Benchmark of the VByte decode hot path on one MI355X.

A step is one pass of the whole hot path over the benchmark workload: the
differential decode (VByte gaps -> uint32 document identifiers, wrapping
prefix sum) of two synthetic single streams of 64Mi gaps each, one with
geometric gaps of mean 8 (almost only 1-byte codes) and one of mean 300
(a 35/65 mix of 1- and 2-byte codes).  The inputs are generated, VByte-encoded
on the GPU by the library's encoder and resident in HBM before timing starts.

Printed: one JSON line with throughput (Gints/s), the HBM roofline of the
decode kernel (algorithmic bytes in + 4n out per launch over the launch's
HIP-event time), and the scalar CPU oracle timed on the host as a baseline.

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
COPY_ELEMS = 1 << 26          # calibration copy: 256 MiB read + 256 MiB written
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "decode_delta_64Mi_counters.json")
PROFILE_TRACE = os.path.join(ROOT, "profiles", "decode_delta_64Mi_kernel_trace.md")
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


def cpu_baseline(streams, budget_s=15.0):
    """The scalar oracle (plain C, one thread) on the same workload: decode of
    whole streams, repeated until about budget_s of CPU work is spent."""
    import oracle
    host = [(s["bytes"].cpu().numpy(), s["gaps"].size) for s in streams]
    ints = 0
    t0 = time.perf_counter()
    passes = 0
    while True:
        for b, n in host:
            st, _ = oracle.decode_delta(b, n, 0)
            if st != oracle.OK:
                raise RuntimeError("oracle failed on the benchmark stream")
            ints += n
        passes += 1
        el = time.perf_counter() - t0
        if el >= budget_s or passes >= 10:
            break
    return {"value": ints / el / 1e9, "unit": "Gints/s", "cores": 1, "kind": "oracle",
            "sample": f"{passes} pass(es) over both 64Mi-gap streams (the full workload), "
                      f"scalar C oracle (Algorithm 1 + wrapping prefix sum), 1 thread, "
                      f"{el:.1f}s wall"}


# Kernels of one single-stream decode call: the look-back kernel alone, the
# chunked kernel alone, or the two-pass sequence (tile sums, scan, decode);
# a call ends with its last kernel.
DECODE_KERNELS = ("k_stream<", "k_chunks<", "k_tile_agg<", "k_tile_scan", "k_known<")
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
    mode = ("two-pass: k_tile_agg + k_tile_scan + k_known" if c < 0 else
            "look-back: k_stream" if c == 0 else f"chunks of {c} tiles: k_chunks")
    return f"{mode} (segs {t['segs_per_wave']}, waves {t['waves_per_block']})"


def summarize_pmc(fetch_csv, write_csv, out_json, out_md, command_lines):
    """Turn two rocprofv3 --pmc runs of `bench.py --calibrate-copy` (one with
    FETCH_SIZE, one with WRITE_SIZE; values in KiB per dispatch) into HBM
    bytes per decode launch.  Each counter is scaled by what it reads for the
    256 MiB calibration copy (known bytes / counted bytes)."""
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
    # dispatches alternate: gap-mean-8 stream, gap-mean-300 stream
    f, w = res["FETCH_SIZE"]["decode_bytes"], res["WRITE_SIZE"]["decode_bytes"]
    per = []
    for k in range(2):
        fk = f[k::2]
        wk = w[k::2]
        per.append({"fetch_bytes": sum(fk) / len(fk), "write_bytes": sum(wk) / len(wk),
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
        fh.write("# HBM traffic of the differential decode, 2 x 64Mi-gap streams\n\n")
        fh.write("Counters from two rocprofv3 runs (one counter each), scaled by the same counter\n"
                 "read for a plain 256 MiB device copy in the same process, summed over the\n"
                 "kernels of one decode call.\n\n")
        for c in command_lines:
            fh.write(f"    {c}\n")
        fh.write(f"\nFETCH_SIZE factor {out['fetch_factor']:.4f}, WRITE_SIZE factor {out['write_factor']:.4f}\n\n")
        fh.write("| stream | fetch MB | write MB | HBM MB |\n|---|---|---|---|\n")
        for name, p in zip(("gap mean 8", "gap mean 300"), per):
            fh.write(f"| {name} | {p['fetch_bytes'] / 1e6:.1f} | {p['write_bytes'] / 1e6:.1f} | "
                     f"{p['hbm_bytes'] / 1e6:.1f} |\n")
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
    """List intersection by the consumer of resumable pieces
    (vbyte_intersect_async): the gap-mean-8 stream (64Mi identifiers) against
    a sorted list of 1Mi identifiers (half drawn from the long list), for
    several piece sizes; a piece of the whole list is the decode-then-consume
    baseline.  Checked against torch.isin."""
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
    vbyte.set_tuning(2, 8, 0)
    rows = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for piece in (1 << 18, 1 << 20, 1 << 22, n):
        vbyte.intersect(s["bytes"], n, b32, piece=piece, out=out, count=cnt, status=st, check=False)
        torch.cuda.synchronize()
        c = int(cnt.item())
        if int(st.item()) != 0 or c != want.numel() or \
                not torch.equal(out[:c].to(torch.int64) & 0xFFFFFFFF, want):
            raise RuntimeError(f"intersection differs from torch.isin (piece {piece})")
        e0.record()
        for _ in range(reps):
            vbyte.intersect(s["bytes"], n, b32, piece=piece, out=out, count=cnt, status=st,
                            check=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rows.append({"piece": piece, "pieces": (n + piece - 1) // piece,
                     "piece_buffer_bytes": piece * 5, "ms": round(ms, 4),
                     "gints_per_s": round(n / (ms / 1e3) / 1e9, 2)})
    return {"workload": "64Mi-identifier list (gap mean 8) intersected with 1Mi sorted identifiers",
            "matches": int(want.numel()), "points": rows}


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
            "speedup_batched_vs_per_list": round(res[False][0] / batched_ms, 1),
            "speedup_graph_vs_per_list": round(res[False][0] / graph_ms, 1)}


def bench_serving(torch, vbyte, serve, workloads, idx, nq=3000, warm=300):
    """Config 4: Poisson queries of 2-8 Zipf(1.0) terms over the config-3
    index; p50/p99 latency and throughput at fractions of saturation QPS."""
    import numpy as np
    d = idx["lists"]
    pos_of_rank = np.argsort(d["rank_of"])
    bo = idx["byte_off"].cpu().numpy()
    counts = d["lengths"].astype("int64")
    nl = counts.size

    def make(qps, n, seed):
        arr, ranks = workloads.query_stream(n, qps, nlists=nl, seed=seed)
        return arr, [pos_of_rank[r] for r in ranks]

    def run(srv, arr, terms):
        lat, stt, _ = srv.run(arr, terms)
        if stt["worst_status"] != 0 or stt["rejected"]:
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
            "saturation_qps": round(sat_qps, 1), "integers_per_query": round(ints_per_query, 1),
            "points": points, "per_list_launches_at_half_saturation": per_list}


def summarize_trace(trace_csv, stats_csv, out_md, command_line):
    """Turn a rocprofv3 --kernel-trace --stats run of bench.py (with a fixed
    --tuning, so that every decode call runs the same kernels) into the
    per-stream duration table of profiles/decode_delta_64Mi_kernel_trace.md:
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

    with open(out_md, "w") as fh:
        fh.write("# Kernel trace: differential decode, 2 x 64Mi-gap streams (bench.py workload)\n\n")
        fh.write("Command (run from the repository root on one MI355X):\n\n")
        fh.write(f"    {command_line}\n\n")
        fh.write("Kernels of one decode call: " + ", ".join(f"`{n}`" for n in names) + ".\n")
        fh.write("Calls alternate between the gap-mean-8 stream and the gap-mean-300 stream "
                 "(first the warm-up steps, then the timed ones).\n\n")
        fh.write("| stream | calls | kernel sum avg us | span avg us | span min us | span max us |\n"
                 "|---|---|---|---|---|---|\n")
        for k, name in enumerate(("gap mean 8", "gap mean 300")):
            cs = calls[k::2]
            if not cs:
                continue
            ksum = [sum(dur(r) for r in c) for c in cs]
            span = [(int(c[-1]["End_Timestamp"]) - int(c[0]["Start_Timestamp"])) / 1e3 for c in cs]
            fh.write(f"| {name} | {len(cs)} | {sum(ksum) / len(ksum):.1f} | {sum(span) / len(span):.1f} | "
                     f"{min(span):.1f} | {max(span):.1f} |\n")
        fh.write("\nPer kernel (average us per call):\n\n| stream | " + " | ".join(names) + " |\n|---|"
                 + "---|" * len(names) + "\n")
        for k, name in enumerate(("gap mean 8", "gap mean 300")):
            cs = calls[k::2]
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
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true", help="skip the config-3 batched comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the config-4 serving run")
    ap.add_argument("--no-decode64", action="store_true", help="skip the 64-bit decode line")
    ap.add_argument("--no-delta4", action="store_true", help="skip the blocks-of-four decode line")
    ap.add_argument("--no-intersect", action="store_true", help="skip the intersection line")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune each stream's tiling first instead of using the library's "
                         "default (two passes, 2 segments x 8 wavefronts)")
    ap.add_argument("--tuning", default=None,
                    help="SEGS,WAVES,CHUNK (both streams) or SEGS,WAVES,CHUNK/SEGS,WAVES,CHUNK "
                         "(gap-mean-8 stream / gap-mean-300 stream): use this tiling and "
                         "single-stream kernel instead of autotuning (profiling runs)")
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
    streams = make_streams(torch, vbyte, workloads)
    alg_bytes = [s["bytes"].numel() + 4 * N_STREAM for s in streams]
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        a = torch.arange(COPY_ELEMS, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # the tiling of each stream picked by the library's autotuner (untimed)
    tunings = []
    fixed = args.tuning.split("/") if args.tuning else []
    for i, s in enumerate(streams):
        if fixed:
            sg, wv, ch = (int(x) for x in fixed[min(i, len(fixed) - 1)].split(","))
            vbyte.set_tuning(sg, wv, 0, tiles_per_chunk=ch)
        elif args.autotune:
            vbyte.autotune_decode(s["bytes"], N_STREAM, delta=True, out=s["out"], reps=3)
        tunings.append(vbyte.get_tuning())
        log(f"stream mean {s['mean']}: tuning {tunings[-1]}")

    def decode_call(i):
        s = streams[i]
        vbyte.set_tuning(**tunings[i])
        vbyte.decode(s["bytes"], N_STREAM, delta=True, prev=0, out=s["out"],
                     status=s["status"], check=False)

    def step(events=None):
        for i in range(len(streams)):
            if events is not None:
                events[i][0].record(stream)
            decode_call(i)
            if events is not None:
                events[i][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    verify(torch, streams)

    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in streams] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    verify(torch, streams)

    kernel_ms = [[evs[k][i][0].elapsed_time(evs[k][i][1]) for k in range(args.steps)]
                 for i in range(len(streams))]
    avg_ms = [sum(v) / len(v) for v in kernel_ms]
    ms_per_step = wall * 1e3 / args.steps
    ints_per_step = N_STREAM * len(streams)
    value = ints_per_step / (ms_per_step / 1e3) / 1e9
    achieved = sum(alg_bytes) / (sum(avg_ms) / 1e3) / 1e9   # GB/s over both launches
    per_stream = []
    for i, s in enumerate(streams):
        per_stream.append({
            "gap_mean": s["mean"], "n": N_STREAM, "bytes_in": int(s["bytes"].numel()),
            "tuning": tunings[i],
            "kernel_ms": round(avg_ms[i], 4),
            "gints_per_s": round(N_STREAM / (avg_ms[i] / 1e3) / 1e9, 2),
            "alg_gbps": round(alg_bytes[i] / (avg_ms[i] / 1e3) / 1e9, 1),
            "pct_hbm_peak": round(100 * alg_bytes[i] / (avg_ms[i] / 1e3) / 1e9 / HBM_PEAK_GBPS, 1),
        })
    traffic = measured_traffic(alg_bytes)
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
        "config": {"workload": "differential VByte decode of two single streams of 64Mi uint32 "
                               "gaps each (geometric gaps, mean 8 and mean 300), wrapping prefix sum",
                   "n_per_stream": N_STREAM, "streams": 2, "gap_means": [8, 300],
                   "tuning": tunings},
        "hbm_gbps": round(achieved, 1),
        "pct_hbm_peak": round(100 * achieved / HBM_PEAK_GBPS, 2),
        "streams": per_stream,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "kernel": "the whole decode call of each stream, all its launches: "
                               + "; ".join(f"mean {s['mean']}: {describe_tuning(t)}"
                                           for s, t in zip(streams, tunings)),
                     "alg_bytes_per_launch": alg_bytes},
    }
    if not args.no_decode64:
        log("64-bit decode ...")
        res["decode64"] = bench_decode64(torch, vbyte, streams)
    if not args.no_delta4:
        log("blocks-of-four decode ...")
        res["delta4"] = bench_delta4(torch, vbyte, streams)
    if not args.no_intersect:
        log("intersection by pieces ...")
        res["intersect"] = bench_intersect(torch, vbyte, streams)
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
        res["cpu_baseline"] = cpu_baseline(streams, args.cpu_budget)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
