"""CPU checks of bench.py's host logic: the one-GPU contract, the counter
summary (scaling by the calibration copy, grouping dispatches into decode
calls) and the rule that traffic figures are withdrawn once the kernel
source changes.  Nothing here touches a GPU."""
import csv
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) { return x + 1; }\n")
    b.write_text("// a comment\nint f(int x) {  /* inline */ return x + 1;   }\n\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    hashes = []
    for p in (a, b, c):
        monkeypatch.setattr(bench, "KERNEL_SRC", str(p))
        hashes.append(bench.kernel_source_hash())
    assert hashes[0] == hashes[1] != hashes[2]


def test_traffic_is_withdrawn_when_the_kernels_change(tmp_path, monkeypatch):
    prof = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "PROFILE_COUNTERS", str(prof))
    assert bench.measured_traffic([1, 2]) is None            # no profile
    prof.write_text(json.dumps({"kernel_source_sha256_16": "0" * 16, "hbm_bytes_per_launch": 5.0}))
    assert bench.measured_traffic([1, 2]) is None            # taken on other kernels
    prof.write_text(json.dumps({"kernel_source_sha256_16": bench.kernel_source_hash(),
                                "hbm_bytes_per_launch": 5.0}))
    assert bench.measured_traffic([1, 2]) == 5.0


def write_pmc(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": kib})


def test_counter_summary_scales_by_the_copy_and_groups_calls(tmp_path):
    copy_kib = bench.COPY_ELEMS * 4 / 1024
    agg, scan, known = "void vb::k_tile_agg<1, 2>(x)", "vb::k_tile_block_scan(x)", "void vb::k_known<1, 2>(x)"
    other = "void at::native::elementwise_kernel(x)"
    # FETCH counts half the copy (factor 2); WRITE counts all of it (factor 1)
    fetch = [(bench.COPY_KERNEL, copy_kib / 2), (other, 999.0),
             (agg, 10.0), (scan, 1.0), (known, 20.0),      # call 1: gap mean 8
             (agg, 30.0), (scan, 2.0), (known, 40.0),      # call 2: gap mean 300
             (agg, 12.0), (scan, 1.0), (known, 22.0),      # call 3: gap mean 8
             (agg, 32.0), (scan, 2.0), (known, 42.0)]      # call 4: gap mean 300
    write = [(bench.COPY_KERNEL, copy_kib), (other, 5.0),
             (agg, 0.0), (scan, 1.0), (known, 100.0),
             (agg, 0.0), (scan, 1.0), (known, 200.0),
             (agg, 0.0), (scan, 1.0), (known, 100.0),
             (agg, 0.0), (scan, 1.0), (known, 200.0)]
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    write_pmc(fcsv, "FETCH_SIZE", fetch)
    write_pmc(wcsv, "WRITE_SIZE", write)
    out = bench.summarize_pmc(str(fcsv), str(wcsv), str(tmp_path / "c.json"), str(tmp_path / "c.md"),
                              ["cmd-f", "cmd-w"], kinds=("gap mean 8", "gap mean 300"))
    assert abs(out["fetch_factor"] - 2.0) < 1e-12 and abs(out["write_factor"] - 1.0) < 1e-12
    kib = 1024.0
    p8, p300 = out["per_stream"]
    assert abs(p8["fetch_bytes"] - 2 * kib * (31 + 35) / 2) < 1e-6
    assert abs(p300["fetch_bytes"] - 2 * kib * (72 + 76) / 2) < 1e-6
    assert abs(p8["write_bytes"] - kib * 101) < 1e-6
    assert abs(p300["write_bytes"] - kib * 201) < 1e-6
    assert out["kernel_source_sha256_16"] == bench.kernel_source_hash()
    assert json.load(open(tmp_path / "c.json"))["commands"] == ["cmd-f", "cmd-w"]
    assert "cmd-f" in open(tmp_path / "c.md").read()
    # one kind: every call alike, averaged over all four
    one = bench.summarize_pmc(str(fcsv), str(wcsv), str(tmp_path / "d.json"), str(tmp_path / "d.md"),
                              ["cmd"])
    assert len(one["per_stream"]) == 1 and one["per_stream"][0]["calls"] == 4
    assert abs(one["per_stream"][0]["write_bytes"] - kib * 151) < 1e-6


def test_shards_cut_at_code_boundaries():
    import numpy as np
    import oracle
    x = np.random.default_rng(3).integers(0, 1 << 32, 5000, dtype=np.uint64).astype(np.uint32)
    x[::3] &= 0x7F
    b = oracle.encode(x)
    for parts in (1, 2, 7, 64):
        cuts = bench.shard_starts(b, parts)
        assert cuts[0] == 0 and cuts[-1] == b.size and (np.diff(cuts) >= 0).all()
        got = []
        for k in range(parts):
            sh = b[cuts[k]:cuts[k + 1]]
            assert sh.size == 0 or (sh[-1] < 0x80 and (k == 0 or b[cuts[k] - 1] < 0x80))
            st, y = oracle.decode(sh, oracle.count(sh))
            assert st == oracle.OK
            got.append(y)
        assert np.array_equal(np.concatenate(got), x)
