"""Plant plausible mistakes in copies of the oracle (CPU only) and check that
the pins catch every one of them.

Each mutant is the oracle source with one textual change, compiled with gcc
into a temporary directory and exercised in a child process, so a mutant that
misbehaves cannot take the test run down.  The real oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "vbyte_oracle.c")

# (name, original text, mutated text); each original must occur exactly once.
MUTANTS = [
    ("enc_shift_8", "((x >> (7 * j)) & 0x7Fu)", "((x >> (8 * j)) & 0x7Fu)"),
    ("enc_cont_on_last", "(j < len - 1) ? (uint8_t)(group | 0x80u)", "(j < len) ? (uint8_t)(group | 0x80u)"),
    ("len_threshold_14", "if (x < (1u << 14)) return 2;", "if (x < (1u << 15)) return 2;"),
    ("len_threshold_28", "if (x < (1u << 28)) return 4;", "if (x < (1u << 27)) return 4;"),
    ("dec_shift_8", "c = c + ((byte & 0x7Fu) << (7 * j));", "c = c + ((byte & 0x7Fu) << (8 * j));"),
    ("dec_drop_mask", "c = c + ((byte & 0x7Fu) << (7 * j));", "c = c + (byte << (7 * j));"),
    ("dec_four_bytes", "for (int j = 0; j < 5; j++) {", "for (int j = 0; j < 4; j++) {"),
    ("dec_terminator_le", "if (byte < 128) {\n                /*", "if (byte <= 128) {\n                /*"),
    ("val_run6", "if (run >= 5) malformed = 1;", "if (run >= 6) malformed = 1;"),
    ("val_no_lastbyte", "if ((nbytes > 0 && b[nbytes - 1] >= 128) || count < (uint64_t)n)",
     "if (count < (uint64_t)n)"),
    ("val_swap_trunc_count", "if (count > (uint64_t)n) return ORC_ECOUNT;", "if (count > (uint64_t)n) return ORC_ETRUNC;"),
    ("count_le", "if (b[i] < 128) count++;", "if (b[i] <= 128) count++;"),
    ("delta_no_prev", "uint32_t s = prev;", "uint32_t s = 0;"),
    ("delta_exclusive", "s = s + y[k];\n        y[k] = s;", "uint32_t g = y[k];\n        y[k] = s;\n        s = s + g;"),
    ("delta_sign", "s = s + y[k];", "s = s - y[k];"),
    ("encdelta_sign", "uint32_t gap = x[i] - last;", "uint32_t gap = last - x[i];"),
    ("batch_no_prev", "uint32_t prev = prevs ? prevs[i] : 0u;", "uint32_t prev = 0u;"),
    ("m1_first_too", "uint32_t step = y[k] + (k > 0 ? 1u : 0u);", "uint32_t step = y[k] + 1u;"),
    ("m1_no_one", "uint32_t step = y[k] + (k > 0 ? 1u : 0u);", "uint32_t step = y[k];"),
    ("encm1_first_too", "uint32_t gap = x[i] - last - (i > 0 ? 1u : 0u);", "uint32_t gap = x[i] - last - 1u;"),
    ("next_window_4k", "if (w / 5 >= k) w = 5 * k;", "if (w / 4 >= k) w = 4 * k;"),
    ("next_cursor_plus1", "*next_off = off + used;", "*next_off = off + used + 1;"),
    ("next_m1_first", "id = id + y[i] + (i > 0 ? 1u : 0u);", "id = id + y[i] + 1u;"),
    ("next_prev_no_one", "*next_prev = y[m - 1] + (delta == 2 ? 1u : 0u);", "*next_prev = y[m - 1];"),
    ("next_trunc_ignored", "if (m < k && w > 0 && p[w - 1] >= 128) return ORC_ETRUNC;", "(void)0;"),
    ("batch_m1_as_delta", "int st = delta == 2 ? orc_decode_delta_m1(b, nb, y, n, prev)",
     "int st = delta == 3 ? orc_decode_delta_m1(b, nb, y, n, prev)"),
    ("batch_no_einval", "return ORC_EINVAL;\n    }\n    int worst", "(void)0;\n    }\n    int worst"),
    ("d4_stride2", "uint32_t v = y[i] + back[i % 4];\n        back[i % 4] = v;",
     "uint32_t v = y[i] + back[i % 2];\n        back[i % 2] = v;"),
    ("d4_no_prev", "for (int r = 0; r < 4; r++) back[r] = prev4[r];", "(void)0;"),
    ("d4_prev_reversed", "for (int r = 0; r < 4; r++) back[r] = prev4[r];",
     "for (int r = 0; r < 4; r++) back[r] = prev4[3 - r];"),
    ("encd4_stride3", "uint32_t before = i >= 4 ? x[i - 4] : (prev4 ? prev4[i] : 0u);",
     "uint32_t before = i >= 3 ? x[i - 3] : (prev4 ? prev4[i] : 0u);"),
    ("len64_nine", "while (len < 10 && (x >> (7 * len)) != 0) len++;",
     "while (len < 9 && (x >> (7 * len)) != 0) len++;"),
    ("enc64_shift_8", "uint8_t group = (uint8_t)((x[i] >> (7 * j)) & 0x7Fu);",
     "uint8_t group = (uint8_t)((x[i] >> (8 * j)) & 0x7Fu);"),
    ("val64_run9", "if (run >= 10) malformed = 1;", "if (run >= 9) malformed = 1;"),
    ("val64_run11", "if (run >= 10) malformed = 1;", "if (run >= 11) malformed = 1;"),
    ("dec64_nine_groups", "for (int j = 0; j < 10; j++) {\n            uint64_t byte",
     "for (int j = 0; j < 9; j++) {\n            uint64_t byte"),
    ("dec64_keep_top", "acc += (byte & 0x7Fu) << (7 * j);", "acc += byte << (7 * j);"),
    ("dec64_32bit_acc", "uint64_t acc = 0;\n        for (int j = 0; j < 10; j++)",
     "uint32_t acc = 0;\n        for (int j = 0; j < 10; j++)"),
    ("delta64_no_prev", "uint64_t run = prev;", "uint64_t run = 0;"),
    ("enc64_cont_on_last", "dst[pos++] = (j + 1 < len) ? (uint8_t)(group | 0x80u) : group;",
     "dst[pos++] = (j < len) ? (uint8_t)(group | 0x80u) : group;"),
    ("size64_skip_first", "for (size_t i = 0; i < n; i++) total += (size_t)orc_code_length64(x[i]);",
     "for (size_t i = 1; i < n; i++) total += (size_t)orc_code_length64(x[i]);"),
    ("size64_len32", "total += (size_t)orc_code_length64(x[i]);",
     "total += (size_t)orc_code_length((uint32_t)x[i]);"),
    ("encdelta64_sign", "uint64_t gap = x[i] - last;", "uint64_t gap = last - x[i];"),
]

RUNNER = r"""
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle.oracle as oo
import pins
lib = oo.load({lib!r})
for p in pins.ALL_PINS:
    try:
        p(lib)
    except AssertionError:
        print("CAUGHT", p.__name__)
        sys.exit(0)
print("SURVIVED")
sys.exit(0)
"""


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, orig, mut):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor for {name} not unique"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(orig, mut))
    mlib = str(tmp_path / "libmutant.so")
    oracle.build(src=str(msrc), out=mlib, extra_flags=("-w",))
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=mlib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    # a crash of the mutant also counts as caught, but say so
    assert "SURVIVED" not in out, f"mutant {name} passed every pin"
    assert r.returncode == 0 or r.returncode < 0 or "CAUGHT" in out
