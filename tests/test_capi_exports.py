"""CPU checks of the boundary: libvbyte builds, loads, and exports every
symbol that include/vbyte.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vbyte.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vbyte_[a-z0-9_]+)\s*\(", text)))


def _lib_path():
    from paper_1503_07387_amd import vbyte
    if not os.path.exists(vbyte.LIB_PATH):
        from paper_1503_07387_amd import build
        build.build()
    return vbyte.LIB_PATH


def test_header_declares_expected_calls():
    names = declared_functions()
    for must in ("vbyte_decode", "vbyte_decode_delta", "vbyte_decode_batch", "vbyte_count"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_header():
    from paper_1503_07387_amd import vbyte
    assert sorted(vbyte.EXPORTS) == declared_functions()


def test_exported_symbols_are_c_linkage():
    out = subprocess.run(["nm", "-D", "--defined-only", _lib_path()], capture_output=True,
                         text=True, check=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in declared_functions():
        assert n in syms, n


def test_status_strings_without_gpu():
    from paper_1503_07387_amd import vbyte
    lib = vbyte.load(_lib_path())
    for code, name in vbyte.STATUS_NAMES.items():
        assert lib.vbyte_status_str(code).decode() == name


def test_tuning_argument_checks_without_gpu():
    from paper_1503_07387_amd import vbyte
    lib = vbyte.load(_lib_path())
    assert lib.vbyte_set_tuning(3, 0, 0) == vbyte.EINVAL
    assert lib.vbyte_set_tuning(0, 9, 0) == vbyte.EINVAL
    assert lib.vbyte_set_tuning(0, 0, -1) == vbyte.EINVAL
    assert lib.vbyte_set_tuning(0, 0, 0) == vbyte.OK


def test_header_status_numbers_match_oracle_readings():
    # the oracle defines its own numbers (it shares no header with the
    # library); both follow the precedence EMALFORMED > ETRUNC > ECOUNT
    import oracle
    text = open(HEADER).read()
    nums = dict((k, int(v)) for k, v in re.findall(r"VBYTE_(\w+)\s*=\s*(\d+)", text))
    assert nums["OK"] == oracle.OK and nums["ECOUNT"] == oracle.ECOUNT
    assert nums["ETRUNC"] == oracle.ETRUNC and nums["EMALFORMED"] == oracle.EMALFORMED
    assert nums["EINVAL"] == oracle.EINVAL


def test_status_numbers_are_fixed():
    # the numbering is part of the ABI: data errors ordered by precedence
    # (ECOUNT < ETRUNC < EMALFORMED), the binding's constants the same
    from paper_1503_07387_amd import vbyte
    text = open(HEADER).read()
    text = text[text.index("typedef enum vbyte_status {"):text.index("} vbyte_status;")]
    nums = dict((k, int(v)) for k, v in re.findall(r"VBYTE_(\w+)\s*=\s*(\d+)", text))
    want = {"OK": 0, "EINVAL": 1, "ECOUNT": 2, "ETRUNC": 3, "EMALFORMED": 4, "EHIP": 5,
            "ENOMEM": 6, "ESTALLED": 7}
    assert nums == want
    for k, v in want.items():
        assert getattr(vbyte, k) == v
    lib = vbyte.load(_lib_path())
    for k, v in want.items():
        assert lib.vbyte_status_str(v).decode() == "VBYTE_" + k


def test_workspace_size_covers_every_single_stream_form():
    # the 32-bit decode's 16-byte tile descriptors, the 64-bit decode's
    # 16-byte unit and group slots and the blocks-of-four decode's 32-byte
    # unit, group and block slots, at the smallest tiles (1 KiB segments,
    # one wavefront per workgroup, 15 bytes of misalignment)
    from paper_1503_07387_amd import vbyte
    lib = vbyte.load(_lib_path())
    import ctypes as C
    segs, wpb, small = C.c_int(), C.c_int(), C.c_int64()
    lib.vbyte_get_tuning(C.byref(segs), C.byref(wpb), C.byref(small))
    try:
        assert lib.vbyte_set_tuning(1, 1, 0) == vbyte.OK
        prev = 0
        for nbytes in (0, 1, 1023, 8192, 123457, 1 << 20, 111_023_732):
            ws = lib.vbyte_workspace_size(nbytes)
            tiles = -(-(15 + nbytes) // 1024)
            units = -(-(15 + nbytes) // 8192)
            assert ws >= 256 + 16 * tiles
            assert ws >= 256 + 16 * 9 * units
            assert ws >= 256 + 32 * (9 * units + units)
            assert ws >= prev
            prev = ws
    finally:
        lib.vbyte_set_tuning(segs.value, wpb.value, small.value)


def test_tuning_defaults_from_the_environment():
    """VBYTE_* variables set the process-wide defaults when the library is
    loaded (no GPU call involved); out-of-range values are ignored."""
    import subprocess
    import sys
    code = ("import ctypes, sys; sys.path.insert(0, %r); from paper_1503_07387_amd import vbyte; "
            "L = vbyte.load(); s, w, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64(); "
            "L.vbyte_get_tuning(ctypes.byref(s), ctypes.byref(w), ctypes.byref(m)); "
            "print(s.value, w.value, m.value, L.vbyte_get_chunk_tiles())") % ROOT
    def run(env):
        e = dict(os.environ)
        e.update(env)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=e, timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        return [int(t) for t in r.stdout.split()]
    base = run({})
    assert base == [2, 8, 16384, -1]
    assert run({"VBYTE_SEGS_PER_WAVE": "4", "VBYTE_WAVES_PER_BLOCK": "4",
                "VBYTE_SMALL_LIST_BYTES": "2048", "VBYTE_SCHEDULE": "-2"}) == [4, 4, 2048, -2]
    assert run({"VBYTE_SEGS_PER_WAVE": "3", "VBYTE_WAVES_PER_BLOCK": "9",
                "VBYTE_SMALL_LIST_BYTES": "x", "VBYTE_SCHEDULE": "65"}) == base
