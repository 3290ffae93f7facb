"""Scalar CPU oracle for VByte coding of uint32 (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports it and
shares no code with it.  The arithmetic lives in ``vbyte_oracle.c`` (plain C,
built with gcc); this module is a ctypes wrapper over numpy arrays.

Every function follows Plaisance, Kurz, Lemire, "Vectorized VByte Decoding":
the byte format of section 1 and Table 1, Algorithm 1 for decoding, and the
differential coding of section 1 / section 4 (inclusive prefix sum mod 2^32),
and the same format for 64-bit integers (section 1; reading R13).
The readings taken where the paper is silent (R1-R15) are listed at the top of
``vbyte_oracle.c``.  All functions are pinned by ``tests/test_oracle_pins.py``.
"""
from .oracle import (  # noqa: F401
    OK, EINVAL, ECOUNT, ETRUNC, EMALFORMED, STATUS_NAMES,
    build, lib_path, code_length, encode, encode_delta, encoded_size, count,
    validate, decode, decode_delta, decode_delta_m1, encode_delta_m1, decode_next, decode_batch,
    code_length64, encoded_size64, encode64, encode_delta64, validate64, decode64, decode64_delta,
    decode_delta4, encode_delta4, intersect_pieces,
)
