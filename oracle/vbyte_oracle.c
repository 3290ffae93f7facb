/*
 * vbyte_oracle.c -- plain scalar CPU oracle for VByte coding of uint32.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the HIP library.
 *
 * Source: Plaisance, Kurz, Lemire, "Vectorized VByte Decoding"
 * (arXiv 1503.07387).
 *
 *   - Byte format (section 1, Table 1): an integer is written 7 bits per
 *     byte, least-significant group first; the top bit of a byte is 1 on
 *     every byte of the code except the last, where it is 0.
 *   - 32-bit scope (section 1): at most 5 bytes per uint32; the fifth byte
 *     carries the top 4 bits (section 4, the 2-integer case).
 *   - Decoder (Algorithm 1): read a byte, finish the integer when the byte
 *     is below 128, otherwise accumulate its low 7 bits at weight 2^(7j).
 *   - Differential coding (section 1, "Differential coding"; section 4,
 *     "Differential Coding"): gaps are successive differences, decoding is
 *     an inclusive prefix sum carried in a 32-bit integer.
 *
 * Readings where the paper is silent:
 *   R1  0 encodes as the single byte 00.
 *   R3  five or more consecutive bytes with the top bit set anywhere in the
 *       buffer -> EMALFORMED (a uint32 code is never longer than 5 bytes).
 *   R4  a fifth byte in [16,128) is accepted; its weight 2^28 wraps mod 2^32
 *       exactly as Algorithm 1 does in 32-bit arithmetic.
 *   R5  over-long codes (e.g. 80 00) are accepted and decode to the sum of
 *       their 7-bit groups.
 *   R11 differences minus one: only differences after the first are
 *       reduced, as in the section's example x_1 - 0, x_2 - x_1 - 1; a
 *       stream continued from an earlier piece passes prev + 1.
 *   R12 a resumable piece of k integers is validated over its window of
 *       5k bytes (or the rest of the buffer); its cursor moves only on
 *       success.
 *   R14 differences between blocks of four (section 1, "Differential
 *       coding": x_1, ..., x_4, x_5 - x_1, x_6 - x_2, ...): y_i = g_i +
 *       y_(i-4) mod 2^32, the four values before the stream given as prev4
 *       (zero for a list coded from its start, which makes x_1..x_4 coded
 *       as themselves); a stream continued from an earlier piece passes the
 *       piece's last four values.
 *   R15 a list intersection consumer of resumable pieces (oracle.py,
 *       intersect_pieces): a failing piece leaves the cursor; the status is
 *       the worst piece status, else ETRUNC for fewer codes than the list's
 *       count, else ECOUNT for bytes left after its last code.
 *   R13 64-bit integers (section 1: the format applies to 64-bit integers
 *       as well): at most 10 bytes per code, the tenth carrying bit 63; ten
 *       or more consecutive continuation bytes -> EMALFORMED; a tenth byte
 *       above 1 is accepted, its weight 2^63 wrapping mod 2^64 (only its
 *       low bit counts); the differential sum wraps mod 2^64.  Truncation
 *       and count statuses as in R6.
 *   R6  exact consumption: the buffer must hold exactly n codes ending at
 *       its last byte; a last byte >= 0x80 or fewer than n terminators ->
 *       ETRUNC, more than n terminators -> ECOUNT.  Precedence when several
 *       apply: EMALFORMED, then ETRUNC, then ECOUNT.
 *   R7  the differential sum wraps mod 2^32.
 *   R8  y_i = y_{i-1} + g_i with y_0 = prev (default 0): inclusive scan.
 *   R9  in a batch every list restarts from its own prev (default 0).
 *
 * Status numbering is fixed by the readings above (a larger data-error code
 * takes precedence): OK 0, EINVAL 1, ECOUNT 2, ETRUNC 3, EMALFORMED 4.
 */
#include <stddef.h>
#include <stdint.h>

enum {
    ORC_OK = 0,
    ORC_EINVAL = 1,
    ORC_ECOUNT = 2,
    ORC_ETRUNC = 3,
    ORC_EMALFORMED = 4
};

/* Code length L(x) from section 1: [0,2^7) -> 1 byte, [2^7,2^14) -> 2 bytes,
 * and so on; a uint32 needs at most 5. */
int orc_code_length(uint32_t x)
{
    if (x < (1u << 7)) return 1;
    if (x < (1u << 14)) return 2;
    if (x < (1u << 21)) return 3;
    if (x < (1u << 28)) return 4;
    return 5;
}

/* ENC(x) (section 1, Table 1): groups of 7 bits, least significant first,
 * top bit set on every byte but the last.  Returns the number of bytes. */
int orc_encode_one(uint32_t x, uint8_t *dst)
{
    int len = orc_code_length(x);
    for (int j = 0; j < len; j++) {
        uint8_t group = (uint8_t)((x >> (7 * j)) & 0x7Fu);
        dst[j] = (j < len - 1) ? (uint8_t)(group | 0x80u) : group;
    }
    return len;
}

/* Concatenation of ENC(x_i) in sequence order.  dst must hold at least
 * orc_encoded_size(x, n) bytes.  Returns the number of bytes written. */
size_t orc_encode(const uint32_t *x, size_t n, uint8_t *dst)
{
    size_t pos = 0;
    for (size_t i = 0; i < n; i++)
        pos += (size_t)orc_encode_one(x[i], dst + pos);
    return pos;
}

size_t orc_encoded_size(const uint32_t *x, size_t n)
{
    size_t total = 0;
    for (size_t i = 0; i < n; i++)
        total += (size_t)orc_code_length(x[i]);
    return total;
}

/* Differential encoding (section 1): write the gaps x_i - x_{i-1} with
 * x_0 = prev, computed mod 2^32 so any uint32 sequence round-trips. */
size_t orc_encode_delta(const uint32_t *x, size_t n, uint32_t prev, uint8_t *dst)
{
    size_t pos = 0;
    uint32_t last = prev;
    for (size_t i = 0; i < n; i++) {
        uint32_t gap = x[i] - last;  /* unsigned: wraps mod 2^32 */
        pos += (size_t)orc_encode_one(gap, dst + pos);
        last = x[i];
    }
    return pos;
}

/* Number of terminator bytes (top bit 0) in the buffer: one per code. */
uint64_t orc_count(const uint8_t *b, size_t nbytes)
{
    uint64_t count = 0;
    for (size_t i = 0; i < nbytes; i++)
        if (b[i] < 128) count++;
    return count;
}

/* Pass 1 of DEC: classify the buffer against n (readings R3, R6). */
int orc_validate(const uint8_t *b, size_t nbytes, size_t n)
{
    int malformed = 0;
    int run = 0;
    uint64_t count = 0;
    for (size_t i = 0; i < nbytes; i++) {
        if (b[i] >= 128) {
            run++;
            if (run >= 5) malformed = 1;
        } else {
            run = 0;
            count++;
        }
    }
    if (malformed) return ORC_EMALFORMED;
    if ((nbytes > 0 && b[nbytes - 1] >= 128) || count < (uint64_t)n)
        return ORC_ETRUNC;
    if (count > (uint64_t)n) return ORC_ECOUNT;
    return ORC_OK;
}

/* Pass 2 of DEC: Algorithm 1, byte by byte, in uint32 arithmetic.  The
 * caller has validated the buffer, so every code ends on a byte below 128
 * within 5 bytes and the loop consumes the buffer exactly. */
static void alg1_decode(const uint8_t *b, size_t n, uint32_t *y)
{
    size_t i = 0;
    for (size_t k = 0; k < n; k++) {
        uint32_t c = 0;
        for (int j = 0; j < 5; j++) {
            uint32_t byte = b[i++];
            if (byte < 128) {
                /* j = 4: weight 2^28, only the low 4 bits survive (R4). */
                y[k] = c + (byte << (7 * j));
                break;
            }
            c = c + ((byte & 0x7Fu) << (7 * j));
        }
    }
}

/* DEC: returns a status; y[0..n) holds the integers when the status is OK
 * and is left untouched otherwise. */
int orc_decode(const uint8_t *b, size_t nbytes, uint32_t *y, size_t n)
{
    int st = orc_validate(b, nbytes, n);
    if (st != ORC_OK) return st;
    alg1_decode(b, n, y);
    return ORC_OK;
}

/* DEC_DELTA: DEC, then the inclusive prefix sum y_i = y_{i-1} + g_i with
 * y_0 = prev, mod 2^32 (R7, R8). */
int orc_decode_delta(const uint8_t *b, size_t nbytes, uint32_t *y, size_t n,
                     uint32_t prev)
{
    int st = orc_decode(b, nbytes, y, n);
    if (st != ORC_OK) return st;
    uint32_t s = prev;
    for (size_t k = 0; k < n; k++) {
        s = s + y[k];
        y[k] = s;
    }
    return ORC_OK;
}

/* Differences minus one (section 1, "Differential coding": for lists with
 * no repeated value, every difference after the first is reduced by one,
 * x_1 - 0, x_2 - x_1 - 1, x_3 - x_2 - 1, ...; reading R11).  Decoding adds
 * the one back: y_0 = prev + g_0 and y_k = y_(k-1) + g_k + 1, mod 2^32. */
int orc_decode_delta_m1(const uint8_t *b, size_t nbytes, uint32_t *y, size_t n,
                        uint32_t prev)
{
    int status = orc_decode(b, nbytes, y, n);
    if (status != ORC_OK) return status;
    uint32_t id = prev;
    for (size_t k = 0; k < n; k++) {
        uint32_t step = y[k] + (k > 0 ? 1u : 0u);
        id = id + step;
        y[k] = id;
    }
    return ORC_OK;
}

/* The matching encoder: gap_0 = x_0 - prev, gap_k = x_k - x_(k-1) - 1. */
size_t orc_encode_delta_m1(const uint32_t *x, size_t n, uint32_t prev, uint8_t *dst)
{
    size_t pos = 0;
    uint32_t last = prev;
    for (size_t i = 0; i < n; i++) {
        uint32_t gap = x[i] - last - (i > 0 ? 1u : 0u);   /* wraps mod 2^32 */
        pos += (size_t)orc_encode_one(gap, dst + pos);
        last = x[i];
    }
    return pos;
}

/* Resumable decode in pieces of at most k integers (section 5 decodes long
 * lists piece by piece into a buffer that stays in cache; reading R12).
 * The piece starts at byte off and looks at the window
 * b[off, off + min(nbytes - off, 5k)), which holds k whole codes whenever
 * the data is well formed (a code has at most 5 bytes):
 *   a run of 5 continuation bytes in the window   -> EMALFORMED
 *   fewer than k codes and the window's last byte continues -> ETRUNC
 *   otherwise the first m = min(k, codes in window) integers are decoded,
 *   *next_off is the byte after the m-th code, *m_out = m, and *next_prev
 *   is the value to pass as prev for the next piece: the last integer
 *   (plus one for differences minus one), or prev if m = 0.
 * delta: 0 plain, 1 differences from prev, 2 differences minus one (the
 * first integer of the piece is prev + g_0).  On an error nothing is
 * written to the outputs. */
int orc_decode_next(const uint8_t *b, size_t nbytes, size_t off, size_t k, uint32_t prev,
                    int delta, uint32_t *y, size_t *next_off, size_t *m_out,
                    uint32_t *next_prev)
{
    if (k == 0 || off > nbytes) return ORC_EINVAL;
    const uint8_t *p = b + off;
    size_t w = nbytes - off;
    if (w / 5 >= k) w = 5 * k;
    int run = 0;
    size_t codes = 0;
    for (size_t i = 0; i < w; i++) {
        if (p[i] >= 128) {
            if (++run >= 5) return ORC_EMALFORMED;
        } else {
            run = 0;
            codes++;
        }
    }
    size_t m = codes < k ? codes : k;
    if (m < k && w > 0 && p[w - 1] >= 128) return ORC_ETRUNC;
    alg1_decode(p, m, y);
    size_t used = 0, seen = 0;
    while (seen < m) {
        if (p[used] < 128) seen++;
        used++;
    }
    uint32_t id = prev;
    for (size_t i = 0; i < m; i++) {
        if (delta == 1) {
            id = id + y[i];
            y[i] = id;
        } else if (delta == 2) {
            id = id + y[i] + (i > 0 ? 1u : 0u);
            y[i] = id;
        }
    }
    *next_off = off + used;
    *m_out = m;
    if (m == 0)
        *next_prev = prev;
    else
        *next_prev = y[m - 1] + (delta == 2 ? 1u : 0u);
    return ORC_OK;
}

/* BATCH (R9): list i is bytes[byte_off[i], byte_off[i+1]) and decodes to
 * out[out_off[i], out_off[i+1]), independently of every other list.
 * prevs may be NULL (all 0).  delta: 0 plain, 1 differences, 2 differences
 * minus one.  list_status[i] receives each list's status.
 * Returns EINVAL for decreasing offsets (nothing decoded), else the largest
 * per-list status. */
int orc_decode_batch(const uint8_t *bytes, const int64_t *byte_off,
                     uint32_t *out, const int64_t *out_off, size_t nlists,
                     const uint32_t *prevs, int delta, int32_t *list_status)
{
    for (size_t i = 0; i < nlists; i++) {
        if (byte_off[i + 1] < byte_off[i] || out_off[i + 1] < out_off[i])
            return ORC_EINVAL;
    }
    int worst = ORC_OK;
    for (size_t i = 0; i < nlists; i++) {
        const uint8_t *b = bytes + byte_off[i];
        size_t nb = (size_t)(byte_off[i + 1] - byte_off[i]);
        size_t n = (size_t)(out_off[i + 1] - out_off[i]);
        uint32_t *y = out + out_off[i];
        uint32_t prev = prevs ? prevs[i] : 0u;
        int st = delta == 2 ? orc_decode_delta_m1(b, nb, y, n, prev)
               : delta ? orc_decode_delta(b, nb, y, n, prev)
                       : orc_decode(b, nb, y, n);
        list_status[i] = st;
        if (st > worst) worst = st;
    }
    return worst;
}

/* Differences between blocks of four (reading R14): y_i = g_i + y_(i-4)
 * mod 2^32, with y_(-4..-1) = prev4[0..3] (all zero when prev4 is NULL). */
int orc_decode_delta4(const uint8_t *b, size_t nbytes, uint32_t *y, size_t n,
                      const uint32_t *prev4)
{
    int st = orc_decode(b, nbytes, y, n);
    if (st != ORC_OK) return st;
    uint32_t back[4] = {0, 0, 0, 0};   /* the value four positions earlier, by i mod 4 */
    if (prev4)
        for (int r = 0; r < 4; r++) back[r] = prev4[r];
    for (size_t i = 0; i < n; i++) {
        uint32_t v = y[i] + back[i % 4];
        back[i % 4] = v;
        y[i] = v;
    }
    return ORC_OK;
}

/* ENC of x_i - x_(i-4) (x_(-4..-1) = prev4, zero when NULL), mod 2^32. */
size_t orc_encode_delta4(const uint32_t *x, size_t n, const uint32_t *prev4, uint8_t *dst)
{
    size_t pos = 0;
    for (size_t i = 0; i < n; i++) {
        uint32_t before = i >= 4 ? x[i - 4] : (prev4 ? prev4[i] : 0u);
        uint32_t g = x[i] - before;
        pos += orc_encode(&g, 1, dst + pos);
    }
    return pos;
}

/* ------------------------------------------------------------------------
 * 64-bit integers (reading R13).  The same byte format with up to ten
 * 7-bit groups; the code length, the encoder, the validation pass and the
 * decoder are written out again for uint64 rather than shared with the
 * 32-bit routines above, so that each can be read against the format on
 * its own.
 * ------------------------------------------------------------------------ */

/* L(x) for uint64: the number of 7-bit groups up to the highest set bit, at
 * least 1; 2^63 and above need 10. */
int orc_code_length64(uint64_t x)
{
    int len = 1;
    while (len < 10 && (x >> (7 * len)) != 0) len++;
    return len;
}

size_t orc_encode64(const uint64_t *x, size_t n, uint8_t *dst)
{
    size_t pos = 0;
    for (size_t i = 0; i < n; i++) {
        int len = orc_code_length64(x[i]);
        for (int j = 0; j < len; j++) {
            uint8_t group = (uint8_t)((x[i] >> (7 * j)) & 0x7Fu);
            dst[pos++] = (j + 1 < len) ? (uint8_t)(group | 0x80u) : group;   /* last: top bit 0 */
        }
    }
    return pos;
}

size_t orc_encoded_size64(const uint64_t *x, size_t n)
{
    size_t total = 0;
    for (size_t i = 0; i < n; i++) total += (size_t)orc_code_length64(x[i]);
    return total;
}

/* Gaps of a uint64 sequence, then ENC: g_0 = x_0 - prev, g_i = x_i - x_(i-1),
 * mod 2^64. */
size_t orc_encode_delta64(const uint64_t *x, size_t n, uint64_t prev, uint8_t *dst)
{
    size_t pos = 0;
    uint64_t last = prev;
    for (size_t i = 0; i < n; i++) {
        uint64_t gap = x[i] - last;
        last = x[i];
        pos += orc_encode64(&gap, 1, dst + pos);
    }
    return pos;
}

/* Validation for 64-bit codes: a run of 10 continuation bytes is
 * malformed; truncation and count as in R6. */
int orc_validate64(const uint8_t *b, size_t nbytes, size_t n)
{
    int malformed = 0;
    int run = 0;
    uint64_t terminators = 0;
    for (size_t i = 0; i < nbytes; i++) {
        if (b[i] & 0x80u) {
            run++;
            if (run >= 10) malformed = 1;
        } else {
            run = 0;
            terminators++;
        }
    }
    if (malformed) return ORC_EMALFORMED;
    if ((nbytes > 0 && (b[nbytes - 1] & 0x80u)) || terminators < (uint64_t)n) return ORC_ETRUNC;
    if (terminators > (uint64_t)n) return ORC_ECOUNT;
    return ORC_OK;
}

/* Algorithm 1 widened to uint64: up to ten groups, group j at weight
 * 2^(7j) mod 2^64. */
int orc_decode64(const uint8_t *b, size_t nbytes, uint64_t *y, size_t n)
{
    int st = orc_validate64(b, nbytes, n);
    if (st != ORC_OK) return st;
    size_t i = 0;
    for (size_t k = 0; k < n; k++) {
        uint64_t acc = 0;
        for (int j = 0; j < 10; j++) {
            uint64_t byte = b[i++];
            acc += (byte & 0x7Fu) << (7 * j);
            if (byte < 128) break;
        }
        y[k] = acc;
    }
    return ORC_OK;
}

/* Differential decode of uint64 gaps: inclusive prefix sum from prev,
 * mod 2^64. */
int orc_decode64_delta(const uint8_t *b, size_t nbytes, uint64_t *y, size_t n, uint64_t prev)
{
    int st = orc_decode64(b, nbytes, y, n);
    if (st != ORC_OK) return st;
    uint64_t run = prev;
    for (size_t k = 0; k < n; k++) {
        run += y[k];
        y[k] = run;
    }
    return ORC_OK;
}
