/* Host-side check of the CPU oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure, built and run by
 * tests/test_oracle_sanitizers.py with gcc): random 32- and 64-bit values of
 * every code length round-trip through every encoder and decoder of the
 * oracle, and random byte buffers (runs of continuation bytes, cut tails,
 * wrong counts) go through every decoder, each input in a heap buffer of
 * exactly its size, so that a read or write past either end is reported.
 * Exits 0 when every round trip holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_code_length(uint32_t x);
size_t orc_encode(const uint32_t *x, size_t n, uint8_t *dst);
size_t orc_encoded_size(const uint32_t *x, size_t n);
size_t orc_encode_delta(const uint32_t *x, size_t n, uint32_t prev, uint8_t *dst);
size_t orc_encode_delta_m1(const uint32_t *x, size_t n, uint32_t prev, uint8_t *dst);
size_t orc_encode_delta4(const uint32_t *x, size_t n, const uint32_t *prev4, uint8_t *dst);
uint64_t orc_count(const uint8_t *b, size_t nbytes);
int orc_decode(const uint8_t *b, size_t nbytes, uint32_t *y, size_t n);
int orc_decode_delta(const uint8_t *b, size_t nbytes, uint32_t *y, size_t n, uint32_t prev);
int orc_decode_delta_m1(const uint8_t *b, size_t nbytes, uint32_t *y, size_t n, uint32_t prev);
int orc_decode_delta4(const uint8_t *b, size_t nbytes, uint32_t *y, size_t n, const uint32_t *prev4);
int orc_decode_next(const uint8_t *b, size_t nbytes, size_t off, size_t k, uint32_t prev, int delta,
                    uint32_t *y, size_t *next_off, size_t *m_out, uint32_t *next_prev);
int orc_decode_batch(const uint8_t *bytes, const int64_t *byte_off, uint32_t *out,
                     const int64_t *out_off, size_t nlists, const uint32_t *prevs, int delta,
                     int32_t *list_status);
size_t orc_encode64(const uint64_t *x, size_t n, uint8_t *dst);
size_t orc_encoded_size64(const uint64_t *x, size_t n);
size_t orc_encode_delta64(const uint64_t *x, size_t n, uint64_t prev, uint8_t *dst);
int orc_decode64(const uint8_t *b, size_t nbytes, uint64_t *y, size_t n);
int orc_decode64_delta(const uint8_t *b, size_t nbytes, uint64_t *y, size_t n, uint64_t prev);

static uint64_t s_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) {   /* xorshift64* */
    s_state ^= s_state >> 12;
    s_state ^= s_state << 25;
    s_state ^= s_state >> 27;
    return s_state * 0x2545F4914F6CDD1Dull;
}
static uint32_t rnd_value(void) {   /* code length uniform in 1..5 */
    const int l = 1 + (int)(rnd() % 5);
    const uint64_t lo = l == 1 ? 0 : 1ull << (7 * (l - 1));
    const uint64_t hi = l == 5 ? (1ull << 32) : 1ull << (7 * l);
    return (uint32_t)(lo + rnd() % (hi - lo));
}
static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) exit(3);
    return p;
}
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(void) {
    for (int it = 0; it < 3000; ++it) {
        const size_t n = rnd() % 300;
        uint32_t *x = xmalloc(n * 4);
        for (size_t i = 0; i < n; ++i) x[i] = rnd_value();
        const size_t nb = orc_encoded_size(x, n);
        uint8_t *b = xmalloc(nb);
        CHECK(orc_encode(x, n, b) == nb);
        CHECK(orc_count(b, nb) == n);
        uint32_t *y = xmalloc(n * 4);
        CHECK(orc_decode(b, nb, y, n) == 0);
        CHECK(n == 0 || memcmp(x, y, n * 4) == 0);
        /* differential forms: x as identifiers */
        uint8_t *bd = xmalloc(5 * n);
        const uint32_t prev = (uint32_t)rnd();
        const size_t nd = orc_encode_delta(x, n, prev, bd);
        CHECK(nd <= 5 * n);
        CHECK(orc_decode_delta(bd, nd, y, n, prev) == 0);
        CHECK(n == 0 || memcmp(x, y, n * 4) == 0);
        const size_t nm = orc_encode_delta_m1(x, n, prev, bd);
        CHECK(orc_decode_delta_m1(bd, nm, y, n, prev) == 0);
        CHECK(n == 0 || memcmp(x, y, n * 4) == 0);
        const uint32_t p4[4] = {(uint32_t)rnd(), (uint32_t)rnd(), 0u, 7u};
        const size_t n4 = orc_encode_delta4(x, n, p4, bd);
        CHECK(orc_decode_delta4(bd, n4, y, n, p4) == 0);
        CHECK(n == 0 || memcmp(x, y, n * 4) == 0);
        /* resumable pieces of k integers over the plain stream */
        if (n) {
            const size_t k = 1 + rnd() % 40;
            uint32_t *piece = xmalloc(k * 4);
            size_t off = 0, done = 0, m = 0;
            uint32_t pv = 0, npv = 0;
            while (done < n) {
                size_t noff = 0;
                CHECK(orc_decode_next(b, nb, off, k, pv, 0, piece, &noff, &m, &npv) == 0);
                CHECK(m > 0 && done + m <= n + k);
                for (size_t i = 0; i < m && done + i < n; ++i) CHECK(piece[i] == x[done + i]);
                done += m;
                off = noff;
                pv = npv;
            }
            free(piece);
        }
        /* a batch of three lists cut from the stream at code boundaries */
        {
            int64_t bo[4], oo[4];
            const size_t c1 = n ? rnd() % (n + 1) : 0, c2 = c1 + (n - c1 ? rnd() % (n - c1 + 1) : 0);
            oo[0] = 0; oo[1] = (int64_t)c1; oo[2] = (int64_t)c2; oo[3] = (int64_t)n;
            for (int q = 0; q < 4; ++q) bo[q] = (int64_t)orc_encoded_size(x, (size_t)oo[q]);
            int32_t ls[3];
            CHECK(orc_decode_batch(b, bo, y, oo, 3, NULL, 0, ls) == 0);
            CHECK(n == 0 || memcmp(x, y, n * 4) == 0);
        }
        /* 64-bit values */
        {
            uint64_t *x64 = xmalloc(n * 8), *y64 = xmalloc(n * 8);
            for (size_t i = 0; i < n; ++i) x64[i] = rnd() >> (rnd() % 64);
            const size_t n64 = orc_encoded_size64(x64, n);
            uint8_t *b64 = xmalloc(n64);
            CHECK(orc_encode64(x64, n, b64) == n64);
            CHECK(orc_decode64(b64, n64, y64, n) == 0);
            CHECK(n == 0 || memcmp(x64, y64, n * 8) == 0);
            uint8_t *bd64 = xmalloc(10 * n);
            const size_t nd64 = orc_encode_delta64(x64, n, 5, bd64);
            CHECK(orc_decode64_delta(bd64, nd64, y64, n, 5) == 0);
            CHECK(n == 0 || memcmp(x64, y64, n * 8) == 0);
            free(x64); free(y64); free(b64); free(bd64);
        }
        /* random bytes through every decoder: statuses only, no overruns */
        {
            const size_t rb = rnd() % 64;
            uint8_t *r = xmalloc(rb);
            for (size_t i = 0; i < rb; ++i) r[i] = (uint8_t)(rnd() % 4 ? rnd() | 0x80 : rnd() & 0x7F);
            const size_t rn = rnd() % 40;
            uint32_t *ry = xmalloc(rn * 4);
            uint64_t *ry64 = xmalloc(rn * 8);
            (void)orc_decode(r, rb, ry, rn);
            (void)orc_decode_delta(r, rb, ry, rn, 3);
            (void)orc_decode_delta_m1(r, rb, ry, rn, 3);
            (void)orc_decode_delta4(r, rb, ry, rn, NULL);
            (void)orc_decode64(r, rb, ry64, rn);
            (void)orc_decode64_delta(r, rb, ry64, rn, 9);
            if (rn) {
                size_t no = 0, mo = 0;
                uint32_t np = 0;
                (void)orc_decode_next(r, rb, rb ? rnd() % rb : 0, rn, 0, (int)(rnd() % 3), ry, &no, &mo, &np);
            }
            (void)orc_count(r, rb);
            free(r); free(ry); free(ry64);
        }
        free(x); free(b); free(y); free(bd);
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
