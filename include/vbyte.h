/*
 * vbyte.h -- C ABI of libvbyte, VByte decoding of uint32 on AMD Instinct
 * MI355X (gfx950).
 *
 * The operation is the one of Plaisance, Kurz, Lemire, "Vectorized VByte
 * Decoding" (arXiv 1503.07387):
 *   - byte format, section 1 and Table 1: an integer is written 7 bits per
 *     byte, least-significant group first; the top bit of a byte is 1 on
 *     every byte of a code except its last ("terminator", top bit 0); a
 *     uint32 takes 1 to 5 bytes;
 *   - decoding, Algorithm 1 (the conventional decoder): each terminator ends
 *     one integer, the value is the sum of the 7-bit groups at weights
 *     2^0, 2^7, 2^14, 2^21, 2^28, in uint32 arithmetic;
 *   - differential coding, section 1 ("Differential coding") and section 4
 *     ("Differential Coding"): the stream holds gaps; decoding adds each gap
 *     to the last value decoded, carried in a 32-bit integer.
 *
 * Conventions shared by every call below.
 *   Memory.  Every data pointer (bytes, out, offsets, prevs, status words)
 *     is a DEVICE pointer on the current HIP device, allocated and owned by
 *     the caller; the library never frees or retains it.  `bytes` may have
 *     any alignment; `out` must be 4-byte aligned; inputs and outputs must
 *     not overlap.  The library keeps its own device workspace per
 *     (device, stream), grown on demand; it frees it at process exit.
 *   Streams.  `stream` is a hipStream_t passed as void*; NULL means the null
 *     stream.  Work is enqueued in stream order; calls on one stream are
 *     ordered, calls on different streams are independent (each stream has
 *     its own workspace).
 *   Threads.  Calls may come from several host threads.  A call that uses
 *     a stream's workspace holds that (device, stream)'s lock from its first
 *     look at the workspace to its last enqueue, and a synchronous call until
 *     it returns, so calls on one stream from two threads are serialised and
 *     never share descriptors or a status slot while in flight.  The tuning
 *     set by vbyte_set_* and the autotuners is process-wide; changing it
 *     while another thread decodes changes that thread's next call.
 *   Strict semantics (the paper is silent on these).  A stream is valid iff
 *     bytes[0..nbytes) is exactly n codes ending at its last byte:
 *       VBYTE_EMALFORMED  five or more consecutive bytes >= 0x80 anywhere;
 *       VBYTE_ETRUNC      last byte >= 0x80, or fewer than n terminators;
 *       VBYTE_ECOUNT      more than n terminators.
 *     When several hold, the larger code wins (EMALFORMED > ETRUNC >
 *     ECOUNT), the same classification as the CPU oracle.  A fifth byte in
 *     [16,128) is accepted and wraps mod 2^32; over-long codes such as
 *     80 00 are accepted.
 *   Errors.  Argument errors (VBYTE_EINVAL) are returned before anything is
 *     enqueued.  Data errors of *_async calls land in the caller's device
 *     status word, written once by the kernel (no zero-initialisation
 *     needed) and valid after the stream reaches that point; synchronous
 *     calls wait and return them.  On a data error out[0..n) is
 *     unspecified, but no element outside out[0..n) is ever written and no
 *     16-byte block that holds no byte of bytes[0..nbytes) is ever read;
 *     bytes outside the stream never influence a result.
 *   Limits.  nbytes < 2^36.
 */
#ifndef VBYTE_H
#define VBYTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  The three data errors are numbered by precedence,
 * VBYTE_ECOUNT 2 < VBYTE_ETRUNC 3 < VBYTE_EMALFORMED 4, so that the status of
 * a stream with several faults, and the worst status of a batch, is the
 * numerically largest one.  This differs from an earlier draft of this
 * interface that numbered them in the order a decoder meets them
 * (ETRUNC 2, EMALFORMED 3, ECOUNT 4): compare against the names, never
 * against literal numbers.  The values below are fixed by this header. */
typedef enum vbyte_status {
    VBYTE_OK = 0,
    VBYTE_EINVAL = 1,      /* bad argument: NULL pointer, misaligned out, size limit, bad offsets */
    VBYTE_ECOUNT = 2,      /* more terminators than n */
    VBYTE_ETRUNC = 3,      /* last byte >= 0x80 or fewer terminators than n */
    VBYTE_EMALFORMED = 4,  /* a run of >= 5 continuation bytes */
    VBYTE_EHIP = 5,        /* a HIP runtime call failed */
    VBYTE_ENOMEM = 6,      /* workspace allocation failed */
    VBYTE_ESTALLED = 7     /* a look-back gave up waiting (vbyte_set_spin_limit): output unreliable */
} vbyte_status;

/* ------------------------------------------------------------ single stream */

/* DEC (Algorithm 1): decode n uint32 from bytes[0..nbytes) into out[0..n).
 * Synchronous on the null stream: returns the data status. */
vbyte_status vbyte_decode(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n);

/* DEC_DELTA (section 1 "Differential coding", section 4 "Differential
 * Coding"): out[i] = prev + g_0 + ... + g_i mod 2^32, where g_i are the
 * decoded gaps; prev is the value before the first gap (0 for a list coded
 * from x_1 - 0), or the last value of a previous part of the same stream,
 * which makes decoding resumable.  Synchronous on the null stream. */
vbyte_status vbyte_decode_delta(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                uint32_t prev);

/* Asynchronous forms of the two calls above, enqueued on `stream`.
 * d_status: device int32 that receives the vbyte_status of the data. */
vbyte_status vbyte_decode_async(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                int32_t *d_status, void *stream);
vbyte_status vbyte_decode_delta_async(const uint8_t *bytes, size_t nbytes, uint32_t *out,
                                      size_t n, uint32_t prev, int32_t *d_status, void *stream);

/* Kernel tuning of one single-stream decode, for vbyte_decode_ex.  A call
 * that passes its own tuning is unaffected by the process-wide defaults
 * (vbyte_set_tuning, vbyte_set_chunk_tiles, vbyte_set_flow_grid), so calls
 * on different streams, or threads, can use different tilings at once.
 *   segs_per_wave    1 KiB segments per wavefront of a tile: 1, 2 or 4
 *   waves_per_block  wavefronts per workgroup (a tile): 1 .. 8
 *   schedule         how tiles learn their prefix (count of integers and
 *                    gap sum of the stream before them):
 *                    VBYTE_SCHED_ONE_READ  one persistent launch, every
 *                        input byte read once: each tile's aggregate is
 *                        published as soon as its bytes arrive and the tile
 *                        is decoded two rounds later from registers;
 *                    VBYTE_SCHED_TWO_PASS  tile aggregates, a one-workgroup
 *                        scan, then the decode (the input is read twice);
 *                    VBYTE_SCHED_LOOKBACK  one launch, a decoupled look-back
 *                        per tile;
 *                    k = 1..64  chunks of k tiles per workgroup
 *   grid             VBYTE_SCHED_ONE_READ only: workgroups (0 = 16
 *                    wavefronts per compute unit; at most 512)
 *   recompute        VBYTE_SCHED_ONE_READ only, diagnostic: 1 makes every
 *                    workgroup compute the aggregates it needs from the
 *                    bytes instead of reading them (same result, slower);
 *                    0 otherwise */
typedef struct vbyte_tuning {
    int segs_per_wave;
    int waves_per_block;
    int schedule;
    int grid;
    int recompute;
} vbyte_tuning;

enum {
    VBYTE_SCHED_ONE_READ = -2,
    VBYTE_SCHED_TWO_PASS = -1,
    VBYTE_SCHED_LOOKBACK = 0
};

/* DEC, DEC_DELTA or differences minus one (mode 0, 1, 2; see
 * vbyte_decode_async, vbyte_decode_delta_async, vbyte_decode_delta_m1_async)
 * with an explicit tuning (NULL = the process-wide defaults).  Arguments,
 * statuses and ownership as in vbyte_decode_async; VBYTE_EINVAL for a
 * tuning field out of range, a mode outside 0..2 or d_status NULL. */
vbyte_status vbyte_decode_ex(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                             uint32_t prev, int mode, const vbyte_tuning *tuning, int32_t *d_status,
                             void *stream);

/* Fills *t with the current process-wide defaults. */
void vbyte_tuning_default(vbyte_tuning *t);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * decode of vbyte_decode_ex (mode 0 plain, 1 differential, 2 differences
 * minus one) with the two-pass schedule at the default tiling (2 segments x
 * 8 wavefronts), whose tile slots live in a fixed device array of 4 MiB per
 * GPU inside the library instead of the per-stream workspace.  It calls no
 * hipMalloc, hipFree or other allocating routine.  Limit: 262,016 tiles of
 * 16 KiB (one 16-byte slot per tile plus one per 2048 tiles), i.e. nbytes
 * (plus the misalignment of `bytes`, 0..15) just under 4 GiB (4,292,870,144
 * bytes); larger streams get VBYTE_EINVAL (with vbyte_last_error saying so)
 * before anything is enqueued.  Every call on a GPU shares that GPU's array:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must be serialised by the caller; calls on one stream are ordered.
 * The array needs no initialisation (every slot a call reads it writes
 * first).  Asynchronous: data errors land in d_status (required). */
vbyte_status vbyte_decode_noalloc(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                  uint32_t prev, int mode, int32_t *d_status, void *stream);

/* Differences minus one (section 1, "Differential coding": with no repeated
 * value, every difference after the first is coded less one, x_1 - 0,
 * x_2 - x_1 - 1, ...): out[0] = prev + g_0 and out[i] = out[i-1] + g_i + 1
 * mod 2^32, i.e. out[i] = prev + g_0 + ... + g_i + i.  To continue a stream
 * decoded in parts, pass the previous part's last value plus one as prev.
 * Arguments and errors as in vbyte_decode_delta(_async). */
vbyte_status vbyte_decode_delta_m1(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                   uint32_t prev);
vbyte_status vbyte_decode_delta_m1_async(const uint8_t *bytes, size_t nbytes, uint32_t *out,
                                         size_t n, uint32_t prev, int32_t *d_status,
                                         void *stream);

/* Differences between blocks of four (section 1, "Differential coding":
 * x_1, x_2, x_3, x_4, x_5 - x_1, x_6 - x_2, ...): out[i] = g_i + out[i-4]
 * mod 2^32, the four values before the stream taken from prev4[0..3] (a
 * host array; NULL means zeros, which decodes a list coded from its start).
 * To continue a stream decoded in parts, pass the last four values of the
 * previous part.  Arguments, statuses and the synchronous/asynchronous
 * split otherwise as in vbyte_decode_delta(_async).  Uses at most 2
 * segments per wavefront of the current tuning. */
vbyte_status vbyte_decode_delta4(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                 const uint32_t *prev4);
vbyte_status vbyte_decode_delta4_async(const uint8_t *bytes, size_t nbytes, uint32_t *out,
                                       size_t n, const uint32_t *prev4, int32_t *d_status,
                                       void *stream);

/* 64-bit integers (section 1: the format applies to 64-bit integers too).
 * A code has at most 10 bytes, the tenth carrying bit 63; ten consecutive
 * continuation bytes are VBYTE_EMALFORMED; a tenth byte above 1 is accepted
 * and only its low bit counts (its weight 2^63 wraps mod 2^64); the
 * differential form is out[i] = prev + g_0 + ... + g_i mod 2^64.
 *   bytes: device, any alignment; out: device uint64[n], 8-byte aligned.
 * Statuses, exact consumption, precedence and the synchronous/asynchronous
 * split as in vbyte_decode(_async); nothing is written outside out[0..n)
 * and no byte outside bytes[0..nbytes) is read.  Uses at most 2 segments
 * per wavefront of the current tuning. */
vbyte_status vbyte_decode64(const uint8_t *bytes, size_t nbytes, uint64_t *out, size_t n);
vbyte_status vbyte_decode64_delta(const uint8_t *bytes, size_t nbytes, uint64_t *out, size_t n,
                                  uint64_t prev);
vbyte_status vbyte_decode64_async(const uint8_t *bytes, size_t nbytes, uint64_t *out, size_t n,
                                  int32_t *d_status, void *stream);
vbyte_status vbyte_decode64_delta_async(const uint8_t *bytes, size_t nbytes, uint64_t *out,
                                        size_t n, uint64_t prev, int32_t *d_status, void *stream);

/* Resumable decode in pieces (section 5 decodes long lists piece by piece
 * into a buffer that stays in cache): each call decodes the next piece of at
 * most k integers of bytes[0..nbytes) into out[0..k), starting where the
 * cursor *d_in points, and writes the advanced cursor to *d_out.  Both
 * cursors live in device memory and the call never synchronizes, so a
 * caller can chain pieces (alternating two cursors) with a consumer of
 * out[] between them.
 *   vbyte_cursor: byte_offset = first byte of the piece; decoded = integers
 *     decoded by all pieces so far; prev = the start value of the piece's
 *     differences (low 32 bits; set it to the list's prev before the first
 *     piece).  On success the piece's integers are out[0..m) with
 *     m = d_out->decoded - d_in->decoded; m < k only at the end of the data.
 *   delta: 0 plain, 1 differences, 2 differences minus one.
 *   d_status: device int32: VBYTE_OK, or VBYTE_EMALFORMED for a run of 5
 *     continuation bytes within the piece's window of 5k bytes,
 *     VBYTE_ETRUNC when the data ends inside a code before k integers,
 *     VBYTE_EINVAL when the cursor lies past nbytes; on an error *d_out is
 *     a copy of *d_in.
 * d_in and d_out must differ.  Pieces of one stream must run in order (one
 * stream).  Always uses one look-back per tile, and at most 2 segments per
 * wavefront whatever vbyte_set_tuning chose. */
typedef struct vbyte_cursor {
    uint64_t byte_offset;
    uint64_t decoded;
    uint64_t prev;
} vbyte_cursor;
vbyte_status vbyte_decode_next_async(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t k,
                                     int delta, const vbyte_cursor *d_in, vbyte_cursor *d_out,
                                     int32_t *d_status, void *stream);

/* List intersection with the decode fused into its consumer (section 5
 * decodes long lists into a buffer that stays in cache and consumes them
 * from there; here the buffer is the registers of the workgroup that decodes
 * a tile, so the list's identifiers are never written out).  Every
 * identifier of the differential list a (na identifiers, from a_prev) that
 * occurs in the sorted array b[0..nb) is written, in list order, to out.
 * Two passes over a's bytes give each tile its rank and running identifier
 * (as the two-pass decode); each tile is then decoded twice, once to count
 * its matches and, after a scan of the counts, once to store them.  Each
 * identifier is tested by a binary search in the window of b between the
 * smallest and largest identifiers of its wavefront, held in LDS when it
 * has at most 1152 entries.
 *   a: device bytes; b, out: device uint32, 4-byte aligned; b sorted
 *   ascending (duplicates allowed), nb < 2^32.  Every identifier of a that
 *   occurs in b is kept (duplicates in a too).
 *   *d_count (device uint64): the number of matches; only out[0..out_cap)
 *   is written, so a count above out_cap means matches were dropped.
 *   *d_status (device int32): the status that decoding a in pieces of
 *   `piece` integers (vbyte_decode_next_async from the start, a failing
 *   piece leaving the cursor) gives: the worst piece status, else
 *   VBYTE_ETRUNC when a holds fewer than na codes, else VBYTE_ECOUNT when
 *   codes or bytes remain after its na-th code, else VBYTE_OK.  VBYTE_OK
 *   holds exactly when a is na well-formed codes.  On a data error out and
 *   *d_count are unspecified.
 *   piece: 1 .. 2^26 integers; it changes only the status of a bad list.
 *   Workspace: 32 bytes per 16 KiB of a, per stream.
 * Returns VBYTE_EINVAL for bad arguments before enqueuing anything. */
vbyte_status vbyte_intersect_async(const uint8_t *a, size_t a_nbytes, size_t na, uint32_t a_prev,
                                   const uint32_t *b, size_t nb, size_t piece, uint32_t *out,
                                   size_t out_cap, uint64_t *d_count, int32_t *d_status,
                                   void *stream);

/* Number of terminator bytes (top bit 0) in bytes[0..nbytes), i.e. the
 * number of codes a valid stream holds (section 1: one terminator per
 * integer).  Written to the device word *d_count. */
vbyte_status vbyte_count(const uint8_t *bytes, size_t nbytes, uint64_t *d_count, void *stream);

/* ------------------------------------------------------------ batched lists */

/* Batched CSR decode of posting lists (section 1: each list of sorted
 * document identifiers is coded independently, from x_1 - 0).  List i is
 * bytes[byte_off[i], byte_off[i+1]) and decodes to out[out_off[i],
 * out_off[i+1]) with n_i = out_off[i+1] - out_off[i] integers.
 *   bytes, nbytes: the byte array that holds every list (device).
 *   byte_off, out_off: device int64[nlists+1].  A list whose byte range
 *     leaves [0, nbytes), whose output range leaves [0, nout), or whose
 *     offsets decrease gets VBYTE_EINVAL and is not decoded (checked on the
 *     device, so nothing outside the buffers is touched).
 *   out, nout: output array of nout uint32 (device).
 *   prevs: device uint32[nlists] start values for delta lists, or NULL (0).
 *   delta: 0 plain, 1 differential, 2 differences minus one (each list as
 *     in vbyte_decode_delta_m1 with its own prev).
 *   d_list_status: device int32[nlists], required; receives each list's
 *     status under the strict semantics above.
 * A small prep kernel classifies the lists and builds a work table.  Lists
 * larger than small_list_bytes (vbyte_set_tuning) are cut into pieces of
 * segs_per_wave KiB, one wavefront each, and decoded in two passes with no
 * look-back, as a single stream: each piece's count and byte sum, one scan
 * over all pieces, then each piece decodes with its prefix within its list
 * (a list of one piece skips the first pass).  A last launch decodes the
 * smaller lists, several to a wavefront (each on its own lanes) when they
 * fit in 64 x 16 bytes, else one wavefront each.  Asynchronous on
 * `stream`. */
vbyte_status vbyte_decode_batch(const uint8_t *bytes, size_t nbytes, const int64_t *byte_off,
                                uint32_t *out, size_t nout, const int64_t *out_off, size_t nlists,
                                const uint32_t *prevs, int delta, int32_t *d_list_status,
                                void *stream);

/* Gather form of the batch, for lists that are not adjacent in memory (the
 * serving loop decodes the lists of several queries out of a resident
 * index; a list may appear more than once).
 *   lists: device int64[nlists][4] rows (byte_begin, byte_end, out_begin, n);
 *     list i is bytes[byte_begin, byte_end) and decodes to
 *     out[out_begin, out_begin + n).
 *   list_bytes: an upper bound on the sum of byte_end - byte_begin over the
 *     rows; it sizes the work table.  If the rows need more, every list
 *     gets VBYTE_EINVAL.
 * Everything else as in vbyte_decode_batch. */
vbyte_status vbyte_decode_lists(const uint8_t *bytes, size_t nbytes, const int64_t *lists,
                                size_t nlists, size_t list_bytes, uint32_t *out, size_t nout,
                                const uint32_t *prevs, int delta, int32_t *d_list_status,
                                void *stream);

/* The batched decode captured once into a HIP graph and replayed: a replay
 * enqueues the same two kernels as vbyte_decode_batch with the arguments
 * given here, so callers that run the same batch shape repeatedly (a fixed
 * index, new contents in the same buffers) pay one graph launch per batch.
 *   Arguments as in vbyte_decode_batch; the pointers and sizes are fixed at
 *   creation and their contents are read at each replay.
 *   *graph receives the handle; the graph owns a workspace of its own,
 *   allocated here (VBYTE_ENOMEM if that fails), so replays allocate
 *   nothing.  The tuning in force at creation is baked in.
 * vbyte_batch_graph_launch enqueues one replay on `stream` (asynchronous);
 * replays of one graph must not overlap (enqueue them on one stream or
 * order them).  vbyte_batch_graph_destroy frees the graph; the caller
 * synchronizes first.  Errors: VBYTE_EINVAL for bad arguments, VBYTE_EHIP
 * when capture or launch fails. */
typedef struct vbyte_batch_graph vbyte_batch_graph;
vbyte_status vbyte_batch_graph_create(const uint8_t *bytes, size_t nbytes, const int64_t *byte_off,
                                      uint32_t *out, size_t nout, const int64_t *out_off,
                                      size_t nlists, const uint32_t *prevs, int delta,
                                      int32_t *d_list_status, vbyte_batch_graph **graph);
vbyte_status vbyte_batch_graph_launch(vbyte_batch_graph *graph, void *stream);
void vbyte_batch_graph_destroy(vbyte_batch_graph *graph);

/* ------------------------------------------------------------ serving */

/* Continuous-batching request loop over an index resident in HBM.  A
 * request asks for the decoded posting lists of several terms; its result is
 * the concatenation, in term order, of those lists, each decoded on its own
 * (differential lists restart from 0: section 1).  The loop releases
 * requests at their arrival times, admits them FIFO when the device output
 * pool has room for their result, and launches every admitted request on an
 * idle stream as one vbyte_decode_lists batch; batches on different streams
 * overlap on the GPU.  With batching = 0 each list is one single-stream
 * launch instead (the per-list baseline). */
typedef struct vbyte_server vbyte_server;

typedef struct vbyte_server_config {
    size_t pool_bytes;       /* device output pool (admission budget) */
    int nstreams;            /* 1..8 streams for overlapping batches */
    int max_batch_requests;  /* requests per launch, at most */
    int batching;            /* 1: one batched launch per batch; 0: one launch per list */
    int delta;               /* 1: differential decode */
} vbyte_server_config;

typedef struct vbyte_serve_stats {
    double wall_s;               /* first arrival origin to last completion */
    uint64_t integers;           /* integers decoded for admitted requests */
    uint64_t batches;
    uint64_t launches;           /* decode launches issued */
    double mean_batch_requests;
    int32_t worst_status;        /* largest per-list status seen (VBYTE_OK if all good) */
    uint64_t rejected;           /* requests larger than the whole pool */
} vbyte_serve_stats;

/* index_bytes: device pointer to the whole index (nbytes); byte_off: HOST
 * int64[nlists+1] list boundaries; counts: HOST int64[nlists] integers per
 * list.  The server copies the host metadata and allocates the pool, the
 * streams and pinned staging; vbyte_server_destroy releases them. */
vbyte_status vbyte_server_create(const uint8_t *index_bytes, size_t nbytes, const int64_t *byte_off,
                                 const int64_t *counts, size_t nlists,
                                 const vbyte_server_config *cfg, vbyte_server **out);
void vbyte_server_destroy(vbyte_server *server);

/* Open-loop run of nreq requests (HOST arrays): request r arrives
 * arrival_s[r] seconds after the start (non-decreasing) and asks for lists
 * terms[term_off[r] .. term_off[r+1]).  latency_s[r] (HOST) receives
 * completion minus arrival on the host steady clock, or -1 if the request
 * could never fit the pool; with batching, a request completes when the
 * last of its own lists is decoded (the batched kernel decodes small lists
 * first and stamps each request's completion in host memory), else when
 * its batch's launches end.  req_status (HOST int32[nreq], may be NULL)
 * receives each request's status: the largest status of its lists, or
 * VBYTE_ENOMEM for a request larger than the pool.  If results (DEVICE
 * uint32) is not NULL, request r's result is copied to
 * results[result_off[r] ..] (result_off: HOST int64[nreq]).  Blocks until
 * every request has completed. */
vbyte_status vbyte_server_run(vbyte_server *server, size_t nreq, const double *arrival_s,
                              const int64_t *term_off, const int64_t *terms, double *latency_s,
                              int32_t *req_status, uint32_t *results, const int64_t *result_off,
                              vbyte_serve_stats *stats);

/* ------------------------------------------------------------ encoder */

/* ENC (section 1, Table 1) on the GPU: writes the concatenated canonical
 * codes of values[0..n) to bytes[0..*d_nbytes).  capacity is the size of
 * `bytes`; 5*n always suffices.  If the codes need more than capacity
 * bytes, nothing past capacity is written and *d_nbytes receives the size
 * that was needed.  d_nbytes: device uint64. */
vbyte_status vbyte_encode_async(const uint32_t *values, size_t n, uint8_t *bytes, size_t capacity,
                                uint64_t *d_nbytes, void *stream);

/* Differential ENC (section 1): encodes the gaps x_i - x_{i-1} mod 2^32
 * with x_{-1} = prev. */
vbyte_status vbyte_encode_delta_async(const uint32_t *values, size_t n, uint32_t prev,
                                      uint8_t *bytes, size_t capacity, uint64_t *d_nbytes,
                                      void *stream);

/* ENC of differences minus one: x_0 - prev, then x_i - x_{i-1} - 1, mod
 * 2^32 (the inverse of vbyte_decode_delta_m1). */
vbyte_status vbyte_encode_delta_m1_async(const uint32_t *values, size_t n, uint32_t prev,
                                         uint8_t *bytes, size_t capacity, uint64_t *d_nbytes,
                                         void *stream);

/* Batched ENC for CSR lists: encodes values[0..n) (all lists concatenated;
 * list i is values[vals_off[i], vals_off[i+1])) in one pass and writes the
 * byte offset of every list boundary to byte_off[0..nlists] (device int64),
 * so that list i's codes are bytes[byte_off[i], byte_off[i+1]).  Plain
 * encoding: for differential lists, pass the gaps.  vals_off: device int64,
 * non-decreasing, values > n are clamped to n. */
vbyte_status vbyte_encode_batch(const uint32_t *values, size_t n, const int64_t *vals_off,
                                size_t nlists, uint8_t *bytes, size_t capacity, int64_t *byte_off,
                                uint64_t *d_nbytes, void *stream);

/* ------------------------------------------------------------ utilities */

/* Bytes of device workspace that a single-stream call (32-bit, 64-bit or
 * blocks-of-four decode) on nbytes input uses at most under the current
 * tuning.  The library allocates and keeps one workspace per stream; this
 * reports its size, it allocates nothing. */
size_t vbyte_workspace_size(size_t nbytes);

/* Tuning knobs of the decode kernels (0 keeps a value unchanged):
 * segs_per_wave: 1 KiB segments one wavefront decodes per tile (1, 2, 4);
 * waves_per_block: wavefronts per workgroup (1..8);
 * small_list_bytes: lists up to this size take the small-list path in the
 * batched forms.  Returns VBYTE_EINVAL for an unsupported value.
 * The process-wide defaults (2, 8, 16384, the two-pass schedule, a spin
 * limit of 2^20) can also be set from the environment when the library is
 * loaded: VBYTE_SEGS_PER_WAVE, VBYTE_WAVES_PER_BLOCK, VBYTE_SMALL_LIST_BYTES,
 * VBYTE_SCHEDULE (as vbyte_set_chunk_tiles) and VBYTE_SPIN_LIMIT; values
 * out of range are ignored. */
vbyte_status vbyte_set_tuning(int segs_per_wave, int waves_per_block, int64_t small_list_bytes);
void vbyte_get_tuning(int *segs_per_wave, int *waves_per_block, int64_t *small_list_bytes);

/* Kernel of the single-stream decodes (vbyte_decode*, not the batched
 * forms): -2 (VBYTE_SCHED_ONE_READ) decodes in one persistent launch that
 * reads every input byte once (see vbyte_tuning); its waits are bounded (an
 * aggregate not published in time is computed from the bytes by the
 * reader), so it needs neither a ticket nor co-resident workgroups.
 * -1 (the default) decodes in two passes, four launches, with no
 * look-back: every tile's terminator count and byte sum, a scan of them
 * (block totals, then every block of 2048 tiles from the totals before it),
 * then every tile with its prefix known (the input is read twice; no
 * workgroup ever waits for another); 0 gives every tile its own
 * look-back; k in 1..64 gives each workgroup a chunk of k consecutive
 * tiles, which it first reads for their counts and sums, then looks back
 * once for the chunk, then reads again and decodes.  The look-back kernels
 * number their tiles by an atomic ticket, so they are safe next to any
 * other work on the device, at the cost of that atomic.  Returns
 * VBYTE_EINVAL outside -2..64. */
vbyte_status vbyte_set_chunk_tiles(int tiles_per_chunk);
int vbyte_get_chunk_tiles(void);

/* Bound of the look-back waits (the look-back, chunked and resumable-piece
 * decodes, the batched decode and the encoder): a tile that has read its
 * predecessors' descriptors `rounds` times without finding one ready gives
 * up, and the call reports VBYTE_ESTALLED (its output is then unreliable;
 * vbyte_count reports a count of UINT64_MAX) instead of waiting forever.
 * The tickets that number the tiles make every wait end in practice; the
 * bound guards against a lost predecessor.  0 restores the default
 * (2^20 round trips, a second or more).  A status written by the last tile
 * before a stall elsewhere was seen can still read VBYTE_OK only if the
 * stalled tile's predecessor published in the instant between; the stalled
 * tile then overwrites it with VBYTE_ESTALLED when it finishes.  Applies to
 * calls enqueued afterwards; for testing the bound, a small value makes
 * tiles give up quickly. */
vbyte_status vbyte_set_spin_limit(uint32_t rounds);

/* Workgroups of the one-launch decode (schedule -2) by default: 0 (the
 * default) gives 16 wavefronts per compute unit; at most 512.  Returns
 * VBYTE_EINVAL outside 0..512. */
vbyte_status vbyte_set_flow_grid(int grid);

/* Autotuner of the tiling.  Times the caller's workload under each candidate
 * tiling (reps calls each after one untimed call, HIP events on `stream`),
 * then applies the fastest with vbyte_set_tuning and returns VBYTE_OK.
 *   vbyte_autotune_decode: single-stream decode of bytes[0, nbytes) into
 *     out[0, n) (plain or delta, prev 0); d_status is a device int32 the
 *     calls write.  Candidates: segs_per_wave {2, 4} x waves_per_block
 *     {4, 8} x tiles_per_chunk {-1, 0, 2, 4, 8, 16}.
 *   vbyte_autotune_batch: vbyte_decode_batch of the given lists (prevs 0);
 *     d_list_status is device int32[nlists].  Candidates: segs_per_wave
 *     {2, 4} x waves_per_block {4, 8} x small_list_bytes {1, 4, 16, 64} KiB.
 *   points, max_points: optional host array that receives each candidate
 *     and its mean time; *npoints (optional) the number written.
 * If the workload does not decode (a data status other than VBYTE_OK) that
 * status is returned and the previous tuning is restored.  The tuning is
 * process-wide: run no other decode meanwhile.  Synchronous. */
typedef struct vbyte_tune_point {
    int segs_per_wave;
    int waves_per_block;
    int64_t small_list_bytes;
    int tiles_per_chunk;
    double ms;        /* mean time of one call */
    int32_t status;   /* worst data status the timed calls produced */
} vbyte_tune_point;
vbyte_status vbyte_autotune_decode(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                   int delta, int reps, int32_t *d_status,
                                   vbyte_tune_point *points, size_t max_points, size_t *npoints,
                                   void *stream);
vbyte_status vbyte_autotune_batch(const uint8_t *bytes, size_t nbytes, const int64_t *byte_off,
                                  uint32_t *out, size_t nout, const int64_t *out_off,
                                  size_t nlists, int delta, int reps, int32_t *d_list_status,
                                  vbyte_tune_point *points, size_t max_points, size_t *npoints,
                                  void *stream);

/* Static name of a status code. */
const char *vbyte_status_str(vbyte_status st);

/* Text of the last HIP error seen by this thread (after VBYTE_EHIP). */
const char *vbyte_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VBYTE_H */
