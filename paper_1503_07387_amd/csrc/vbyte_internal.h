// Internal definitions shared by the HIP kernels and the C-ABI host layer of
// libvbyte.  Not installed; callers use include/vbyte.h.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "vbyte.h"

namespace vb {

// One wavefront segment: 64 lanes x 16 bytes, loaded with one 128-bit load
// per lane.  A tile is wpb x SEGS consecutive segments decoded by one
// workgroup of wpb wavefronts (SEGS each); it takes one ticket and owns one
// look-back descriptor.
constexpr int kWave = 64;
constexpr int kSegBytes = 1024;
// Per-wavefront LDS rows of one segment: one candidate integer per input
// byte, 16 per lane in rows of 18 words (padding against bank conflicts).
constexpr int kStageWords = 64 * 18;

// Workspace layout: a 256-byte header, then one look-back descriptor per
// tile (or per work item of a batched launch), then batch work tables.
constexpr size_t kHeaderBytes = 512;
// Header bytes [256, 512): the completion counters of the one-launch decode.
constexpr size_t kFlowCtrOff = 256;

// Look-back descriptor of one tile: two self-contained 64-bit words, each
// holding a tag that names the launch, an "inclusive" flag and a payload.
// A tile first publishes its own aggregate (flag 0), later its inclusive
// prefix (flag 1), each time with one 64-bit atomic store per word; a reader
// accepts a descriptor only when both words carry this launch's tag and the
// same flag, so no fence is needed to order a payload against a flag.
//   c: [63:38] tag (26 bits), [37] malformed seen, [36] flag, [35:0] count
//   s: [63:38] tag, [32] flag, [31:0] wrapping uint32 sum
struct Desc {
    uint64_t c;
    uint64_t s;
};
static_assert(sizeof(Desc) == 16, "descriptor is 16 bytes");

constexpr int kTicketWord = 3;   // zero between launches (take_ticket)
// Header word 4: the stall word (epoch + 1 once a look-back of that launch
// gave up).  Look-backs give up after this many round trips that found a
// predecessor not ready (about a second or more); vbyte_set_spin_limit
// changes it for later calls.
constexpr int kStallWord = 4;
constexpr uint32_t kDefaultSpinLimit = 1u << 20;
uint32_t spin_limit();

// Header words: [0] launch epoch, [1] batched large-span queue, [2] batched
// small-chunk queue, [3] tile ticket.  Tiles of a single-stream launch are
// numbered by ticket in the order their workgroups start (so a tile's
// predecessors are running when it looks back); each launch reads the epoch, tags its
// descriptors with it, and the tile that finishes the chain stores epoch+1,
// which retires the launch's descriptors for the next one.  Descriptors carry
// the low 25 bits of the epoch (the one-launch decode's aggregate words the
// low 13 bits), so the host re-zeroes a workspace before 2^13 launches.
constexpr uint64_t kEpochLaunchLimit = (1ull << 13);

struct StreamArgs {
    const uint8_t *base;   // 16-byte aligned, <= bytes
    uint64_t vstart;       // bytes - base (0..15)
    uint64_t vend;         // vstart + nbytes
    uint32_t *out;
    uint64_t n;
    uint32_t prev;
    uint32_t ntiles;
    uint64_t *hdr;
    Desc *desc;
    int32_t *d_status;     // may be null (count mode)
    uint64_t *d_count;     // count mode only
    // Resumable pieces (vbyte_decode_next_async): base/vstart/vend describe
    // the whole buffer; the piece starts at cursor_in[0] (byte offset), its
    // prev is cursor_in[2], it looks at most `window` bytes ahead, and the
    // kernel leaves the byte offset of the code of rank n (relative to the
    // piece) in scratch[0] and the piece's code count in scratch[1].
    const uint64_t *cursor_in;
    uint64_t window;
    uint64_t *scratch;
    uint32_t spin_limit = kDefaultSpinLimit;   // look-back round trips before giving up
    // Block scans only: the number of slots, read on the device when set
    // (written by an earlier kernel), else ntiles, which then bounds it.
    const uint64_t *d_nslots = nullptr;
};

// Single-stream decode in one persistent launch of `grid` workgroups that
// reads the input once (k_flow): tile (k, r) = k * grid + r, s.desc holds one
// tagged aggregate per tile; ctr points at kFlowMaxGroups + 1 completion
// counters (zero between launches).
constexpr int kFlowMaxGroups = 16;
constexpr int kFlowMaxGrid = kFlowMaxGroups * 64;
constexpr int kScheduleFlow = -2;   // the schedule number of the one-launch decode
struct FlowArgs {
    StreamArgs s;
    uint64_t *ctr;
    uint32_t rounds;      // ceil(s.ntiles / grid), set by launch_flow
    uint32_t recompute;   // diagnostic: take every aggregate from the bytes
};

// Single-stream decode of 64-bit codes, in units of
// kUnit64Groups x SEGS segments per wavefront with one 16-byte slot per unit
// in `slots`.
constexpr int kUnit64Groups = 8;
struct Stream64Args {
    const uint8_t *base;   // 16-byte aligned, <= bytes
    uint64_t vstart;       // bytes - base (0..15)
    uint64_t vend;         // vstart + nbytes
    uint64_t *out;
    uint64_t n;
    uint64_t prev;
    uint32_t nunits;
    uint4 *slots;    // per unit: its totals, then its exclusive prefix
    uint4 *gslots;   // per group (kUnit64Groups per unit): the totals of the groups before it in the unit
    int32_t *d_status;
};

// Single-stream decode with differences between blocks of four (y_i = g_i +
// y_(i-4)), in the layout of Stream64Args; a slot is 32 bytes (count and the
// four class sums by rank mod 4).
struct Stream4Args {
    const uint8_t *base;   // 16-byte aligned, <= bytes
    uint64_t vstart;       // bytes - base (0..15)
    uint64_t vend;         // vstart + nbytes
    uint32_t *out;
    uint64_t n;
    uint32_t prev4[4];
    uint32_t nunits;
    uint32_t nblocks;       // aggregate workgroups: block_units units each
    uint32_t block_units;
    uint4 *slots;    // 2 per unit: its exclusive prefix within its block
    uint4 *gslots;   // 2 per group (kUnit64Groups per unit): the summary of the groups before it in the unit
    uint4 *bslots;   // 2 per block: its summary, then its exclusive prefix
    int32_t *d_status;
};

// Intersection consumer of resumable pieces (vbyte_intersect_async).
// List intersection fused with the decode (vbyte_intersect_async).
struct IsectArgs {
    StreamArgs s;           // the list as one differential stream; s.desc: its tile slots
    Desc *mdesc;            // per tile: matches (bit 37: the tile's bytes end a run of five
                            // continuation bytes), then the tile's first output position
    uint64_t na;            // identifiers in the list
    uint64_t piece;         // piece size whose status the call reports
    const uint32_t *b;      // sorted short list
    uint64_t nb;
    uint32_t *out;
    uint64_t out_cap;
    uint64_t *d_count;
    int32_t *d_status;
    uint64_t *total;        // terminators in the stream (from the stream's scan)
    int32_t *scan_status;   // the stream scan's status, and a spare word after it
};
constexpr int kIsectSegs = 2, kIsectWaves = 8;   // the intersection's tiling

// One list of a batched launch, resolved on the device from either CSR
// offsets or gather rows.
// A list item of the batched decode: the list's byte and output ranges, its
// start value and its index (ti is unused, 0; the size stays 48 bytes).
struct BatchItem {
    int64_t bb, be, ob, n;
    uint32_t li, ti, prev, pad;
};
static_assert(sizeof(BatchItem) == 48, "work item is 48 bytes");

struct ListArgs {
    const uint8_t *bytes;
    uint64_t nbytes;           // size of `bytes`; every list must lie inside
    uint64_t nout;             // size of `out` in uint32; every list must lie inside
    const int64_t *byte_off;   // CSR form (nullptr in gather form)
    const int64_t *out_off;    // CSR form
    const int64_t *rows;       // gather form: [nlists][4] (byte_begin, byte_end, out_begin, n)
    uint32_t *out;
    const uint32_t *prevs;     // may be null
    int32_t *list_status;
    uint64_t nlists;
    int delta;
    uint64_t small_bytes;      // lists of at most this many bytes go to the small-list kernel
    uint64_t max_items;        // capacity of the work table
    uint64_t max_large;        // capacity for large-list pieces (items [0, L), L <= max_large)
    uint64_t *hdr;             // header: epoch (word 0), prep ticket (3), stall word (4)
    Desc *desc;                // a slot per large-list piece, then the scan's block totals
    Desc *prep_desc;           // one per prep block
    BatchItem *items;          // work table: a large list's item at its first piece's index,
                               // small lists from the back
    uint32_t *pmap;            // per large-list piece: the index of its list's first piece
    uint64_t *totals;          // [0] large-list pieces L, [1] small lists S, [2] 1 if the
                               // table overflowed, 2 if the prep stalled (written by the
                               // prep kernel); [4] a spare status word
    uint32_t wpb;              // wavefronts per workgroup of the list kernels
    uint32_t spin_limit = kDefaultSpinLimit;   // look-back round trips before giving up
};

// Encoder (k_enc_*): values addressed from the 16-byte-aligned element at
// or below values[0]; chunks of kEncChunk aligned elements.
constexpr uint64_t kEncChunk = 256;
constexpr uint64_t kEncLenChunks = 32;   // chunks per workgroup of the length pass
constexpr uint32_t kEncStageWords = (kEncChunk * 5 + 16 + 3) / 4 + 8;   // a chunk's bytes, 16-byte shifted, zeroed in 16-byte units
struct EncArgs {
    const uint32_t *vbase;   // 16-byte aligned, <= values
    uint64_t e0;             // values - vbase (0..3 elements)
    uint64_t n;
    uint32_t prev;
    int delta;               // 0 values, 1 differences, 2 differences minus one after the first
    uint8_t *bytes;
    uint64_t capacity;
    uint64_t *d_nbytes;
    uint64_t nchunks;        // ceil((e0 + n) / kEncChunk)
    uint32_t *csum;          // per chunk: bytes of its codes
    uint64_t *cpre;          // per chunk: exclusive byte offset
    uint32_t *gsum;          // per k_enc_len workgroup (kEncLenChunks chunks): bytes
};

// Launchers (kernels.hip).
hipError_t launch_stream(const StreamArgs &a, int delta, int count_only, int segs, int wpb,
                         hipStream_t s);
hipError_t launch_batch(const ListArgs &a, int segs, int wpb, int grid_blocks, hipStream_t s);
// Cursor update after a resumable piece (one thread).
hipError_t launch_resume_finish(const uint8_t *bytes, const uint64_t *cursor_in, uint64_t *cursor_out,
                                const uint64_t *scratch, const int32_t *d_status,
                                const uint32_t *out, uint64_t k, uint64_t nbytes, uint64_t window,
                                int delta, hipStream_t s);
// Chunked single-stream decode: a.ntiles tiles in nchunks chunks (one
// descriptor per chunk).
hipError_t launch_chunks(const StreamArgs &a, int delta, int segs, int wpb, uint32_t nchunks,
                         hipStream_t s);
// Single-stream decode in four launches with no look-back: tile aggregates,
// block totals of the tile slots, a scan of every block from the totals
// before it (the last block writes the status), decode with the prefix
// known.  Slots: one per tile, then one per block of kTwoPassScanSpan tiles
// (two_pass_slots).
hipError_t launch_two_pass(const StreamArgs &a, int delta, int segs, int wpb, hipStream_t s);
constexpr uint64_t kTwoPassScanSpan = 2048;
inline uint64_t two_pass_slots(uint64_t ntiles) {
    return ntiles + (ntiles + kTwoPassScanSpan - 1) / kTwoPassScanSpan;
}
// Single-stream decode in one launch of `grid` persistent workgroups (0: as
// many as are resident at once on `cus` compute units; at most
// kFlowMaxGrid), every input byte read once (k_flow); f.rounds is set here.
hipError_t launch_flow(const FlowArgs &f, int delta, int segs, int wpb, int grid, int cus,
                       hipStream_t s);
// 64-bit decode: unit aggregates, a one-workgroup scan (status), decode;
// segs 1 or 2.
hipError_t launch64(const Stream64Args &a, int delta, int segs, int wpb, hipStream_t s);
// Blocks-of-four decode: group and unit summaries, a one-workgroup scan
// (status), decode; segs 1 or 2.
hipError_t launch4(const Stream4Args &a, int segs, int wpb, hipStream_t s);
hipError_t launch_isect(const IsectArgs &a, hipStream_t s);
hipError_t launch_encode(const EncArgs &a, hipStream_t s);
hipError_t launch_encode_bounds(const EncArgs &a, const int64_t *vals_off, int64_t *byte_off,
                                uint64_t nb, hipStream_t s);
hipError_t launch_set_status(int32_t *d_status, int32_t value, hipStream_t s);

// Allocation-free decode (vbyte_decode_noalloc): the two-pass schedule at
// the default tiling with its tile slots (16 bytes each) in a file-scope
// device array of kNoAllocScratchBytes per GPU.  noalloc_scratch returns
// that array's address on the current device (hipGetSymbolAddress, taken
// once per device and kept).
constexpr size_t kNoAllocScratchBytes = (size_t)4 << 20;
constexpr int kNoAllocMaxDevices = 64;
constexpr int kNoAllocSegs = 2, kNoAllocWaves = 8;
hipError_t noalloc_scratch(void **ptr);
hipError_t launch_set_u64(uint64_t *p, uint64_t value, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_fill_i64(int64_t *p, uint64_t n, int64_t value, hipStream_t s);

// Host side of the batched decode (capi.cpp), shared with the graph form.
// batch_plan checks the arguments, fills the work-table sizing fields of
// `a` from the current tuning and lays out the workspace; batch_bind points
// `a` into a workspace of plan.bytes (zero-filled before its first use).
struct BatchPlan {
    size_t bytes, desc_off, prep_off, items_off, pmap_off;
    int segs, wpb, grid;
};
vbyte_status batch_plan(ListArgs &a, size_t list_bytes, BatchPlan *plan);
void batch_bind(ListArgs &a, const BatchPlan &plan, uint8_t *ws);
// Records a HIP failure for vbyte_last_error and returns VBYTE_EHIP.
vbyte_status hip_error(hipError_t e, const char *what);

// Tiles of a single-stream decode of nbytes starting at misalignment vstart.
inline uint64_t stream_tiles(uint64_t vstart, uint64_t nbytes, int segs, int wpb) {
    uint64_t tb = (uint64_t)segs * wpb * kSegBytes;
    return (vstart + nbytes + tb - 1) / tb;
}

constexpr int kPrepBlock = 256;           // lists per prep workgroup
constexpr int kSmallChunk = 64;           // small lists per batched work item
constexpr int kBatchWavesPerCu = 16;      // resident wavefronts per CU of the persistent batched decode

}  // namespace vb
