// Internal definitions shared by the HIP kernels and the C-ABI host layer of
// libvbyte.  Not installed; callers use include/vbyte.h.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace vb {

// One wavefront segment: 64 lanes x 16 bytes, loaded with one 128-bit load
// per lane.  A tile is SEGS consecutive segments decoded by one wavefront.
constexpr int kWave = 64;
constexpr int kSegBytes = 1024;
// Per-wavefront LDS staging for one segment's outputs: at most one integer
// per input byte, plus up to 3 slots to align global stores to 16 bytes.
constexpr int kStageWords = 1040;

// Workspace layout: a 256-byte header, then one look-back descriptor per
// tile (or per work item of a batched launch), then batch work tables.
constexpr size_t kHeaderBytes = 256;

// Look-back descriptor of one tile.  Each word is self-contained (a tag that
// names the launch, a flag and a payload), published with one 64-bit atomic
// store and read with one 64-bit atomic load, so no fence orders a payload
// against a flag.
//   c_*: [63:38] tag (26 bits), [37] malformed seen, [36:0] count
//   s_*: [57:32] tag, [31:0] wrapping uint32 sum
// *_agg hold the tile's own aggregate, *_inc the inclusive prefix up to and
// including the tile.
struct Desc {
    uint64_t c_agg;
    uint64_t s_agg;
    uint64_t c_inc;
    uint64_t s_inc;
};
static_assert(sizeof(Desc) == 32, "descriptor is 32 bytes");

// The header word holds (epoch << 32) | ticket.  Every launch takes exactly
// a known number of tickets; the wavefront that takes the last one stores
// ((epoch + 1) << 32), which both resets the ticket counter and retires the
// descriptors of this launch for the next one.  Descriptors carry the low 25
// bits of the epoch, so the host re-zeroes a workspace before 2^24 launches.
constexpr uint64_t kEpochLaunchLimit = (1ull << 24);

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
};

// One list of a batched launch, resolved on the device from either CSR
// offsets or gather rows.
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
    uint64_t small_bytes;      // lists of at most this many bytes take one wavefront
    uint64_t max_items;        // capacity of the work table / descriptor array
    uint64_t *hdr;             // persistent-queue header (ticket word)
    Desc *desc;                // one per work item
    Desc *prep_desc;           // one per prep block
    int2 *items;               // work table: (list, tile) per item
    uint64_t *totals;          // [0] large items, [1] all items, [2] 1 if the table overflowed
    uint32_t nwaves;           // wavefronts of the persistent launch
};

struct EncodeArgs {
    const uint32_t *values;
    uint64_t n;
    uint32_t prev;
    int delta;
    uint8_t *bytes;
    uint64_t capacity;
    uint64_t *d_nbytes;
    uint32_t ntiles;
    uint64_t *hdr;
    Desc *desc;
};

// Launchers (kernels.hip).
hipError_t launch_stream(const StreamArgs &a, int delta, int count_only, int segs, int wpb,
                         hipStream_t s);
hipError_t launch_batch(const ListArgs &a, int segs, int wpb, int grid_blocks, hipStream_t s);
hipError_t launch_encode(const EncodeArgs &a, hipStream_t s);
hipError_t launch_set_status(int32_t *d_status, int32_t value, hipStream_t s);
hipError_t launch_set_u64(uint64_t *p, uint64_t value, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);

// Tiles of a single-stream decode of nbytes starting at misalignment vstart.
inline uint64_t stream_tiles(uint64_t vstart, uint64_t nbytes, int segs) {
    uint64_t tb = (uint64_t)segs * kSegBytes;
    return (vstart + nbytes + tb - 1) / tb;
}

constexpr int kEncodeWaveValues = 1024;   // values per encoder tile (one wavefront)
constexpr int kPrepBlock = 256;           // lists per prep workgroup

}  // namespace vb
