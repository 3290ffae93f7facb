// kernels.hip -- gfx950 (MI355X) kernels of libvbyte: VByte decoding of
// uint32 (plain and differential, differences minus one), terminator
// counting, encoding, the batched / persistent decode of many posting
// lists, resumable decoding in pieces with a list-intersection consumer,
// differences between blocks of four, and 64-bit integers.
//
// Method: Plaisance, Kurz, Lemire, "Vectorized VByte Decoding".  The byte
// format is that of section 1 / Table 1; a code ends at its terminator byte
// (top bit 0) and its value is the sum of its 7-bit groups at weights
// 2^(7j) in uint32 arithmetic (Algorithm 1).  Differential decoding is an
// inclusive prefix sum of the gaps carried in 32 bits (section 1,
// "Differential coding"; section 4, "Differential Coding").
//
// GPU design (the paper's x86 Masked VByte is prior art, not the design):
//  * A wavefront owns tiles of SEGS x 1 KiB.  Each lane loads 16 bytes of a
//    segment with one 128-bit load; the dword before a lane's 16 bytes and
//    the dword after them come from the neighbouring lanes by DPP (at the
//    wavefront's ends from 4-byte halo loads).  Codes are at most 5 bytes,
//    so the 4 bytes after a lane complete any code that begins in it (the
//    paper's decoder likewise relies on a segment beginning with a whole
//    code, section 4).
//  * The terminator mask of a lane's 16 bytes plays the role of the paper's
//    pmovmskb continuation mask (complemented).  A lane owns the integers
//    whose code begins in its bytes (the byte before is a terminator); their
//    count is a popcount and the wave sum gives the segment's count.
//  * Ranks across tiles come, by default, from two passes: per-tile
//    terminator counts and byte sums that need no decoding, one scan over
//    the tiles, then the decode with each tile's prefix given (the input is
//    read twice, nothing waits).  The one-launch alternative is a decoupled
//    look-back over per-tile descriptors (tile count, tile gap sum,
//    malformed flag), tiles numbered by an atomic ticket; the batched decode
//    and the resumable pieces use it.
//  * Each lane evaluates Algorithm 1's sum for every byte position at once,
//    in Horner form from its last byte down, so that each code's integer is
//    left at the code's first byte (the fifth group's weight 2^28 wraps mod
//    2^32 like Algorithm 1).  The wavefront writes one candidate per byte to
//    LDS and stores each 64-byte row of the segment with one masked store of
//    consecutive words, the slots given by mbcnt over the row's mask.
//  * The differential form keeps lane-local suffix sums during assembly and
//    adds a wave scan of lane sums, the tile's exclusive prefix sum and the
//    caller's start value, all mod 2^32 (the wave-level counterpart of the
//    4-wide shift-and-add prefix sum of section 4).
//  * Descriptor words are published and read with relaxed agent-scope 64-bit
//    atomics that bypass the per-XCD L2, so no cache-flushing fence is
//    needed between tiles on different XCDs.

#include <atomic>
#include <mutex>

#include "vbyte_internal.h"
#include "vbyte.h"

namespace vb {
namespace {

typedef uint8_t u8;
typedef uint32_t u32;
typedef uint64_t u64;
typedef int64_t i64;
// pointers into global memory (address space 1), for stores addressed as
// scalar base + 32-bit offset
typedef __attribute__((address_space(1))) u8 gbyte;
typedef __attribute__((address_space(1))) u32 gword;

constexpr u64 kCountMask = (1ull << 36) - 1;
constexpr int kLookbackWindows = 4;   // most 64-descriptor windows read per round trip

// ------------------------------------------------------------------ atomics
__device__ __forceinline__ u64 aload(const u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(u64 *p, u64 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 aadd(u64 *p, u64 v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tiles of a look-back launch are numbered in the order their workgroups
// (or wavefronts) start, by an atomic ticket: a tile then only ever waits
// for tiles whose tickets running workgroups already hold, whatever else
// the device is running (a workgroup index would not do: with other
// kernels resident, a later index can start while an earlier one waits for
// room on another XCD).  The taker of the last ticket resets the counter
// for the next launch on this workspace; no ticket is taken after it.
__device__ __forceinline__ u32 take_ticket(u64 *ctr, u64 total) {
    const u64 t = aadd(ctr, 1);
    if (t == total - 1) astore(ctr, 0);
    return (u32)t;
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ u32 lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ u32 first_lane(u32 v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ u32 read_lane(u32 v, u32 l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ u64 ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ u32 dpp_zero(u32 x) {
    return (u32)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, true);
}

// Inclusive wave64 prefix sum, mod 2^32: four row shifts inside each row of
// 16 lanes, then row broadcasts of lanes 15 and 31.
__device__ __forceinline__ u32 wave_scan(u32 x) {
    x += dpp_zero<0x111>(x);        // row_shr:1
    x += dpp_zero<0x112>(x);        // row_shr:2
    x += dpp_zero<0x114>(x);        // row_shr:4
    x += dpp_zero<0x118>(x);        // row_shr:8
    x += dpp_zero<0x142, 0xA>(x);   // row_bcast:15 -> rows 1, 3
    x += dpp_zero<0x143, 0xC>(x);   // row_bcast:31 -> rows 2, 3
    return x;
}
__device__ __forceinline__ u32 wave_sum(u32 x) { return read_lane(wave_scan(x), 63); }

// Value of lane-1 (wave_shr:1); lane 0 receives `lane0`.
__device__ __forceinline__ u32 from_lane_below(u32 x, u32 lane0) {
    return (u32)__builtin_amdgcn_update_dpp((int)lane0, (int)x, 0x138, 0xF, 0xF, false);
}
// Value of lane+1 (wave_shl:1); lane 63 receives `lane63`.
__device__ __forceinline__ u32 from_lane_above(u32 x, u32 lane63) {
    return (u32)__builtin_amdgcn_update_dpp((int)lane63, (int)x, 0x130, 0xF, 0xF, false);
}

// LDS written by some lanes of a wavefront and read by others: LDS
// instructions of one wavefront execute in order, so a compiler barrier at
// wavefront scope is all that is needed.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ descriptors
// c word: [63:38] tag, [37] malformed seen, [36] inclusive flag, [35:0] count
// s word: [63:38] tag, [32] inclusive flag, [31:0] wrapping sum
__device__ __forceinline__ u32 make_tag(u32 epoch) { return (1u << 25) | (epoch & 0x1FFFFFFu); }
__device__ __forceinline__ u64 pack_c(u32 tag, bool inc, bool mal, u64 c) {
    return ((u64)tag << 38) | ((u64)(mal ? 1 : 0) << 37) | ((u64)(inc ? 1 : 0) << 36) | (c & kCountMask);
}
__device__ __forceinline__ u64 pack_s(u32 tag, bool inc, u32 s) {
    return ((u64)tag << 38) | ((u64)(inc ? 1 : 0) << 32) | s;
}

// Publish a tile's aggregate (inc = false) or inclusive prefix (inc = true):
// the sum word first, the count word last.
template <bool SUM>
__device__ __forceinline__ void publish(Desc *d, u32 tag, bool inc, bool mal, u64 c, u32 s) {
    if (SUM) astore(&d->s, pack_s(tag, inc, s));
    astore(&d->c, pack_c(tag, inc, mal, c));
}

struct Prefix {
    u64 c;
    u32 s;
    bool mal;
    bool stalled;   // the look-back gave up after its round limit (the prefix is wrong)
};

// Decoupled look-back: exclusive prefix of descriptor `idx` over the chain
// that starts at descriptor `first` (which always publishes an inclusive
// value).  Each round trip reads nw windows of 64 predecessors (one per lane
// per window, two 64-bit atomic loads each), then walks them nearest first:
// aggregates are summed until an inclusive prefix ends the walk; a
// predecessor that has published nothing yet (or is between its two stores)
// stops the walk and the remaining ones are read again.  A round that walks
// a whole window without meeting an inclusive prefix widens the next round
// to kLookbackWindows windows, so that a look-back far behind the chain of
// inclusive prefixes catches up in one more round trip instead of one per 64
// tiles.  The wait is bounded: after `limit` round trips that found a
// predecessor not ready, the look-back gives up and says so (stalled), so
// that a lost predecessor ends the launch with a status instead of a hang.
template <bool SUM>
__device__ __forceinline__ Prefix lookback(const Desc *desc, i64 idx, i64 first, u32 tag, u32 limit) {
    const u32 ln = lane_id();
    u64 acc_c = 0;
    u32 acc_s = 0;
    bool acc_m = false;
    i64 pos = idx - 1;
    u32 nw = 1;
    u32 waits = 0;
    for (;;) {
        u64 cw[kLookbackWindows], sw[kLookbackWindows];
#pragma unroll
        for (int k = 0; k < kLookbackWindows; ++k) {
            const i64 p = pos - (i64)ln - 64 * k;
            cw[k] = 0;
            sw[k] = 0;
            if ((u32)k < nw && p >= first) {
                cw[k] = aload(&desc[p].c);
                if (SUM) sw[k] = aload(&desc[p].s);
            }
        }
        i64 consumed = 0;
        bool done = false, stopped = false;
#pragma unroll
        for (int k = 0; k < kLookbackWindows; ++k) {
            if ((u32)k >= nw) break;
            const i64 p = pos - (i64)ln - 64 * k;
            const u64 c = cw[k];
            const bool vc = (u32)(c >> 38) == tag;
            const bool ic = (c >> 36) & 1;
            bool ok = vc;
            if (SUM) {
                const bool vs = (u32)(sw[k] >> 38) == tag;
                const bool is = (sw[k] >> 32) & 1;
                ok = vc && vs && ic == is;
            }
            // 0 not ready, 1 aggregate, 2 inclusive (or before the chain)
            const u32 state = p < first ? 2u : (ok ? (ic ? 2u : 1u) : 0u);
            const u64 m_inc = ballot(state == 2);
            const u64 m_nr = ballot(state == 0);
            const u32 fi = m_inc ? (u32)__builtin_ctzll(m_inc) : 64u;
            const u32 fn = m_nr ? (u32)__builtin_ctzll(m_nr) : 64u;
            const u32 lim = fi < fn ? fi : fn;
            const bool take = ln < lim;
            acc_c += wave_sum(take ? (u32)(c & kCountMask) : 0u);
            if (SUM) acc_s += wave_sum(take ? (u32)sw[k] : 0u);
            acc_m |= ballot(take && ((c >> 37) & 1)) != 0;
            consumed += lim;
            if (fi < fn) {
                const u64 ci = ((u64)read_lane((u32)(c >> 32), fi) << 32) | read_lane((u32)c, fi);
                acc_c += ci & kCountMask;
                acc_m |= ((ci >> 37) & 1) != 0;
                if (SUM) acc_s += read_lane((u32)sw[k], fi);
                done = true;
                break;
            }
            if (fn < 64) {
                stopped = true;
                break;
            }
        }
        if (done) break;
        pos -= consumed;
        if (consumed == 0) {
            if (++waits > limit) return Prefix{acc_c, acc_s, acc_m, true};
            __builtin_amdgcn_s_sleep(1);
        }
        nw = stopped ? 1u : (u32)kLookbackWindows;
    }
    return Prefix{acc_c, acc_s, acc_m, false};
}

// The stall word of a workspace holds epoch + 1 once a look-back of that
// launch gave up; later launches (other epochs) ignore it.
__device__ __forceinline__ void mark_stalled(u64 *stall, u32 epoch) {
    astore(stall, (u64)epoch + 1);
}
__device__ __forceinline__ bool launch_stalled(const u64 *stall, u32 epoch) {
    return aload(stall) == (u64)epoch + 1;
}

// ------------------------------------------------------------ byte loads
__device__ __forceinline__ void load16(const u8 *p, u32 (&w)[4]) {
    const uint4 q = *(const uint4 *)p;
    w[0] = q.x;
    w[1] = q.y;
    w[2] = q.z;
    w[3] = q.w;
}

// 0xFF in each byte k of the result whose bit k of m (0..3) is set.
__device__ __forceinline__ u32 byte_mask4(u32 m) {
    return ((m & 1u) * 0xFFu) | ((m & 2u) * 0x7F80u) | ((m & 4u) * 0x3FC000u) | ((m & 8u) * 0x1FE00000u);
}

// Bytes [v, v+16) of the aligned base: those in [lo, hi) are marked valid,
// the others read as zero.  A chunk that holds a byte of [lo, hi) is loaded
// with one 16-byte load (an aligned chunk never crosses a page, so it is
// mapped whenever one of its bytes is) and its other bytes are cleared
// before any use; a chunk with none is not loaded.
__device__ __forceinline__ void load16_guarded(const u8 *base, u64 v, u64 lo, u64 hi, u32 (&w)[4],
                                               u32 &valid) {
    w[0] = w[1] = w[2] = w[3] = 0;
    valid = 0;
    if (v + 16 <= lo || v >= hi) return;
    load16(base + v, w);
    const u32 a = v < lo ? (u32)(lo - v) : 0u;         // first byte in range, 0..15
    const u32 e = v + 16 > hi ? (u32)(hi - v) : 16u;   // one past the last, 1..16
    valid = (0xFFFFu >> (16u - e)) & (0xFFFFu << a) & 0xFFFFu;
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] &= byte_mask4((valid >> (4 * k)) & 0xFu);
}

// 4 bytes [v, v+4) (v a multiple of 4) with validity bits at 0..3, loaded
// as one dword when it holds a byte of [lo, hi) (same reasoning as above).
__device__ __forceinline__ void load4_guarded(const u8 *base, i64 v, u64 lo, u64 hi, u32 &w,
                                              u32 &valid4) {
    w = 0;
    valid4 = 0;
    if (v + 4 <= (i64)lo || v >= (i64)hi) return;
    w = *(const u32 *)(base + v);
    const u32 a = v < (i64)lo ? (u32)((i64)lo - v) : 0u;         // 0..3
    const u32 e = (u64)v + 4 > hi ? (u32)((i64)hi - v) : 4u;     // 1..4
    valid4 = (0xFu >> (4u - e)) & (0xFu << a) & 0xFu;
    w &= byte_mask4(valid4);
}

// Top bit of each byte (bit 7 of byte k -> bit k), by dot products of the
// isolated top bits (0 or 0x80 per byte) with byte weights 1, 2, 4, 8 and
// 16, 32, 64, 128: each product sum is 128 times the mask.
__device__ __forceinline__ u32 top4(u32 w) {
    return __builtin_amdgcn_udot4(w & 0x80808080u, 0x08040201u, 0u, false) >> 7;
}
__device__ __forceinline__ u32 top16(const u32 (&w)[4]) {
    u32 lo = __builtin_amdgcn_udot4(w[0] & 0x80808080u, 0x08040201u, 0u, false);
    lo = __builtin_amdgcn_udot4(w[1] & 0x80808080u, 0x80402010u, lo, false);
    u32 hi = __builtin_amdgcn_udot4(w[2] & 0x80808080u, 0x08040201u, 0u, false);
    hi = __builtin_amdgcn_udot4(w[3] & 0x80808080u, 0x80402010u, hi, false);
    return (lo >> 7) | (hi << 1);
}

// a & sext(byte K of w): one VALU instruction with a sub-dword operand
// select (SDWA) that sign-extends the selected byte, so a byte with its top
// bit set acts as "all ones above bit 6" and a byte below 0x80 as itself.
template <int K>
__device__ __forceinline__ u32 and_sbyte(u32 a, u32 w);
#define VB_AND_SBYTE(K)                                                                           \
    template <>                                                                                   \
    __device__ __forceinline__ u32 and_sbyte<K>(u32 a, u32 w) {                                   \
        u32 r;                                                                                    \
        asm("v_and_b32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD "                \
            "src0_sel:DWORD src1_sel:BYTE_" #K                                                    \
            : "=v"(r)                                                                             \
            : "v"(a), "v"(w));                                                                    \
        return r;                                                                                 \
    }
VB_AND_SBYTE(0)
VB_AND_SBYTE(1)
VB_AND_SBYTE(2)
VB_AND_SBYTE(3)
#undef VB_AND_SBYTE

// Per-lane summary of the lane's 16 bytes, given the byte before them (top
// byte of `below`, valid when `below_ok`) and the 4 bytes after them
// (`above`, valid bytes flagged in bits 0..3 of `above_valid`).
//  term:  valid bytes below 0x80 (terminators; their popcount is the number
//         of integers the lane's bytes end).
//  emit:  bytes that begin a code -- the byte before is a terminator or lies
//         outside the stream -- whose terminator lies inside the stream.  A
//         lane's integers are attributed to the lanes holding their first
//         byte; every code has exactly one first byte and one terminator, so
//         the counts agree over a whole stream.
//  mal:   a run of 5 continuation bytes begins in the lane's bytes (a code of
//         more than 5 bytes, which no uint32 has).
struct SegMask {
    u32 term;
    u32 emit;
    bool mal;
};
template <bool EDGE>
__device__ __forceinline__ SegMask seg_mask(const u32 (&w)[4], u32 valid, u32 below, bool below_ok,
                                            u32 above, u32 above_valid) {
    const u32 top = top16(w);
    const u32 topa = top4(above);
    const u32 cont = EDGE ? top & valid : top;
    const u32 term = EDGE ? ~top & valid : ~top & 0xFFFFu;
    const u32 conta = EDGE ? topa & above_valid : topa;
    // the byte before the lane ends a code, or is not part of the stream
    const u32 tb = (EDGE && !below_ok) ? 1u : ((below >> 31) ^ 1u);
    SegMask m;
    m.term = term;
    if (EDGE) {
        const u32 start = ((((term | ~valid) << 1) | tb) & valid) & 0xFFFFu;
        // a code beginning at byte j is terminated when some terminator
        // lies at or after j within the lane's 20-byte window
        const u32 t20 = term | ((~topa & above_valid & 0xFu) << 16);
        const u32 hi = 31u - (u32)__builtin_clz(t20 | 1u);
        m.emit = t20 ? start & ((2u << hi) - 1u) : 0u;
    } else {
        m.emit = ((term << 1) | tb) & 0xFFFFu;
    }
    const u32 c20 = cont | (conta << 16);
    const u32 run5 = c20 & (c20 >> 1) & (c20 >> 2) & (c20 >> 3) & (c20 >> 4);
    m.mal = (run5 & 0xFFFFu) != 0;
    return m;
}

// Assembly of the lane's codes from the last byte down (Horner form of
// Algorithm 1's sum): walking bytes j = 19 .. 0 of the window "own 16 bytes
// then the 4 after", acc becomes the integer formed by the groups from byte
// j up to the first terminator at or after j:
//     acc = ((acc << 7) | 0x7F) & sext8(byte j)
// which keeps (acc << 7) | group for a continuation byte and restarts at the
// group for a terminator.  At a code's first byte acc is the code's integer,
// with the fifth group's weight 2^28 wrapping mod 2^32 as in Algorithm 1.
// Plain: r[j] = acc at byte j.  DELTA: r[j] = -(sum of the integers of codes
// beginning after byte j), and the lane sum T is returned, so that T + r[j]
// is the lane-local inclusive sum at a code beginning at j (bit j of emit).
template <bool DELTA>
__device__ __forceinline__ u32 horner(const u32 (&w)[4], u32 above, u32 emit, u32 (&r)[16]) {
    u32 acc = and_sbyte<3>(0x7Fu, above);
    acc = and_sbyte<2>((acc << 7) | 0x7Fu, above);
    acc = and_sbyte<1>((acc << 7) | 0x7Fu, above);
    acc = and_sbyte<0>((acc << 7) | 0x7Fu, above);
    u32 nu = 0;
#define VB_STEP(J)                                                               \
    acc = and_sbyte<(J) & 3>((acc << 7) | 0x7Fu, w[(J) >> 2]);                   \
    if (DELTA) {                                                                 \
        r[J] = nu;                                                               \
        nu -= acc & (u32)__builtin_amdgcn_sbfe(emit, (J), 1);                    \
    } else {                                                                     \
        r[J] = acc;                                                              \
    }
    VB_STEP(15) VB_STEP(14) VB_STEP(13) VB_STEP(12)
    VB_STEP(11) VB_STEP(10) VB_STEP(9) VB_STEP(8)
    VB_STEP(7) VB_STEP(6) VB_STEP(5) VB_STEP(4)
    VB_STEP(3) VB_STEP(2) VB_STEP(1) VB_STEP(0)
#undef VB_STEP
    return 0u - nu;
}

// Per-wavefront LDS rows: lane L's 16 candidate integers (one per byte) at
// words kRowStride*L .. +15, written as 8-byte pairs.  The stride of 18
// words puts the pairs of 16 consecutive lanes on 32 distinct banks.
constexpr u32 kRowStride = 18;
static_assert(kRowStride * kWave <= kStageWords, "row buffer exceeds the staging area");

// Store the integers of the codes flagged in `emit` (one candidate u[j] per
// byte j of the lane), compacted and in byte order, to out_seg[0 ..), with
// slots below `lim` only when GUARD; RANK adds rbase + slot to each (the
// rank term of differences minus one).  The segment's 1024 bytes are taken 64
// at a time: row k covers bytes 64k .. 64k+63, i.e. the masks of lanes
// 4k .. 4k+3; lane i of the wavefront handles byte 64k + i, and its output
// slot is the row's base plus the number of flagged bytes below it in the
// row (mbcnt of the row mask).  Each row is one masked store of consecutive
// words.
template <bool GUARD, bool RANK>
__device__ __forceinline__ void store_rows(u32 *rows, const u32 (&u)[16], u32 emit, u32 *out_seg,
                                           u32 lim, u32 rbase) {
    const u32 ln = lane_id();
    uint2 *dst = (uint2 *)(rows + kRowStride * ln);
#pragma unroll
    for (int m = 0; m < 8; ++m) dst[m] = make_uint2(u[2 * m], u[2 * m + 1]);
    // even lanes: their mask in bits 0..15, the next lane's in bits 16..31
    const u32 e2 = emit | (dpp_zero<0x101>(emit) << 16);   // row_shl:1
    wave_lds_sync();
    const u32 rd = kRowStride * (ln >> 4) + (ln & 15u);
    u32 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = rows[rd + 4 * kRowStride * k];
    // out_seg is the same on every lane: keep it in scalar registers so each
    // row's store takes a 32-bit byte offset from a scalar base
    const u64 op = (u64)(uintptr_t)out_seg;
    gbyte *ob = (gbyte *)(uintptr_t)(((u64)first_lane((u32)(op >> 32)) << 32) | first_lane((u32)op));
    u32 base = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const u32 lo = read_lane(e2, 4 * k), hi = read_lane(e2, 4 * k + 2);
        const u64 rm = ((u64)hi << 32) | lo;
        if (__builtin_amdgcn_inverse_ballot_w64(rm)) {
            const u32 slot = base + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            if (!GUARD || slot < lim) *(gword *)(ob + (slot << 2)) = RANK ? v[k] + rbase + slot : v[k];
        }
        base += (u32)__builtin_popcountll(rm);
    }
    wave_lds_sync();
}

// Misalignment (in uint32 elements, 0..3) of out + gbase against 16 bytes.
__device__ __forceinline__ u32 out_mis(const u32 *out, u64 gbase) {
    return (u32)((((uintptr_t)out >> 2) + gbase) & 3u);
}
// Store phase of a dense segment: 1024 one-byte codes, whose integers are
// the bytes themselves.  The segment's bytes sit in stage (as bytes, in
// order); lane q of each row expands the 4 bytes of elements 4q - amis ..
// 4q - amis + 3 and stores them with one aligned 16-byte store.  DELTA: the
// integers are the running sums, from a 4-wide local scan plus a wave scan of
// the lane sums, carried across rows (the 4-wide shift-and-add prefix sum of
// the paper's section 4, widened to the wavefront).
template <bool DELTA, bool RANK>
__device__ __forceinline__ void store_dense(const u32 *stage, u32 amis, u32 *out, u64 gbase, u64 n,
                                            u32 add) {
    const u32 ln = lane_id();
    const u8 *sb = (const u8 *)stage;
    u32 carry = add;
    const u32 nq = (amis + kSegBytes + 3) >> 2;
    for (u32 q0 = 0; q0 < nq; q0 += kWave) {
        const u32 q = q0 + ln;
        const int e0 = (int)(q << 2) - (int)amis;
        u32 b4;
        const bool inner = e0 >= 0 && e0 + 4 <= kSegBytes;
        if (inner) {
            const u32 lo = stage[e0 >> 2];
            const u32 hi = (e0 & 3) ? stage[(e0 >> 2) + 1] : 0u;
            b4 = __builtin_amdgcn_alignbyte(hi, lo, (u32)(e0 & 3));   // byte shift
        } else {
            b4 = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int e = e0 + t;
                if (e >= 0 && e < kSegBytes) b4 |= (u32)sb[e] << (8 * t);
            }
        }
        uint4 v;
        v.x = b4 & 0xFFu;
        v.y = (b4 >> 8) & 0xFFu;
        v.z = (b4 >> 16) & 0xFFu;
        v.w = b4 >> 24;
        if (DELTA) {
            v.y += v.x;
            v.z += v.y;
            v.w += v.z;
            const u32 incl = wave_scan(v.w);
            const u32 base = carry + incl - v.w;
            carry += read_lane(incl, 63);
            v.x += base;
            v.y += base;
            v.z += base;
            v.w += base;
        }
        if (RANK) {
            const u32 rk = (u32)gbase + (u32)e0;
            v.x += rk;
            v.y += rk + 1u;
            v.z += rk + 2u;
            v.w += rk + 3u;
        }
        if (q < nq) {
            if (inner && gbase + (u64)e0 + 4 <= n) {
                *(uint4 *)(out + gbase + e0) = v;
            } else {
                const u32 vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int e = e0 + t;
                    if (e >= 0 && e < kSegBytes && gbase + (u64)e < n) out[gbase + e] = vv[t];
                }
            }
        }
    }
}

// ------------------------------------------------------------ byte sums
// The sum of a run of integers in byte form.  Byte j of a code holds the
// group of weight 2^(7 p), where p is the number of continuation bytes
// right before it (0 for the code's first byte), so the integers of any
// whole codes add up to the sum over their bytes of (byte & 0x7F) * 2^(7 p)
// (mod 2^32; a fifth group's 2^28 wraps as in Algorithm 1).  Over a prefix
// [start, x) of the stream, that byte sum counts every code that begins
// before x except the bytes at or after x of the code that straddles x, and
// the terminators before x count the codes that end before x.  k_tile_agg
// produces both per tile, the block scans add them up, and the tile at x adds
// the straddling code from its own first bytes (straddle()).
//
// seg_bytes adds a lane's 16 bytes w (with the 4 bytes before them in
// `below`) to its running number of continuation bytes and byte sum, and
// flags a run of 5 continuation bytes that ends in the lane.  The terms
// 2^(7 p) = 1 + sum over q = 1..p of (2^(7q) - 2^(7(q-1))) are taken as
// byte sums over the bytes with at least q continuation bytes before them,
// each a dot product of the 7-bit groups with 0/1 byte marks; q >= 2 only
// where the wavefront has such a byte at all.
template <bool SUM>
__device__ __forceinline__ void seg_bytes(const u32 (&w)[4], u32 below, u32 &cont, u32 &sum,
                                          bool &mal) {
    u32 c[5];   // 0x01 per continuation byte: c[0] the 4 bytes below, c[k + 1] dword k
    c[0] = (below >> 7) & 0x01010101u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k + 1] = (w[k] >> 7) & 0x01010101u;
        cont += __builtin_popcount(c[k + 1]);
    }
    u32 g[4], m1[4], m2[4], any2 = 0, t0 = 0, t1 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        g[k] = w[k] & 0x7F7F7F7Fu;
        // byte i of alignbyte(c[k+1], c[k], 3 - d) is the mark d + 1 bytes back
        m1[k] = __builtin_amdgcn_alignbyte(c[k + 1], c[k], 3);
        m2[k] = m1[k] & __builtin_amdgcn_alignbyte(c[k + 1], c[k], 2);
        any2 |= m2[k];
        if (SUM) {
            t0 = __builtin_amdgcn_sad_u8(g[k], 0u, t0);
            t1 = __builtin_amdgcn_udot4(g[k], m1[k], t1, false);
        }
    }
    u32 s = t0 + 127u * t1;
    if (ballot(any2 != 0) != 0) {
        u32 t2 = 0, t3 = 0, t4 = 0, run5 = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u32 m3 = m2[k] & __builtin_amdgcn_alignbyte(c[k + 1], c[k], 1);
            const u32 m4 = m3 & c[k];
            run5 |= m4 & c[k + 1];
            if (SUM) {
                t2 = __builtin_amdgcn_udot4(g[k], m2[k], t2, false);
                t3 = __builtin_amdgcn_udot4(g[k], m3, t3, false);
                t4 = __builtin_amdgcn_udot4(g[k], m4, t4, false);
            }
        }
        s += 16256u * t2 + 2080768u * t3 + 266338304u * t4;
        mal |= run5 != 0;
    }
    if (SUM) sum += s;
}

// The code that straddles the start of a tile: `below` holds the 4 bytes
// before the tile (zero outside the stream), f0 and f1 its first 8 bytes.
// code = 1 when a code begins before the tile and ends in it; rest = the
// byte-sum terms of its bytes in the tile.
struct Straddle {
    u32 code, rest;
};
__device__ __forceinline__ Straddle straddle(u32 below, u32 f0, u32 f1) {
    // continuation bytes right before the tile (at most 4 are seen)
    const u32 p0 = (u32)__builtin_clz(~(top4(below) << 28));
    Straddle r{p0 ? 1u : 0u, 0u};
    if (p0) {
        const u64 f = ((u64)f1 << 32) | f0;
        for (u32 j = 0; j < 8; ++j) {
            const u32 b = (u32)(f >> (8 * j)) & 0xFFu;
            const u32 sh = 7u * (p0 + j);
            if (sh < 32) r.rest += (b & 0x7Fu) << sh;
            if (b < 0x80u) break;
        }
    }
    return r;
}

// ------------------------------------------------------------ one tile
// A tile is the run of wpb x SEGS segments that one workgroup decodes;
// wavefront w owns segments [w*SEGS, (w+1)*SEGS) of it.  `base` is 16-byte
// aligned; valid bytes are [vstart, vend); the tile starts at tv.  One
// look-back descriptor per tile.
struct TileIn {
    const u8 *base;
    u64 vstart, vend, tv;
    u32 *out;
    u64 n;
    u32 prev;
    Desc *desc;
    i64 didx, dfirst;
    u32 tag;
    // kKnown: exclusive prefix of the tile (count, sum, malformed so far)
    u64 known_c;
    u32 known_s;
    bool known_mal;
    // resumable pieces: receives the offset (from vstart) of the code of rank n
    u64 *pos_out;
    // look-back bound and the workspace's stall word
    u32 spin_limit;
    u64 *stall;
};

struct TileOut {
    u64 total;   // integers up to and including this tile (kAgg: of the wavefront)
    bool mal;
    u32 sum;     // inclusive wrapping sum (kAgg: of the wavefront)
    bool stalled = false;   // this tile's look-back gave up
};

// What run_tile does with a tile.
constexpr int kFull = 0;    // decode, prefix from the look-back
constexpr int kCount = 1;   // count terminators only, prefix from the look-back
constexpr int kAgg = 2;     // this wavefront's count and sum only; no synchronisation
constexpr int kKnown = 3;   // decode with the exclusive prefix given in TileIn
constexpr int kPiece = 4;   // kFull, and record where the code of rank n begins
constexpr int kKnownB = 5;  // kKnown with the prefix in byte form (see k_tile_agg)
constexpr int kKnownW = 6;  // every wavefront alone, its own prefix in byte form given (no barrier)
constexpr int kConsume = 7; // kKnownB, each segment's integers handed to a consumer instead of stored

// The consumer of kinds other than kConsume: never called.
struct NoConsumer {
    __device__ void take(int, const u32 (&)[16], u32, u64, u64, u32) {}
};

constexpr int kMaxWaves = 16;
constexpr int kMaxBlock = 8 * kWave;   // at most 8 wavefronts per workgroup

// Workgroup-shared scratch of the tile protocol.
struct WgShared {
    u32 wcnt[kMaxWaves];
    u32 wsum[kMaxWaves];
    u32 wmal[kMaxWaves];
    u64 excl_c;
    u32 excl_s;
    u32 excl_mal;
    u32 epoch;
    u64 item;
    u64 cur;    // resumable pieces: the piece's first byte and its prev
    u32 cprev;
    u32 stalled;   // the tile's look-back gave up
};

// Totals of the tile's wavefronts, read from `sh`.
struct TileSum {
    u32 c, s;
    bool mal;
};
__device__ __forceinline__ TileSum tile_sum(const WgShared &sh, u32 wpb) {
    TileSum r{0, 0, false};
    for (u32 k = 0; k < wpb; ++k) {
        r.c += sh.wcnt[k];
        r.s += sh.wsum[k];
        r.mal |= sh.wmal[k] != 0;
    }
    return r;
}

// A wavefront's share of a tile in registers: its SEGS segments (16 bytes
// per lane each, with validity bits for the guarded edge form), the 4 bytes
// before them and the 4 after them.
template <int SEGS>
struct TileRegs {
    u32 w[SEGS][4];
    u32 valid[SEGS];
    u32 hb, hbv, ha, hav;
};

// Loads the wavefront's share of the tile whose wavefront range starts at
// byte wv of the aligned base: unguarded in the interior, byte by byte at the
// stream's edges.  AFTER: also the 4 bytes after the range.
template <int SEGS, bool EDGE, bool AFTER>
__device__ __forceinline__ void load_tile(const u8 *base, u64 vstart, u64 vend, u64 wv,
                                          TileRegs<SEGS> &x) {
    const u32 ln = lane_id();
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u64 v = wv + (u64)s * kSegBytes + 16u * ln;
        if (EDGE) {
            load16_guarded(base, v, vstart, vend, x.w[s], x.valid[s]);
        } else {
            load16(base + v, x.w[s]);
            x.valid[s] = 0xFFFFu;
        }
    }
    x.ha = 0;
    x.hav = 0;
    if (EDGE) {
        load4_guarded(base, (i64)wv - 4, vstart, vend, x.hb, x.hbv);
        if (AFTER) load4_guarded(base, (i64)(wv + SEGS * kSegBytes), vstart, vend, x.ha, x.hav);
    } else {
        x.hb = *(const u32 *)(base + wv - 4);
        x.hbv = 0xFu;
        if (AFTER) x.ha = *(const u32 *)(base + wv + SEGS * kSegBytes);
        x.hav = 0xFu;
    }
}

// D: 0 plain, 1 differences (inclusive prefix sum), 2 differences minus one
// (the prefix sum plus each integer's rank).  The tile's bytes come in `x`.
template <int D, int KIND, int SEGS, bool EDGE, class CONS = NoConsumer>
__device__ __forceinline__ TileOut run_tile_regs(const TileIn &t, const TileRegs<SEGS> &x, u32 *rows,
                                                 WgShared &sh, u32 wib, u32 wpb,
                                                 CONS *cons = nullptr) {
    constexpr bool DELTA = D != 0, RANK = D == 2;
    constexpr bool COUNT = KIND == kCount, AGG = KIND == kAgg;
    constexpr bool CONSUME = KIND == kConsume;
    constexpr bool KNOWN = KIND == kKnown || KIND == kKnownB || CONSUME;
    static_assert(!CONSUME || D == 1, "the consumer takes differential lists");
    constexpr bool PIECE = KIND == kPiece;
    constexpr bool WAVE = KIND == kKnownW;
    const u32 ln = lane_id();
    const u64 wv = t.tv + (u64)wib * (SEGS * kSegBytes);   // this wavefront's first byte
    const auto &w = x.w;
    const auto &valid = x.valid;
    const u32 hb = x.hb, hbv = x.hbv, ha = x.ha, hav = x.hav;

    // Phase 1: masks, counts (and for DELTA the integers and sums).
    u32 emit[SEGS], above[SEGS], segbase[SEGS], segcnt[SEGS];
    u32 lincl[SEGS], sbase[SEGS];
    u32 r[DELTA ? SEGS : 1][16];
    u32 ctot = 0, stot = 0, dmask = 0;
    bool mal = false;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u32 l0w = s == 0 ? hb : read_lane(w[s - 1][3], 63);
        const u32 below = from_lane_below(w[s][3], l0w);
        bool below_ok = true;
        if (EDGE) {
            const u32 l0v = s == 0 ? (hbv << 12) : read_lane(valid[s - 1], 63);
            below_ok = ((from_lane_below(valid[s], l0v) >> 15) & 1u) != 0;
        }
        u32 ab = 0, abv = 0;
        if (!COUNT) {
            ab = from_lane_above(w[s][0], s + 1 < SEGS ? read_lane(w[s + 1][0], 0) : ha);
            abv = EDGE ? from_lane_above(valid[s], s + 1 < SEGS ? read_lane(valid[s + 1], 0) : hav) & 0xFu
                       : 0xFu;
        }
        above[s] = ab;
        const SegMask m = seg_mask<EDGE>(w[s], valid[s], below, below_ok, ab, abv);
        emit[s] = m.emit;
        mal |= m.mal;
        // dense: all 1024 bytes are terminators and no code enters from below
        const bool dense = !COUNT && !CONSUME && !EDGE && ballot(m.term == 0xFFFFu) == ~0ull &&
                           (l0w >> 31) == 0;
        dmask |= dense ? (1u << s) : 0u;
        segcnt[s] = wave_sum(__builtin_popcount(COUNT ? m.term : m.emit));
        segbase[s] = ctot;
        ctot += segcnt[s];
        if (DELTA) {
            u32 ls;
            if (dense) {
                ls = __builtin_amdgcn_sad_u8(w[s][0], 0u, 0u);
                ls = __builtin_amdgcn_sad_u8(w[s][1], 0u, ls);
                ls = __builtin_amdgcn_sad_u8(w[s][2], 0u, ls);
                ls = __builtin_amdgcn_sad_u8(w[s][3], 0u, ls);
            } else {
                ls = horner<true>(w[s], ab, m.emit, r[s]);
            }
            const u32 si = wave_scan(ls);
            lincl[s] = si;
            sbase[s] = stot;
            stot += read_lane(si, 63);
        }
    }
    const bool wmal = ballot(mal) != 0;
    if (AGG) return TileOut{ctot, wmal, stot};
    u64 exc;
    u32 exs, wex_c = 0, wex_s = 0;
    TileOut res;
    if constexpr (WAVE) {
        // the wavefront's own prefix plus the code straddling its first byte
        const Straddle st = straddle(hb, read_lane(w[0][0], 0), read_lane(w[0][1], 0));
        exc = t.known_c + st.code;
        exs = t.known_s + st.rest;
        res = TileOut{exc + ctot, wmal, exs + stot};
    } else {
        if (ln == 0) {
            sh.wcnt[wib] = ctot;
            sh.wsum[wib] = stot;
            sh.wmal[wib] = wmal ? 1u : 0u;
        }
        __syncthreads();
        for (u32 k = 0; k < wib; ++k) {
            wex_c += sh.wcnt[k];
            wex_s += sh.wsum[k];
        }
        const TileSum tsum = tile_sum(sh, wpb);

        // Wavefront 0 publishes the aggregate, looks back, publishes the
        // inclusive prefix and hands the exclusive prefix to the others; the
        // aggregate and the inclusive prefix are stored by the same wavefront,
        // in that order.
        if (wib == 0) {
            Prefix ex;
            if (KNOWN) {
                ex = Prefix{t.known_c, t.known_s, t.known_mal};
                if (KIND == kKnownB || CONSUME) {
                    const Straddle st = straddle(hb, read_lane(w[0][0], 0), read_lane(w[0][1], 0));
                    ex.c += st.code;
                    ex.s += st.rest;
                }
            } else if (t.didx == t.dfirst) {
                ex = Prefix{0, t.prev, false};
            } else {
                if (ln == 0) publish<DELTA>(&t.desc[t.didx], t.tag, false, tsum.mal, tsum.c, tsum.s);
                ex = lookback<DELTA>(t.desc, t.didx, t.dfirst, t.tag, t.spin_limit);
                if (ex.stalled && ln == 0) mark_stalled(t.stall, t.tag & 0x1FFFFFFu);
            }
            if (ln == 0) {
                if (!KNOWN)
                    publish<DELTA>(&t.desc[t.didx], t.tag, true, ex.mal || tsum.mal, ex.c + tsum.c,
                                   ex.s + tsum.s);
                sh.excl_c = ex.c;
                sh.excl_s = ex.s;
                sh.excl_mal = ex.mal ? 1u : 0u;
                sh.stalled = ex.stalled ? 1u : 0u;
            }
        }
        __syncthreads();
        exc = sh.excl_c;
        exs = sh.excl_s;
        res = TileOut{exc + tsum.c, sh.excl_mal != 0 || tsum.mal, exs + tsum.s, sh.stalled != 0};
    }
    if (COUNT) return res;

    // Phase 2: store each segment's integers.
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u64 gbase = exc + wex_c + segbase[s];
        if (PIECE && gbase <= t.n && t.n < gbase + segcnt[s]) {
            // The code of rank n begins in this segment: where a resumed
            // piece starts.  Its lane is found by a scan of the lanes'
            // counts, its byte as the right set bit of the lane's mask.
            const u32 kk = (u32)(t.n - gbase);
            const u32 cnt = __builtin_popcount(emit[s]);
            const u32 ci = wave_scan(cnt);
            if (kk >= ci - cnt && kk < ci) {
                u32 e = emit[s];
                for (u32 q = kk - (ci - cnt); q > 0; --q) e &= e - 1u;
                *t.pos_out = wv + (u64)s * kSegBytes + 16u * ln + (u32)__builtin_ctz(e) - t.vstart;
            }
        }
        if (gbase >= t.n || segcnt[s] == 0) continue;
        if constexpr (CONSUME) {
            u32 u[16];
            const u32 add = exs + wex_s + sbase[s] + lincl[s];
#pragma unroll
            for (int j = 0; j < 16; ++j) u[j] = r[s][j] + add;
            cons->take(s, u, emit[s], gbase, t.n, segcnt[s]);
            continue;
        }
        if (dmask & (1u << s)) {
            *(uint4 *)(rows + 4 * ln) = make_uint4(w[s][0], w[s][1], w[s][2], w[s][3]);
            wave_lds_sync();
            store_dense<DELTA, RANK>(rows, out_mis(t.out, gbase), t.out, gbase, t.n,
                                     DELTA ? exs + wex_s + sbase[s] : 0u);
            wave_lds_sync();
            continue;
        }
        u32 u[16];
        if (DELTA) {
            // exclusive sum before the lane plus the lane's own sum T
            const u32 add = exs + wex_s + sbase[s] + lincl[s];
#pragma unroll
            for (int j = 0; j < 16; ++j) u[j] = r[s][j] + add;
        } else {
            horner<false>(w[s], above[s], emit[s], u);
        }
        u32 *out_seg = t.out + gbase;
        if (gbase + segcnt[s] <= t.n)
            store_rows<false, RANK>(rows, u, emit[s], out_seg, 0u, (u32)gbase);
        else
            store_rows<true, RANK>(rows, u, emit[s], out_seg, (u32)(t.n - gbase), (u32)gbase);
    }
    return res;
}

// run_tile_regs with the wavefront's bytes loaded first.
template <int D, int KIND, int SEGS, bool EDGE, class CONS = NoConsumer>
__device__ __forceinline__ TileOut run_tile(const TileIn &t, u32 *rows, WgShared &sh, u32 wib,
                                            u32 wpb, CONS *cons = nullptr) {
    TileRegs<SEGS> x;
    load_tile<SEGS, EDGE, KIND != kCount>(t.base, t.vstart, t.vend,
                                          t.tv + (u64)wib * (SEGS * kSegBytes), x);
    return run_tile_regs<D, KIND, SEGS, EDGE, CONS>(t, x, rows, sh, wib, wpb, cons);
}

// Status of a finished stream or list: malformed first,
// then truncated (last byte continues, or too few integers), then count.
__device__ __forceinline__ int32_t final_status(bool mal, u8 last_byte, u64 total, u64 n) {
    if (mal) return VBYTE_EMALFORMED;
    if (last_byte >= 0x80 || total < n) return VBYTE_ETRUNC;
    if (total > n) return VBYTE_ECOUNT;
    return VBYTE_OK;
}

// ------------------------------------------------------------ single stream
// PIECE: a resumable piece (the window and prev come from the cursor); its
// own instantiation, so that the whole-stream kernels carry none of it.
template <int D, bool COUNT, int SEGS, bool PIECE>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(D ? 4 : 8))) void k_stream(StreamArgs a) {
    constexpr int KIND = COUNT ? kCount : PIECE ? kPiece : kFull;
    extern __shared__ __align__(16) u32 lds[];
    __shared__ WgShared sh;
    const u32 tid = threadIdx.x;
    const u32 wib = tid >> 6;
    const u32 wpb = blockDim.x >> 6;
    u32 *stage = lds + wib * kStageWords;

    if (tid == 0) {
        sh.item = take_ticket(a.hdr + kTicketWord, a.ntiles);
        sh.epoch = (u32)aload(a.hdr);
        if (PIECE) {
            sh.cur = a.cursor_in[0];
            sh.cprev = (u32)a.cursor_in[2];
        }
    }
    __syncthreads();
    const u32 epoch = sh.epoch;
    const u32 tile = (u32)sh.item;

    const u64 tb = (u64)wpb * SEGS * kSegBytes;
    TileIn t{};
    t.base = a.base;
    t.vstart = a.vstart;
    t.vend = a.vend;
    t.prev = a.prev;
    bool bad_cursor = false;
    if (PIECE) {
        // the piece: at most `window` bytes from the cursor
        const u64 total_bytes = a.vend - a.vstart;
        u64 cur = sh.cur;
        bad_cursor = cur > total_bytes;
        if (bad_cursor) cur = total_bytes;
        const u8 *p0 = a.base + a.vstart + cur;
        t.base = (const u8 *)((uintptr_t)p0 & ~(uintptr_t)15);
        t.vstart = (u64)(p0 - t.base);
        const u64 remain = total_bytes - cur;
        t.vend = t.vstart + (remain < a.window ? remain : a.window);
        t.prev = sh.cprev;
        t.pos_out = a.scratch;
    }
    t.tv = (u64)tile * tb;
    t.out = a.out;
    t.n = a.n;
    t.desc = a.desc;
    t.didx = tile;
    t.dfirst = 0;
    t.tag = make_tag(epoch);
    t.spin_limit = a.spin_limit;
    t.stall = a.hdr + kStallWord;
    const bool interior = tile > 0 && t.tv + tb + 4 <= t.vend;
    TileOut r;
    if (interior)
        r = run_tile<D, KIND, SEGS, false>(t, stage, sh, wib, wpb);
    else
        r = run_tile<D, KIND, SEGS, true>(t, stage, sh, wib, wpb);

    if (tile == a.ntiles - 1 && tid == 0) {
        const bool stalled = launch_stalled(t.stall, epoch);
        if (COUNT) {
            *a.d_count = stalled ? ~0ull : r.total;
        } else if (PIECE) {
            // a piece: more codes than n are fine; a short piece that ends
            // inside a code is truncated
            a.scratch[1] = r.total;
            const bool cut = r.total < a.n && t.vend > t.vstart && t.base[t.vend - 1] >= 0x80;
            *a.d_status = stalled    ? VBYTE_ESTALLED
                          : bad_cursor ? VBYTE_EINVAL
                          : r.mal    ? VBYTE_EMALFORMED
                          : cut      ? VBYTE_ETRUNC
                                     : VBYTE_OK;
        } else {
            const u8 last = a.base[a.vend - 1];
            *a.d_status = stalled ? VBYTE_ESTALLED : final_status(r.mal, last, r.total, a.n);
        }
        // The last tile's look-back has ended, so every tile has published
        // and therefore read the epoch: retire this launch's descriptors.
        astore(a.hdr, (u64)epoch + 1);
    }
    // a tile whose look-back gave up after the status was written says so
    // itself, once its stores are done
    if (r.stalled && tid == 0) {
        if (COUNT)
            __hip_atomic_store(a.d_count, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_store(a.d_status, (int32_t)VBYTE_ESTALLED, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------ chunked stream
// Single stream in chunks of whole tiles, one chunk per workgroup (chunk =
// workgroup index, so a chunk only ever waits for chunks dispatched before
// it).  Pass 1 reads the chunk's tiles for their counts and sums only; the
// chunk then publishes one aggregate and looks back once over the chunks
// before it; pass 2 decodes the chunk's tiles in order with the prefix
// known, re-reading their bytes (mostly from cache).  One look-back per
// chunk instead of one per tile, and none of pass 2 waits on other
// workgroups.
template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(D ? 4 : 8))) void k_chunks(StreamArgs a) {
    constexpr bool DELTA = D != 0;
    extern __shared__ __align__(16) u32 lds[];
    __shared__ WgShared sh;
    const u32 tid = threadIdx.x;
    const u32 ln = lane_id();
    const u32 wib = tid >> 6;
    const u32 wpb = blockDim.x >> 6;
    u32 *stage = lds + wib * kStageWords;
    const u32 nch = gridDim.x;
    if (tid == 0) {
        sh.item = take_ticket(a.hdr + kTicketWord, nch);
        sh.epoch = (u32)aload(a.hdr);
    }
    __syncthreads();
    const u32 epoch = sh.epoch;
    const u32 chunk = (u32)sh.item;
    const u64 tb = (u64)wpb * SEGS * kSegBytes;
    const u64 t0 = (u64)chunk * a.ntiles / nch, t1 = (u64)(chunk + 1) * a.ntiles / nch;
    TileIn t{};
    t.base = a.base;
    t.vstart = a.vstart;
    t.vend = a.vend;
    t.out = a.out;
    t.n = a.n;
    t.prev = a.prev;
    t.desc = a.desc;
    t.tag = make_tag(epoch);

    // pass 1: this wavefront's count and sum over the chunk
    u64 cc = 0;
    u32 cs = 0;
    bool cm = false;
    for (u64 ti = t0; ti < t1; ++ti) {
        t.tv = ti * tb;
        const bool interior = ti > 0 && t.tv + tb + 4 <= a.vend;
        const TileOut g = interior ? run_tile<D, kAgg, SEGS, false>(t, stage, sh, wib, wpb)
                                   : run_tile<D, kAgg, SEGS, true>(t, stage, sh, wib, wpb);
        cc += g.total;
        cs += g.sum;
        cm |= g.mal;
    }
    if (ln == 0) {
        sh.wcnt[wib] = (u32)cc;
        sh.wsum[wib] = cs;
        sh.wmal[wib] = cm ? 1u : 0u;
    }
    __syncthreads();
    const TileSum csum = tile_sum(sh, wpb);
    if (wib == 0) {
        Prefix ex;
        if (chunk == 0) {
            ex = Prefix{0, a.prev, false};
        } else {
            if (ln == 0) publish<DELTA>(&a.desc[chunk], t.tag, false, csum.mal, csum.c, csum.s);
            ex = lookback<DELTA>(a.desc, chunk, 0, t.tag, a.spin_limit);
            if (ex.stalled && ln == 0) mark_stalled(a.hdr + kStallWord, epoch);
        }
        if (ln == 0) {
            publish<DELTA>(&a.desc[chunk], t.tag, true, ex.mal || csum.mal, ex.c + csum.c,
                           ex.s + csum.s);
            sh.excl_c = ex.c;
            sh.excl_s = ex.s;
            sh.excl_mal = ex.mal ? 1u : 0u;
            sh.stalled = ex.stalled ? 1u : 0u;
        }
    }
    __syncthreads();
    const bool chunk_stalled = sh.stalled != 0;
    t.known_c = sh.excl_c;
    t.known_s = sh.excl_s;
    t.known_mal = sh.excl_mal != 0;

    // pass 2: decode the chunk's tiles in order
    TileOut r{t.known_c, t.known_mal, t.known_s};
    for (u64 ti = t0; ti < t1; ++ti) {
        t.tv = ti * tb;
        const bool interior = ti > 0 && t.tv + tb + 4 <= a.vend;
        r = interior ? run_tile<D, kKnown, SEGS, false>(t, stage, sh, wib, wpb)
                     : run_tile<D, kKnown, SEGS, true>(t, stage, sh, wib, wpb);
        t.known_c = r.total;
        t.known_s = r.sum;
        t.known_mal = r.mal;
    }
    if (chunk == nch - 1 && tid == 0) {
        const u8 last = a.base[a.vend - 1];
        *a.d_status = launch_stalled(a.hdr + kStallWord, epoch) ? VBYTE_ESTALLED
                                                                : final_status(r.mal, last, r.total, a.n);
        // the last chunk's look-back has ended: every chunk has read the epoch
        astore(a.hdr, (u64)epoch + 1);
    }
    if (chunk_stalled && tid == 0)
        __hip_atomic_store(a.d_status, (int32_t)VBYTE_ESTALLED, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ two passes
// Single stream in four launches with no look-back: k_tile_agg stores every
// tile's number of terminators, byte sum (seg_bytes) and malformed flag in
// its descriptor slot, k_tile_block_sums and k_tile_block_scan turn them
// into exclusive prefixes in place (block totals, then every block scanned
// from the totals before it) and write the status (the number of integers
// of a stream is its number of terminators), and k_known decodes every tile
// with that prefix plus the code that straddles the tile's start.  The
// slots hold plain values with bits 63:38 clear, which no tagged descriptor
// has, so a later look-back launch on the same workspace never accepts
// them.
// One wavefront's share of a tile aggregate: SEGS segments from byte wv of
// the aligned base (valid bytes [vstart, vend); EDGE: guarded loads), their
// continuation bytes, byte sum and whether a run of five continuation bytes
// ends in them, all wavefront-uniform.
template <int D, int SEGS, bool EDGE>
__device__ __forceinline__ void wave_agg(const u8 *base, u64 vstart, u64 vend, u64 wv, u32 &cont,
                                         u32 &sum, bool &mal) {
    const u32 ln = lane_id();
    u32 w[SEGS][4];
    u32 hb, hbv, valid;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u64 v = wv + (u64)s * kSegBytes + 16u * ln;
        if (EDGE)
            load16_guarded(base, v, vstart, vend, w[s], valid);
        else
            load16(base + v, w[s]);
    }
    if (EDGE)
        load4_guarded(base, (i64)wv - 4, vstart, vend, hb, hbv);
    else
        hb = *(const u32 *)(base + wv - 4);
    cont = 0;
    sum = 0;
    bool m = false;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u32 below = from_lane_below(w[s][3], s == 0 ? hb : read_lane(w[s - 1][3], 63));
        seg_bytes<D != 0>(w[s], below, cont, sum, m);
    }
    cont = wave_sum(cont);
    if (D) sum = wave_sum(sum);
    mal = ballot(m) != 0;
}

template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock) void k_tile_agg(StreamArgs a) {
    __shared__ u32 wc[kMaxWaves], ws[kMaxWaves], wm[kMaxWaves];
    const u32 tid = threadIdx.x;
    const u32 wib = tid >> 6;
    const u32 wpb = blockDim.x >> 6;
    const u32 ln = lane_id();
    const u32 tile = blockIdx.x;
    const u64 tb = (u64)wpb * SEGS * kSegBytes;
    const u64 tv = (u64)tile * tb;
    const u64 wv = tv + (u64)wib * (SEGS * kSegBytes);
    // interior: the tile and the 4 bytes before it lie inside the stream
    const bool interior = tile > 0 && tv + tb <= a.vend;
    u32 cont, sum;
    bool wmal;
    if (interior)
        wave_agg<D, SEGS, false>(a.base, a.vstart, a.vend, wv, cont, sum, wmal);
    else
        wave_agg<D, SEGS, true>(a.base, a.vstart, a.vend, wv, cont, sum, wmal);
    if (ln == 0) {
        wc[wib] = cont;
        ws[wib] = sum;
        wm[wib] = wmal ? 1u : 0u;
    }
    __syncthreads();
    if (tid == 0) {
        u32 ct = 0, st = 0, mt = 0;
        for (u32 k = 0; k < wpb; ++k) {
            ct += wc[k];
            st += ws[k];
            mt |= wm[k];
        }
        const u64 lo = tv > a.vstart ? tv : a.vstart;
        const u64 hi = tv + tb < a.vend ? tv + tb : a.vend;
        const u64 terms = hi - lo - ct;   // bytes of the stream in the tile minus continuations
        a.desc[tile].c = terms | ((u64)mt << 37);
        a.desc[tile].s = st;
    }
}

constexpr int kScanBlock = 1024;

constexpr int kScanPer = 8;   // slots per lane per round

// The scans below run in one workgroup, so one CU's memory pipeline carries
// all their slot traffic and one CU issues all their instructions: every
// access is coalesced and a round has only as many rows as it needs.  A
// round of R rows (R = 8, or fewer for the last round) gives wavefront w
// the kWave x R consecutive slots from b0 + w kWave R, lane l the slots l,
// l + 64, ... of them; a wavefront's exclusive prefix is taken in that
// order by one wave scan per row of 64, and rows past R are skipped.
__device__ __forceinline__ u32 scan_rows(u64 left) {
    return left >= (u64)kScanBlock * kScanPer ? (u32)kScanPer : (u32)((left + kScanBlock - 1) / kScanBlock);
}
// Exclusive prefixes, in place, of the tile slots [i_begin, i_end), from
// the carry (count, sum, malformed) before i_begin; the carry leaves with
// the totals through i_end.  One workgroup of kScanBlock threads.
__device__ __forceinline__ void scan_span(const StreamArgs &a, u64 i_begin, u64 i_end, u64 &carry_c,
                                          u32 &carry_s, bool &carry_m) {
    __shared__ u32 wc[kScanBlock / kWave], ws[kScanBlock / kWave], wm[kScanBlock / kWave];
    const u32 tid = threadIdx.x, wib = tid >> 6, ln = lane_id();
    const u64 last = i_end - 1;   // i_end > i_begin
    for (u64 b0 = i_begin, rows = 0; b0 < i_end; b0 += (u64)kScanBlock * rows) {
        rows = scan_rows(i_end - b0);
        const u64 i0 = b0 + (u64)wib * (kWave * rows) + ln;
        // every load issued before the first use: indexes past the end read
        // the last slot and count as zero
        Desc d[kScanPer];
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const u64 i = i0 + (u64)q * kWave;
            d[q] = a.desc[i < last ? i : last];
        }
        u32 pc[kScanPer], ps[kScanPer];
        u32 rc = 0, rs = 0;   // the wavefront's running totals (64 x 8 tiles fit 32 bits)
        bool m = false;
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            if ((u32)q >= rows) break;
            const bool in = i0 + (u64)q * kWave < i_end;
            const u32 c = in ? (u32)(d[q].c & kCountMask) : 0u;   // at most the tile's bytes
            const u32 sm = in ? (u32)d[q].s : 0u;
            m |= in && ((d[q].c >> 37) & 1u) != 0;
            const u32 ci = wave_scan(c), si = wave_scan(sm);
            pc[q] = rc + ci - c;
            ps[q] = rs + si - sm;
            rc += read_lane(ci, 63);
            rs += read_lane(si, 63);
        }
        const bool anym = ballot(m) != 0;
        if (ln == 0) {
            wc[wib] = rc;
            ws[wib] = rs;
            wm[wib] = anym ? 1u : 0u;
        }
        __syncthreads();
        u64 oc = carry_c;
        u32 os = carry_s;
        for (u32 k = 0; k < kScanBlock / kWave; ++k) {
            if (k == wib) {
                oc = carry_c;
                os = carry_s;
            }
            carry_c += wc[k];
            carry_s += ws[k];
            carry_m |= wm[k] != 0;
        }
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const u64 i = i0 + (u64)q * kWave;
            if ((u32)q < rows && i < i_end) {
                a.desc[i].c = oc + pc[q];
                a.desc[i].s = os + ps[q];
            }
        }
        __syncthreads();   // wc, ws and wm are rewritten by the next round
    }
}

// The scan of the tile slots over many workgroups, in two launches:
// k_tile_block_sums writes the totals of every block of kScanSpan slots
// (count with the malformed flag in bit 37, sum) to bsum; k_tile_block_scan
// gives each block its carry from the totals before it and scans the block
// in place; the block holding the last tile writes the stream's status.
constexpr u64 kScanSpan = kTwoPassScanSpan;   // tile slots per scan workgroup
static_assert(kScanSpan == 2 * kScanBlock, "two slots per thread");

// Slots of a block scan: ntiles, or the count an earlier kernel wrote (at
// most ntiles, which sized the grid).
__device__ __forceinline__ u64 scan_slots(const StreamArgs &a) {
    if (!a.d_nslots) return a.ntiles;
    const u64 n = *a.d_nslots;
    return n < a.ntiles ? n : a.ntiles;
}

__global__ __launch_bounds__(kScanBlock) void k_tile_block_sums(StreamArgs a, Desc *bsum) {
    __shared__ u64 bc[kScanBlock / kWave];
    __shared__ u32 bs[kScanBlock / kWave], bm[kScanBlock / kWave];
    const u32 tid = threadIdx.x, wib = tid >> 6, ln = lane_id();
    const u64 nt = scan_slots(a);
    const u64 i0 = (u64)blockIdx.x * kScanSpan;
    if (i0 >= nt) return;   // past the slots written this launch
    const u64 i1 = i0 + kScanSpan < nt ? i0 + kScanSpan : nt;
    u64 c = 0;
    u32 sm = 0;
    bool m = false;
    for (u64 i = i0 + tid; i < i1; i += kScanBlock) {
        const Desc d = a.desc[i];
        c += d.c & kCountMask;
        sm += (u32)d.s;
        m |= ((d.c >> 37) & 1u) != 0;
    }
    const u32 clo = wave_sum((u32)c);   // a span's count fits 32 bits
    sm = wave_sum(sm);
    const bool wm = ballot(m) != 0;
    if (ln == 0) {
        bc[wib] = clo;
        bs[wib] = sm;
        bm[wib] = wm ? 1u : 0u;
    }
    __syncthreads();
    if (tid == 0) {
        u64 tc = 0;
        u32 ts = 0, tm = 0;
        for (u32 k = 0; k < kScanBlock / kWave; ++k) {
            tc += bc[k];
            ts += bs[k];
            tm |= bm[k];
        }
        bsum[blockIdx.x].c = tc | ((u64)tm << 37);
        bsum[blockIdx.x].s = ts;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_tile_block_scan(StreamArgs a, const Desc *bsum) {
    __shared__ u64 pc_sh;
    __shared__ u32 ps_sh, pm_sh, all_m_sh;
    const u32 tid = threadIdx.x, ln = lane_id();
    const u64 nt = scan_slots(a);
    const u32 b = blockIdx.x, nb = (u32)((nt + kScanSpan - 1) / kScanSpan);
    if (b >= nb) return;   // past the slots written this launch
    const u8 lastb = a.base[a.vend - 1];
    if (tid < kWave) {
        // the carry: totals of the blocks before this one (and the
        // malformed flag of all blocks, for the last block's status)
        u64 c = 0;
        u32 sm = 0;
        bool m = false, mall = false;
        for (u32 k = ln; k < nb; k += kWave) {
            const Desc d = bsum[k];
            const bool mk = ((d.c >> 37) & 1u) != 0;
            mall |= mk;
            if (k < b) {
                c += d.c & kCountMask;
                sm += (u32)d.s;
                m |= mk;
            }
        }
        // 64-bit lane counts summed as 24 low bits and the rest (each part
        // fits 32 bits over 64 lanes for counts below 2^56)
        const u32 clo = wave_sum((u32)c & 0xFFFFFFu), chi = wave_sum((u32)(c >> 24));
        sm = wave_sum(sm);
        const bool bmal = ballot(m) != 0, amal = ballot(mall) != 0;
        if (tid == 0) {
            pc_sh = ((u64)chi << 24) + clo;
            ps_sh = a.prev + sm;
            pm_sh = bmal ? 1u : 0u;
            all_m_sh = amal ? 1u : 0u;
        }
    }
    __syncthreads();
    u64 carry_c = pc_sh;
    u32 carry_s = ps_sh;
    bool carry_m = pm_sh != 0;
    const u64 i0 = (u64)b * kScanSpan;
    const u64 i1 = i0 + kScanSpan < nt ? i0 + kScanSpan : nt;
    scan_span(a, i0, i1, carry_c, carry_s, carry_m);
    if (b == nb - 1 && tid == 0) {
        *a.d_status = final_status(all_m_sh != 0, lastb, carry_c, a.n);
        if (a.d_count) *a.d_count = carry_c;   // the stream's terminators, when asked for
    }
}

template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(D ? 4 : 8))) void k_known(StreamArgs a) {
    extern __shared__ __align__(16) u32 lds[];
    __shared__ WgShared sh;
    const u32 tid = threadIdx.x;
    const u32 wib = tid >> 6;
    const u32 wpb = blockDim.x >> 6;
    u32 *stage = lds + wib * kStageWords;
    const u32 tile = blockIdx.x;
    const u64 tb = (u64)wpb * SEGS * kSegBytes;
    TileIn t{};
    t.base = a.base;
    t.vstart = a.vstart;
    t.vend = a.vend;
    t.tv = (u64)tile * tb;
    t.out = a.out;
    t.n = a.n;
    t.known_c = a.desc[tile].c & kCountMask;
    t.known_s = (u32)a.desc[tile].s;
    t.known_mal = false;
    const bool interior = tile > 0 && t.tv + tb + 4 <= t.vend;
    if (interior)
        (void)run_tile<D, kKnownB, SEGS, false>(t, stage, sh, wib, wpb);
    else
        (void)run_tile<D, kKnownB, SEGS, true>(t, stage, sh, wib, wpb);
}

// ============================================================ one launch, one read
// Single stream in one persistent launch that reads every input byte once
// and never waits without bound.  Workgroup r (of G) owns tiles k G + r,
// k = 0, 1, ...: in round k it loads tile k G + r into registers and
// publishes that tile's aggregate (terminator count, byte sum, malformed
// flag: the slot k_tile_agg writes, tagged with the launch), and it decodes
// the tile it loaded two rounds earlier, whose bytes are still in registers.
// The exclusive prefix of tile (k-2) G + r is the running total of rounds
// before k-2 plus the aggregates of ranks below r in round k-2; one
// wavefront reads round k-2's G aggregates (at most 16 per lane), which were
// published a round ago, and also adds all of them to the running total.
// An aggregate that is not there yet is read again a few times from the
// coherent level, then computed from the tile's bytes by the reader itself,
// so a workgroup that has not been scheduled (another kernel holds the
// device) delays no other: forward progress needs no co-residency and no
// ticket.  The last workgroup to finish (counted in groups of 64) writes the
// status and advances the launch epoch.
constexpr int kFlowMaxSlots = kFlowMaxGrid / kWave;   // aggregates per lane
// How long a reader waits for a missing aggregate before it takes the
// producer to be absent (not scheduled, because other work holds the
// device) and computes the value itself: 200 us of the 100 MHz reference
// clock.  A producer found absent is not waited for again in later rounds
// (unless its values show up at the first read).
constexpr u64 kFlowWaitTicks = 20000;
// LDS words of one ring slot of one wavefront: SEGS segments, then the two
// halo words (padded to 16 bytes).
template <int SEGS>
constexpr u32 kFlowSlotWords = SEGS * kWave * 4 + 4;

struct FlowVal {
    u32 c, s;
    bool m;
};

// A tile's aggregate in one 64-bit word, stored and read whole:
// [63:50] tag (valid bit and the low 13 bits of the epoch), [49] malformed,
// [48:32] terminators (a tile holds at most 32 KiB), [31:0] byte sum.
__device__ __forceinline__ u32 flow_tag(u32 epoch) { return 0x2000u | (epoch & 0x1FFFu); }
__device__ __forceinline__ u64 flow_pack(u32 tag, bool mal, u32 c, u32 s) {
    return ((u64)tag << 50) | ((u64)(mal ? 1u : 0u) << 49) | ((u64)(c & 0x1FFFFu) << 32) | s;
}

// The aggregate of one tile computed by one wavefront from the bytes (the
// value k_tile_agg and the flow's own aggregate step produce): terminators
// in the tile's part of the stream, byte sum, malformed run.
template <int D, int SEGS>
__device__ FlowVal tile_agg_alone(const StreamArgs &a, u64 tile, u32 wpb) {
    const u32 ln = lane_id();
    const u64 tb = (u64)wpb * SEGS * kSegBytes;
    const u64 tv = tile * tb;
    u32 cont = 0, sum = 0;
    bool mal = false;
    for (u32 q = 0; q < wpb; ++q) {
        const u64 wv = tv + (u64)q * (SEGS * kSegBytes);
        u32 w[SEGS][4], valid, hb, hbv;
#pragma unroll
        for (int s = 0; s < SEGS; ++s)
            load16_guarded(a.base, wv + (u64)s * kSegBytes + 16u * ln, a.vstart, a.vend, w[s], valid);
        load4_guarded(a.base, (i64)wv - 4, a.vstart, a.vend, hb, hbv);
#pragma unroll
        for (int s = 0; s < SEGS; ++s) {
            const u32 below = from_lane_below(w[s][3], s == 0 ? hb : read_lane(w[s - 1][3], 63));
            seg_bytes<D != 0>(w[s], below, cont, sum, mal);
        }
    }
    const u64 lo = tv > a.vstart ? tv : a.vstart;
    const u64 hi = tv + tb < a.vend ? tv + tb : a.vend;
    FlowVal v;
    v.c = (u32)(hi - lo) - wave_sum(cont);
    v.s = D ? wave_sum(sum) : 0u;
    v.m = ballot(mal) != 0;
    return v;
}

// Sums round kk's aggregates (tiles t0 .. t0 + nr - 1; lane l slot q holds
// rank l + 64 q) over the ranks below `r` (below) and over all ranks (all):
// a first read through the caches, then for what it lacked coherent
// re-reads or the bytes themselves.
template <int D, int SEGS>
__device__ void flow_round_sums(const StreamArgs &a, u64 *agg, u64 t0, u32 nr, u32 r, u32 tag,
                                u32 wpb, bool recompute, u32 &absent, FlowVal &below,
                                FlowVal &all) {
    const u32 ln = lane_id();
    u32 pend = 0;   // slots not read yet
    below = FlowVal{0, 0, false};
    all = FlowVal{0, 0, false};
    auto take = [&](u32 q, u64 w) {
        const u32 cc = (u32)(w >> 32) & 0x1FFFFu, ss = (u32)w;
        const bool mm = ((w >> 49) & 1u) != 0;
        all.c += cc;
        all.s += ss;
        all.m |= mm;
        if (ln + 64u * q < r) {
            below.c += cc;
            below.s += ss;
            below.m |= mm;
        }
    };
    // first read through the caches, in batches of 8 slots per lane: one
    // line serves every workgroup of an XCD, and a stale line only means a
    // coherent re-read below
    constexpr int kBatch = 8;
#pragma unroll
    for (int q0 = 0; q0 < kFlowMaxSlots; q0 += kBatch) {
        if (64u * q0 >= nr) break;
        u64 v[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            const u32 rho = ln + 64u * (q0 + q);
            v[q] = (!recompute && rho < nr) ? agg[t0 + rho] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            if (ln + 64u * (q0 + q) >= nr) continue;
            if (!recompute && (u32)(v[q] >> 50) == tag)
                take(q0 + q, v[q]);
            else
                pend |= 1u << (q0 + q);
        }
    }
    // producers that are running publish soon: wait for them (coherent
    // re-reads), up to kFlowWaitTicks; those already found absent are not
    // waited for
    absent &= pend;
    u32 wait = recompute ? 0u : pend & ~absent;
    const u64 t_start = __builtin_amdgcn_s_memrealtime();
    while (ballot(wait != 0) != 0) {
        if (__builtin_amdgcn_s_memrealtime() - t_start > kFlowWaitTicks) {
            absent |= wait;
            break;
        }
        __builtin_amdgcn_s_sleep(2);
        u32 p = wait;
        while (p) {
            const u32 q = (u32)__builtin_ctz(p);
            p &= p - 1u;
            const u64 w = aload(&agg[t0 + ln + 64u * q]);
            if ((u32)(w >> 50) == tag) {
                take(q, w);
                pend &= ~(1u << q);
                wait &= ~(1u << q);
            }
        }
    }
    // still missing: computed from the bytes, one tile at a time by the
    // whole wavefront, and published (the value its producer would publish),
    // so that other readers find it instead of computing it again
    for (u64 m = ballot(pend != 0); m; m = ballot(pend != 0)) {
        const u32 l = (u32)__builtin_ctzll(m);
        const u32 q = (u32)__builtin_ctz(read_lane(pend, l));
        const FlowVal fv = tile_agg_alone<D, SEGS>(a, t0 + l + 64u * q, wpb);
        if (ln == l) {
            const u64 w = flow_pack(tag, fv.m, fv.c, fv.s);
            if (!recompute) astore(&agg[t0 + l + 64u * q], w);
            take(q, w);
            pend &= ~(1u << q);
        }
    }
    below.c = wave_sum(below.c);
    all.c = wave_sum(all.c);
    if (D) {
        below.s = wave_sum(below.s);
        all.s = wave_sum(all.s);
    }
    below.m = ballot(below.m) != 0;
    all.m = ballot(all.m) != 0;
}

// Per-wavefront partial of a tile's aggregate: terminators in the
// wavefront's range, its byte sum, malformed run seen.
template <int D, int SEGS, bool EDGE>
__device__ __forceinline__ FlowVal wave_partial(const StreamArgs &a, const TileRegs<SEGS> &x, u64 wv) {
    u32 cont = 0, sum = 0;
    bool mal = false;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u32 below = from_lane_below(x.w[s][3], s == 0 ? x.hb : read_lane(x.w[s - 1][3], 63));
        seg_bytes<D != 0>(x.w[s], below, cont, sum, mal);
    }
    const u64 lo = wv > a.vstart ? wv : a.vstart;
    const u64 hi = wv + SEGS * kSegBytes < a.vend ? wv + SEGS * kSegBytes : a.vend;
    FlowVal v;
    v.c = (hi > lo ? (u32)(hi - lo) : 0u) - wave_sum(cont);
    v.s = D ? wave_sum(sum) : 0u;
    v.m = ballot(mal) != 0;
    return v;
}

// Workgroup layout: wavefront 0 is the control wavefront, wavefronts
// 1 .. nd (nd = blockDim / 64 - 1) decode; a tile is nd x SEGS segments,
// decode wavefront d + 1 owning segments [d SEGS, (d + 1) SEGS).  Round k:
//  * decode wavefront d loads its share of tile k G + r into registers,
//    decodes its share of the tile of round k - 3 (kept in an LDS ring)
//    with its own exclusive prefix (computed by the control wavefront in
//    round k - 1), writes its partial aggregate of tile k and the tile's
//    bytes to LDS;
//  * the control wavefront publishes the aggregate of the tile of round
//    k - 1 (the sum of its partials), reads round k - 2's aggregates of all
//    G workgroups (published one round earlier), and turns them, with the
//    partials of its own tile of round k - 2, into the exclusive prefix of
//    every decode wavefront's share of that tile;
//  * one barrier ends the round.
// No wavefront holds both roles' registers, and the decode waits on nothing
// but the round's barrier.
template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock + kWave) __attribute__((amdgpu_waves_per_eu(4))) void k_flow(FlowArgs f) {
    constexpr u32 kRing = 3;   // tiles of rounds k - 3 .. k - 1
    extern __shared__ __align__(16) u32 lds[];
    __shared__ WgShared sh;    // unused by the per-wavefront decode
    __shared__ u32 p_c[kRing][kMaxWaves], p_s[kRing][kMaxWaves], p_m[kRing][kMaxWaves];
    __shared__ u64 w_c[2][kMaxWaves];
    __shared__ u32 w_s[2][kMaxWaves];
    __shared__ u32 f_epoch;
    const StreamArgs &a = f.s;
    const u32 tid = threadIdx.x, wib = tid >> 6, ln = lane_id();
    const u32 nd = (blockDim.x >> 6) - 1;   // decode wavefronts
    const u32 d = wib - 1;                 // decode wavefront index (wib >= 1)
    const u32 G = gridDim.x, r = blockIdx.x;
    const u64 tb = (u64)nd * SEGS * kSegBytes;
    if (tid == 0) f_epoch = (u32)aload(a.hdr);
    __syncthreads();
    const u32 epoch = f_epoch;
    const u32 tag = flow_tag(epoch);
    u64 *const agg = (u64 *)a.desc;   // one word per tile
    const u32 rounds = f.rounds;

    if (wib == 0) {
        // ---------------------------------------------------- control
        u64 bc = 0;
        u32 bs = a.prev;
        bool bm = false;
        u32 absent = 0;
        for (u32 k = 0; k < rounds + 3; ++k) {
            // round k-2's aggregates (read below)
            const bool rd = k >= 2 && k - 2 < rounds;
            const u64 t0 = rd ? (u64)(k - 2) * G : 0;
            const u64 left = a.ntiles - t0;
            const u32 nr = left < G ? (u32)left : G;
            // publish the aggregate of this workgroup's tile of round k-1
            if (k >= 1 && k - 1 < rounds) {
                const u64 tp = (u64)(k - 1) * G + r;
                if (tp < a.ntiles && ln == 0) {
                    const u32 sl = (k - 1) % kRing;
                    u32 ct = 0, st = 0, mt = 0;
                    for (u32 q = 0; q < nd; ++q) {
                        ct += p_c[sl][q];
                        st += p_s[sl][q];
                        mt |= p_m[sl][q];
                    }
                    astore(&agg[tp], flow_pack(tag, mt != 0, ct, st));
                }
            }
            if (rd) {
                FlowVal below, all;
                flow_round_sums<D, SEGS>(a, agg, t0, nr, r, tag, nd, f.recompute != 0, absent,
                                         below, all);
                // exclusive prefixes of the decode wavefronts' shares of
                // tile (k-2) G + r, for its decode in round k+1
                if (t0 + r < a.ntiles && ln == 0) {
                    const u32 sl = (k - 2) % kRing;
                    u64 c = bc + below.c;
                    u32 sm = bs + below.s;
                    for (u32 q = 0; q < nd; ++q) {
                        w_c[k & 1u][q] = c;
                        w_s[k & 1u][q] = sm;
                        c += p_c[sl][q];
                        sm += p_s[sl][q];
                    }
                }
                bc += all.c;
                bs += all.s;
                bm |= all.m;
            }
            __syncthreads();
        }
        // Completion, counted per group of 64 workgroups then over the
        // groups: the last one writes the status (every control wavefront
        // holds the same totals) and advances the epoch, after which no
        // workgroup of this launch reads an aggregate again.
        if (ln == 0) {
            const u32 ng = (G + 63) / 64, grp = r / 64;
            const u32 gsize = grp + 1 < ng ? 64u : G - 64u * grp;
            if (aadd(&f.ctr[grp], 1) == gsize - 1) {
                astore(&f.ctr[grp], 0);
                if (aadd(&f.ctr[kFlowMaxGroups], 1) == ng - 1) {
                    astore(&f.ctr[kFlowMaxGroups], 0);
                    *a.d_status = final_status(bm, a.base[a.vend - 1], bc, a.n);
                    astore(a.hdr, (u64)epoch + 1);
                }
            }
        }
        return;
    }

    // -------------------------------------------------------- decode
    u32 *stage = lds + d * kStageWords;
    u32 *ring = lds + nd * kStageWords + d * kRing * kFlowSlotWords<SEGS>;
    TileIn t{};
    t.base = a.base;
    t.vstart = a.vstart;
    t.vend = a.vend;
    t.out = a.out;
    t.n = a.n;
    // the loads of a round's tile are issued one round ahead, so that a
    // whole round of work hides their latency
    auto tile_of = [&](u32 k, u64 &tv, u64 &wv, bool &has, bool &inner) {
        const u64 ta = (u64)k * G + r;
        has = k < rounds && ta < a.ntiles;
        tv = ta * tb;
        wv = tv + (u64)d * (SEGS * kSegBytes);
        inner = has && ta > 0 && tv + tb + 4 <= a.vend;
    };
    TileRegs<SEGS> xc, xn;   // this round's tile, the next round's
    u64 tvc, wvc;
    bool hasc, inc;
    tile_of(0, tvc, wvc, hasc, inc);
    if (inc) load_tile<SEGS, false, true>(a.base, a.vstart, a.vend, wvc, xc);
    for (u32 k = 0; k < rounds + 3; ++k) {
        u64 tvn, wvn;
        bool hasn, inn;
        tile_of(k + 1, tvn, wvn, hasn, inn);
        if (inn) load_tile<SEGS, false, true>(a.base, a.vstart, a.vend, wvn, xn);

        // partial aggregate of this round's tile, and its bytes to the ring
        if (hasc) {
            FlowVal v;
            if (inc) {
                v = wave_partial<D, SEGS, false>(a, xc, wvc);
            } else {
                TileRegs<SEGS> e;
                load_tile<SEGS, true, false>(a.base, a.vstart, a.vend, wvc, e);
                v = wave_partial<D, SEGS, true>(a, e, wvc);
            }
            if (ln == 0) {
                p_c[k % kRing][d] = v.c;
                p_s[k % kRing][d] = v.s;
                p_m[k % kRing][d] = v.m ? 1u : 0u;
            }
        }

        // decode this wavefront's share of the tile of round k - 3, then
        // put this round's tile in its ring slot
        u32 *slot = ring + (k % kRing) * kFlowSlotWords<SEGS>;
        if (k >= 3) {
            const u64 td = (u64)(k - 3) * G + r;
            if (td < a.ntiles) {
                t.tv = td * tb;
                t.known_c = w_c[(k - 1) & 1u][d];
                t.known_s = w_s[(k - 1) & 1u][d];
                if (td > 0 && t.tv + tb + 4 <= a.vend) {   // interior: its bytes are in the ring
                    TileRegs<SEGS> x3;
#pragma unroll
                    for (int sg = 0; sg < SEGS; ++sg) {
                        const uint4 q = *(const uint4 *)(slot + (sg * kWave + ln) * 4);
                        x3.w[sg][0] = q.x;
                        x3.w[sg][1] = q.y;
                        x3.w[sg][2] = q.z;
                        x3.w[sg][3] = q.w;
                        x3.valid[sg] = 0xFFFFu;
                    }
                    x3.hb = slot[SEGS * kWave * 4];
                    x3.ha = slot[SEGS * kWave * 4 + 1];
                    x3.hbv = x3.hav = 0xFu;
                    (void)run_tile_regs<D, kKnownW, SEGS, false>(t, x3, stage, sh, d, nd);
                } else {
                    (void)run_tile<D, kKnownW, SEGS, true>(t, stage, sh, d, nd);
                }
            }
        }
        if (inc) {
#pragma unroll
            for (int sg = 0; sg < SEGS; ++sg)
                *(uint4 *)(slot + (sg * kWave + ln) * 4) =
                    make_uint4(xc.w[sg][0], xc.w[sg][1], xc.w[sg][2], xc.w[sg][3]);
            if (ln == 0) {
                slot[SEGS * kWave * 4] = xc.hb;
                slot[SEGS * kWave * 4 + 1] = xc.ha;
            }
        }
        __syncthreads();
        xc = xn;
        tvc = tvn;
        wvc = wvn;
        hasc = hasn;
        inc = inn;
    }
}

// Launches k_flow with wpb decode wavefronts and the control wavefront per
// workgroup.  grid 0: the workgroups that can be resident at once per CU
// (the occupancy the runtime reports for this kernel, its workgroup size
// and LDS; one less when it reports 3 or more, because it rounds the
// register allocation more finely than the hardware and a workgroup that
// is not resident is one whose aggregates the others must compute) times
// the CU count, at most kFlowMaxGrid and one per tile.
template <int D, int SEGS>
hipError_t launch_flow_t(FlowArgs f, int wpb, int grid, int cus, hipStream_t s) {
    const size_t lds = (size_t)wpb * (kStageWords + 3 * kFlowSlotWords<SEGS>) * sizeof(u32);
    const int threads = (wpb + 1) * kWave;
    if (grid <= 0) {
        static std::atomic<int> occ[9];   // per wpb (zero-initialised statics)
        int b = occ[wpb].load(std::memory_order_relaxed);
        if (b <= 0) {
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_flow<D, SEGS>, threads, lds);
            if (e != hipSuccess) return e;
            b = b >= 3 ? b - 1 : (b > 0 ? b : 1);
            occ[wpb].store(b, std::memory_order_relaxed);
        }
        grid = cus * b;
    }
    if (grid > kFlowMaxGrid) grid = kFlowMaxGrid;
    if ((u64)grid > f.s.ntiles) grid = (int)f.s.ntiles;
    if (grid < 1) grid = 1;
    f.rounds = (u32)((f.s.ntiles + grid - 1) / grid);
    hipLaunchKernelGGL((k_flow<D, SEGS>), dim3(grid), dim3(threads), lds, s, f);
    return hipGetLastError();
}
template <int SEGS>
hipError_t launch_flow_s(const FlowArgs &f, int delta, int wpb, int grid, int cus, hipStream_t s) {
    return delta == 2 ? launch_flow_t<2, SEGS>(f, wpb, grid, cus, s)
           : delta   ? launch_flow_t<1, SEGS>(f, wpb, grid, cus, s)
                     : launch_flow_t<0, SEGS>(f, wpb, grid, cus, s);
}

// ============================================================ 64-bit codes
// The byte format for 64-bit integers: up to ten 7-bit
// groups, a run of ten continuation bytes is malformed, a tenth group
// wraps mod 2^64, differences are summed mod 2^64.  Decoded in two passes
// with no look-back, one unit of kUnitGroups x SEGS 1 KiB segments per
// wavefront (taken a group of SEGS segments at a time):
// k64_agg gives every unit its number of terminators, its byte sum (each
// byte's group at weight 2^(7p), p the continuation bytes right before it,
// capped at 9) and a malformed flag, and every group of it the
// terminators and byte sum of the groups before it in the unit; k64_scan
// makes the units' totals exclusive
// prefixes and writes the status; k64_known decodes one group per
// wavefront from its unit's prefix, the groups before it in the unit and
// the code that straddles the group's start (the same identity as the
// 32-bit two-pass schedule).  No wavefront waits for another.

constexpr u32 kRow64Stride = 36;   // words per lane of u64 candidates (16-byte aligned rows)
constexpr u32 kUnitGroups = kUnit64Groups;   // groups of SEGS segments per unit, in turn
constexpr u32 kStage64Words = kWave * kRow64Stride;

__device__ __forceinline__ int32_t sbyte(u32 w, u32 k) {   // byte k of w, sign-extended
    return __builtin_amdgcn_sbfe((int32_t)w, 8 * k, 8);
}

// Continuation bytes right before a lane's byte 0 given the 12 bytes before
// it (bytes -12..-1 in p1, p2, p3), capped at 9.
__device__ __forceinline__ u32 run_before(u32 p1, u32 p2, u32 p3) {
    const u32 cb = top4(p1) | (top4(p2) << 4) | (top4(p3) << 8);   // bit 11 = byte -1
    const u32 r = (u32)__builtin_clz(~(cb << 20));
    return r < 9 ? r : 9;
}

// A lane's 16 bytes into its running continuation count, byte sum and
// malformed flag (a continuation byte with 9 continuation bytes before it).
template <bool SUM>
__device__ __forceinline__ void lane_bytes64(const u32 (&w)[4], u32 p1, u32 p2, u32 p3, u32 &cont,
                                             u64 &sum, bool &mal) {
    u32 pos = run_before(p1, p2, p3);
    cont += __builtin_popcount(top16(w));
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const u32 b = (w[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        if (SUM) sum += (u64)(b & 0x7Fu) << (7 * pos);
        const bool c = b >= 0x80u;
        mal |= c && pos >= 9;
        pos = c ? (pos < 9 ? pos + 1 : 9) : 0;
    }
}

// The same for a wavefront whose bytes have at most one continuation byte
// before them (no code longer than 2 bytes, no malformed run): the byte sum
// is the groups' sum plus 127 times the groups that follow a continuation
// byte (dot products over 0/1 byte marks, as in seg_bytes).  Returns false,
// having done nothing, when some lane of the wavefront has a deeper byte.
template <bool SUM>
__device__ __forceinline__ bool lane_bytes64_short(const u32 (&w)[4], u32 p3, u32 &cont, u64 &sum) {
    u32 c[5];
    c[0] = (p3 >> 7) & 0x01010101u;
    u32 any2 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k + 1] = (w[k] >> 7) & 0x01010101u;
        any2 |= __builtin_amdgcn_alignbyte(c[k + 1], c[k], 3) & __builtin_amdgcn_alignbyte(c[k + 1], c[k], 2);
    }
    if (ballot(any2 != 0) != 0) return false;
    u32 t0 = 0, t1 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cont += __builtin_popcount(c[k + 1]);
        if (SUM) {
            const u32 g = w[k] & 0x7F7F7F7Fu;
            t0 = __builtin_amdgcn_sad_u8(g, 0u, t0);
            t1 = __builtin_amdgcn_udot4(g, __builtin_amdgcn_alignbyte(c[k + 1], c[k], 3), t1, false);
        }
    }
    if (SUM) sum += (u64)t0 + 127ull * t1;
    return true;
}

// 12 bytes from v (a multiple of 4), zero outside [lo, hi).
__device__ __forceinline__ void load12(const u8 *base, i64 v, u64 lo, u64 hi, bool guarded,
                                       u32 (&w)[3], u32 &valid) {
    valid = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (guarded) {
            u32 vk;
            load4_guarded(base, v + 4 * k, lo, hi, w[k], vk);
            valid |= vk << (4 * k);
        } else {
            w[k] = *(const u32 *)(base + v + 4 * k);
            valid |= 0xFu << (4 * k);
        }
    }
}

// One step of a 64-bit wavefront scan: add the DPP-selected lane's value.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ void add64_dpp(u32 &lo, u32 &hi) {
    const u32 yl = dpp_zero<CTRL, ROWS>(lo), yh = dpp_zero<CTRL, ROWS>(hi);
    lo += yl;
    hi += yh + (lo < yl ? 1u : 0u);
}
// Inclusive wave64 prefix sum mod 2^64: the steps of wave_scan on both
// halves, with the carry of the low half.
__device__ __forceinline__ u64 wave_scan64(u64 x) {
    u32 lo = (u32)x, hi = (u32)(x >> 32);
    add64_dpp<0x111>(lo, hi);
    add64_dpp<0x112>(lo, hi);
    add64_dpp<0x114>(lo, hi);
    add64_dpp<0x118>(lo, hi);
    add64_dpp<0x142, 0xA>(lo, hi);
    add64_dpp<0x143, 0xC>(lo, hi);
    return ((u64)hi << 32) | lo;
}
// Wavefront sum of 64-bit values (the same on every lane).
__device__ __forceinline__ u64 wave_sum64(u64 x) {
    const u64 t = wave_scan64(x);
    return ((u64)read_lane((u32)(t >> 32), 63) << 32) | read_lane((u32)t, 63);
}

template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock) void k64_agg(Stream64Args a) {
    constexpr u32 W = SEGS * kSegBytes;
    const u32 wib = threadIdx.x >> 6, wpb = blockDim.x >> 6, ln = lane_id();
    const u64 u = (u64)blockIdx.x * wpb + wib;
    if (u >= a.nunits) return;   // whole wavefronts only: no workgroup barrier below
    u32 ucont = 0;
    u64 usum = 0;
    bool mal = false;
    for (u32 g = 0; g < kUnitGroups; ++g) {
        const u64 wv = (u * kUnitGroups + g) * W;
        if (wv >= a.vend) break;
        // interior: the group and the 12 bytes before it are inside the stream
        const bool interior = wv >= 1024 && wv + W <= a.vend;
        u32 w[SEGS][4], valid, bl[3], blv;
#pragma unroll
        for (int s = 0; s < SEGS; ++s) {
            const u64 v = wv + (u64)s * kSegBytes + 16u * ln;
            if (interior)
                load16(a.base + v, w[s]);
            else
                load16_guarded(a.base, v, a.vstart, a.vend, w[s], valid);
        }
        load12(a.base, (i64)wv - 12, a.vstart, a.vend, !interior, bl, blv);
        u32 cont = 0;
        u64 sum = 0;
#pragma unroll
        for (int s = 0; s < SEGS; ++s) {
            const u32 p1 = from_lane_below(w[s][1], s == 0 ? bl[0] : read_lane(w[s - 1][1], 63));
            const u32 p2 = from_lane_below(w[s][2], s == 0 ? bl[1] : read_lane(w[s - 1][2], 63));
            const u32 p3 = from_lane_below(w[s][3], s == 0 ? bl[2] : read_lane(w[s - 1][3], 63));
            if (!lane_bytes64_short<D != 0>(w[s], p3, cont, sum))
                lane_bytes64<D != 0>(w[s], p1, p2, p3, cont, sum, mal);
        }
        // the group's own terminators and byte sum, for k64_known
        cont = wave_sum(cont);
        if (D) sum = wave_sum64(sum);
        const u64 lo = wv > a.vstart ? wv : a.vstart;
        const u64 hi = wv + W < a.vend ? wv + W : a.vend;
        const u32 terms = (u32)(hi - lo) - cont;
        // the group's slot: the terminators and byte sum of the groups before it in the unit
        if (ln == 0) a.gslots[u * kUnitGroups + g] = make_uint4(ucont, 0u, (u32)usum, (u32)(usum >> 32));
        ucont += terms;
        usum += sum;
    }
    const bool wmal = ballot(mal) != 0;
    if (ln == 0) a.slots[u] = make_uint4(ucont, wmal ? 1u : 0u, (u32)usum, (u32)(usum >> 32));
}


__global__ __launch_bounds__(kScanBlock) void k64_scan(Stream64Args a) {
    __shared__ u32 wc[kScanBlock / kWave], wm[kScanBlock / kWave];
    __shared__ u64 ws[kScanBlock / kWave];
    const u32 tid = threadIdx.x, wib = tid >> 6, ln = lane_id();
    const u8 lastb = a.base[a.vend - 1];   // one address for all: in flight with the first slots
    const u64 lastu = a.nunits - 1;        // nunits >= 1
    u64 carry_c = 0, carry_s = a.prev;
    bool carry_m = false;
    // the layout of scan_span: coalesced rows of 64 slots per wavefront
    for (u64 b0 = 0, rows = 0; b0 < a.nunits; b0 += (u64)kScanBlock * rows) {
        rows = scan_rows(a.nunits - b0);
        const u64 i0 = b0 + (u64)wib * (kWave * rows) + ln;
        uint4 q[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const u64 i = i0 + (u64)k * kWave;
            q[k] = a.slots[i < lastu ? i : lastu];   // past the end: counted as zero
        }
        u32 pc[kScanPer];
        u64 ps[kScanPer];
        u32 rc = 0;   // 64 x 8 units of at most 16 KiB: the counts fit 32 bits
        u64 rs = 0;
        bool m = false;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if ((u32)k >= rows) break;
            const bool in = i0 + (u64)k * kWave < a.nunits;
            const u32 c = in ? q[k].x : 0u;
            const u64 sm = in ? (q[k].z | ((u64)q[k].w << 32)) : 0ull;
            m |= in && q[k].y != 0;
            const u32 ci = wave_scan(c);
            const u64 si = wave_scan64(sm);
            pc[k] = rc + ci - c;
            ps[k] = rs + si - sm;
            rc += read_lane(ci, 63);
            rs += ((u64)read_lane((u32)(si >> 32), 63) << 32) | read_lane((u32)si, 63);
        }
        const bool anym = ballot(m) != 0;
        if (ln == 0) {
            wc[wib] = rc;
            ws[wib] = rs;
            wm[wib] = anym ? 1u : 0u;
        }
        __syncthreads();
        u64 oc = carry_c, os = carry_s;
        for (u32 k = 0; k < kScanBlock / kWave; ++k) {
            if (k == wib) {
                oc = carry_c;
                os = carry_s;
            }
            carry_c += wc[k];
            carry_s += ws[k];
            carry_m |= wm[k] != 0;
        }
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const u64 i = i0 + (u64)k * kWave;
            const u64 c = oc + pc[k], sv = os + ps[k];
            if ((u32)k < rows && i < a.nunits) a.slots[i] = make_uint4((u32)c, (u32)(c >> 32), (u32)sv, (u32)(sv >> 32));
        }
        __syncthreads();   // wc, ws and wm are rewritten by the next round
    }
    if (tid == 0) *a.d_status = final_status(carry_m, lastb, carry_c, a.n);
}

// Assembly of a lane's 64-bit codes from byte 24 down to byte 0 of the
// window "own 16 bytes, then the 9 after" (a0, a1 and byte 0 of a2): the
// Horner form of the sum, acc = ((acc << 7) | 0x7F) & sext(byte), in 64
// bits.  Plain: r[j] = acc at byte j; DELTA: r[j] = -(sum of the integers of
// emitted codes beginning after byte j), and the lane sum is returned.
template <bool DELTA>
__device__ __forceinline__ u64 horner64(const u32 (&w)[4], u32 a0, u32 a1, u32 a2, u32 emit,
                                        u64 (&r)[16]) {
    u64 acc = (u64)(i64)sbyte(a2, 0) & 0x7Fu;
#define VB64_STEP(WORD, K) acc = ((acc << 7) | 0x7Fu) & (u64)(i64)sbyte((WORD), (K));
    VB64_STEP(a1, 3) VB64_STEP(a1, 2) VB64_STEP(a1, 1) VB64_STEP(a1, 0)
    VB64_STEP(a0, 3) VB64_STEP(a0, 2) VB64_STEP(a0, 1) VB64_STEP(a0, 0)
#undef VB64_STEP
    u64 nu = 0;
#pragma unroll
    for (int j = 15; j >= 0; --j) {
        acc = ((acc << 7) | 0x7Fu) & (u64)(i64)sbyte(w[j >> 2], j & 3);
        if (DELTA) {
            r[j] = nu;
            if ((emit >> j) & 1u) nu -= acc;
        } else {
            r[j] = acc;
        }
    }
    return 0 - nu;
}

typedef __attribute__((address_space(1))) u64 gdword;

// store_rows for 64-bit candidates: lane L's 16 candidates sit at words
// kRow64Stride * L + 2 j of `rows`; row k covers bytes 64k .. 64k+63 (the
// masks of lanes 4k .. 4k+3), lane i of the wavefront takes byte 64k + i,
// whose slot is the row's base plus the flagged bytes below it (mbcnt of the
// row mask, which also becomes the exec mask of the row's store).  Slots
// below `lim` only when GUARD.
template <bool GUARD>
__device__ __forceinline__ void store_rows64(const u32 *rows, u32 emit, u64 *out_seg, u32 lim) {
    const u32 ln = lane_id();
    const u32 e2 = emit | (dpp_zero<0x101>(emit) << 16);   // row_shl:1
    const u32 src = kRow64Stride * (ln >> 4) + 2u * (ln & 15u);
    const u64 op = (u64)(uintptr_t)out_seg;
    gbyte *ob = (gbyte *)(uintptr_t)(((u64)first_lane((u32)(op >> 32)) << 32) | first_lane((u32)op));
    u32 base = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const u32 lo = read_lane(e2, 4 * k), hi = read_lane(e2, 4 * k + 2);
        const u64 rm = ((u64)hi << 32) | lo;
        if (__builtin_amdgcn_inverse_ballot_w64(rm)) {
            const u32 slot = base + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            if (!GUARD || slot < lim)
                *(gdword *)(ob + (slot << 3)) = *(const u64 *)(rows + src + 4u * kRow64Stride * k);
        }
        base += (u32)__builtin_popcountll(rm);
    }
}

template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock) void k64_known(Stream64Args a) {
    constexpr bool DELTA = D != 0;
    constexpr u32 W = SEGS * kSegBytes;
    extern __shared__ __align__(16) u32 lds[];
    // wib as a scalar: the prefix slots are scalar loads
    const u32 wib = first_lane(threadIdx.x >> 6), wpb = blockDim.x >> 6, ln = lane_id();
    // one group of SEGS segments per wavefront: group gi = unit uu, group g of it
    const u64 gi = (u64)blockIdx.x * wpb + wib;
    const u64 wv = gi * W;
    if (wv >= a.vend) return;   // whole wavefronts only: no workgroup barrier below
    u32 *rows = lds + wib * kStage64Words;
    const u64 uu = gi / kUnitGroups;
    const u32 g = (u32)(gi % kUnitGroups);
    // prefix: the unit's (scanned from prev) plus the groups before g in it
    const uint4 pre = a.slots[uu], gpre = a.gslots[uu * kUnitGroups + g];
    u64 cnt = (pre.x | ((u64)pre.y << 32)) + gpre.x;
    u64 sum = (pre.z | ((u64)pre.w << 32)) + (gpre.z | ((u64)gpre.w << 32));
    // interior: the group, 12 bytes before and 12 after lie inside the stream
    const bool interior = wv >= 1024 && wv + W + 12 <= a.vend;
    u32 w[SEGS][4], valid[SEGS], bl[3], blv, af[3], afv;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u64 v = wv + (u64)s * kSegBytes + 16u * ln;
        if (interior) {
            load16(a.base + v, w[s]);
            valid[s] = 0xFFFFu;
        } else {
            load16_guarded(a.base, v, a.vstart, a.vend, w[s], valid[s]);
        }
    }
    load12(a.base, (i64)wv - 12, a.vstart, a.vend, !interior, bl, blv);
    load12(a.base, (i64)(wv + W), a.vstart, a.vend, !interior, af, afv);
    {
        // the code that begins before the group and ends in it
        const u32 p0 = run_before(bl[0], bl[1], bl[2]);
        if (p0) {
            cnt += 1;
            const u32 f[3] = {read_lane(w[0][0], 0), read_lane(w[0][1], 0), read_lane(w[0][2], 0)};
            u64 rest = 0;
            for (u32 j = 0; j < 12; ++j) {
                const u32 b = (f[j >> 2] >> (8 * (j & 3))) & 0xFFu;
                const u32 sh = 7u * (p0 + j);
                if (sh < 64) rest += (u64)(b & 0x7Fu) << sh;
                if (b < 0x80u) break;
            }
            sum += rest;
        }
    }
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u32 lw = s == 0 ? bl[2] : read_lane(w[s - 1][3], 63);
        const u32 below = from_lane_below(w[s][3], lw);
        bool below_ok = true;
        if (!interior) {
            const u32 lv = s == 0 ? (blv >> 8) << 12 : read_lane(valid[s - 1], 63);
            below_ok = ((from_lane_below(valid[s], lv) >> 15) & 1u) != 0;
        }
        const bool ls = s + 1 < SEGS;
        const u32 a0 = from_lane_above(w[s][0], ls ? read_lane(w[s + 1][0], 0) : af[0]);
        const u32 a1 = from_lane_above(w[s][1], ls ? read_lane(w[s + 1][1], 0) : af[1]);
        const u32 a2 = from_lane_above(w[s][2], ls ? read_lane(w[s + 1][2], 0) : af[2]);
        const u32 top = top16(w[s]);
        const u32 term = ~top & valid[s] & 0xFFFFu;
        const u32 tb = below_ok ? ((below >> 31) ^ 1u) : 1u;   // byte -1 ends a code or is outside
        u32 emit;
        if (interior) {
            emit = ((term << 1) | tb) & 0xFFFFu;
        } else {
            // a code counts only if its terminator is in the stream: within
            // the lane's 16 bytes or the 9 after them
            u32 av = from_lane_above(valid[s], ls ? read_lane(valid[s + 1], 0) : afv) & 0x1FFu;
            const u32 ta = ~(top4(a0) | (top4(a1) << 4) | (top4(a2) << 8)) & av;
            const u32 t25 = term | (ta << 16);
            const u32 start = ((((term | ~valid[s]) << 1) | tb) & valid[s]) & 0xFFFFu;
            const u32 hi = 31u - (u32)__builtin_clz(t25 | 1u);
            emit = t25 ? start & ((2u << hi) - 1u) : 0u;
        }
        u64 r[16];
        const u64 tl = horner64<DELTA>(w[s], a0, a1, a2, emit, r);
        const u32 cl = __builtin_popcount(emit);
        const u32 ci = wave_scan(cl);
        const u32 segcnt = read_lane(ci, 63);
        if (DELTA) {
            const u64 si = wave_scan64(tl);
            const u64 add = sum + si;   // exclusive lane sum + the lane's own sum
#pragma unroll
            for (int j = 0; j < 16; ++j) r[j] += add;
            sum += (u64)read_lane((u32)si, 63) | ((u64)read_lane((u32)(si >> 32), 63) << 32);
        }
        if (cnt < a.n && segcnt) {
            // candidates to LDS rows, then one masked 8-byte store per lane
            // for each 64-byte row of input bytes
            u64 *row = (u64 *)(rows + ln * kRow64Stride);
#pragma unroll
            for (int j = 0; j < 16; j += 2)
                *(uint4 *)(row + j) = make_uint4((u32)r[j], (u32)(r[j] >> 32), (u32)r[j + 1],
                                                 (u32)(r[j + 1] >> 32));
            wave_lds_sync();
            if (cnt + segcnt <= a.n)
                store_rows64<false>(rows, emit, a.out + cnt, 0u);
            else
                store_rows64<true>(rows, emit, a.out + cnt, (u32)(a.n - cnt));
            wave_lds_sync();
        }
        cnt += segcnt;
    }
}

template <int D, int SEGS>
hipError_t launch64_t(const Stream64Args &a, int wpb, hipStream_t s) {
    const u32 blocks = (a.nunits + wpb - 1) / wpb;
    k64_agg<D, SEGS><<<blocks, wpb * kWave, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k64_scan<<<1, kScanBlock, 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const u64 ngroups = (a.vend + SEGS * kSegBytes - 1) / (SEGS * kSegBytes);
    const u32 gblocks = (u32)((ngroups + wpb - 1) / wpb);
    k64_known<D, SEGS><<<gblocks, wpb * kWave, (size_t)wpb * kStage64Words * sizeof(u32), s>>>(a);
    return hipGetLastError();
}

// ============================================================ blocks of four
// Differences between blocks of four: y_i = g_i + y_(i-4),
// i.e. four interleaved prefix sums by rank mod 4, from the four values
// prev4.  A code's class is its rank mod 4, known only once the count of
// the codes before it is, so a run of codes is summarised by (count, S[4])
// with S[c] the sum of its codes of rank = c mod 4 counted from the run's
// first code; two runs combine as (cA + cB, SA[c] + SB[(c - cA) mod 4]).
// Same layout as the 64-bit decode: units of kUnitGroups groups of SEGS
// segments, one unit per wavefront of the aggregate; k4_agg gives every
// group the summary of the groups before it in its unit, and every unit
// the summary of the units before it in its workgroup (block); k4_scan
// turns the blocks into exclusive prefixes (absolute classes, from prev4)
// and writes the status; k4_known decodes one group per wavefront from
// those three prefixes.  A group's codes are those that begin in it and
// end in the stream: the aggregate takes them as byte sums by class
// (d4_sums), the decode assembles them (d4_group).

struct Run4 {
    u64 c;
    u32 s[4];
};

// s rotated by r: t[c] = s[(c - r) mod 4]
__device__ __forceinline__ void rot4(const u32 (&s)[4], u32 r, u32 (&t)[4]) {
    r &= 3u;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const u32 k = (c - r) & 3u;
        t[c] = k == 0 ? s[0] : k == 1 ? s[1] : k == 2 ? s[2] : s[3];
    }
}

__device__ __forceinline__ Run4 join4(const Run4 &a, const Run4 &b) {
    u32 t[4];
    rot4(b.s, (u32)a.c, t);
    return Run4{a.c + b.c, {a.s[0] + t[0], a.s[1] + t[1], a.s[2] + t[2], a.s[3] + t[3]}};
}

__device__ __forceinline__ void put4(uint4 *slot, const Run4 &r) {
    slot[0] = make_uint4((u32)r.c, (u32)(r.c >> 32), r.s[0], r.s[1]);
    slot[1] = make_uint4(r.s[2], r.s[3], 0u, 0u);
}
__device__ __forceinline__ Run4 get4(const uint4 *slot) {
    const uint4 a = slot[0], b = slot[1];
    return Run4{a.x | ((u64)a.y << 32), {a.z, a.w, b.x, b.y}};
}

// One group's segments: masks and values of every segment, and what the
// caller does with them (the decode).  Returns the malformed flag.
struct D4Seg {
    u32 emit;
    u32 u[16];
};

template <bool EDGE, int SEGS, class F>
__device__ __forceinline__ bool d4_group(const Stream4Args &a, u64 wv, F &&f) {
    const u32 ln = lane_id();
    u32 w[SEGS][4], valid[SEGS];
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u64 v = wv + (u64)s * kSegBytes + 16u * ln;
        if (EDGE) {
            load16_guarded(a.base, v, a.vstart, a.vend, w[s], valid[s]);
        } else {
            load16(a.base + v, w[s]);
            valid[s] = 0xFFFFu;
        }
    }
    u32 hb, hbv, ha, hav;
    if (EDGE) {
        load4_guarded(a.base, (i64)wv - 4, a.vstart, a.vend, hb, hbv);
        load4_guarded(a.base, (i64)(wv + SEGS * kSegBytes), a.vstart, a.vend, ha, hav);
    } else {
        hb = *(const u32 *)(a.base + wv - 4);
        ha = *(const u32 *)(a.base + wv + SEGS * kSegBytes);
        hbv = hav = 0xFu;
    }
    bool mal = false;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u32 l0w = s == 0 ? hb : read_lane(w[s - 1][3], 63);
        const u32 below = from_lane_below(w[s][3], l0w);
        bool below_ok = true;
        if (EDGE) {
            const u32 l0v = s == 0 ? (hbv << 12) : read_lane(valid[s - 1], 63);
            below_ok = ((from_lane_below(valid[s], l0v) >> 15) & 1u) != 0;
        }
        const u32 ab = from_lane_above(w[s][0], s + 1 < SEGS ? read_lane(w[s + 1][0], 0) : ha);
        const u32 abv = EDGE ? from_lane_above(valid[s], s + 1 < SEGS ? read_lane(valid[s + 1], 0) : hav) & 0xFu
                             : 0xFu;
        const SegMask m = seg_mask<EDGE>(w[s], valid[s], below, below_ok, ab, abv);
        mal |= m.mal;
        D4Seg g;
        g.emit = m.emit;
        horner<false>(w[s], ab, m.emit, g.u);
        f(g);
    }
    return mal;
}

// A lane's byte sums by class.  The class of a byte is the rank mod 4, from
// the group's first code, of the code that holds it: B (the class of the
// code running into the lane) plus the codes beginning at or before the
// byte in the lane.  Each class sum is the byte-sum identity of seg_bytes
// over the bytes of that class, the class masks coming from a byte lookup
// (v_perm) of the per-byte class; classes 0..2 are added to s[0..2] and
// all bytes to s[3].  Away from the stream's ends (not EDGE) every byte
// after a terminator begins a code, so the start marks are the complement
// of the marks of bytes after a continuation byte; at the ends they come
// from emit.
template <bool EDGE>
__device__ __forceinline__ void class_bytes(const u32 (&w)[4], u32 below, u32 emit, u32 B,
                                            u32 (&s)[4]) {
    u32 c[5];
    c[0] = (below >> 7) & 0x01010101u;
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k + 1] = (w[k] >> 7) & 0x01010101u;
    u32 g[4], m1[4], cls[4], any2 = 0;
    u32 q = B * 0x01010101u;
    u32 t0[4] = {0, 0, 0, 0}, t1[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        g[k] = w[k] & 0x7F7F7F7Fu;
        m1[k] = __builtin_amdgcn_alignbyte(c[k + 1], c[k], 3);
        any2 |= m1[k] & __builtin_amdgcn_alignbyte(c[k + 1], c[k], 2);
        // code starts of the dword as 0x01 bytes, then per byte B + the
        // starts at or before it (at most 3 + 16, no carry between bytes)
        const u32 st = EDGE ? ((((emit >> (4 * k)) & 0xFu) * 0x00204081u) & 0x01010101u)
                            : m1[k] ^ 0x01010101u;
        const u32 p = st * 0x01010101u + q;
        q = __builtin_amdgcn_perm(p, p, 0x03030303u);   // byte 3 of p in every byte
        cls[k] = p & 0x03030303u;
        t0[3] = __builtin_amdgcn_sad_u8(g[k], 0u, t0[3]);
        t1[3] = __builtin_amdgcn_udot4(g[k], m1[k], t1[3], false);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const u32 mk = __builtin_amdgcn_perm(0u, 1u << (8 * cc), cls[k]);
            t0[cc] = __builtin_amdgcn_udot4(g[k], mk, t0[cc], false);
            t1[cc] = __builtin_amdgcn_udot4(g[k], mk & m1[k], t1[cc], false);
        }
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) s[cc] += t0[cc] + 127u * t1[cc];
    if (ballot(any2 != 0) != 0) {
        u32 t2[4] = {0, 0, 0, 0}, t3[4] = {0, 0, 0, 0}, t4[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u32 m2 = m1[k] & __builtin_amdgcn_alignbyte(c[k + 1], c[k], 2);
            const u32 m3 = m2 & __builtin_amdgcn_alignbyte(c[k + 1], c[k], 1);
            const u32 m4 = m3 & c[k];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                const u32 mk = cc < 3 ? __builtin_amdgcn_perm(0u, 1u << (8 * cc), cls[k]) : 0x01010101u;
                t2[cc] = __builtin_amdgcn_udot4(g[k], mk & m2, t2[cc], false);
                t3[cc] = __builtin_amdgcn_udot4(g[k], mk & m3, t3[cc], false);
                t4[cc] = __builtin_amdgcn_udot4(g[k], mk & m4, t4[cc], false);
            }
        }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) s[cc] += 16256u * t2[cc] + 2080768u * t3[cc] + 266338304u * t4[cc];
    }
}

// The code that runs across a boundary, seen from before it: last4 holds
// the 4 bytes before the boundary, ha the 4 after (valid bytes flagged in
// bits 0..3 of hav).  rest = the byte-sum terms of the code's bytes after
// the boundary; returns whether such a code ends in the valid bytes.
__device__ __forceinline__ bool code_tail(u32 last4, u32 ha, u32 hav, u32 &rest) {
    const u32 p0 = (u32)__builtin_clz(~(top4(last4) << 28));
    rest = 0;
    if (!p0) return false;
#pragma unroll
    for (u32 j = 0; j < 4; ++j) {
        if (!((hav >> j) & 1u)) return false;
        const u32 b = (ha >> (8 * j)) & 0xFFu;
        const u32 sh = 7u * (p0 + j);
        if (sh < 32) rest += (b & 0x7Fu) << sh;
        if (b < 0x80u) return true;
    }
    return false;
}

// One group's summary (its count and class sums, from its first code) by
// byte sums, no code assembled: per-lane class sums, then the bytes of the
// code that runs into the group (all of class 3, i.e. rank -1) taken out
// of class 3 and the bytes after the group of the code that runs out of it
// added to that code's class.  Returns the malformed flag.
template <bool EDGE, int SEGS>
__device__ __forceinline__ bool d4_sums(const Stream4Args &a, u64 wv, Run4 &grp) {
    const u32 ln = lane_id();
    u32 w[SEGS][4], valid[SEGS];
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u64 v = wv + (u64)s * kSegBytes + 16u * ln;
        if (EDGE) {
            load16_guarded(a.base, v, a.vstart, a.vend, w[s], valid[s]);
        } else {
            load16(a.base + v, w[s]);
            valid[s] = 0xFFFFu;
        }
    }
    u32 hb, hbv, ha, hav;
    if (EDGE) {
        load4_guarded(a.base, (i64)wv - 4, a.vstart, a.vend, hb, hbv);
        load4_guarded(a.base, (i64)(wv + SEGS * kSegBytes), a.vstart, a.vend, ha, hav);
    } else {
        hb = *(const u32 *)(a.base + wv - 4);
        ha = *(const u32 *)(a.base + wv + SEGS * kSegBytes);
        hbv = hav = 0xFu;
    }
    bool mal = false;
    u32 acc[4] = {0, 0, 0, 0};
    u32 cnt = 0;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u32 l0w = s == 0 ? hb : read_lane(w[s - 1][3], 63);
        const u32 below = from_lane_below(w[s][3], l0w);
        bool below_ok = true;
        if (EDGE) {
            const u32 l0v = s == 0 ? (hbv << 12) : read_lane(valid[s - 1], 63);
            below_ok = ((from_lane_below(valid[s], l0v) >> 15) & 1u) != 0;
        }
        const u32 ab = from_lane_above(w[s][0], s + 1 < SEGS ? read_lane(w[s + 1][0], 0) : ha);
        const u32 abv = EDGE ? from_lane_above(valid[s], s + 1 < SEGS ? read_lane(valid[s + 1], 0) : hav) & 0xFu
                             : 0xFu;
        const SegMask m = seg_mask<EDGE>(w[s], valid[s], below, below_ok, ab, abv);
        mal |= m.mal;
        const u32 cl = __builtin_popcount(m.emit);
        const u32 ci = wave_scan(cl);
        class_bytes<EDGE>(w[s], below, m.emit, (cnt + ci - cl - 1u) & 3u, acc);
        cnt += read_lane(ci, 63);
    }
    u32 S[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) S[c] = wave_sum(acc[c]);
    S[3] -= S[0] + S[1] + S[2];
    S[3] -= straddle(hb, read_lane(w[0][0], 0), read_lane(w[0][1], 0)).rest;
    u32 rest;
    if (code_tail(read_lane(w[SEGS - 1][3], 63), ha, hav, rest)) {
        const u32 lc = (cnt - 1u) & 3u;
#pragma unroll
        for (int c = 0; c < 4; ++c) S[c] += lc == (u32)c ? rest : 0u;
    }
    grp = Run4{cnt, {S[0], S[1], S[2], S[3]}};
    return mal;
}

// One wavefront per unit; the block (workgroup) then combines its units
// through LDS: each unit's slot gets its exclusive prefix within the
// block, the block's slot the block's summary and malformed flag, so that
// the scan runs over blocks only.  No wavefront waits for the others: each
// posts its unit and takes a ticket, and the one that takes the last
// ticket combines the block.
template <int SEGS>
__global__ __launch_bounds__(kMaxBlock) void k4_agg(Stream4Args a) {
    constexpr u32 W = SEGS * kSegBytes;
    __shared__ u32 uc[kMaxWaves], us[4][kMaxWaves], um[kMaxWaves], done;
    const u32 wib = first_lane(threadIdx.x >> 6), wpb = blockDim.x >> 6, ln = lane_id();   // wib: scalar
    if (threadIdx.x == 0) done = 0;
    __syncthreads();
    const u64 u = (u64)blockIdx.x * wpb + wib;
    Run4 unit{0, {0, 0, 0, 0}};
    bool mal = false;
    if (u < a.nunits) {
        for (u32 g = 0; g < kUnitGroups; ++g) {
            const u64 wv = (u * kUnitGroups + g) * W;
            if (wv >= a.vend) break;
            Run4 grp;
            const bool interior = wv >= 16 && wv + W + 4 <= a.vend;
            mal |= interior ? d4_sums<false, SEGS>(a, wv, grp) : d4_sums<true, SEGS>(a, wv, grp);
            if (ln == 0) put4(a.gslots + 2 * (u * kUnitGroups + g), unit);   // the groups before it
            unit = join4(unit, grp);
        }
    }
    const bool wmal = ballot(mal) != 0;
    u32 ticket = 0;
    if (ln == 0) {
        uc[wib] = (u32)unit.c;   // at most the unit's bytes
#pragma unroll
        for (int c = 0; c < 4; ++c) us[c][wib] = unit.s[c];
        um[wib] = wmal ? 1u : 0u;
        ticket = __hip_atomic_fetch_add(&done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (read_lane(ticket, 0) != wpb - 1 || ln != 0) return;
    const u64 u0 = (u64)blockIdx.x * wpb;
    Run4 pre{0, {0, 0, 0, 0}};
    u32 mt = 0;
    for (u32 k = 0; k < wpb; ++k) {
        if (u0 + k < a.nunits) put4(a.slots + 2 * (u0 + k), pre);
        pre = join4(pre, Run4{uc[k], {us[0][k], us[1][k], us[2][k], us[3][k]}});
        mt |= um[k];
    }
    put4(a.bslots + 2 * blockIdx.x, pre);
    a.bslots[2 * blockIdx.x + 1].z = mt;
}

// Exclusive prefixes of the blocks in absolute classes, in the coalesced
// layout of scan_span.  Each round scans the counts first (plain sums); a
// unit's class sums, rotated by the count of the codes before it, are then
// in absolute classes, and four plain scans finish the round: the rotating
// combination never enters a scan.
__global__ __launch_bounds__(kScanBlock) void k4_scan(Stream4Args a) {
    __shared__ u32 wc[kScanBlock / kWave], wm[kScanBlock / kWave];
    __shared__ u32 wsc[4][kScanBlock / kWave];
    const u32 tid = threadIdx.x, wib = tid >> 6, ln = lane_id();
    const u8 lastb = a.base[a.vend - 1];   // one address for all: in flight with the first slots
    const u64 lastu = a.nblocks - 1;       // nblocks >= 1
    u64 carry_c = 0;
    u32 carry_s[4] = {a.prev4[0], a.prev4[1], a.prev4[2], a.prev4[3]};
    bool carry_m = false;
    for (u64 b0 = 0, rows = 0; b0 < a.nblocks; b0 += (u64)kScanBlock * rows) {
        rows = scan_rows(a.nblocks - b0);
        const u64 i0 = b0 + (u64)wib * (kWave * rows) + ln;
        uint4 lo[kScanPer], hi[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const u64 i = i0 + (u64)k * kWave;
            const u64 j = i < lastu ? i : lastu;   // past the end: counted as zero
            lo[k] = a.bslots[2 * j];
            hi[k] = a.bslots[2 * j + 1];
        }
        // counts
        u32 pc[kScanPer];
        u32 rc = 0;   // 64 x 8 blocks of at most 16 units of 16 KiB
        bool m = false;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if ((u32)k >= rows) break;
            const bool in = i0 + (u64)k * kWave < a.nblocks;
            const u32 c = in ? lo[k].x : 0u;   // a block's count: at most its bytes
            m |= in && hi[k].z != 0;
            const u32 ci = wave_scan(c);
            pc[k] = rc + ci - c;
            rc += read_lane(ci, 63);
        }
        const bool anym = ballot(m) != 0;
        if (ln == 0) {
            wc[wib] = rc;
            wm[wib] = anym ? 1u : 0u;
        }
        __syncthreads();
        u64 oc = carry_c;
        for (u32 k = 0; k < kScanBlock / kWave; ++k) {
            if (k == wib) oc = carry_c;
            carry_c += wc[k];
            carry_m |= wm[k] != 0;
        }
        // class sums in absolute classes, then their scans
        u32 ps[kScanPer][4];
        u32 rs[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if ((u32)k >= rows) break;
            const bool in = i0 + (u64)k * kWave < a.nblocks;
            const u32 s4[4] = {in ? lo[k].z : 0u, in ? lo[k].w : 0u, in ? hi[k].x : 0u, in ? hi[k].y : 0u};
            u32 t[4];
            rot4(s4, (u32)(oc + pc[k]), t);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const u32 si = wave_scan(t[c]);
                ps[k][c] = rs[c] + si - t[c];
                rs[c] += read_lane(si, 63);
            }
        }
        if (ln == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) wsc[c][wib] = rs[c];
        }
        __syncthreads();
        u32 os[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) os[c] = carry_s[c];
        for (u32 k = 0; k < kScanBlock / kWave; ++k) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (k == wib) os[c] = carry_s[c];
                carry_s[c] += wsc[c][k];
            }
        }
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const u64 i = i0 + (u64)k * kWave;
            if ((u32)k < rows && i < a.nblocks)
                put4(a.bslots + 2 * i, Run4{oc + pc[k], {os[0] + ps[k][0], os[1] + ps[k][1], os[2] + ps[k][2],
                                                        os[3] + ps[k][3]}});
        }
        __syncthreads();   // wc, wm and wsc are rewritten by the next round
    }
    if (tid == 0) *a.d_status = final_status(carry_m, lastb, carry_c, a.n);
}

template <int SEGS>
__global__ __launch_bounds__(kMaxBlock) void k4_known(Stream4Args a) {
    constexpr u32 W = SEGS * kSegBytes;
    extern __shared__ __align__(16) u32 lds[];
    // wib is the same on every lane: as a scalar, the prefix slots below are
    // scalar loads and their joins scalar arithmetic
    const u32 wib = first_lane(threadIdx.x >> 6), wpb = blockDim.x >> 6;
    const u64 gi = (u64)blockIdx.x * wpb + wib;
    const u64 wv = gi * W;
    if (wv >= a.vend) return;   // whole wavefronts only: no workgroup barrier below
    u32 *rows = lds + wib * kStageWords;
    const u64 uu = gi / kUnitGroups;
    const u32 g = (u32)(gi % kUnitGroups);
    // prefix: the block's (absolute classes, from prev4), the unit's within
    // the block, then the groups before g in the unit
    Run4 run = join4(join4(get4(a.bslots + 2 * (uu / a.block_units)), get4(a.slots + 2 * uu)),
                     get4(a.gslots + 2 * (uu * kUnitGroups + g)));
    // A segment's codes are compacted in LDS by their rank p in the
    // segment (16 ranks per lane, 18 words per lane so that 8-byte reads of
    // consecutive lanes hit distinct banks; the two spare words of a lane
    // take the writes of its bytes that begin no code).  A code's class is
    // then fixed by p mod 4 = its index mod 4 in the lane's 16, so the
    // running values are per-index sums: 3 adds per index in the lane, 4 wave
    // scans, the carried values rotated by the class of the segment's first
    // code.  The rows of 64 ranks are then stored as consecutive words.
    auto f = [&](const D4Seg &sg) {
        const u32 ln = lane_id();
        const u32 cl = __builtin_popcount(sg.emit);
        const u32 ci = wave_scan(cl);
        const u32 segcnt = read_lane(ci, 63);
        const u32 cls0 = (u32)run.c & 3u;
        uint2 *mine = (uint2 *)(rows + kRowStride * ln);
#pragma unroll
        for (int m = 0; m < 8; ++m) mine[m] = make_uint2(0u, 0u);
        wave_lds_sync();
        const u32 spare = kRowStride * ln + 16u;
        u32 p = ci - cl;   // rank of the lane's first code in the segment
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const u32 e = (sg.emit >> j) & 1u;
            rows[e ? p + ((p >> 4) << 1) : spare] = sg.u[j];
            p += e;
        }
        wave_lds_sync();
        u32 v[16];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const uint2 t = mine[m];
            v[2 * m] = t.x;
            v[2 * m + 1] = t.y;
        }
#pragma unroll
        for (int k = 4; k < 16; ++k) v[k] += v[k - 4];
        // index class r holds the codes of class (cls0 + r) mod 4
        u32 carried[4], tot[4];
        rot4(run.s, 4u - cls0, carried);   // carried[r] = run.s[(cls0 + r) mod 4]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const u32 inc = wave_scan(v[12 + r]);
            tot[r] = read_lane(inc, 63);
            carried[r] += inc - v[12 + r];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] += carried[k & 3];
        u32 add[4];
        rot4(tot, cls0, add);   // add[c] = tot[(c - cls0) mod 4]
#pragma unroll
        for (int c = 0; c < 4; ++c) run.s[c] += add[c];
#pragma unroll
        for (int m = 0; m < 8; ++m) mine[m] = make_uint2(v[2 * m], v[2 * m + 1]);
        wave_lds_sync();
        // ranks below lim are stored: rank 64 q + ln sits at word 72 q + wl;
        // the stores take a scalar base and the lane's byte offset
        const u64 gbase = run.c;
        const u64 room = gbase < a.n ? a.n - gbase : 0;
        const u32 lim = first_lane(room < segcnt ? (u32)room : segcnt);
        const u64 op = (u64)(uintptr_t)(a.out + (gbase < a.n ? gbase : 0));
        gbyte *ob = (gbyte *)(uintptr_t)(((u64)first_lane((u32)(op >> 32)) << 32) | first_lane((u32)op));
        const u32 wl = ln + ((ln >> 4) << 1);
        const u32 nr = (lim + kWave - 1) / kWave;
        u32 yv[16];   // all 16 rows read first (words of this wavefront's area)
#pragma unroll
        for (u32 q = 0; q < 16; ++q) yv[q] = rows[wl + 72u * q];
#pragma unroll
        for (u32 q = 0; q < 16; ++q) {
            if (q >= nr) break;
            if (q * kWave + ln < lim) *(gword *)(ob + ((q * kWave + ln) << 2)) = yv[q];
        }
        wave_lds_sync();   // the next segment rewrites the rows
        run.c += segcnt;
    };
    const bool interior = wv >= 16 && wv + W + 4 <= a.vend;
    if (interior)
        (void)d4_group<false, SEGS>(a, wv, f);
    else
        (void)d4_group<true, SEGS>(a, wv, f);
}

template <int SEGS>
hipError_t launch4_t(const Stream4Args &a, int wpb, hipStream_t s) {
    if (a.block_units != (u32)wpb || a.nblocks != (a.nunits + wpb - 1) / wpb) return hipErrorInvalidValue;
    k4_agg<SEGS><<<a.nblocks, wpb * kWave, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k4_scan<<<1, kScanBlock, 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const u64 ngroups = (a.vend + SEGS * kSegBytes - 1) / (SEGS * kSegBytes);
    const u32 gblocks = (u32)((ngroups + wpb - 1) / wpb);
    k4_known<SEGS><<<gblocks, wpb * kWave, (size_t)wpb * kStageWords * sizeof(u32), s>>>(a);
    return hipGetLastError();
}

// ============================================================ intersection
// List intersection with the decode and the consumer fused, so that the
// list's identifiers never leave the chip (section 5 consumes a list from a
// buffer that stays in cache; here the buffer is a tile's registers).  The
// tile slots come from the two-pass aggregate and scan (k_tile_agg,
// k_tile_block_sums, k_tile_block_scan): each tile knows the rank and the
// running identifier at its first byte.  k_isect_tiles decodes a tile with
// that prefix and tests each identifier of rank below na against the sorted
// array b: the wavefront's smallest and largest identifiers bound a window
// of b (a 32-way search per bound), the window goes to LDS when it fits,
// and each lane walks the entries between its smallest and largest
// identifiers, comparing each with all of its identifiers.  The first run counts
// each tile's matches into a second row of slots; the same block scans turn
// those into each tile's first output position; the second run decodes and
// tests the tile again and stores its matches there, in list order.
// k_isect_status gives the status that decoding in pieces of `piece`
// integers gives (reading R15), from the stream's totals.
constexpr u32 kIsectWin = kStageWords;   // entries of b a wavefront holds in LDS

// The wavefront's identifiers, as the tile decode hands them over: the
// candidate of every byte and, per segment, the lane's code starts of rank
// below n.
template <int SEGS>
struct IsectCons {
    u32 u[SEGS][16];
    u32 m[SEGS];
    __device__ __forceinline__ void take(int s, const u32 (&v)[16], u32 emit, u64 gbase, u64 n,
                                         u32 segcnt) {
        u32 e = emit;
        if (gbase + segcnt > n) {
            // the codes of rank n and above are not the list's
            const u32 c = (u32)__builtin_popcount(emit);
            const u64 r0 = gbase + (wave_scan(c) - c);   // rank of the lane's first code
            const u32 keep = r0 >= n ? 0u : (n - r0 < c ? (u32)(n - r0) : c);
            while ((u32)__builtin_popcount(e) > keep) e &= ~(0x80000000u >> __builtin_clz(e));
        }
        m[s] = e;
#pragma unroll
        for (int j = 0; j < 16; ++j) u[s][j] = v[j];
    }
};

__device__ __forceinline__ u32 wave_min(u32 x) {
#pragma unroll
    for (int o = 32; o; o >>= 1) {
        const u32 y = (u32)__shfl_xor((int)x, o);
        x = y < x ? y : x;
    }
    return first_lane(x);
}
__device__ __forceinline__ u32 wave_max(u32 x) {
#pragma unroll
    for (int o = 32; o; o >>= 1) {
        const u32 y = (u32)__shfl_xor((int)x, o);
        x = y > x ? y : x;
    }
    return first_lane(x);
}

// first = the first index with b[i] >= lo, last = the first index with
// b[i] > hi (b sorted ascending), by lanes 0..31 and 32..63 at once: each
// round, lane l of a half probes the l-th of up to 32 evenly spaced entries
// of the range where its answer lies; the probes below the answer form a
// prefix, counted by a ballot, and the range shrinks to the gap between the
// last of them and the next probe.
__device__ __forceinline__ void wave_bounds(const u32 *b, u64 nb, u32 lo, u32 hi, u64 &first,
                                            u64 &last) {
    const u32 ln = lane_id(), half = ln >> 5, l = ln & 31u;
    const u32 x = half ? hi : lo;
    u64 a0 = 0, a1 = nb, c0 = 0, c1 = nb;   // answers in [a0, a1] and [c0, c1]
    while (a0 < a1 || c0 < c1) {
        const u64 sa = (a1 - a0 + 31) >> 5, sc = (c1 - c0 + 31) >> 5;
        const u64 r0 = half ? c0 : a0, r1 = half ? c1 : a1, st = half ? sc : sa;
        const u64 p = r0 + (u64)l * st;
        bool below = false;
        if (p < r1) {
            const u32 v = b[p];
            below = half ? v <= x : v < x;
        }
        const u64 bm = ballot(below);
        const u64 ka = (u64)__builtin_popcount((u32)bm), kc = (u64)__builtin_popcount((u32)(bm >> 32));
        if (a0 < a1) {
            const u64 nhi = a0 + ka * sa;
            a1 = nhi < a1 ? nhi : a1;
            a0 = ka ? a0 + (ka - 1) * sa + 1 : a0;
        }
        if (c0 < c1) {
            const u64 nhi = c0 + kc * sc;
            c1 = nhi < c1 ? nhi : c1;
            c0 = kc ? c0 + (kc - 1) * sc + 1 : c0;
        }
    }
    first = a0;
    last = c0;
}

// Entries of win[0, W) (sorted, W >= 1) below x, by steps of top, top/2,
// ..., 1 (top the highest power of two <= W).
template <class P>
__device__ __forceinline__ u32 count_below(P win, u32 W, u32 top, u32 x) {
    u32 pos = 0;
    for (u32 step = top; step; step >>= 1) {
        const u32 q = pos + step;
        const u32 v = win[(q <= W ? q : W) - 1];
        pos = (q <= W && v < x) ? q : pos;
    }
    return pos;
}

// Match masks of the wavefront's identifiers against win[0, W).  A lane
// walks the entries between the smallest and the largest of its valid
// identifiers in a segment (lo[s], hi[s]) and compares each with all 16 of
// its identifiers; with sorted identifiers that range holds a few entries.
// After kMergeRounds entries the lanes that still have some (identifiers
// that wrap mod 2^32, or a short list much denser than the list) test each
// identifier by a binary search instead.
constexpr u32 kMergeRounds = 16;
template <int SEGS, class P>
__device__ __forceinline__ void match_window(P win, u32 W, u32 top, const IsectCons<SEGS> &c,
                                             const u32 (&lo)[SEGS], const u32 (&hi)[SEGS],
                                             u32 (&mt)[SEGS]) {
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u32 m = c.m[s];
        u32 pos = count_below(win, W, top, lo[s]);
        u32 f = 0;
        bool act = m != 0;
        for (u32 it = 0;; ++it) {
            u32 x = 0;
            if (act) {
                x = win[pos < W ? pos : W - 1];
                act = pos < W && x <= hi[s];
            }
            if (ballot(act) == 0 || it == kMergeRounds) break;
            if (act) {
#pragma unroll
                for (int j = 0; j < 16; ++j) f |= (c.u[s][j] == x) ? (1u << j) : 0u;
                ++pos;
            }
        }
        if (ballot(act) != 0 && act) {
            f = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const u32 q = count_below(win, W, top, c.u[s][j]);
                f |= (q < W && win[q < W ? q : W - 1] == c.u[s][j]) ? (1u << j) : 0u;
            }
        }
        mt[s] = f & m;
    }
}

template <bool WRITE>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_isect_tiles(IsectArgs a) {
    constexpr int SEGS = kIsectSegs;
    extern __shared__ __align__(16) u32 lds[];
    __shared__ WgShared sh;
    __shared__ u32 wmatch[kMaxWaves];
    const u32 tid = threadIdx.x, ln = lane_id();
    const u32 wib = tid >> 6;
    const u32 wpb = blockDim.x >> 6;
    u32 *stage = lds + wib * kStageWords;
    const u32 tile = blockIdx.x;
    const u64 tb = (u64)wpb * SEGS * kSegBytes;
    TileIn t{};
    t.base = a.s.base;
    t.vstart = a.s.vstart;
    t.vend = a.s.vend;
    t.tv = (u64)tile * tb;
    t.n = a.na;
    t.known_c = a.s.desc[tile].c & kCountMask;
    t.known_s = (u32)a.s.desc[tile].s;
    t.known_mal = false;
    IsectCons<SEGS> c;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) c.m[s] = 0;
    const bool interior = tile > 0 && t.tv + tb + 4 <= t.vend;
    TileOut r;
    if (interior)
        r = run_tile<1, kConsume, SEGS, false>(t, stage, sh, wib, wpb, &c);
    else
        r = run_tile<1, kConsume, SEGS, true>(t, stage, sh, wib, wpb, &c);

    // each segment's smallest and largest valid identifier of the lane
    u32 lo[SEGS], hi[SEGS];
    u32 mn = ~0u, mx = 0u;
    bool any = false;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        lo[s] = ~0u;
        hi[s] = 0u;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const bool v = (c.m[s] >> j) & 1u;
            lo[s] = v && c.u[s][j] < lo[s] ? c.u[s][j] : lo[s];
            hi[s] = v && c.u[s][j] > hi[s] ? c.u[s][j] : hi[s];
        }
        mn = lo[s] < mn ? lo[s] : mn;
        mx = hi[s] > mx ? hi[s] : mx;
        any = any || c.m[s] != 0;
    }
    u32 mt[SEGS];
#pragma unroll
    for (int s = 0; s < SEGS; ++s) mt[s] = 0;
    if (ballot(any) != 0 && a.nb > 0) {
        mn = wave_min(mn);
        mx = wave_max(mx);
        u64 first, last;
        wave_bounds(a.b, a.nb, mn, mx, first, last);
        const u32 W = (u32)(last - first);
        if (W > 0) {
            const u32 top = 0x80000000u >> __builtin_clz(W);
            if (W <= kIsectWin) {
                for (u32 i = ln; i < W; i += kWave) stage[i] = a.b[first + i];
                wave_lds_sync();
                match_window<SEGS>(stage, W, top, c, lo, hi, mt);
            } else {
                match_window<SEGS>(a.b + first, W, top, c, lo, hi, mt);
            }
        }
    }
    u32 cnt = 0;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) cnt += (u32)__builtin_popcount(mt[s]);
    const u32 wcount = wave_sum(cnt);
    if (ln == 0) wmatch[wib] = wcount;
    __syncthreads();
    if (!WRITE) {
        if (tid == 0) {
            u64 tot = 0;
            for (u32 k = 0; k < wpb; ++k) tot += wmatch[k];
            // the tile's own malformed flag rides in bit 37, as in the tile slots
            a.mdesc[tile].c = tot | ((u64)(r.mal ? 1u : 0u) << 37);
            a.mdesc[tile].s = 0;
        }
        return;
    }
    u64 base = a.mdesc[tile].c & kCountMask;   // the tile's first output position
    for (u32 k = 0; k < wib; ++k) base += wmatch[k];
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const u32 cs = (u32)__builtin_popcount(mt[s]);
        const u32 inc = wave_scan(cs);
        u64 pos = base + (inc - cs);
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if ((mt[s] >> j) & 1u) {
                if (pos < a.out_cap) a.out[pos] = c.u[s][j];
                ++pos;
            }
        base += read_lane(inc, 63);
    }
    if (tile == gridDim.x - 1 && wib == wpb - 1 && ln == 0) *a.d_count = base;
}

// The status of the list decoded in pieces of k = piece integers (reading
// R15), from the stream's totals: C terminators, the first run of five
// continuation bytes (at byte q0, if any) and the last byte.  A piece starts
// at the end c_j of code j = p k and looks at bytes [c_j, c_j + 5k); it fails
// as malformed once that window holds the whole run, i.e. for the first p
// with c_(pk) >= q0 + 5 - 5k, and that is p = T / k + 1 for T the
// terminators before byte q0 + 4 - 5k (p = 0 when that byte is before the
// stream).  Without a run: truncated when the last byte continues and the
// piece holding the last code (p = C / k) is among the P = ceil(na / k)
// pieces; else the pieces decode min(P k, C) codes, too few for na
// (truncated) or leaving codes or bytes behind (count).  One workgroup; the
// byte searches run only for a malformed stream.
constexpr u32 kStatusBlock = 256;
__global__ __launch_bounds__(kStatusBlock) void k_isect_status(IsectArgs a, u32 tb) {
    __shared__ u64 first_tile, q0_sh, t_sh;
    const u32 tid = threadIdx.x;
    const u64 C = *a.total, na = a.na, k = a.piece, P = (na + k - 1) / k;
    const u64 vs = a.s.vstart, ve = a.s.vend;
    const bool lastc = a.s.base[ve - 1] >= 0x80;   // the stream is not empty
    const bool mal = *a.scan_status == VBYTE_EMALFORMED;
    if (!mal) {
        if (tid == 0) {
            int32_t st;
            if (lastc) {
                st = C / k < P ? VBYTE_ETRUNC : VBYTE_ECOUNT;
            } else {
                const u64 done = P * k < C ? P * k : C;
                st = done < na ? VBYTE_ETRUNC : (done < C || done > na) ? VBYTE_ECOUNT : VBYTE_OK;
            }
            *a.d_status = st;
        }
        return;
    }
    if (tid == 0) {
        first_tile = ~0ull;
        q0_sh = ~0ull;
        t_sh = 0;
    }
    __syncthreads();
    // the first tile flagged in its match slot (bit 37): the tile decode flags
    // a run at the lane that holds its first byte, so the first run starts
    // in that tile and no run starts before it
    const u64 ntiles = a.s.ntiles;
    for (u64 i = tid; i < ntiles; i += kStatusBlock)
        if ((a.mdesc[i].c >> 37) & 1u) {
            atomicMin((unsigned long long *)&first_tile, (unsigned long long)i);
            break;
        }
    __syncthreads();
    // (should no tile be flagged, the status stays malformed and nothing is
    // searched; the search also covers the 4 bytes before the tile)
    const u64 tm = first_tile;
    if (tm >= ntiles) {
        if (tid == 0) *a.d_status = VBYTE_EMALFORMED;
        return;
    }
    const u64 lo0 = tm * tb >= vs + 4 ? tm * tb - 4 : vs;
    const u64 hi0 = (tm + 1) * tb < ve ? (tm + 1) * tb : ve;
    for (u64 p = lo0 + tid; p < hi0 && p + 5 <= ve; p += kStatusBlock) {
        bool run = true;
        for (u32 j = 0; j < 5; ++j) run = run && a.s.base[p + j] >= 0x80;
        if (run) {
            atomicMin((unsigned long long *)&q0_sh, (unsigned long long)p);
            break;
        }
    }
    __syncthreads();
    if (q0_sh >= ve) {
        if (tid == 0) *a.d_status = VBYTE_EMALFORMED;
        return;
    }
    const u64 q0 = q0_sh - vs;   // stream-relative
    const i64 X = (i64)q0 + 5 - 5 * (i64)k;
    u64 pm = 0;
    if (X > 0) {
        // terminators in stream bytes [0, X - 1): the tile slot's prefix and
        // the tile's bytes before X - 1
        const u64 ya = vs + (u64)X - 1, ty = ya / tb;
        const u64 from = ty * tb > vs ? ty * tb : vs;
        u32 cnt = 0;
        for (u64 p = from + tid; p < ya; p += kStatusBlock) cnt += a.s.base[p] < 0x80 ? 1u : 0u;
        atomicAdd((unsigned long long *)&t_sh, (unsigned long long)cnt);
        __syncthreads();
        const u64 T = (a.s.desc[ty].c & kCountMask) + t_sh;
        pm = T / k + 1;
    }
    if (tid == 0) *a.d_status = pm < P ? VBYTE_EMALFORMED : VBYTE_ECOUNT;
}

// ------------------------------------------------------------ batched lists
struct ListDesc {
    i64 bb, be, ob, n;
};

__device__ __forceinline__ ListDesc list_desc(const ListArgs &a, u64 i) {
    ListDesc d;
    if (a.rows) {
        const int64_t *r = a.rows + 4 * i;
        d.bb = r[0];
        d.be = r[1];
        d.ob = r[2];
        d.n = r[3];
    } else {
        d.bb = a.byte_off[i];
        d.be = a.byte_off[i + 1];
        d.ob = a.out_off[i];
        d.n = a.out_off[i + 1] - d.ob;
    }
    return d;
}

__device__ __forceinline__ bool list_ok(const ListArgs &a, const ListDesc &d) {
    return d.bb >= 0 && d.be >= d.bb && (u64)d.be <= a.nbytes && d.ob >= 0 && d.n >= 0 &&
           (u64)d.ob + (u64)d.n <= a.nout && (d.be - d.bb) < (1ll << 36);
}

// Prep: classify every list (empty / small / large) and build the work
// table with a decoupled look-back scan over blocks of kPrepBlock lists.
// Large lists get pieces of ub bytes, numbered [0, L), a list's pieces
// consecutive, with the list's item at its first piece (see pmap below); small lists get one slot each, counted down from
// max_items - 1 (so a slot needs no knowledge of L).
__global__ __launch_bounds__(kPrepBlock) void k_prep(ListArgs a, u32 nblocks, u64 ub) {
    __shared__ u32 sh_c[kPrepBlock / kWave], sh_s[kPrepBlock / kWave];
    __shared__ u32 sh_epoch;
    __shared__ u64 sh_exc;
    __shared__ u32 sh_exs;
    const u32 tid = threadIdx.x;
    const u32 ln = lane_id();
    const u32 wib = tid >> 6;
    __shared__ u32 sh_blk;
    if (tid == 0) {
        sh_blk = take_ticket(a.hdr + kTicketWord, gridDim.x);
        sh_epoch = (u32)aload(a.hdr);
    }
    __syncthreads();
    const u32 epoch = sh_epoch;
    const u32 blk = sh_blk;
    const u32 tag = make_tag(epoch);

    const u64 i = (u64)blk * kPrepBlock + tid;
    u32 nlarge = 0, nsmall = 0;
    if (i < a.nlists) {
        const ListDesc d = list_desc(a, i);
        if (!list_ok(a, d)) {
            a.list_status[i] = VBYTE_EINVAL;
        } else if (d.be == d.bb) {
            a.list_status[i] = d.n == 0 ? VBYTE_OK : VBYTE_ETRUNC;
        } else if ((u64)(d.be - d.bb) <= a.small_bytes) {
            nsmall = 1;
        } else {
            const u64 vs = (u64)(uintptr_t)(a.bytes + d.bb) & 15u;
            nlarge = (u32)((vs + (u64)(d.be - d.bb) + ub - 1) / ub);
            a.list_status[i] = VBYTE_OK;   // raised by the tile kernels (atomic max)
        }
    }
    const u32 cl = wave_scan(nlarge), cs = wave_scan(nsmall);
    if (ln == 63) {
        sh_c[wib] = cl;
        sh_s[wib] = cs;
    }
    __syncthreads();
    u32 wl = 0, ws = 0, bl = 0, bs = 0;
    for (u32 k = 0; k < kPrepBlock / kWave; ++k) {
        if (k < wib) {
            wl += sh_c[k];
            ws += sh_s[k];
        }
        bl += sh_c[k];
        bs += sh_s[k];
    }
    if (wib == 0) {
        Prefix ex;
        if (blk == 0) {
            ex = Prefix{0, 0, false};
        } else {
            if (ln == 0) publish<true>(&a.prep_desc[blk], tag, false, false, bl, bs);
            ex = lookback<true>(a.prep_desc, blk, 0, tag, a.spin_limit);
            if (ex.stalled && ln == 0) {
                mark_stalled(a.hdr + kStallWord, epoch);
                astore(&a.totals[2], 2);   // read by the decode launch after this one
            }
        }
        if (ln == 0) {
            publish<true>(&a.prep_desc[blk], tag, true, false, ex.c + bl, ex.s + bs);
            sh_exc = ex.c;
            sh_exs = ex.s;
            if (blk == nblocks - 1) {
                const u64 L = ex.c + bl, S = (u64)ex.s + bs;
                const bool fits = L + S <= a.max_items && L <= a.max_large;
                const bool stalled = launch_stalled(a.hdr + kStallWord, epoch);
                astore(&a.totals[0], fits && !stalled ? L : 0);
                astore(&a.totals[1], fits && !stalled ? S : 0);
                astore(&a.totals[2], stalled ? 2 : fits ? 0 : 1);
                astore(a.hdr, (u64)epoch + 1);   // every block has published
            }
        }
    }
    __syncthreads();
    const u64 lstart = sh_exc + wl + (cl - nlarge);
    const u64 sslot = (u64)sh_exs + ws + (cs - nsmall);
    if (nlarge || nsmall) {
        const ListDesc d = list_desc(a, i);
        const BatchItem it{d.bb, d.be, d.ob, d.n, (u32)i, 0u, a.prevs ? a.prevs[i] : 0u, 0u};
        if (nsmall && sslot < a.max_items) a.items[a.max_items - 1 - sslot] = it;
        if (nlarge && lstart < a.max_large) a.items[lstart] = it;   // the head
    }
    // every piece of a large list points at its head; the map is written by
    // the whole wavefront, lane l taking pieces l, l + 64, ..., so a list of
    // many pieces does not keep one lane busy long after the others
    for (u64 big = ballot(nlarge != 0); big; big &= big - 1) {
        const u32 j = (u32)__builtin_ctzll(big);
        const u32 nj = read_lane(nlarge, j);
        const u64 sj = ((u64)read_lane((u32)(lstart >> 32), j) << 32) | read_lane((u32)lstart, j);
        for (u32 k = ln; k < nj; k += kWave)
            if (sj + k < a.max_large) a.pmap[sj + k] = (u32)sj;
    }
}

// Large lists of a batch: each list is cut into pieces of SEGS KiB, one per
// wavefront.  The prep numbers the pieces of all large lists [0, L), a
// list's pieces consecutive, stores each large list's item once, at the
// index of its first piece (its head), and maps every piece to its head
// (pmap[k] = head, 4 bytes a piece, so a list of many pieces costs little to
// lay out); piece k is then the list's piece k - head.  Two passes with no
// look-back and no queue, as for a single stream: k_list_agg stores each
// piece's terminator count and byte sum in slot k, the block scans turn the
// slots into exclusive prefixes over all pieces, and k_list_known decodes
// each piece alone with its prefix within its list, the slot's prefix minus
// that of the list's head (a list of one piece needs no slot: k_list_agg
// skips it and k_list_known finds its malformed runs).  A run of five
// continuation bytes raises its list's status to malformed (atomic max); the
// wavefront holding a list's last byte raises it to the list's truncation
// or count status the same way, so the list ends with the larger code.  Both
// kernels launch one wavefront per piece the table can hold (those past L
// return at once) and keep a grid stride for grids that are capped.
__device__ __forceinline__ void list_geometry(const ListArgs &a, const BatchItem &d, const u8 *&base,
                                              u64 &vstart, u64 &vend) {
    const u8 *p0 = a.bytes + d.bb;
    base = (const u8 *)((uintptr_t)p0 & ~(uintptr_t)15);
    vstart = (u64)(p0 - base);
    vend = vstart + (u64)(d.be - d.bb);
}

constexpr u64 kListGridCap = 1u << 16;   // workgroups of the piece kernels

template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock) void k_list_agg(ListArgs a) {
    const u32 ln = lane_id();
    const u64 ub = (u64)SEGS * kSegBytes;
    u64 L = aload(&a.totals[0]);
    L = L < a.max_large ? L : a.max_large;
    // the wavefront's index made uniform, so the table loads are scalar
    const u64 W = (u64)gridDim.x * (blockDim.x >> 6);
    const u64 k0 = (u64)blockIdx.x * (blockDim.x >> 6) + (u32)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (u64 k = k0; k < L; k += W) {
        const u32 head = a.pmap[k];
        const BatchItem d = a.items[head];
        const u8 *base;
        u64 vstart, vend;
        list_geometry(a, d, base, vstart, vend);
        const u64 wv = (k - head) * ub;   // < vend: the prep makes no empty piece
        if (vend <= ub) {
            // a list of one piece: its prefix is the list's start, so the
            // decode pass needs no slot (it also finds a malformed run)
            if (ln == 0) {
                a.desc[k].c = 0;
                a.desc[k].s = 0;
            }
            continue;
        }
        u32 cont, sum;
        bool mal;
        if (wv >= vstart + 4 && wv + ub <= vend)
            wave_agg<D, SEGS, false>(base, vstart, vend, wv, cont, sum, mal);
        else
            wave_agg<D, SEGS, true>(base, vstart, vend, wv, cont, sum, mal);
        const u64 lo = wv > vstart ? wv : vstart, hi = wv + ub < vend ? wv + ub : vend;
        if (mal && ln == 0) atomicMax(&a.list_status[d.li], (int32_t)VBYTE_EMALFORMED);
        if (ln == 0) {
            a.desc[k].c = hi - lo - cont;
            a.desc[k].s = sum;
        }
    }
}

template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(D ? 4 : 8))) void k_list_known(ListArgs a) {
    extern __shared__ __align__(16) u32 lds[];
    __shared__ WgShared sh;   // not used by wavefronts that decode alone
    const u32 wib = (u32)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = lane_id();
    u32 *stage = lds + wib * kStageWords;
    const u64 ub = (u64)SEGS * kSegBytes;
    u64 L = aload(&a.totals[0]);
    L = L < a.max_large ? L : a.max_large;
    const u64 W = (u64)gridDim.x * (blockDim.x >> 6);
    const u64 k0 = (u64)blockIdx.x * (blockDim.x >> 6) + wib;
    for (u64 k = k0; k < L; k += W) {
        const u32 head = a.pmap[k];
        const BatchItem d = a.items[head];
        TileIn t{};
        list_geometry(a, d, t.base, t.vstart, t.vend);
        const u64 wv = (k - head) * ub;
        const Desc sq = a.desc[k], s0 = a.desc[head];
        t.tv = wv;
        t.out = a.out + d.ob;
        t.n = (u64)d.n;
        t.known_c = (sq.c & kCountMask) - (s0.c & kCountMask);
        t.known_s = d.prev + ((u32)sq.s - (u32)s0.s);
        TileOut r;
        // the piece is its own one-wavefront tile (wavefront index 0 of 1)
        if (wv >= t.vstart + 4 && wv + ub + 4 <= t.vend)
            r = run_tile<D, kKnownW, SEGS, false>(t, stage, sh, 0, 1);
        else
            r = run_tile<D, kKnownW, SEGS, true>(t, stage, sh, 0, 1);
        if (t.vend <= ub && r.mal && ln == 0) atomicMax(&a.list_status[d.li], (int32_t)VBYTE_EMALFORMED);
        if (wv + ub >= t.vend && ln == 0)
            atomicMax(&a.list_status[d.li], final_status(false, t.base[t.vend - 1], r.total, t.n));
    }
}

// Small list: one wavefront walks its segments in order, carrying the rank
// and the running sum, with no look-back.
template <int D>
__device__ __forceinline__ void run_small(const ListArgs &a, const BatchItem &d, u32 *rows) {
    constexpr bool DELTA = D != 0, RANK = D == 2;
    const u32 ln = lane_id();
    const u8 *p0 = a.bytes + d.bb;
    const u8 *base = (const u8 *)((uintptr_t)p0 & ~(uintptr_t)15);
    const u64 vstart = (u64)(p0 - base);
    const u64 vend = vstart + (u64)(d.be - d.bb);
    const u8 last = base[vend - 1];   // for the status, loaded with the first segment
    u32 *out = a.out + d.ob;
    const u64 n = (u64)d.n;
    u64 rank = 0;
    u32 run = d.prev;
    bool mal = false;
    u32 pw = 0, pv = 0;   // lane 63's last dword and validity of the previous segment
    for (u64 tv = 0; tv < vend; tv += kSegBytes) {
        u32 w[4], valid, nw, nv;
        load16_guarded(base, tv + 16u * ln, vstart, vend, w, valid);
        load4_guarded(base, (i64)(tv + kSegBytes), vstart, vend, nw, nv);
        const u32 below = from_lane_below(w[3], pw);
        const bool below_ok = ((from_lane_below(valid, pv) >> 15) & 1u) != 0;
        const u32 ab = from_lane_above(w[0], nw);
        const u32 abv = from_lane_above(valid, nv) & 0xFu;
        const SegMask m = seg_mask<true>(w, valid, below, below_ok, ab, abv);
        mal |= m.mal;
        const u32 segcnt = wave_sum(__builtin_popcount(m.emit));
        u32 r[16];
        const u32 ls = horner<DELTA>(w, ab, m.emit, r);
        u32 segsum = 0;
        if (DELTA) {
            const u32 si = wave_scan(ls);
            segsum = read_lane(si, 63);
            const u32 add = run + si;
#pragma unroll
            for (int j = 0; j < 16; ++j) r[j] += add;
        }
        if (segcnt && rank < n) {
            if (rank + segcnt <= n)
                store_rows<false, RANK>(rows, r, m.emit, out + rank, 0u, (u32)rank);
            else
                store_rows<true, RANK>(rows, r, m.emit, out + rank, (u32)(n - rank), (u32)rank);
        }
        rank += segcnt;
        run += segsum;
        pw = read_lane(w[3], 63);
        pv = read_lane(valid, 63);
    }
    const bool anymal = ballot(mal) != 0;
    // every lane stores the same (uniform) status word
    a.list_status[d.li] = final_status(anymal, last, rank, n);
}

// Several small lists in one wavefront: list q of the pack (q < m) takes the
// c_q lanes from lane s_q = (c_0 + ... + c_(q-1)), one aligned 16-byte chunk
// of its bytes per lane (c_q = ceil((vstart + bytes) / 16) <= 64), so a lane
// never holds two lists.  The halos stop at the list's first and last lanes;
// the count and sum scans run over the whole wavefront and each lane takes
// off the value at its list's first lane; the integers are compacted in LDS
// in wavefront order and each list's run is copied to its output.  Lane q
// brings list q's item (`it`, `need` = c_q, `incl` = s_q + c_q).
__device__ __forceinline__ u32 lane_u32(u32 v, u32 l) {
    return (u32)__builtin_amdgcn_ds_bpermute((int)(l << 2), (int)v);
}
__device__ __forceinline__ u64 lane_u64(u64 v, u32 l) {
    return ((u64)lane_u32((u32)(v >> 32), l) << 32) | lane_u32((u32)v, l);
}
__device__ __forceinline__ u32 wave_scan_max(u32 x) {   // x >= 0: 0 is the identity
    x = max(x, dpp_zero<0x111>(x));
    x = max(x, dpp_zero<0x112>(x));
    x = max(x, dpp_zero<0x114>(x));
    x = max(x, dpp_zero<0x118>(x));
    x = max(x, dpp_zero<0x142, 0xA>(x));
    x = max(x, dpp_zero<0x143, 0xC>(x));
    return x;
}

template <int D>
__device__ __forceinline__ void run_packed(const ListArgs &a, const BatchItem &it, u32 need, u32 incl,
                                           u32 m, u32 *stage) {
    constexpr bool DELTA = D != 0, RANK = D == 2;
    const u32 ln = lane_id();
    // lane -> list of the pack: list q marks its first lane, a max scan spreads it
    stage[ln] = 0;
    wave_lds_sync();
    if (ln < m) stage[incl - need] = ln + 1;
    wave_lds_sync();
    const u32 q1 = wave_scan_max(stage[ln]);   // 1 + the lane's list, 0 past the pack
    wave_lds_sync();
    const u32 q = q1 ? q1 - 1 : 0;
    const u32 used = read_lane(incl, m - 1);   // lanes the pack takes
    const bool in = ln < used;
    // the list's fields from lane q
    const u64 bb = lane_u64((u64)it.bb, q), be = lane_u64((u64)it.be, q);
    const u32 prev = lane_u32(it.prev, q);
    const u32 s0 = lane_u32(incl - need, q), cq = lane_u32(need, q);
    const u32 o = ln - s0;   // the lane's chunk within its list
    const u8 *p0 = a.bytes + bb;
    const u8 *base = (const u8 *)((uintptr_t)p0 & ~(uintptr_t)15);
    const u64 vstart = (u64)(p0 - base);
    const u64 vend = vstart + (be - bb);
    u32 w[4] = {0, 0, 0, 0}, valid = 0;
    if (in) load16_guarded(base, 16u * o, vstart, vend, w, valid);
    const bool first = o == 0, last = o + 1 == cq;
    // cross-lane reads in uniform control flow, then the list edges applied
    u32 below = from_lane_below(w[3], 0u);
    const u32 bv = from_lane_below(valid, 0u);
    const bool below_ok = !first && ((bv >> 15) & 1u) != 0;
    if (first) below = 0;
    u32 ab = from_lane_above(w[0], 0u);
    u32 abv = from_lane_above(valid, 0u) & 0xFu;
    if (last || !in) {
        ab = 0;
        abv = 0;
    }
    const SegMask mk = seg_mask<true>(w, valid, below, below_ok, ab, abv);
    // the list's last byte, from the lane that holds it
    u32 lastb = 0;
    if (in && last) {
        const u32 k = (u32)(vend - 1 - 16u * o);   // 0..15
        const u32 word = k < 4 ? w[0] : k < 8 ? w[1] : k < 12 ? w[2] : w[3];
        lastb = (word >> (8 * (k & 3))) & 0xFFu;
    }
    const u32 cnt = (u32)__builtin_popcount(mk.emit);
    const u32 ci = wave_scan(cnt);
    const u32 cx = ci - cnt;                  // codes of the wavefront before the lane
    const u32 cbase = lane_u32(cx, s0);       // ... before the list's first lane
    u32 r[16];
    if (DELTA) {
        const u32 ls = horner<true>(w, ab, mk.emit, r);
        const u32 si = wave_scan(ls);
        const u32 sx = si - ls;
        const u32 add = prev + (sx - lane_u32(sx, s0)) + ls;
#pragma unroll
        for (int j = 0; j < 16; ++j) r[j] += add;
    } else {
        horner<false>(w, ab, mk.emit, r);
    }
    // compact the integers in wavefront order (rank term for differences
    // minus one: the code's rank within its list)
    u32 pos = cx;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if ((mk.emit >> j) & 1u) {
            stage[pos] = RANK ? r[j] + (pos - cbase) : r[j];
            ++pos;
        }
    wave_lds_sync();
    const u64 malm = ballot(mk.mal);
    for (u32 k = 0; k < m; ++k) {
        const u32 ks = read_lane(incl - need, k), kc = read_lane(need, k);
        const u32 from = read_lane(cx, ks), to = read_lane(ci, ks + kc - 1);
        const u64 n = ((u64)read_lane((u32)((u64)it.n >> 32), k) << 32) | read_lane((u32)it.n, k);
        const u64 ob = ((u64)read_lane((u32)((u64)it.ob >> 32), k) << 32) | read_lane((u32)it.ob, k);
        const u32 total = to - from;
        const u32 lim = (u64)total < n ? total : (u32)n;
        for (u32 i = ln; i < lim; i += kWave) a.out[ob + i] = stage[from + i];
        const u64 lm = (kc >= 64 ? ~0ull : ((1ull << kc) - 1)) << ks;
        if (ln == 0)
            a.list_status[read_lane(it.li, k)] =
                final_status((malm & lm) != 0, (u8)read_lane(lastb, ks + kc - 1), total, n);
    }
    wave_lds_sync();
}

// Persistent decode of the small lists of a batch: each wavefront of the
// grid takes a fixed share of them (below).
template <int D, int SEGS>
__global__ __launch_bounds__(kMaxBlock) void k_batch(ListArgs a) {
    extern __shared__ __align__(16) u32 lds[];
    const u32 tid = threadIdx.x;
    const u32 wib = (u32)__builtin_amdgcn_readfirstlane(tid >> 6);
    u32 *stage = lds + wib * kStageWords;
    const u64 S = aload(&a.totals[1]);
    const u64 fail_code = aload(&a.totals[2]);   // 1: the work table was too small; 2: prep stalled
    const bool failed = fail_code != 0;
    const u64 G = gridDim.x;

    // Wavefront w of the W in the grid takes the consecutive small lists
    // [w S / W, (w + 1) S / W) (no queue: the lists need no ordering).  It
    // packs the next lists that fit in 64 lanes (16 bytes each) into one
    // pass; a list of more than 64 lanes decodes alone, segment by segment.
    const u32 ln = lane_id();
    const u64 W = G * (blockDim.x >> 6);
    const u64 wid = (u64)blockIdx.x * (blockDim.x >> 6) + wib;
    {
        const u64 lo = wid * S / W;
        const u64 hi = (wid + 1) * S / W;
        for (u64 p = lo; p < hi;) {
            BatchItem it{};
            u32 need = 65;   // lanes of the list at lane t (65: none, never fits)
            if (p + ln < hi) {
                it = a.items[a.max_items - 1 - (p + ln)];
                const u64 vs = (u64)(uintptr_t)(a.bytes + it.bb) & 15u;
                const u64 l = (vs + (u64)(it.be - it.bb) + 15) >> 4;
                need = l < 65 ? (u32)l : 65u;
            }
            if (read_lane(need, 0) > 64) {
                const BatchItem d = a.items[a.max_items - 1 - p];
                run_small<D>(a, d, stage);
                ++p;
                continue;
            }
            const u32 incl = wave_scan(need);
            const u32 m = (u32)__builtin_popcountll(ballot(incl <= 64 && p + ln < hi));
            run_packed<D>(a, it, need, incl, m, stage);
            p += m;
        }
    }
    if (failed) {
        const u64 nthreads = (u64)gridDim.x * blockDim.x;
        for (u64 i = (u64)blockIdx.x * blockDim.x + tid; i < a.nlists; i += nthreads)
            a.list_status[i] = fail_code == 2 ? VBYTE_ESTALLED : VBYTE_EINVAL;
    }
}

// ------------------------------------------------------------ encoder
// Canonical ENC (section 1): L(x) bytes, 7 bits each, least significant
// first, top bit set on all but the last.  delta: 1 codes x_i - x_(i-1),
// 2 codes x_i - x_(i-1) - 1 after the first (x_(-1) = prev).
//
// Two passes over the values with no look-back.  The values are addressed
// from the 16-byte-aligned element at or below values[0] (e0 elements
// before it); chunk c is aligned elements [256 c, 256 c + 256): one 128-bit
// load per lane of a wavefront.  k_enc_len stores each chunk's byte count
// and each of its workgroups' totals; k_enc_bscan turns the counts into
// exclusive byte offsets (a scan workgroup's carry is the sum of the length
// workgroups' totals before it; the last block writes the total);
// k_enc_write loads the chunk again and gives
// every value its byte offset (lane scan plus the chunk offset).  A chunk
// whose codes are all one byte, or all one or two bytes, is stored straight
// from registers as dwords (a lane's codes then span at least four bytes, so
// a dword holds bytes of at most two lanes); any other chunk is built in LDS
// by OR-ing each code, shifted to its byte offset, into the one or two dwords
// it touches (codes never overlap, so the ORs assemble the bytes exactly) and
// stored from there.  Dwords shared with the neighbouring chunks go out byte
// by byte in every form.  k_enc_bounds gives every CSR
// list boundary its byte offset: the chunk offset plus the lengths of the
// values before it in its chunk.
constexpr int kEncPerWave = 8;        // chunks per wavefront in k_enc_len
constexpr int kEncWritePerWave = 1;   // chunks per wavefront in k_enc_write

__device__ __forceinline__ u32 code_len(u32 x) {
    return 1u + (x >= (1u << 7)) + (x >= (1u << 14)) + (x >= (1u << 21)) + (x >= (1u << 28));
}

// The code of x in a 64-bit word (bytes 0..L-1, the rest zero): the five
// 7-bit groups spread to bytes 0..4, continuation bits on bytes 0..L-2.
__device__ __forceinline__ u64 code_bytes(u32 x, u32 len) {
    const u32 lo = (x & 0x7Fu) | ((x << 1) & 0x7F00u) | ((x << 2) & 0x7F0000u) | ((x << 3) & 0x7F000000u);
    const u64 c = ((u64)(x >> 28) << 32) | lo;
    const u64 cont = 0x8080808080ull & ((1ull << (8 * (len - 1))) - 1);   // len >= 1
    return (c | cont) & ((1ull << (8 * len)) - 1);
}

// Lane l's four values of chunk c (aligned elements 256 c + 4 l .. + 3) as
// the integers to code (values, or their differences), with a validity
// mask (bit j: element j is values[i] for some 0 <= i < n).
__device__ __forceinline__ u32 enc_load(const EncArgs &a, u64 c, u32 (&v)[4]) {
    const u32 ln = lane_id();
    const u64 a0 = c * kEncChunk + 4u * ln;   // aligned index of element 0
    const u64 lo = a.e0, hi = a.e0 + a.n;     // valid aligned indices
    u32 valid = 0;
    if (a0 >= lo && a0 + 4 <= hi) {
        const uint4 q = *(const uint4 *)(a.vbase + a0);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
        valid = 0xFu;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u64 ai = a0 + k;
            v[k] = 0;
            if (ai >= lo && ai < hi) {
                v[k] = a.vbase[ai];
                valid |= 1u << k;
            }
        }
    }
    if (a.delta) {
        // the value before each element: the lane's own, the lane below's
        // last, or (lane 0) the element before the chunk, or prev
        const u64 c0 = c * kEncChunk;
        u32 before_chunk = a.prev;
        if (c0 > lo && c0 - 1 < hi) before_chunk = a.vbase[c0 - 1];
        const u32 below = from_lane_below(v[3], before_chunk);
        const u32 m1 = a.delta == 2 ? 1u : 0u;
        u32 p = below;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u64 ai = a0 + k;
            const u32 x = v[k];
            // the first value takes prev, with no minus one
            const bool first = ai == lo;
            v[k] = first ? x - a.prev : x - p - m1;
            p = x;
        }
    }
    return valid;
}

// A wavefront takes kEncPerWave consecutive chunks, all loads issued first;
// a workgroup (kEncLenWaves wavefronts, kEncLenChunks chunks) also stores
// its chunks' total for the scan.
constexpr u32 kEncLenWaves = kEncLenChunks / kEncPerWave;
static_assert(kEncLenWaves * kEncPerWave == kEncLenChunks, "a length workgroup's chunks");

__global__ __launch_bounds__(kEncLenWaves * kWave) void k_enc_len(EncArgs a) {
    __shared__ u32 wt[kEncLenWaves];
    const u32 ln = lane_id(), wib = threadIdx.x >> 6;
    const u64 c0 = ((u64)blockIdx.x * kEncLenWaves + wib) * kEncPerWave;
    u32 v[kEncPerWave][4], valid[kEncPerWave];
#pragma unroll
    for (int q = 0; q < kEncPerWave; ++q)
        valid[q] = c0 + q < a.nchunks ? enc_load(a, c0 + q, v[q]) : 0u;
    u32 mine = 0;   // lane q ends up with chunk q's count
    u32 tot = 0;
#pragma unroll
    for (int q = 0; q < kEncPerWave; ++q) {
        u32 len = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) len += (valid[q] >> k) & 1u ? code_len(v[q][k]) : 0u;
        len = wave_sum(len);
        mine = ln == (u32)q ? len : mine;
        tot += len;
    }
    if (ln < (u32)kEncPerWave && c0 + ln < a.nchunks) a.csum[c0 + ln] = mine;
    if (ln == 0) wt[wib] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;   // at most kEncLenChunks x 1280
        for (u32 k = 0; k < kEncLenWaves; ++k) t += wt[k];
        a.gsum[blockIdx.x] = t;
    }
}

constexpr u64 kEncScanSpan = 8 * kScanBlock;   // chunk counts per scan workgroup (8 per thread)
static_assert(kEncScanSpan % kEncLenChunks == 0, "a scan block holds whole length workgroups");

// Scan workgroup b: its carry is the sum of the length workgroups' totals
// before its first chunk (every thread adds a strided share), then each
// thread scans 8 consecutive chunk counts.
__global__ __launch_bounds__(kScanBlock) void k_enc_bscan(EncArgs a) {
    __shared__ u64 carry_sh, part[kScanBlock / kWave];
    __shared__ u32 wtot[kScanBlock / kWave];
    const u32 tid = threadIdx.x, wib = tid >> 6, ln = lane_id();
    const u32 b = blockIdx.x, nb = gridDim.x;
    {
        const u64 ng = (u64)b * (kEncScanSpan / kEncLenChunks);
        u64 c = 0;
        for (u64 k = tid; k < ng; k += kScanBlock) c += a.gsum[k];
        // 64-bit lane sums as 24 low bits and the rest
        const u32 lo = wave_sum((u32)c & 0xFFFFFFu), hi = wave_sum((u32)(c >> 24));
        if (ln == 0) part[wib] = ((u64)hi << 24) + lo;
    }
    // thread t holds the 8 consecutive counts 8 t .. 8 t + 7 of the block
    const u64 i0 = (u64)b * kEncScanSpan + 8u * tid;
    u32 cnt[8], lsum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        cnt[k] = i0 + k < a.nchunks ? a.csum[i0 + k] : 0u;
        lsum += cnt[k];
    }
    const u32 incl = wave_scan(lsum);   // a wavefront's 512 counts fit 32 bits
    if (ln == 63) wtot[wib] = incl;
    __syncthreads();
    if (tid == 0) {
        u64 t = 0;
        for (u32 k = 0; k < kScanBlock / kWave; ++k) t += part[k];
        carry_sh = t;
    }
    __syncthreads();
    u64 off = carry_sh;
    for (u32 k = 0; k < wib; ++k) off += wtot[k];
    off += incl - lsum;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (i0 + k < a.nchunks) a.cpre[i0 + k] = off;
        off += cnt[k];
    }
    if (b == nb - 1 && tid == kScanBlock - 1) *a.d_nbytes = off;   // the last thread's end: the total
}

// Writes one chunk's codes: lane values v (valid mask), chunk byte offset
// `base`; st is the wavefront's LDS stage.
__device__ __forceinline__ void enc_write_chunk(const EncArgs &a, u32 *st, const u32 (&v)[4],
                                                u32 valid, u64 base) {
    const u32 ln = lane_id();
    if (ballot(valid != 0xFu || (v[0] | v[1] | v[2] | v[3]) >= 128u) == 0) {
        // Every code of the chunk is one byte: its 256 bytes are the values
        // in order, lane l's four at base + 4 l.  Dword j of the dword-aligned
        // window holds lane j's bytes shifted up by the window's offset m
        // and lane j - 1's top m bytes; the first and last dwords also hold
        // bytes of the neighbouring chunks, so their own bytes go out one by
        // one.  No LDS.
        const u32 m = (u32)(((uintptr_t)a.bytes + base) & 3u);
        const u32 p = v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
        const u32 below = from_lane_below(p, 0u);
        const u32 dw = m ? (p << (8u * m)) | (below >> (32u - 8u * m)) : p;
        const u64 g0 = base - m + 4u * ln;   // byte index of the lane's dword
        if ((ln > 0 || m == 0) && g0 + 4 <= a.capacity) {
            *(u32 *)(a.bytes + g0) = dw;
        } else {
            for (u32 t = ln == 0 ? m : 0u; t < 4; ++t)
                if (g0 + t < a.capacity) a.bytes[g0 + t] = (u8)(dw >> (8 * t));
        }
        if (ln == 63 && m) {   // lane 63's top m bytes start the dword after
            const u32 top = p >> (32u - 8u * m);
            for (u32 t = 0; t < m; ++t)
                if (g0 + 4 + t < a.capacity) a.bytes[g0 + 4 + t] = (u8)(top >> (8 * t));
        }
        return;
    }
    if (ballot(valid != 0xFu || (v[0] | v[1] | v[2] | v[3]) >= 16384u) == 0) {
        // Every code is one or two bytes, so a lane's codes take 4..8 bytes
        // and a dword of the window holds bytes of at most two lanes.  Dword
        // j is written by the lane that holds its first byte of the chunk:
        // its own bytes there, ORed with the first dword of the lane above
        // when that lane starts inside it.  The window's first and last
        // dwords, shared with the neighbouring chunks, go out byte by byte.
        const u32 m = (u32)(((uintptr_t)a.bytes + base) & 3u);
        u64 pk = 0;
        u32 nb = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u32 x = v[k];
            const u32 two = x >= 128u ? 1u : 0u;
            const u32 c = two ? ((x & 0x7Fu) | 0x80u | ((x >> 7) << 8)) : x;
            pk |= (u64)c << (8 * nb);
            nb += 1 + two;
        }
        const u32 incl = wave_scan(nb);
        const u32 endb = m + read_lane(incl, 63);   // one past the chunk's last window byte
        const u32 off = m + incl - nb;              // the lane's first window byte
        const u32 sh = off & 3u, w = off >> 2, e = (off + nb - 1) >> 2;
        const u64 lo = pk << (8 * sh);
        const u32 q[3] = {(u32)lo, (u32)(lo >> 32), sh ? (u32)(pk >> (64 - 8 * sh)) : 0u};
        const u32 up = from_lane_above((u32)lo, 0u);   // the lane above's first dword
        const u32 nxt = ((off + nb) & 3u) && ln < 63 ? up : 0u;
        const u32 first = ln == 0 ? 0u : (off + 3) >> 2;
        const u64 gw = base - m;   // byte index of window byte 0
#pragma unroll
        for (u32 j = 0; j < 3; ++j) {
            const u32 idx = w + j;
            if (idx < first || idx > e) continue;
            const u32 val = q[j] | (idx == e ? nxt : 0u);
            const u64 g = gw + 4ull * idx;
            const u32 b0 = 4 * idx < m ? m - 4 * idx : 0u;
            const u32 b1 = 4 * idx + 4 > endb ? endb - 4 * idx : 4u;
            if (b0 == 0 && b1 == 4 && g + 4 <= a.capacity) {
                *(u32 *)(a.bytes + g) = val;
            } else {
                for (u32 t = b0; t < b1; ++t)
                    if (g + t < a.capacity) a.bytes[g + t] = (u8)(val >> (8 * t));
            }
        }
        return;
    }
    u32 len[4], lsum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        len[k] = (valid >> k) & 1u ? code_len(v[k]) : 0u;
        lsum += len[k];
    }
    const u32 incl = wave_scan(lsum);
    const u32 total = read_lane(incl, 63);
    // the stage starts at the 16-byte boundary at or below base
    const u32 mis = (u32)(((uintptr_t)a.bytes + base) & 15u);
    const u32 nwords = (mis + total + 3) >> 2;
    for (u32 q = ln; 4 * q < nwords; q += kWave) *(uint4 *)(st + 4 * q) = make_uint4(0, 0, 0, 0);
    wave_lds_sync();
    u32 off = mis + incl - lsum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (len[k]) {
            const u64 code = code_bytes(v[k], len[k]) << (8 * (off & 3u));
            const u32 w0 = off >> 2;
            atomicOr(&st[w0], (u32)code);
            if ((u32)(code >> 32)) atomicOr(&st[w0 + 1], (u32)(code >> 32));
            off += len[k];
        }
    }
    wave_lds_sync();
    // stores: dwords of the stage, 256 bytes per wavefront instruction; the
    // first and last dwords may hold bytes of the neighbouring chunks, whose
    // bytes of them are written by those chunks, so they go out byte by byte
    const u64 gb = base - mis;   // byte index of stage byte 0
    u8 *ob = a.bytes + gb;
    const u8 *sb = (const u8 *)st;
    const u32 end = mis + total;
    for (u32 q = ln; q < nwords; q += kWave) {
        const u32 b0 = q << 2;
        if (b0 >= mis && b0 + 4 <= end && gb + b0 + 4 <= a.capacity) {
            *(u32 *)(ob + b0) = st[q];
        } else {
#pragma unroll
            for (u32 t = 0; t < 4; ++t) {
                const u32 bb = b0 + t;
                if (bb >= mis && bb < end && gb + bb < a.capacity) ob[bb] = sb[bb];
            }
        }
    }
    wave_lds_sync();   // the stage is zeroed again for the next chunk
}

__global__ __launch_bounds__(256) void k_enc_write(EncArgs a) {
    extern __shared__ __align__(16) u32 lds[];
    const u32 wib = threadIdx.x >> 6;
    // the last chunks first: the length pass read them last, so the device
    // cache (MALL) still holds their values when this pass starts
    const u64 blk = gridDim.x - 1 - blockIdx.x;
    const u64 c0 = (blk * (blockDim.x >> 6) + (threadIdx.x >> 6)) * kEncWritePerWave;
    u32 *st = lds + wib * kEncStageWords;
    u32 vv[kEncWritePerWave][4], vvalid[kEncWritePerWave];
    u64 pre[kEncWritePerWave];
#pragma unroll
    for (int q = 0; q < kEncWritePerWave; ++q) {
        vvalid[q] = c0 + q < a.nchunks ? enc_load(a, c0 + q, vv[q]) : 0u;
        pre[q] = c0 + q < a.nchunks ? a.cpre[c0 + q] : 0ull;
    }
#pragma unroll
    for (int q = 0; q < kEncWritePerWave; ++q) {
        if (c0 + q >= a.nchunks) break;
        enc_write_chunk(a, st, vv[q], vvalid[q], pre[q]);
    }
}

__global__ __launch_bounds__(256) void k_enc_bounds(EncArgs a, const int64_t *vals_off,
                                                    int64_t *byte_off, u64 nb) {
    const u32 ln = lane_id();
    const u64 i = (u64)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= nb) return;
    u64 k = (u64)vals_off[i];
    if (k > a.n) k = a.n;
    const u64 ak = a.e0 + k;   // aligned index of the boundary
    u64 off;
    if (k == a.n) {
        off = *a.d_nbytes;
    } else {
        const u64 c = ak / kEncChunk;
        u32 v[4];
        const u32 valid = enc_load(a, c, v);
        u32 len = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            len += ((valid >> q) & 1u) && c * kEncChunk + 4u * ln + q < ak ? code_len(v[q]) : 0u;
        off = a.cpre[c] + wave_sum(len);
    }
    if (ln == 0) byte_off[i] = (int64_t)off;
}

// ------------------------------------------------------------ small kernels
// Cursor after a resumable piece: on success the piece's first byte moves
// past the last decoded code (to the code of rank k if there is one, else
// to the end of the piece's window less an unfinished code at its end) and
// prev becomes the last integer (plus one for differences minus one); on an
// error the cursor stays.
__global__ void k_resume_finish(const u8 *bytes, const u64 *cin, u64 *cout, const u64 *scratch,
                                const int32_t *d_status, const u32 *out, u64 k, u64 nbytes,
                                u64 window, int delta) {
    const u64 cur = cin[0], done = cin[1], prev = cin[2];
    if (*d_status != VBYTE_OK) {
        cout[0] = cur;
        cout[1] = done;
        cout[2] = prev;
        return;
    }
    const u64 total = scratch[1];
    const u64 m = total < k ? total : k;
    const u64 remain = nbytes - cur;
    const u64 wlen = remain < window ? remain : window;
    u64 tail = 0;   // continuation bytes that end the window (an unfinished code)
    while (tail < wlen && tail < 5 && bytes[cur + wlen - 1 - tail] >= 0x80) ++tail;
    cout[0] = cur + (total > k ? scratch[0] : wlen - tail);
    cout[1] = done + m;
    cout[2] = m ? (u64)(out[m - 1] + (delta == 2 ? 1u : 0u)) : prev;
}


__global__ void k_set_status(int32_t *p, int32_t v) { *p = v; }
__global__ void k_set_u64(uint64_t *p, uint64_t v) { *p = v; }
__global__ void k_fill_i64(int64_t *p, uint64_t n, int64_t v) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_zero(uint4 *p, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

template <int D, bool COUNT, int SEGS>
hipError_t launch_stream_t(const StreamArgs &a, int wpb, hipStream_t s) {
    const size_t lds = COUNT ? 0 : (size_t)wpb * kStageWords * sizeof(u32);
    if (a.cursor_in) {
        // pieces: decode only, at most 2 segments per wavefront
        if constexpr (!COUNT && SEGS <= 2) {
            k_stream<D, false, SEGS, true><<<a.ntiles, wpb * kWave, lds, s>>>(a);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    k_stream<D, COUNT, SEGS, false><<<a.ntiles, wpb * kWave, lds, s>>>(a);
    return hipGetLastError();
}

template <int D, int SEGS>
hipError_t launch_chunks_t(const StreamArgs &a, int wpb, u32 nchunks, hipStream_t s) {
    const size_t lds = (size_t)wpb * kStageWords * sizeof(u32);
    k_chunks<D, SEGS><<<nchunks, wpb * kWave, lds, s>>>(a);
    return hipGetLastError();
}

template <int SEGS>
hipError_t launch_chunks_s(const StreamArgs &a, int delta, int wpb, u32 nchunks, hipStream_t s) {
    if (delta == 2) return launch_chunks_t<2, SEGS>(a, wpb, nchunks, s);
    if (delta) return launch_chunks_t<1, SEGS>(a, wpb, nchunks, s);
    return launch_chunks_t<0, SEGS>(a, wpb, nchunks, s);
}

template <int D, int SEGS>
hipError_t launch_two_pass_t(const StreamArgs &a, int wpb, hipStream_t s) {
    k_tile_agg<D, SEGS><<<a.ntiles, wpb * kWave, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the block totals sit right after the tile slots
    Desc *bsum = a.desc + a.ntiles;
    const u32 nblocks = (u32)((a.ntiles + kScanSpan - 1) / kScanSpan);
    k_tile_block_sums<<<nblocks, kScanBlock, 0, s>>>(a, bsum);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tile_block_scan<<<nblocks, kScanBlock, 0, s>>>(a, bsum);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)wpb * kStageWords * sizeof(u32);
    k_known<D, SEGS><<<a.ntiles, wpb * kWave, lds, s>>>(a);
    return hipGetLastError();
}

template <int SEGS>
hipError_t launch_two_pass_s(const StreamArgs &a, int delta, int wpb, hipStream_t s) {
    if (delta == 2) return launch_two_pass_t<2, SEGS>(a, wpb, s);
    if (delta) return launch_two_pass_t<1, SEGS>(a, wpb, s);
    return launch_two_pass_t<0, SEGS>(a, wpb, s);
}

template <int SEGS>
hipError_t launch_stream_s(const StreamArgs &a, int delta, int count_only, int wpb, hipStream_t s) {
    if (count_only) return launch_stream_t<0, true, SEGS>(a, wpb, s);
    if (delta == 2) return launch_stream_t<2, false, SEGS>(a, wpb, s);
    if (delta) return launch_stream_t<1, false, SEGS>(a, wpb, s);
    return launch_stream_t<0, false, SEGS>(a, wpb, s);
}

// Workgroups of `kernel` resident at once on the device: the tile kernels of
// the batch loop over their items, so a grid larger than that would run in
// rounds, each block's items one after another.
template <class K>
hipError_t resident_grid(K kernel, int wpb, size_t lds, std::atomic<int> (&cache)[9], u32 &grid) {
    int b = cache[wpb].load(std::memory_order_relaxed);
    if (b <= 0) {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, wpb * kWave, lds);
        if (e != hipSuccess) return e;
        b = b > 0 ? b : 1;
        cache[wpb].store(b, std::memory_order_relaxed);
    }
    static std::atomic<int> cus{0};
    int c = cus.load(std::memory_order_relaxed);
    if (c <= 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cus.store(c, std::memory_order_relaxed);
    }
    grid = (u32)(c * b);
    return hipSuccess;
}

template <int D, int SEGS>
hipError_t launch_large_lists_t(const ListArgs &a, int wpb, hipStream_t s) {
    static std::atomic<int> occ_agg[9], occ_known[9];   // per wpb (zero-initialised statics)
    const size_t lds = (size_t)wpb * kStageWords * sizeof(u32);
    u32 ga = 0, gk = 0;
    hipError_t e = resident_grid(k_list_agg<D, SEGS>, wpb, 0, occ_agg, ga);
    if (e != hipSuccess) return e;
    if ((e = resident_grid(k_list_known<D, SEGS>, wpb, lds, occ_known, gk)) != hipSuccess) return e;
    // one wavefront per piece the table can hold (L is known only on the
    // device), at least the resident grid, at most kListGridCap workgroups
    // (the kernels' grid stride takes the rest)
    const u64 want = (a.max_large + wpb - 1) / wpb;
    const u32 g = (u32)(want < kListGridCap ? want : kListGridCap);
    ga = g > ga ? g : ga;
    gk = g > gk ? g : gk;
    k_list_agg<D, SEGS><<<ga, wpb * kWave, 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the slots through the block scans of the two-pass decode (the status
    // they write goes to a spare header word)
    StreamArgs sa{};
    sa.base = (const u8 *)a.hdr;
    sa.vstart = 0;
    sa.vend = 1;
    sa.ntiles = (u32)a.max_large;
    sa.desc = a.desc;
    sa.d_status = (int32_t *)(a.totals + 4);
    sa.d_count = nullptr;
    sa.d_nslots = a.totals + 0;   // L, written by the prep
    const u32 nblocks = (u32)((sa.ntiles + kScanSpan - 1) / kScanSpan);
    k_tile_block_sums<<<nblocks, kScanBlock, 0, s>>>(sa, sa.desc + sa.ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_tile_block_scan<<<nblocks, kScanBlock, 0, s>>>(sa, sa.desc + sa.ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_list_known<D, SEGS><<<gk, wpb * kWave, lds, s>>>(a);
    return hipGetLastError();
}

template <int SEGS>
hipError_t launch_batch_s(const ListArgs &a, int wpb, int grid_blocks, hipStream_t s) {
    const u32 nblocks = (u32)((a.nlists + kPrepBlock - 1) / kPrepBlock);
    if (nblocks) {
        k_prep<<<nblocks, kPrepBlock, 0, s>>>(a, nblocks, (u64)SEGS * kSegBytes);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.max_large) {
        hipError_t e = a.delta == 2 ? launch_large_lists_t<2, SEGS>(a, wpb, s)
                       : a.delta    ? launch_large_lists_t<1, SEGS>(a, wpb, s)
                                    : launch_large_lists_t<0, SEGS>(a, wpb, s);
        if (e != hipSuccess) return e;
    }
    // the small lists: as many workgroups as are resident at once (the
    // decode of a small list waits on memory more than it computes)
    (void)grid_blocks;
    const size_t lds = (size_t)wpb * kStageWords * sizeof(u32);
    static std::atomic<int> occ_small[3][9];
    u32 grid = 0;
    hipError_t e;
    if (a.delta == 2) {
        if ((e = resident_grid(k_batch<2, SEGS>, wpb, lds, occ_small[2], grid)) != hipSuccess) return e;
        k_batch<2, SEGS><<<grid, wpb * kWave, lds, s>>>(a);
    } else if (a.delta) {
        if ((e = resident_grid(k_batch<1, SEGS>, wpb, lds, occ_small[1], grid)) != hipSuccess) return e;
        k_batch<1, SEGS><<<grid, wpb * kWave, lds, s>>>(a);
    } else {
        if ((e = resident_grid(k_batch<0, SEGS>, wpb, lds, occ_small[0], grid)) != hipSuccess) return e;
        k_batch<0, SEGS><<<grid, wpb * kWave, lds, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stream(const StreamArgs &a, int delta, int count_only, int segs, int wpb,
                         hipStream_t s) {
    switch (segs) {
        case 1: return launch_stream_s<1>(a, delta, count_only, wpb, s);
        case 2: return launch_stream_s<2>(a, delta, count_only, wpb, s);
        case 4: return launch_stream_s<4>(a, delta, count_only, wpb, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_isect(const IsectArgs &a, hipStream_t s) {
    constexpr int SEGS = kIsectSegs, wpb = kIsectWaves;
    const u32 ntiles = a.s.ntiles;   // >= 1
    const u32 nblocks = (u32)((ntiles + kScanSpan - 1) / kScanSpan);
    const u32 tb = wpb * SEGS * kSegBytes;
    const size_t lds = (size_t)wpb * kStageWords * sizeof(u32);
    // the stream's tile slots: aggregates, then exclusive prefixes
    StreamArgs sa = a.s;
    sa.d_status = a.scan_status;
    sa.d_count = a.total;
    k_tile_agg<1, SEGS><<<ntiles, wpb * kWave, 0, s>>>(sa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tile_block_sums<<<nblocks, kScanBlock, 0, s>>>(sa, sa.desc + ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_tile_block_scan<<<nblocks, kScanBlock, 0, s>>>(sa, sa.desc + ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_isect_tiles<false><<<ntiles, wpb * kWave, lds, s>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_isect_status<<<1, kStatusBlock, 0, s>>>(a, tb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the match counts through the same scans (their status goes to a spare word)
    StreamArgs ma = sa;
    ma.desc = a.mdesc;
    ma.prev = 0;
    ma.d_status = a.scan_status + 1;
    ma.d_count = nullptr;
    k_tile_block_sums<<<nblocks, kScanBlock, 0, s>>>(ma, ma.desc + ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_tile_block_scan<<<nblocks, kScanBlock, 0, s>>>(ma, ma.desc + ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_isect_tiles<true><<<ntiles, wpb * kWave, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch4(const Stream4Args &a, int segs, int wpb, hipStream_t s) {
    switch (segs) {
        case 1: return launch4_t<1>(a, wpb, s);
        case 2: return launch4_t<2>(a, wpb, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch64(const Stream64Args &a, int delta, int segs, int wpb, hipStream_t s) {
    switch (segs) {
        case 1: return delta ? launch64_t<1, 1>(a, wpb, s) : launch64_t<0, 1>(a, wpb, s);
        case 2: return delta ? launch64_t<1, 2>(a, wpb, s) : launch64_t<0, 2>(a, wpb, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_flow(const FlowArgs &f, int delta, int segs, int wpb, int grid, int cus,
                       hipStream_t s) {
    if (grid < 0 || grid > kFlowMaxGrid || wpb < 1 || wpb > 8) return hipErrorInvalidValue;
    switch (segs) {
    case 1: return launch_flow_s<1>(f, delta, wpb, grid, cus, s);
    case 2: return launch_flow_s<2>(f, delta, wpb, grid, cus, s);
    case 4: return launch_flow_s<4>(f, delta, wpb, grid, cus, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_two_pass(const StreamArgs &a, int delta, int segs, int wpb, hipStream_t s) {
    switch (segs) {
        case 1: return launch_two_pass_s<1>(a, delta, wpb, s);
        case 2: return launch_two_pass_s<2>(a, delta, wpb, s);
        case 4: return launch_two_pass_s<4>(a, delta, wpb, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_chunks(const StreamArgs &a, int delta, int segs, int wpb, uint32_t nchunks,
                         hipStream_t s) {
    switch (segs) {
        case 1: return launch_chunks_s<1>(a, delta, wpb, nchunks, s);
        case 2: return launch_chunks_s<2>(a, delta, wpb, nchunks, s);
        case 4: return launch_chunks_s<4>(a, delta, wpb, nchunks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(const ListArgs &a, int segs, int wpb, int grid_blocks, hipStream_t s) {
    switch (segs) {
        case 1: return launch_batch_s<1>(a, wpb, grid_blocks, s);
        case 2: return launch_batch_s<2>(a, wpb, grid_blocks, s);
        case 4: return launch_batch_s<4>(a, wpb, grid_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_encode(const EncArgs &a, hipStream_t s) {
    const u32 wpb = 4;
    const u64 blocks = (a.nchunks + kEncLenChunks - 1) / kEncLenChunks;
    k_enc_len<<<(unsigned)blocks, kEncLenWaves * kWave, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const u64 nsb = (a.nchunks + kEncScanSpan - 1) / kEncScanSpan;
    k_enc_bscan<<<(unsigned)nsb, kScanBlock, 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const u64 wblocks = (a.nchunks + (u64)wpb * kEncWritePerWave - 1) / ((u64)wpb * kEncWritePerWave);
    k_enc_write<<<(unsigned)wblocks, wpb * kWave, wpb * kEncStageWords * sizeof(u32), s>>>(a);
    return hipGetLastError();
}

hipError_t launch_encode_bounds(const EncArgs &a, const int64_t *vals_off, int64_t *byte_off,
                                uint64_t nb, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    const u32 wpb = 4;
    k_enc_bounds<<<(unsigned)((nb + wpb - 1) / wpb), wpb * kWave, 0, s>>>(a, vals_off, byte_off, nb);
    return hipGetLastError();
}

hipError_t launch_resume_finish(const uint8_t *bytes, const uint64_t *cursor_in, uint64_t *cursor_out,
                                const uint64_t *scratch, const int32_t *d_status,
                                const uint32_t *out, uint64_t k, uint64_t nbytes, uint64_t window,
                                int delta, hipStream_t s) {
    k_resume_finish<<<1, 1, 0, s>>>(bytes, cursor_in, cursor_out, scratch, d_status, out, k, nbytes,
                                    window, delta);
    return hipGetLastError();
}

hipError_t launch_set_status(int32_t *d_status, int32_t value, hipStream_t s) {
    k_set_status<<<1, 1, 0, s>>>(d_status, value);
    return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t *p, uint64_t value, hipStream_t s) {
    k_set_u64<<<1, 1, 0, s>>>(p, value);
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t *p, uint64_t n, int64_t value, hipStream_t s) {
    if (n == 0) return hipSuccess;
    u64 blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    k_fill_i64<<<(unsigned)blocks, 256, 0, s>>>(p, n, value);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_zero<<<(unsigned)blocks, 256, 0, s>>>((uint4 *)p, n16);
    return hipGetLastError();
}

// ------------------------------------------------------------ allocation-free decode
// The tile slots of vbyte_decode_noalloc, one copy per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not a
// device address: host code uses only the address hipGetSymbolAddress
// returns for the current device, taken once per device below.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void **ptr) {
    static std::mutex mu;
    static void *addr[kNoAllocMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace vb
