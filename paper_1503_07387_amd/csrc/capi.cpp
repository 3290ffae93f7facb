// capi.cpp -- the C ABI of libvbyte (include/vbyte.h): argument checks,
// the per-(device, stream) workspace cache, and kernel launches.
//
// Every call validates its arguments on the host and returns VBYTE_EINVAL
// before enqueuing anything; data errors are produced by the kernels into a
// device status word.  The library allocates only its own workspace
// (look-back descriptors, ticket header, batch work tables).

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <cstdlib>
#include <mutex>
#include <utility>

#include <hip/hip_runtime.h>

#include "vbyte.h"
#include "vbyte_internal.h"

namespace vb {
namespace {

thread_local char g_last_error[256] = "";

std::atomic<int> g_segs{2};
std::atomic<int> g_wpb{8};
std::atomic<int64_t> g_small{16384};
std::atomic<int> g_chunk{-1};  // single stream: -1 = two passes, four launches, no look-back (default),
                               // -2 = one launch reading the input once,
                               // 0 = per-tile look-back, k = chunks of k tiles
std::atomic<int> g_flow_grid{0};   // workgroups of the one-launch decode (0: per CU count)
std::atomic<uint32_t> g_spin_limit{kDefaultSpinLimit};

// Process-wide defaults from the environment, read once when the library is
// loaded: VBYTE_SEGS_PER_WAVE (1, 2, 4), VBYTE_WAVES_PER_BLOCK (1..8),
// VBYTE_SMALL_LIST_BYTES (>= 1), VBYTE_SCHEDULE (-2..64, as
// vbyte_set_chunk_tiles), VBYTE_SPIN_LIMIT (>= 1).  A value that is not a
// whole number in range is ignored.
bool env_int(const char *name, long long lo, long long hi, long long *v) {
    const char *t = std::getenv(name);
    if (!t || !*t) return false;
    char *end = nullptr;
    const long long x = std::strtoll(t, &end, 10);
    if (*end != '\0' || x < lo || x > hi) return false;
    *v = x;
    return true;
}
struct EnvDefaults {
    EnvDefaults() {
        long long v = 0;
        if (env_int("VBYTE_SEGS_PER_WAVE", 1, 4, &v) && v != 3) g_segs.store((int)v);
        if (env_int("VBYTE_WAVES_PER_BLOCK", 1, 8, &v)) g_wpb.store((int)v);
        if (env_int("VBYTE_SMALL_LIST_BYTES", 1, 1ll << 40, &v)) g_small.store((int64_t)v);
        if (env_int("VBYTE_SCHEDULE", kScheduleFlow, 64, &v)) g_chunk.store((int)v);
        if (env_int("VBYTE_SPIN_LIMIT", 1, 0xFFFFFFFFll, &v)) g_spin_limit.store((uint32_t)v);
    }
} g_env_defaults;

vbyte_status hip_fail(hipError_t e, const char *what) {
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s", what, hipGetErrorString(e));
    return VBYTE_EHIP;
}

// Workspace layout (bytes):
//   [0, 40)     epoch word (0), ticket word (3), stall word (4)
//   [64, 68)    status slot used by the synchronous calls
//   [128, 168)  batch totals (5 x uint64)
//   [192, 208)  resumable piece: offset of the code of rank k, code count
//   [256, 512)  completion counters of the one-launch decode
//   [512, ...)  descriptors, then batch tables
constexpr size_t kStatusOff = 64;
constexpr size_t kTotalsOff = 128;
constexpr size_t kPieceOff = 192;   // resumable pieces: rank-n offset and code count

struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    uint64_t launches = 0;
    // the intersection consumer's buffers (piece, flags, counts, cursors),
    // apart from `ptr` because the piece decodes use that
    void *aux = nullptr;
    size_t aux_bytes = 0;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
std::map<std::pair<int, hipStream_t>, std::recursive_mutex> g_stream_mu;

// Held by every call that uses a stream's workspace, from its first look at
// the workspace to its last enqueue (synchronous calls: until they return),
// so that calls on one stream from several host threads do not interleave
// their launches on the shared descriptors and status slot.
class StreamGuard {
  public:
    explicit StreamGuard(hipStream_t s) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        {
            std::lock_guard<std::mutex> lk(g_mu);
            mu_ = &g_stream_mu[{dev, s}];
        }
        mu_->lock();
    }
    ~StreamGuard() { mu_->unlock(); }
    StreamGuard(const StreamGuard &) = delete;
    StreamGuard &operator=(const StreamGuard &) = delete;

  private:
    std::recursive_mutex *mu_;
};

struct Cleanup {
    ~Cleanup() {
        // Process exit: the runtime may already be torn down; release quietly.
        for (auto &kv : g_ws) {
            if (kv.second.ptr) (void)hipFree(kv.second.ptr);
            if (kv.second.aux) (void)hipFree(kv.second.aux);
        }
    }
} g_cleanup;

// Returns a workspace of at least `need` bytes for `stream`, zero-filled on
// (re)allocation and re-zeroed before the epoch tag could wrap.  `launches`
// is the number of ticketed launches the caller is about to enqueue.
vbyte_status get_ws(hipStream_t stream, size_t need, int launches, Workspace **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace &w = g_ws[{dev, stream}];
    need = std::max(need, kHeaderBytes);
    if (w.bytes < need) {
        if (w.ptr) {
            e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t sz = std::max(need + need / 2, (size_t)1 << 20);
        sz = (sz + 255) & ~(size_t)255;
        e = hipMalloc(&w.ptr, sz);
        if (e != hipSuccess) {
            w.ptr = nullptr;
            std::snprintf(g_last_error, sizeof g_last_error, "hipMalloc(%zu): %s", sz, hipGetErrorString(e));
            return VBYTE_ENOMEM;
        }
        w.bytes = sz;
        w.launches = 0;
        e = launch_zero(w.ptr, sz, stream);
        if (e != hipSuccess) return hip_fail(e, "zero workspace");
    }
    if (w.launches + (uint64_t)launches >= kEpochLaunchLimit) {
        e = launch_zero(w.ptr, w.bytes, stream);
        if (e != hipSuccess) return hip_fail(e, "re-zero workspace");
        w.launches = 0;
    }
    w.launches += (uint64_t)launches;
    *out = &w;
    return VBYTE_OK;
}

uint8_t *ws_base(Workspace *w) { return (uint8_t *)w->ptr; }

// The consumer buffers of workspace w, at least `need` bytes (grown on
// demand; their contents are initialised by the kernels that use them).
vbyte_status aux_area(Workspace *w, hipStream_t s, size_t need, uint8_t **p) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (w->aux_bytes < need) {
        if (w->aux) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(w->aux);
            w->aux = nullptr;
            w->aux_bytes = 0;
        }
        const size_t sz = (need + 255) & ~(size_t)255;
        hipError_t e = hipMalloc(&w->aux, sz);
        if (e != hipSuccess) {
            w->aux = nullptr;
            std::snprintf(g_last_error, sizeof g_last_error, "hipMalloc(%zu): %s", sz, hipGetErrorString(e));
            return VBYTE_ENOMEM;
        }
        w->aux_bytes = sz;
    }
    *p = (uint8_t *)w->aux;
    return VBYTE_OK;
}

constexpr uint64_t kMaxBytes = 1ull << 36;

// Compute units of the current device (hipDeviceAttributeMultiprocessorCount).
int device_cus() {
    static std::atomic<int> cached[64];   // per device ordinal (zero-initialised)
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev >= 0 && dev < 64 && (v = cached[dev].load(std::memory_order_relaxed)) > 0) return v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
        return 256;
    if (dev >= 0 && dev < 64) cached[dev].store(v, std::memory_order_relaxed);
    return v;
}


// The process-wide defaults as a per-call tuning.
vbyte_tuning default_tuning() {
    vbyte_tuning t{};
    t.segs_per_wave = g_segs.load();
    t.waves_per_block = g_wpb.load();
    t.schedule = g_chunk.load();
    t.grid = g_flow_grid.load();
    t.recompute = 0;
    return t;
}

bool tuning_ok(const vbyte_tuning &t) {
    const int sg = t.segs_per_wave;
    if (sg != 1 && sg != 2 && sg != 4) return false;
    if (t.waves_per_block < 1 || t.waves_per_block > 8) return false;
    if (t.schedule < kScheduleFlow || t.schedule > 64) return false;
    if (t.grid < 0 || t.grid > kFlowMaxGrid) return false;
    return t.recompute == 0 || t.recompute == 1;
}

// Enqueues a single-stream decode with tuning `tu` (nullptr: the process
// defaults).  With d_status == nullptr the status goes to the workspace's
// own slot, returned through *slot (synchronous calls).
vbyte_status decode_stream(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                           uint32_t prev, int delta, int32_t *d_status, hipStream_t s,
                           int32_t **slot = nullptr, const vbyte_tuning *tu = nullptr) {
    const vbyte_tuning tun = tu ? *tu : default_tuning();
    if (!tuning_ok(tun)) return VBYTE_EINVAL;
    if (delta < 0 || delta > 2) return VBYTE_EINVAL;
    if (nbytes >= kMaxBytes) return VBYTE_EINVAL;
    if (nbytes > 0 && !bytes) return VBYTE_EINVAL;
    if (n > 0 && !out) return VBYTE_EINVAL;
    if (((uintptr_t)out & 3u) != 0) return VBYTE_EINVAL;
    if (((uintptr_t)d_status & 3u) != 0) return VBYTE_EINVAL;
    if (!d_status && !slot) return VBYTE_EINVAL;
    const int segs = tun.segs_per_wave, wpb = tun.waves_per_block;
    StreamArgs a{};
    a.spin_limit = spin_limit();
    a.vstart = (uintptr_t)bytes & 15u;
    a.base = bytes - a.vstart;
    a.vend = a.vstart + nbytes;
    a.out = out;
    a.n = n;
    a.prev = prev;
    const uint64_t ntiles = nbytes ? stream_tiles(a.vstart, nbytes, segs, wpb) : 0;
    if (ntiles >= (1ull << 31)) return VBYTE_EINVAL;
    a.ntiles = (uint32_t)ntiles;
    const int chunk = tun.schedule;
    const uint64_t nchunks = chunk > 0 ? (ntiles + chunk - 1) / chunk : 0;
    const uint64_t ndesc = chunk > 0 ? nchunks : chunk == -1 ? two_pass_slots(ntiles) : ntiles;
    Workspace *w = nullptr;
    vbyte_status st = get_ws(s, kHeaderBytes + ndesc * sizeof(Desc), ntiles ? 1 : 0, &w);
    if (st != VBYTE_OK) return st;
    if (!d_status) {
        d_status = (int32_t *)(ws_base(w) + kStatusOff);
        *slot = d_status;
    }
    if (nbytes == 0) {
        hipError_t e = launch_set_status(d_status, n == 0 ? VBYTE_OK : VBYTE_ETRUNC, s);
        return e == hipSuccess ? VBYTE_OK : hip_fail(e, "set status");
    }
    a.hdr = (uint64_t *)ws_base(w);
    a.desc = (Desc *)(ws_base(w) + kHeaderBytes);
    a.d_status = d_status;
    a.d_count = nullptr;
    hipError_t e;
    if (chunk == kScheduleFlow) {
        FlowArgs f{};
        f.s = a;
        f.ctr = (uint64_t *)(ws_base(w) + kFlowCtrOff);
        f.recompute = (uint32_t)tun.recompute;
        e = launch_flow(f, delta, segs, wpb, tun.grid, device_cus(), s);
    } else {
        e = chunk > 0   ? launch_chunks(a, delta, segs, wpb, (uint32_t)nchunks, s)
            : chunk < 0 ? launch_two_pass(a, delta, segs, wpb, s)
                        : launch_stream(a, delta, 0, segs, wpb, s);
    }
    return e == hipSuccess ? VBYTE_OK : hip_fail(e, "decode launch");
}

vbyte_status decode_sync(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n, uint32_t prev,
                         int delta) {
    StreamGuard guard_(nullptr);
    hipStream_t s = nullptr;
    int32_t *slot = nullptr;
    vbyte_status st = decode_stream(bytes, nbytes, out, n, prev, delta, nullptr, s, &slot);
    if (st != VBYTE_OK) return st;
    int32_t h = -1;
    hipError_t e = hipMemcpyAsync(&h, slot, sizeof h, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "status copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return (vbyte_status)h;
}

// Enqueues a 64-bit single-stream decode; status as in
// decode_stream.
vbyte_status decode64_stream(const uint8_t *bytes, size_t nbytes, uint64_t *out, size_t n,
                             uint64_t prev, int delta, int32_t *d_status, hipStream_t s,
                             int32_t **slot = nullptr) {
    if (nbytes >= kMaxBytes) return VBYTE_EINVAL;
    if (nbytes > 0 && !bytes) return VBYTE_EINVAL;
    if (n > 0 && !out) return VBYTE_EINVAL;
    if (((uintptr_t)out & 7u) != 0) return VBYTE_EINVAL;
    if (((uintptr_t)d_status & 3u) != 0) return VBYTE_EINVAL;
    if (!d_status && !slot) return VBYTE_EINVAL;
    const int segs = std::min(g_segs.load(), 2), wpb = g_wpb.load();
    Stream64Args a{};
    a.vstart = (uintptr_t)bytes & 15u;
    a.base = bytes - a.vstart;
    a.vend = a.vstart + nbytes;
    a.out = out;
    a.n = n;
    a.prev = prev;
    const uint64_t unit = (uint64_t)kUnit64Groups * segs * kSegBytes;
    const uint64_t nunits = nbytes ? (a.vstart + nbytes + unit - 1) / unit : 0;
    if (nunits >= (1ull << 31)) return VBYTE_EINVAL;
    a.nunits = (uint32_t)nunits;
    Workspace *w = nullptr;
    vbyte_status st = get_ws(s, kHeaderBytes + nunits * 16 * (1 + kUnit64Groups), 0, &w);
    if (st != VBYTE_OK) return st;
    if (!d_status) {
        d_status = (int32_t *)(ws_base(w) + kStatusOff);
        *slot = d_status;
    }
    if (nbytes == 0) {
        hipError_t e = launch_set_status(d_status, n == 0 ? VBYTE_OK : VBYTE_ETRUNC, s);
        return e == hipSuccess ? VBYTE_OK : hip_fail(e, "set status");
    }
    a.slots = (uint4 *)(ws_base(w) + kHeaderBytes);
    a.gslots = a.slots + nunits;
    a.d_status = d_status;
    hipError_t e = launch64(a, delta, segs, wpb, s);
    return e == hipSuccess ? VBYTE_OK : hip_fail(e, "decode64 launch");
}

// Enqueues a blocks-of-four decode; status as in decode_stream.
vbyte_status decode4_stream(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                            const uint32_t *prev4, int32_t *d_status, hipStream_t s,
                            int32_t **slot = nullptr) {
    if (nbytes >= kMaxBytes) return VBYTE_EINVAL;
    if (nbytes > 0 && !bytes) return VBYTE_EINVAL;
    if (n > 0 && !out) return VBYTE_EINVAL;
    if (((uintptr_t)out & 3u) != 0) return VBYTE_EINVAL;
    if (((uintptr_t)d_status & 3u) != 0) return VBYTE_EINVAL;
    if (!d_status && !slot) return VBYTE_EINVAL;
    const int segs = std::min(g_segs.load(), 2), wpb = g_wpb.load();
    Stream4Args a{};
    a.vstart = (uintptr_t)bytes & 15u;
    a.base = bytes - a.vstart;
    a.vend = a.vstart + nbytes;
    a.out = out;
    a.n = n;
    for (int k = 0; k < 4; ++k) a.prev4[k] = prev4 ? prev4[k] : 0u;
    const uint64_t unit = (uint64_t)kUnit64Groups * segs * kSegBytes;
    const uint64_t nunits = nbytes ? (a.vstart + nbytes + unit - 1) / unit : 0;
    if (nunits >= (1ull << 31)) return VBYTE_EINVAL;
    a.nunits = (uint32_t)nunits;
    const uint64_t nblocks = (nunits + wpb - 1) / wpb;   // aggregate workgroups
    a.nblocks = (uint32_t)nblocks;
    a.block_units = (uint32_t)wpb;
    Workspace *w = nullptr;
    vbyte_status st = get_ws(s, kHeaderBytes + (nunits * (1 + kUnit64Groups) + nblocks) * 32, 0, &w);
    if (st != VBYTE_OK) return st;
    if (!d_status) {
        d_status = (int32_t *)(ws_base(w) + kStatusOff);
        *slot = d_status;
    }
    if (nbytes == 0) {
        hipError_t e = launch_set_status(d_status, n == 0 ? VBYTE_OK : VBYTE_ETRUNC, s);
        return e == hipSuccess ? VBYTE_OK : hip_fail(e, "set status");
    }
    a.slots = (uint4 *)(ws_base(w) + kHeaderBytes);
    a.gslots = a.slots + 2 * nunits;
    a.bslots = a.gslots + 2 * nunits * kUnit64Groups;
    a.d_status = d_status;
    hipError_t e = launch4(a, segs, wpb, s);
    return e == hipSuccess ? VBYTE_OK : hip_fail(e, "decode_delta4 launch");
}

vbyte_status decode64_sync(const uint8_t *bytes, size_t nbytes, uint64_t *out, size_t n,
                           uint64_t prev, int delta) {
    StreamGuard guard_(nullptr);
    hipStream_t s = nullptr;
    int32_t *slot = nullptr;
    vbyte_status st = decode64_stream(bytes, nbytes, out, n, prev, delta, nullptr, s, &slot);
    if (st != VBYTE_OK) return st;
    int32_t h = -1;
    hipError_t e = hipMemcpyAsync(&h, slot, sizeof h, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "status copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return (vbyte_status)h;
}

}  // namespace

uint32_t spin_limit() { return g_spin_limit.load(std::memory_order_relaxed); }

vbyte_status batch_plan(ListArgs &a, size_t list_bytes, BatchPlan *plan) {
    if (!a.list_status || ((uintptr_t)a.list_status & 3u)) return VBYTE_EINVAL;
    if (!a.bytes && a.nbytes) return VBYTE_EINVAL;
    if (!a.out && a.nout) return VBYTE_EINVAL;
    if (((uintptr_t)a.out & 3u) != 0) return VBYTE_EINVAL;
    if (a.nlists >= (1ull << 31)) return VBYTE_EINVAL;
    const int segs = g_segs.load(), wpb = g_wpb.load();
    a.wpb = (uint32_t)wpb;
    a.small_bytes = (uint64_t)std::max<int64_t>(g_small.load(), 0);
    // A large list holds more than small_bytes bytes and needs at most
    // bytes/ub + 2 pieces of ub = segs KiB (one work item and slot each); a
    // small list needs one item.
    const uint64_t ub = (uint64_t)segs * kSegBytes;
    const uint64_t nlarge_max = std::min<uint64_t>(a.nlists, list_bytes / (a.small_bytes + 1));
    a.max_large = list_bytes / ub + 2 * nlarge_max;
    a.max_items = a.max_large + a.nlists + 2;
    if (a.max_items >= (1ull << 31)) return VBYTE_EINVAL;
    const uint32_t nblocks = (uint32_t)((a.nlists + kPrepBlock - 1) / kPrepBlock);
    size_t off = kHeaderBytes;
    plan->desc_off = off;
    off += two_pass_slots(a.max_large) * sizeof(Desc);
    plan->prep_off = off;
    off += (size_t)nblocks * sizeof(Desc);
    off = (off + 63) & ~(size_t)63;
    plan->items_off = off;
    off += a.max_items * sizeof(BatchItem);
    plan->pmap_off = off;   // 48-byte items keep it 16-byte aligned
    off += a.max_large * sizeof(uint32_t);
    plan->bytes = off;
    plan->segs = segs;
    plan->wpb = wpb;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
    }
    plan->grid = cus * std::max(1, kBatchWavesPerCu / wpb);
    return VBYTE_OK;
}

void batch_bind(ListArgs &a, const BatchPlan &plan, uint8_t *ws) {
    a.hdr = (uint64_t *)ws;
    a.totals = (uint64_t *)(ws + kTotalsOff);
    a.desc = (Desc *)(ws + plan.desc_off);
    a.prep_desc = (Desc *)(ws + plan.prep_off);
    a.items = (BatchItem *)(ws + plan.items_off);
    a.pmap = (uint32_t *)(ws + plan.pmap_off);
}

vbyte_status hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }

namespace {

vbyte_status batch_common(ListArgs a, size_t list_bytes, hipStream_t s) {
    if (a.nlists == 0) return VBYTE_OK;
    BatchPlan plan;
    vbyte_status st = batch_plan(a, list_bytes, &plan);
    if (st != VBYTE_OK) return st;
    Workspace *w = nullptr;
    st = get_ws(s, plan.bytes, 2, &w);
    if (st != VBYTE_OK) return st;
    batch_bind(a, plan, ws_base(w));
    hipError_t e = launch_batch(a, plan.segs, plan.wpb, plan.grid, s);
    return e == hipSuccess ? VBYTE_OK : hip_fail(e, "batch launch");
}

}  // namespace
}  // namespace vb

using namespace vb;

extern "C" {

vbyte_status vbyte_decode(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n) {
    return decode_sync(bytes, nbytes, out, n, 0, 0);
}

vbyte_status vbyte_decode_delta(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                uint32_t prev) {
    return decode_sync(bytes, nbytes, out, n, prev, 1);
}

vbyte_status vbyte_decode_async(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                int32_t *d_status, void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return decode_stream(bytes, nbytes, out, n, 0, 0, d_status, (hipStream_t)stream);
}

vbyte_status vbyte_decode_delta_async(const uint8_t *bytes, size_t nbytes, uint32_t *out,
                                      size_t n, uint32_t prev, int32_t *d_status, void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return decode_stream(bytes, nbytes, out, n, prev, 1, d_status, (hipStream_t)stream);
}

vbyte_status vbyte_decode_ex(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                             uint32_t prev, int mode, const vbyte_tuning *tuning, int32_t *d_status,
                             void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    if (!d_status) return VBYTE_EINVAL;
    return decode_stream(bytes, nbytes, out, n, prev, mode, d_status, (hipStream_t)stream, nullptr,
                         tuning);
}

vbyte_status vbyte_decode_noalloc(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                  uint32_t prev, int mode, int32_t *d_status, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (mode < 0 || mode > 2 || !d_status || ((uintptr_t)d_status & 3u) != 0) return VBYTE_EINVAL;
    if (nbytes >= kMaxBytes || (nbytes > 0 && !bytes) || (n > 0 && !out)) return VBYTE_EINVAL;
    if (((uintptr_t)out & 3u) != 0) return VBYTE_EINVAL;
    StreamArgs a{};
    a.spin_limit = spin_limit();
    a.vstart = (uintptr_t)bytes & 15u;
    a.base = bytes - a.vstart;
    a.vend = a.vstart + nbytes;
    a.out = out;
    a.n = n;
    a.prev = prev;
    const uint64_t ntiles = nbytes ? stream_tiles(a.vstart, nbytes, kNoAllocSegs, kNoAllocWaves) : 0;
    if (two_pass_slots(ntiles) * sizeof(Desc) > kNoAllocScratchBytes) {
        std::snprintf(g_last_error, sizeof g_last_error,
                      "vbyte_decode_noalloc: %zu bytes need %llu tile slots, more than the %zu the "
                      "scratch array holds",
                      nbytes, (unsigned long long)ntiles, kNoAllocScratchBytes / sizeof(Desc));
        return VBYTE_EINVAL;
    }
    if (nbytes == 0) {
        hipError_t e = launch_set_status(d_status, n == 0 ? VBYTE_OK : VBYTE_ETRUNC, s);
        return e == hipSuccess ? VBYTE_OK : hip_fail(e, "set status");
    }
    void *scr = nullptr;
    hipError_t e = noalloc_scratch(&scr);
    if (e != hipSuccess) return hip_fail(e, "scratch symbol address");
    a.ntiles = (uint32_t)ntiles;
    a.desc = (Desc *)scr;
    a.hdr = nullptr;
    a.d_status = d_status;
    e = launch_two_pass(a, mode, kNoAllocSegs, kNoAllocWaves, s);
    return e == hipSuccess ? VBYTE_OK : hip_fail(e, "decode launch");
}

void vbyte_tuning_default(vbyte_tuning *t) {
    if (t) *t = default_tuning();
}

vbyte_status vbyte_set_spin_limit(uint32_t rounds) {
    g_spin_limit.store(rounds ? rounds : kDefaultSpinLimit);
    return VBYTE_OK;
}

vbyte_status vbyte_set_flow_grid(int grid) {
    if (grid < 0 || grid > kFlowMaxGrid) return VBYTE_EINVAL;
    g_flow_grid.store(grid);
    return VBYTE_OK;
}

vbyte_status vbyte_decode_delta_m1(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                   uint32_t prev) {
    return decode_sync(bytes, nbytes, out, n, prev, 2);
}

vbyte_status vbyte_decode_delta_m1_async(const uint8_t *bytes, size_t nbytes, uint32_t *out,
                                         size_t n, uint32_t prev, int32_t *d_status,
                                         void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return decode_stream(bytes, nbytes, out, n, prev, 2, d_status, (hipStream_t)stream);
}

vbyte_status vbyte_decode_delta4(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                 const uint32_t *prev4) {
    StreamGuard guard_(nullptr);
    hipStream_t s = nullptr;
    int32_t *slot = nullptr;
    vbyte_status st = decode4_stream(bytes, nbytes, out, n, prev4, nullptr, s, &slot);
    if (st != VBYTE_OK) return st;
    int32_t h = -1;
    hipError_t e = hipMemcpyAsync(&h, slot, sizeof h, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "status copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return (vbyte_status)h;
}

vbyte_status vbyte_decode_delta4_async(const uint8_t *bytes, size_t nbytes, uint32_t *out,
                                       size_t n, const uint32_t *prev4, int32_t *d_status,
                                       void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return decode4_stream(bytes, nbytes, out, n, prev4, d_status, (hipStream_t)stream);
}

vbyte_status vbyte_decode64(const uint8_t *bytes, size_t nbytes, uint64_t *out, size_t n) {
    return decode64_sync(bytes, nbytes, out, n, 0, 0);
}

vbyte_status vbyte_decode64_delta(const uint8_t *bytes, size_t nbytes, uint64_t *out, size_t n,
                                  uint64_t prev) {
    return decode64_sync(bytes, nbytes, out, n, prev, 1);
}

vbyte_status vbyte_decode64_async(const uint8_t *bytes, size_t nbytes, uint64_t *out, size_t n,
                                  int32_t *d_status, void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return decode64_stream(bytes, nbytes, out, n, 0, 0, d_status, (hipStream_t)stream);
}

vbyte_status vbyte_decode64_delta_async(const uint8_t *bytes, size_t nbytes, uint64_t *out,
                                        size_t n, uint64_t prev, int32_t *d_status, void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return decode64_stream(bytes, nbytes, out, n, prev, 1, d_status, (hipStream_t)stream);
}

vbyte_status vbyte_decode_next_async(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t k,
                                     int delta, const vbyte_cursor *d_in, vbyte_cursor *d_out,
                                     int32_t *d_status, void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    hipStream_t s = (hipStream_t)stream;
    if (k == 0 || k > (1ull << 40) || !out || ((uintptr_t)out & 3u)) return VBYTE_EINVAL;
    if (!d_in || !d_out || d_in == d_out || ((uintptr_t)d_in & 7u) || ((uintptr_t)d_out & 7u))
        return VBYTE_EINVAL;
    if (!d_status || ((uintptr_t)d_status & 3u)) return VBYTE_EINVAL;
    if (delta < 0 || delta > 2) return VBYTE_EINVAL;
    if (nbytes >= kMaxBytes || (nbytes > 0 && !bytes)) return VBYTE_EINVAL;
    // at most 2 segments per wavefront: the piece kernel's extra position
    // search does not fit the 4-segment register budget
    const int segs = g_segs.load() > 2 ? 2 : g_segs.load(), wpb = g_wpb.load();
    const uint64_t window = 5ull * k;
    const uint64_t span = nbytes < window ? nbytes : window;
    // tiles for the widest piece at the worst misalignment of its start
    const uint64_t ntiles = stream_tiles(15, span > 0 ? span : 1, segs, wpb);
    if (ntiles >= (1ull << 31)) return VBYTE_EINVAL;
    Workspace *w = nullptr;
    vbyte_status st = get_ws(s, kHeaderBytes + ntiles * sizeof(Desc), 1, &w);
    if (st != VBYTE_OK) return st;
    uint64_t *scratch = (uint64_t *)(ws_base(w) + kPieceOff);
    const uint64_t *cin = (const uint64_t *)d_in;
    StreamArgs a{};
    a.spin_limit = spin_limit();
    const uint8_t *p = nbytes ? bytes : (const uint8_t *)d_in;   // any readable address
    a.vstart = (uintptr_t)p & 15u;
    a.base = p - a.vstart;
    a.vend = a.vstart + nbytes;
    a.out = out;
    a.n = k;
    a.ntiles = (uint32_t)ntiles;
    a.hdr = (uint64_t *)ws_base(w);
    a.desc = (Desc *)(ws_base(w) + kHeaderBytes);
    a.d_status = d_status;
    a.cursor_in = cin;
    a.window = window;
    a.scratch = scratch;
    hipError_t e = launch_stream(a, delta, 0, segs, wpb, s);
    if (e != hipSuccess) return hip_fail(e, "piece launch");
    e = launch_resume_finish(bytes, cin, (uint64_t *)d_out, scratch, d_status, out, k, nbytes,
                             window, delta, s);
    return e == hipSuccess ? VBYTE_OK : hip_fail(e, "cursor update");
}

vbyte_status vbyte_intersect_async(const uint8_t *a, size_t a_nbytes, size_t na, uint32_t a_prev,
                                   const uint32_t *b, size_t nb, size_t piece, uint32_t *out,
                                   size_t out_cap, uint64_t *d_count, int32_t *d_status,
                                   void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    hipStream_t s = (hipStream_t)stream;
    if (piece == 0 || piece > (1ull << 26)) return VBYTE_EINVAL;
    if (a_nbytes >= kMaxBytes || (a_nbytes > 0 && !a) || na >= kMaxBytes) return VBYTE_EINVAL;
    if ((nb > 0 && !b) || ((uintptr_t)b & 3u) || nb >= (1ull << 32)) return VBYTE_EINVAL;
    if ((out_cap > 0 && !out) || ((uintptr_t)out & 3u)) return VBYTE_EINVAL;
    if (!d_count || ((uintptr_t)d_count & 7u) || !d_status || ((uintptr_t)d_status & 3u))
        return VBYTE_EINVAL;
    if (a_nbytes == 0) {
        hipError_t e = launch_set_u64(d_count, 0, s);
        if (e == hipSuccess) e = launch_set_status(d_status, na == 0 ? VBYTE_OK : VBYTE_ETRUNC, s);
        return e == hipSuccess ? VBYTE_OK : hip_fail(e, "intersect of an empty list");
    }
    IsectArgs ia{};
    StreamArgs &sa = ia.s;
    sa.spin_limit = spin_limit();
    sa.vstart = (uintptr_t)a & 15u;
    sa.base = a - sa.vstart;
    sa.vend = sa.vstart + a_nbytes;
    sa.n = na;
    sa.prev = a_prev;
    const uint64_t ntiles = stream_tiles(sa.vstart, a_nbytes, kIsectSegs, kIsectWaves);
    if (ntiles >= (1ull << 31)) return VBYTE_EINVAL;
    sa.ntiles = (uint32_t)ntiles;
    // two rows of tile slots (the stream's, the matches'), then the totals
    const uint64_t nslots = two_pass_slots(ntiles);
    const size_t off_m = kHeaderBytes + nslots * sizeof(Desc);
    const size_t off_tot = off_m + nslots * sizeof(Desc);
    Workspace *w = nullptr;
    vbyte_status st = get_ws(s, off_tot + 64, 0, &w);
    if (st != VBYTE_OK) return st;
    sa.hdr = (uint64_t *)ws_base(w);
    sa.desc = (Desc *)(ws_base(w) + kHeaderBytes);
    ia.mdesc = (Desc *)(ws_base(w) + off_m);
    ia.total = (uint64_t *)(ws_base(w) + off_tot);
    ia.scan_status = (int32_t *)(ws_base(w) + off_tot + 8);
    ia.na = na;
    ia.piece = piece;
    ia.b = b;
    ia.nb = nb;
    ia.out = out;
    ia.out_cap = out_cap;
    ia.d_count = d_count;
    ia.d_status = d_status;
    hipError_t e = launch_isect(ia, s);
    return e == hipSuccess ? VBYTE_OK : hip_fail(e, "intersect launch");
}

vbyte_status vbyte_count(const uint8_t *bytes, size_t nbytes, uint64_t *d_count, void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    hipStream_t s = (hipStream_t)stream;
    if (!d_count || ((uintptr_t)d_count & 7u)) return VBYTE_EINVAL;
    if (nbytes >= kMaxBytes) return VBYTE_EINVAL;
    if (nbytes > 0 && !bytes) return VBYTE_EINVAL;
    if (nbytes == 0) {
        hipError_t e = launch_set_u64(d_count, 0, s);
        return e == hipSuccess ? VBYTE_OK : hip_fail(e, "set count");
    }
    const int segs = g_segs.load(), wpb = g_wpb.load();
    StreamArgs a{};
    a.spin_limit = spin_limit();
    a.vstart = (uintptr_t)bytes & 15u;
    a.base = bytes - a.vstart;
    a.vend = a.vstart + nbytes;
    a.out = nullptr;
    a.n = 0;
    const uint64_t ntiles = stream_tiles(a.vstart, nbytes, segs, wpb);
    if (ntiles >= (1ull << 31)) return VBYTE_EINVAL;
    a.ntiles = (uint32_t)ntiles;
    Workspace *w = nullptr;
    vbyte_status st = get_ws(s, kHeaderBytes + ntiles * sizeof(Desc), 1, &w);
    if (st != VBYTE_OK) return st;
    a.hdr = (uint64_t *)ws_base(w);
    a.desc = (Desc *)(ws_base(w) + kHeaderBytes);
    a.d_status = nullptr;
    a.d_count = d_count;
    hipError_t e = launch_stream(a, 0, 1, segs, wpb, s);
    return e == hipSuccess ? VBYTE_OK : hip_fail(e, "count launch");
}

vbyte_status vbyte_decode_batch(const uint8_t *bytes, size_t nbytes, const int64_t *byte_off,
                                uint32_t *out, size_t nout, const int64_t *out_off, size_t nlists,
                                const uint32_t *prevs, int delta, int32_t *d_list_status,
                                void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    if (nlists > 0 && (!byte_off || !out_off)) return VBYTE_EINVAL;
    if (delta < 0 || delta > 2) return VBYTE_EINVAL;
    ListArgs a{};
    a.spin_limit = spin_limit();
    a.bytes = bytes;
    a.nbytes = nbytes;
    a.nout = nout;
    a.byte_off = byte_off;
    a.out_off = out_off;
    a.rows = nullptr;
    a.out = out;
    a.prevs = prevs;
    a.list_status = d_list_status;
    a.nlists = nlists;
    a.delta = delta;
    return batch_common(a, nbytes, (hipStream_t)stream);
}

vbyte_status vbyte_decode_lists(const uint8_t *bytes, size_t nbytes, const int64_t *lists,
                                size_t nlists, size_t list_bytes, uint32_t *out, size_t nout,
                                const uint32_t *prevs, int delta, int32_t *d_list_status,
                                void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    if (nlists > 0 && !lists) return VBYTE_EINVAL;
    if (delta < 0 || delta > 2) return VBYTE_EINVAL;
    ListArgs a{};
    a.spin_limit = spin_limit();
    a.bytes = bytes;
    a.nbytes = nbytes;
    a.nout = nout;
    a.byte_off = nullptr;
    a.out_off = nullptr;
    a.rows = lists;
    a.out = out;
    a.prevs = prevs;
    a.list_status = d_list_status;
    a.nlists = nlists;
    a.delta = delta;
    return batch_common(a, list_bytes, (hipStream_t)stream);
}

static vbyte_status encode_common(const uint32_t *values, size_t n, uint32_t prev, int delta,
                                  uint8_t *bytes, size_t capacity, uint64_t *d_nbytes,
                                  hipStream_t s, const int64_t *vals_off = nullptr,
                                  int64_t *byte_off = nullptr, size_t nbounds = 0) {
    if (!d_nbytes || ((uintptr_t)d_nbytes & 7u)) return VBYTE_EINVAL;
    if (n > 0 && !values) return VBYTE_EINVAL;
    if (((uintptr_t)values & 3u) != 0) return VBYTE_EINVAL;
    if (capacity > 0 && !bytes) return VBYTE_EINVAL;
    if (n == 0) {
        hipError_t e = launch_set_u64(d_nbytes, 0, s);
        return e == hipSuccess ? VBYTE_OK : hip_fail(e, "set nbytes");
    }
    if (n >= (1ull << 40)) return VBYTE_EINVAL;
    EncArgs a{};
    a.e0 = ((uintptr_t)values >> 2) & 3u;
    a.vbase = values - a.e0;
    a.n = n;
    a.prev = prev;
    a.delta = delta;
    a.bytes = bytes;
    a.capacity = capacity;
    a.d_nbytes = d_nbytes;
    a.nchunks = (a.e0 + n + kEncChunk - 1) / kEncChunk;
    const uint64_t ngs = (a.nchunks + kEncLenChunks - 1) / kEncLenChunks;
    // workspace: chunk counts (4 B), chunk offsets (8 B), length-workgroup totals (4 B)
    const size_t off_pre = kHeaderBytes + ((a.nchunks * 4 + 15) & ~(uint64_t)15);
    const size_t off_gsum = off_pre + a.nchunks * 8;
    Workspace *w = nullptr;
    vbyte_status st = get_ws(s, off_gsum + ngs * 4, 0, &w);
    if (st != VBYTE_OK) return st;
    a.csum = (uint32_t *)(ws_base(w) + kHeaderBytes);
    a.cpre = (uint64_t *)(ws_base(w) + off_pre);
    a.gsum = (uint32_t *)(ws_base(w) + off_gsum);
    hipError_t e = launch_encode(a, s);
    if (e != hipSuccess) return hip_fail(e, "encode launch");
    if (nbounds) {
        e = launch_encode_bounds(a, vals_off, byte_off, nbounds, s);
        if (e != hipSuccess) return hip_fail(e, "encode bounds launch");
    }
    return VBYTE_OK;
}

vbyte_status vbyte_encode_async(const uint32_t *values, size_t n, uint8_t *bytes, size_t capacity,
                                uint64_t *d_nbytes, void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return encode_common(values, n, 0, 0, bytes, capacity, d_nbytes, (hipStream_t)stream);
}

vbyte_status vbyte_encode_delta_async(const uint32_t *values, size_t n, uint32_t prev,
                                      uint8_t *bytes, size_t capacity, uint64_t *d_nbytes,
                                      void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return encode_common(values, n, prev, 1, bytes, capacity, d_nbytes, (hipStream_t)stream);
}

vbyte_status vbyte_encode_delta_m1_async(const uint32_t *values, size_t n, uint32_t prev,
                                         uint8_t *bytes, size_t capacity, uint64_t *d_nbytes,
                                         void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    return encode_common(values, n, prev, 2, bytes, capacity, d_nbytes, (hipStream_t)stream);
}

vbyte_status vbyte_encode_batch(const uint32_t *values, size_t n, const int64_t *vals_off,
                                size_t nlists, uint8_t *bytes, size_t capacity, int64_t *byte_off,
                                uint64_t *d_nbytes, void *stream) {
    StreamGuard guard_((hipStream_t)stream);
    if (nlists > 0 && (!vals_off || !byte_off)) return VBYTE_EINVAL;
    if (((uintptr_t)byte_off & 7u) || ((uintptr_t)vals_off & 7u)) return VBYTE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        if (nlists > 0) {
            hipError_t e = launch_fill_i64(byte_off, nlists + 1, 0, s);
            if (e != hipSuccess) return hip_fail(e, "zero byte offsets");
        }
        return encode_common(values, 0, 0, 0, bytes, capacity, d_nbytes, s);
    }
    return encode_common(values, n, 0, 0, bytes, capacity, d_nbytes, s, vals_off, byte_off,
                         nlists ? nlists + 1 : 0);
}

size_t vbyte_workspace_size(size_t nbytes) {
    // the largest of the single-stream forms at the current segment count
    // and the smallest workgroups: the 32-bit decode's tile descriptors, the
    // 64-bit decode's unit and group slots (16 bytes), the blocks-of-four
    // decode's unit, group and block slots (32 bytes; a block holds at least
    // one unit)
    const uint64_t d32 = two_pass_slots(stream_tiles(15, nbytes, g_segs.load(), 1)) * sizeof(Desc);
    const uint64_t unit = (uint64_t)kUnit64Groups * std::min(g_segs.load(), 2) * kSegBytes;
    const uint64_t nunits = (15 + nbytes + unit - 1) / unit;
    const uint64_t d64 = nunits * 16 * (1 + kUnit64Groups);
    const uint64_t d4 = (nunits * (1 + kUnit64Groups) + nunits) * 32;
    return kHeaderBytes + std::max(d32, std::max(d64, d4));
}

vbyte_status vbyte_set_tuning(int segs_per_wave, int waves_per_block, int64_t small_list_bytes) {
    if (segs_per_wave != 0 && segs_per_wave != 1 && segs_per_wave != 2 && segs_per_wave != 4)
        return VBYTE_EINVAL;
    if (waves_per_block < 0 || waves_per_block > 8) return VBYTE_EINVAL;
    if (small_list_bytes < 0) return VBYTE_EINVAL;
    if (segs_per_wave) g_segs.store(segs_per_wave);
    if (waves_per_block) g_wpb.store(waves_per_block);
    if (small_list_bytes) g_small.store(small_list_bytes);
    return VBYTE_OK;
}

vbyte_status vbyte_set_chunk_tiles(int tiles_per_chunk) {
    if (tiles_per_chunk < kScheduleFlow || tiles_per_chunk > 64) return VBYTE_EINVAL;
    g_chunk.store(tiles_per_chunk);
    return VBYTE_OK;
}

int vbyte_get_chunk_tiles(void) { return g_chunk.load(); }

void vbyte_get_tuning(int *segs_per_wave, int *waves_per_block, int64_t *small_list_bytes) {
    if (segs_per_wave) *segs_per_wave = g_segs.load();
    if (waves_per_block) *waves_per_block = g_wpb.load();
    if (small_list_bytes) *small_list_bytes = g_small.load();
}

const char *vbyte_status_str(vbyte_status st) {
    switch (st) {
        case VBYTE_OK: return "VBYTE_OK";
        case VBYTE_EINVAL: return "VBYTE_EINVAL";
        case VBYTE_ECOUNT: return "VBYTE_ECOUNT";
        case VBYTE_ETRUNC: return "VBYTE_ETRUNC";
        case VBYTE_EMALFORMED: return "VBYTE_EMALFORMED";
        case VBYTE_EHIP: return "VBYTE_EHIP";
        case VBYTE_ENOMEM: return "VBYTE_ENOMEM";
        case VBYTE_ESTALLED: return "VBYTE_ESTALLED";
    }
    return "VBYTE_UNKNOWN";
}

const char *vbyte_last_error(void) { return g_last_error; }

}  // extern "C"
