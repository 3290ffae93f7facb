// serve.cpp -- continuous-batching request loop over a VByte index resident
// in HBM (the served form of the decode; C ABI in include/vbyte.h).
//
// A request asks for the decoded posting lists of several terms; its result
// is the concatenation of those lists, each decoded (optionally with the
// differential prefix sum, every list restarting from 0) in term order.
//
// Loop, on one host thread:
//   * arrivals are released at their scheduled times (open loop);
//   * admission is FIFO by output memory: a request is admitted when a
//     contiguous range of the device output pool can hold its result (first
//     fit); it is never skipped by a later, smaller one;
//   * every stream that is idle takes all admitted requests (up to a cap) as
//     one batch: its lists become gather rows, copied to the device, and one
//     vbyte_decode_lists launch decodes them all; with several streams,
//     batches overlap on the GPU while new requests keep being admitted;
//   * a batch's requests are sorted by output size and cut into up to four
//     groups, smallest first, each decoded by its own launch followed by an
//     event, so that a request's latency (host steady clock) ends with its
//     group, not with the largest request of the batch;
//   * a batch completes when its last event fires: per-list statuses give
//     each request's status, results are optionally copied out, and the
//     pool ranges freed.
// The "per-list launches" mode replaces the batched launch by one
// single-stream launch per list (the baseline the batched form is compared
// against).

#include <rocprofiler-sdk-roctx/roctx.h>
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "vbyte.h"
#include "vbyte_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// A batch is decoded in up to kGroups launches: its requests sorted by
// output size, smallest first, cut into groups of about equal count; each
// group's launch is followed by an event, so a request's completion is its
// group's event, not the end of the whole batch.
constexpr int kGroups = 4;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t gdone[kGroups] = {};
    int64_t *h_rows = nullptr;    // pinned
    int64_t *d_rows = nullptr;
    int32_t *h_status = nullptr;  // pinned
    int32_t *d_status = nullptr;
    size_t cap_rows = 0;
    bool busy = false;
    std::vector<size_t> reqs;        // requests of the batch in flight, in group order
    std::vector<int64_t> req_row0;   // first row of each request of the batch
    std::vector<size_t> gend;        // end (in reqs) of every group
    std::vector<char> gseen;         // group completion already taken
    bool grouped = false;            // the batch's groups have events
    size_t nrows = 0;
};

// First-fit allocator over [0, size) in uint32 elements.
class Pool {
  public:
    explicit Pool(uint64_t size) { free_[0] = size; }
    bool alloc(uint64_t n, uint64_t *off) {
        if (n == 0) {
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        if (n == 0) return;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<uint64_t, uint64_t> free_;
};

}  // namespace

struct vbyte_server {
    const uint8_t *index = nullptr;
    size_t nbytes = 0;
    std::vector<int64_t> byte_off;
    std::vector<int64_t> counts;
    vbyte_server_config cfg{};
    uint32_t *pool = nullptr;
    uint64_t pool_elems = 0;
    std::vector<Slot> slots;
};

// A roctx range for the lifetime of the object (ends on every return path).
struct RoctxRange {
    explicit RoctxRange(const char *what) { roctxRangePushA(what); }
    ~RoctxRange() { roctxRangePop(); }
    RoctxRange(const RoctxRange &) = delete;
    RoctxRange &operator=(const RoctxRange &) = delete;
};

static vbyte_status hip_err(hipError_t e) { return e == hipSuccess ? VBYTE_OK : VBYTE_EHIP; }

static void destroy_slots(vbyte_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_rows) (void)hipHostFree(sl.h_rows);
        if (sl.d_rows) (void)hipFree(sl.d_rows);
        if (sl.h_status) (void)hipHostFree(sl.h_status);
        if (sl.d_status) (void)hipFree(sl.d_status);
        for (hipEvent_t &e : sl.gdone)
            if (e) (void)hipEventDestroy(e);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    s->slots.clear();
}

static vbyte_status ensure_rows(Slot &sl, size_t rows) {
    if (rows <= sl.cap_rows) return VBYTE_OK;
    size_t cap = std::max<size_t>(rows, std::max<size_t>(2 * sl.cap_rows, 1024));
    if (sl.h_rows) (void)hipHostFree(sl.h_rows);
    if (sl.d_rows) (void)hipFree(sl.d_rows);
    if (sl.h_status) (void)hipHostFree(sl.h_status);
    if (sl.d_status) (void)hipFree(sl.d_status);
    sl.h_rows = nullptr;
    sl.d_rows = nullptr;
    sl.h_status = nullptr;
    sl.d_status = nullptr;
    sl.cap_rows = 0;
    if (hipHostMalloc((void **)&sl.h_rows, cap * 4 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&sl.d_rows, cap * 4 * sizeof(int64_t)) != hipSuccess ||
        hipHostMalloc((void **)&sl.h_status, cap * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&sl.d_status, cap * sizeof(int32_t)) != hipSuccess)
        return VBYTE_ENOMEM;
    sl.cap_rows = cap;
    return VBYTE_OK;
}

extern "C" {

vbyte_status vbyte_server_create(const uint8_t *index_bytes, size_t nbytes, const int64_t *byte_off,
                                 const int64_t *counts, size_t nlists,
                                 const vbyte_server_config *cfg, vbyte_server **out) {
    if (!out || !cfg || !byte_off || !counts || (nbytes && !index_bytes)) return VBYTE_EINVAL;
    if (cfg->nstreams < 1 || cfg->nstreams > 8 || cfg->pool_bytes < 4 || cfg->max_batch_requests < 1)
        return VBYTE_EINVAL;
    for (size_t i = 0; i < nlists; ++i) {
        if (byte_off[i + 1] < byte_off[i] || counts[i] < 0) return VBYTE_EINVAL;
    }
    if (nlists && (byte_off[0] < 0 || (uint64_t)byte_off[nlists] > nbytes)) return VBYTE_EINVAL;
    vbyte_server *s = new vbyte_server();
    s->index = index_bytes;
    s->nbytes = nbytes;
    s->byte_off.assign(byte_off, byte_off + nlists + 1);
    s->counts.assign(counts, counts + nlists);
    s->cfg = *cfg;
    s->pool_elems = cfg->pool_bytes / 4;
    if (hipMalloc((void **)&s->pool, s->pool_elems * 4) != hipSuccess) {
        delete s;
        return VBYTE_ENOMEM;
    }
    s->slots.resize(cfg->nstreams);
    for (Slot &sl : s->slots) {
        bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
        for (hipEvent_t &e : sl.gdone) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (!ok || ensure_rows(sl, 1024) != VBYTE_OK) {
            destroy_slots(s);
            (void)hipFree(s->pool);
            delete s;
            return VBYTE_ENOMEM;
        }
    }
    *out = s;
    return VBYTE_OK;
}

void vbyte_server_destroy(vbyte_server *s) {
    if (!s) return;
    destroy_slots(s);
    if (s->pool) (void)hipFree(s->pool);
    delete s;
}

vbyte_status vbyte_server_run(vbyte_server *s, size_t nreq, const double *arrival_s,
                              const int64_t *term_off, const int64_t *terms, double *latency_s,
                              int32_t *req_status, uint32_t *results, const int64_t *result_off,
                              vbyte_serve_stats *stats) {
    if (!s || (nreq && (!arrival_s || !term_off || !terms || !latency_s))) return VBYTE_EINVAL;
    if (results && !result_off) return VBYTE_EINVAL;
    const size_t nlists = s->counts.size();
    for (size_t r = 0; r < nreq; ++r) {
        if (term_off[r + 1] < term_off[r]) return VBYTE_EINVAL;
        if (r && arrival_s[r] < arrival_s[r - 1]) return VBYTE_EINVAL;
        for (int64_t k = term_off[r]; k < term_off[r + 1]; ++k)
            if (terms[k] < 0 || (size_t)terms[k] >= nlists) return VBYTE_EINVAL;
    }
    // per-request output size (uint32 elements) and pool ranges
    std::vector<uint64_t> need(nreq), pool_off(nreq, 0);
    for (size_t r = 0; r < nreq; ++r) {
        uint64_t e = 0;
        for (int64_t k = term_off[r]; k < term_off[r + 1]; ++k) e += (uint64_t)s->counts[terms[k]];
        need[r] = e;
    }
    Pool pool(s->pool_elems);
    std::deque<size_t> pending;
    size_t next = 0, completed = 0;
    vbyte_serve_stats st{};
    int32_t worst = VBYTE_OK;
    uint64_t batches = 0, launches = 0, batched_reqs = 0;
    const bool delta = s->cfg.delta != 0;
    const size_t cap = (size_t)s->cfg.max_batch_requests;

    const Clock::time_point t0 = Clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };
    // roctx ranges (visible with rocprofv3 --marker-trace): the whole run,
    // each batch's admission and launches; a mark per finished group
    const RoctxRange run_range("vbyte_server_run");

    while (completed < nreq) {
        bool progressed = false;
        double now = now_s();
        while (next < nreq && arrival_s[next] <= now) pending.push_back(next++);

        // completions: a request is done when its group's launch has ended
        // (its group event), at the latest with its batch (the batch event,
        // which also ends the status and result copies); the batch's pool
        // ranges are released and its statuses read at the batch event
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            for (size_t g = 0; sl.grouped && g + 1 < sl.gend.size(); ++g) {
                if (sl.gseen[g]) continue;
                hipError_t q = hipEventQuery(sl.gdone[g]);
                if (q == hipErrorNotReady) break;   // groups end in order
                if (q != hipSuccess) return VBYTE_EHIP;
                const double t = now_s();
                for (size_t k = sl.gend[g]; k < sl.gend[g + 1]; ++k) latency_s[sl.reqs[k]] = t - arrival_s[sl.reqs[k]];
                sl.gseen[g] = 1;
                roctxMarkA("vbyte serve: group done");
                progressed = true;
            }
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return VBYTE_EHIP;
            const double t = now_s();
            for (size_t g = 0; g + 1 < sl.gend.size(); ++g) {
                if (sl.gseen[g]) continue;
                for (size_t k = sl.gend[g]; k < sl.gend[g + 1]; ++k) latency_s[sl.reqs[k]] = t - arrival_s[sl.reqs[k]];
                sl.gseen[g] = 1;
            }
            for (size_t k = 0; k < sl.reqs.size(); ++k) {
                const size_t r = sl.reqs[k];
                int32_t rs = VBYTE_OK;
                for (int64_t j = sl.req_row0[k]; j < sl.req_row0[k + 1]; ++j)
                    rs = std::max<int32_t>(rs, sl.h_status[j]);
                if (req_status) req_status[r] = rs;
                worst = std::max<int32_t>(worst, rs);
                pool.release(pool_off[r], need[r]);
                ++completed;
            }
            sl.reqs.clear();
            sl.busy = false;
            progressed = true;
        }

        // admission and launch on idle streams
        for (Slot &sl : s->slots) {
            if (sl.busy || pending.empty()) continue;
            std::vector<size_t> batch;
            size_t rows = 0;
            while (!pending.empty() && batch.size() < cap) {
                const size_t r = pending.front();
                if (need[r] > s->pool_elems) {   // can never fit: reject
                    latency_s[r] = -1.0;
                    if (req_status) req_status[r] = VBYTE_ENOMEM;
                    ++st.rejected;
                    ++completed;
                    pending.pop_front();
                    continue;
                }
                uint64_t off;
                if (!pool.alloc(need[r], &off)) break;   // FIFO: wait for memory
                pool_off[r] = off;
                batch.push_back(r);
                rows += (size_t)(term_off[r + 1] - term_off[r]);
                pending.pop_front();
            }
            if (batch.empty()) break;
            const RoctxRange batch_range("vbyte serve: batch admission and launches");
            vbyte_status es = ensure_rows(sl, rows);
            if (es != VBYTE_OK) return es;
            // groups: the batch's requests by output size, smallest first
            std::stable_sort(batch.begin(), batch.end(),
                             [&](size_t x, size_t y) { return need[x] < need[y]; });
            const size_t ng = s->cfg.batching ? std::min<size_t>(kGroups, batch.size()) : 1;
            sl.gend.assign(ng + 1, 0);
            for (size_t g = 0; g <= ng; ++g) sl.gend[g] = g * batch.size() / ng;
            sl.gseen.assign(ng, 0);
            size_t k = 0;
            sl.req_row0.assign(batch.size() + 1, 0);
            for (size_t b = 0; b < batch.size(); ++b) {
                const size_t r = batch[b];
                uint64_t pos = pool_off[r];
                sl.req_row0[b] = (int64_t)k;
                for (int64_t j = term_off[r]; j < term_off[r + 1]; ++j) {
                    const int64_t t = terms[j];
                    sl.h_rows[4 * k + 0] = s->byte_off[t];
                    sl.h_rows[4 * k + 1] = s->byte_off[t + 1];
                    sl.h_rows[4 * k + 2] = (int64_t)pos;
                    sl.h_rows[4 * k + 3] = s->counts[t];
                    pos += (uint64_t)s->counts[t];
                    ++k;
                }
            }
            sl.req_row0[batch.size()] = (int64_t)k;
            if (rows) {
                if (s->cfg.batching) {
                    if (hipMemcpyAsync(sl.d_rows, sl.h_rows, rows * 4 * sizeof(int64_t),
                                       hipMemcpyHostToDevice, sl.stream) != hipSuccess)
                        return VBYTE_EHIP;
                    for (size_t g = 0; g < ng; ++g) {
                        const int64_t r0 = sl.req_row0[sl.gend[g]], r1 = sl.req_row0[sl.gend[g + 1]];
                        uint64_t gbytes = 0;
                        for (int64_t j = r0; j < r1; ++j)
                            gbytes += (uint64_t)(sl.h_rows[4 * j + 1] - sl.h_rows[4 * j]);
                        if (r1 > r0) {
                            vbyte_status ls = vbyte_decode_lists(
                                s->index, s->nbytes, sl.d_rows + 4 * r0, (size_t)(r1 - r0), gbytes, s->pool,
                                s->pool_elems, nullptr, delta ? 1 : 0, sl.d_status + r0, sl.stream);
                            if (ls != VBYTE_OK) return ls;
                            ++launches;
                        }
                        if (hipEventRecord(sl.gdone[g], sl.stream) != hipSuccess) return VBYTE_EHIP;
                    }
                } else {
                    for (size_t j = 0; j < rows; ++j) {
                        const int64_t *row = sl.h_rows + 4 * j;
                        const uint8_t *b = s->index + row[0];
                        const size_t nb = (size_t)(row[1] - row[0]);
                        uint32_t *o = s->pool + row[2];
                        vbyte_status ls = delta
                            ? vbyte_decode_delta_async(b, nb, o, (size_t)row[3], 0, sl.d_status + j, sl.stream)
                            : vbyte_decode_async(b, nb, o, (size_t)row[3], sl.d_status + j, sl.stream);
                        if (ls != VBYTE_OK) return ls;
                        ++launches;
                    }
                }
                if (results) {
                    for (size_t r : batch) {
                        if (need[r] == 0) continue;
                        if (hipMemcpyAsync(results + result_off[r], s->pool + pool_off[r], need[r] * 4,
                                           hipMemcpyDeviceToDevice, sl.stream) != hipSuccess)
                            return VBYTE_EHIP;
                    }
                }
                if (hipMemcpyAsync(sl.h_status, sl.d_status, rows * sizeof(int32_t), hipMemcpyDeviceToHost,
                                   sl.stream) != hipSuccess)
                    return VBYTE_EHIP;
            }
            // without group launches (one launch per list, or no rows) the
            // requests complete with the batch event only
            sl.grouped = s->cfg.batching && rows;
            if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return VBYTE_EHIP;
            sl.reqs = batch;
            sl.nrows = rows;
            sl.busy = true;
            ++batches;
            batched_reqs += batch.size();
            progressed = true;
        }

        if (!progressed) {
            bool any_busy = false;
            for (Slot &sl : s->slots) any_busy |= sl.busy;
            if (!any_busy && pending.empty() && next < nreq) {
                const double wait = arrival_s[next] - now_s();
                if (wait > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(wait - 100e-6));
            } else {
                std::this_thread::yield();
            }
        }
    }
    for (Slot &sl : s->slots) (void)hipStreamSynchronize(sl.stream);
    st.wall_s = now_s();
    uint64_t ints = 0;
    for (size_t r = 0; r < nreq; ++r)
        if (latency_s[r] >= 0) ints += need[r];
    st.integers = ints;
    st.batches = batches;
    st.launches = launches;
    st.mean_batch_requests = batches ? (double)batched_reqs / (double)batches : 0.0;
    st.worst_status = worst;
    if (stats) *stats = st;
    return VBYTE_OK;
}

}  // extern "C"
