// tune.cpp -- the autotuner of the decode tiling (include/vbyte.h,
// vbyte_autotune_*).
//
// It times the caller's own workload under every candidate tiling with HIP
// events on the caller's stream, keeps the fastest and applies it with
// vbyte_set_tuning / vbyte_set_chunk_tiles.  Candidates: 1 KiB segments per
// wavefront {2, 4} x wavefronts per workgroup {4, 8} x single-stream kernel
// {-1 (two passes), 0 (look-back per tile), chunks of 2, 4, 8, 16
// tiles} for a single stream; for the batched form {2, 4} x
// {4, 8} x small-list threshold {1, 4, 16, 64} KiB.  The
// tuning is process-wide, so no other decode should run meanwhile.

#include <hip/hip_runtime.h>

#include "vbyte.h"
#include "vbyte_internal.h"

using namespace vb;

namespace {

struct Cand {
    int segs, wpb;
    int64_t small;
    int chunk;
};

// Times `reps` calls of fn() on stream s (after one untimed call); the mean
// milliseconds go to *ms.
template <class F>
vbyte_status time_calls(F fn, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double *ms) {
    vbyte_status st = fn();
    if (st != VBYTE_OK) return st;
    hipError_t e = hipEventRecord(e0, s);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord");
    for (int r = 0; r < reps; ++r) {
        st = fn();
        if (st != VBYTE_OK) return st;
    }
    e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) return hip_error(e, "timing events");
    *ms = (double)t / reps;
    return VBYTE_OK;
}

// Runs every candidate, records it, applies the fastest.  `check` reads the
// data status the calls produced (after a synchronisation).
template <class F, class C>
vbyte_status tune(const Cand *cands, int ncand, F call, C check, int reps, hipStream_t s,
                  vbyte_tune_point *points, size_t max_points, size_t *npoints) {
    if (reps < 1 || reps > 1000) return VBYTE_EINVAL;
    int segs0, wpb0;
    int64_t small0;
    vbyte_get_tuning(&segs0, &wpb0, &small0);
    const int chunk0 = vbyte_get_chunk_tiles();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_error(e, "hipEventCreate");
    }
    vbyte_status st = VBYTE_OK;
    int best = -1;
    double best_ms = 0;
    size_t written = 0;
    for (int i = 0; i < ncand && st == VBYTE_OK; ++i) {
        st = vbyte_set_tuning(cands[i].segs, cands[i].wpb, cands[i].small);
        if (st == VBYTE_OK) st = vbyte_set_chunk_tiles(cands[i].chunk);
        double ms = 0;
        if (st == VBYTE_OK) st = time_calls(call, reps, s, e0, e1, &ms);
        int32_t data = VBYTE_OK;
        if (st == VBYTE_OK) st = check(&data);
        if (st != VBYTE_OK) break;
        if (points && (size_t)i < max_points) {
            points[i] = vbyte_tune_point{cands[i].segs, cands[i].wpb, cands[i].small,
                                         cands[i].chunk, ms, data};
            written = (size_t)i + 1;
        }
        if (data != VBYTE_OK) {
            st = (vbyte_status)data;   // the workload itself does not decode
            break;
        }
        if (best < 0 || ms < best_ms) {
            best = i;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (npoints) *npoints = written;
    if (st != VBYTE_OK || best < 0) {
        (void)vbyte_set_tuning(segs0, wpb0, small0);
        (void)vbyte_set_chunk_tiles(chunk0);
        return st != VBYTE_OK ? st : VBYTE_EINVAL;
    }
    const vbyte_status fin = vbyte_set_chunk_tiles(cands[best].chunk);
    return fin != VBYTE_OK ? fin : vbyte_set_tuning(cands[best].segs, cands[best].wpb, cands[best].small);
}

}  // namespace

extern "C" {

vbyte_status vbyte_autotune_decode(const uint8_t *bytes, size_t nbytes, uint32_t *out, size_t n,
                                   int delta, int reps, int32_t *d_status,
                                   vbyte_tune_point *points, size_t max_points, size_t *npoints,
                                   void *stream) {
    if (!d_status || (delta != 0 && delta != 1)) return VBYTE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t small = 0;
    vbyte_get_tuning(nullptr, nullptr, &small);
    Cand cands[24];
    int nc = 0;
    for (int segs : {2, 4})
        for (int wpb : {4, 8})
            for (int chunk : {-1, 0, 2, 4, 8, 16}) cands[nc++] = Cand{segs, wpb, small, chunk};
    auto call = [&]() {
        return delta ? vbyte_decode_delta_async(bytes, nbytes, out, n, 0, d_status, s)
                     : vbyte_decode_async(bytes, nbytes, out, n, d_status, s);
    };
    auto check = [&](int32_t *data) {
        hipError_t e = hipMemcpyAsync(data, d_status, sizeof *data, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e == hipSuccess ? VBYTE_OK : hip_error(e, "status copy");
    };
    return tune(cands, nc, call, check, reps, s, points, max_points, npoints);
}

vbyte_status vbyte_autotune_batch(const uint8_t *bytes, size_t nbytes, const int64_t *byte_off,
                                  uint32_t *out, size_t nout, const int64_t *out_off,
                                  size_t nlists, int delta, int reps, int32_t *d_list_status,
                                  vbyte_tune_point *points, size_t max_points, size_t *npoints,
                                  void *stream) {
    if (!d_list_status || nlists == 0 || delta < 0 || delta > 2) return VBYTE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Cand cands[16];
    int nc = 0;
    for (int segs : {2, 4})
        for (int wpb : {4, 8})
            for (int64_t small : {1024, 4096, 16384, 65536})
                cands[nc++] = Cand{segs, wpb, small, vbyte_get_chunk_tiles()};
    auto call = [&]() {
        return vbyte_decode_batch(bytes, nbytes, byte_off, out, nout, out_off, nlists, nullptr,
                                  delta, d_list_status, s);
    };
    // the worst list status: copied back whole, at most once per candidate
    auto check = [&](int32_t *data) {
        const size_t chunk = 1 << 16;
        static thread_local int32_t host[1 << 16];
        *data = VBYTE_OK;
        for (size_t i = 0; i < nlists; i += chunk) {
            const size_t m = nlists - i < chunk ? nlists - i : chunk;
            hipError_t e = hipMemcpyAsync(host, d_list_status + i, m * sizeof(int32_t),
                                          hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_error(e, "list status copy");
            for (size_t k = 0; k < m; ++k)
                if (host[k] > *data) *data = host[k];
        }
        return VBYTE_OK;
    };
    return tune(cands, nc, call, check, reps, s, points, max_points, npoints);
}

}  // extern "C"
