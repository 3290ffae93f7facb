// graph.cpp -- the batched decode captured once into a HIP graph and
// replayed (include/vbyte.h, vbyte_batch_graph_*).
//
// The graph object owns its workspace, so a replay needs no allocation and
// enqueues exactly the two kernels of vbyte_decode_batch (the prep kernel
// and the persistent decode), with the arguments fixed at capture.  The
// workspace's epoch word advances twice per replay; before the epoch tag
// could wrap, the launch call clears the workspace with a kernel enqueued
// ahead of the graph (never inside it).

#include <cstdio>
#include <new>

#include <hip/hip_runtime.h>

#include "vbyte.h"
#include "vbyte_internal.h"

using namespace vb;

struct vbyte_batch_graph {
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t launches = 0;   // epoch advances since the workspace was cleared
};

namespace {

void release(vbyte_batch_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ws) (void)hipFree(g->ws);
    delete g;
}

}  // namespace

extern "C" {

vbyte_status vbyte_batch_graph_create(const uint8_t *bytes, size_t nbytes, const int64_t *byte_off,
                                      uint32_t *out, size_t nout, const int64_t *out_off,
                                      size_t nlists, const uint32_t *prevs, int delta,
                                      int32_t *d_list_status, vbyte_batch_graph **graph) {
    if (!graph) return VBYTE_EINVAL;
    *graph = nullptr;
    if (nlists == 0 || !byte_off || !out_off) return VBYTE_EINVAL;
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
    BatchPlan plan;
    vbyte_status st = batch_plan(a, nbytes, &plan);
    if (st != VBYTE_OK) return st;

    vbyte_batch_graph *g = new (std::nothrow) vbyte_batch_graph;
    if (!g) return VBYTE_ENOMEM;
    g->ws_bytes = (plan.bytes + 255) & ~(size_t)255;
    hipError_t e = hipMalloc(&g->ws, g->ws_bytes);
    if (e != hipSuccess) {
        g->ws = nullptr;
        release(g);
        return VBYTE_ENOMEM;
    }
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        release(g);
        return hip_error(e, "hipStreamCreateWithFlags");
    }
    // zero the workspace outside the graph, and wait for it
    e = launch_zero(g->ws, g->ws_bytes, cap);
    if (e == hipSuccess) e = hipStreamSynchronize(cap);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        release(g);
        return hip_error(e, "zero graph workspace");
    }
    batch_bind(a, plan, (uint8_t *)g->ws);
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = launch_batch(a, plan.segs, plan.wpb, plan.grid, cap);
        e = hipStreamEndCapture(cap, &g->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        release(g);
        return hip_error(e, "batch graph capture");
    }
    *graph = g;
    return VBYTE_OK;
}

vbyte_status vbyte_batch_graph_launch(vbyte_batch_graph *graph, void *stream) {
    if (!graph || !graph->exec) return VBYTE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (graph->launches + 2 >= kEpochLaunchLimit) {
        hipError_t e = launch_zero(graph->ws, graph->ws_bytes, s);
        if (e != hipSuccess) return hip_error(e, "re-zero graph workspace");
        graph->launches = 0;
    }
    graph->launches += 2;
    hipError_t e = hipGraphLaunch(graph->exec, s);
    return e == hipSuccess ? VBYTE_OK : hip_error(e, "hipGraphLaunch");
}

void vbyte_batch_graph_destroy(vbyte_batch_graph *graph) { release(graph); }

}  // extern "C"
