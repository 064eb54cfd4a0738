// dq_batch.hip - a batch of fields as one HIP graph (host runtime, no kernels
// of its own): the fields' compress and device-count decompress calls are
// captured once over parallel branches and replayed with one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/dq.h"
#include "../../include/dq_batch.h"

struct dq_batch_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> streams;  // [0] capture origin, then the branches
    std::vector<hipEvent_t> events;    // [0] fork, then one join per branch
};

namespace {

void release(dq_batch_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
    for (hipStream_t s : g->streams) (void)hipStreamDestroy(s);
    delete g;
}

uint64_t cells(const dq_params& p) {
    uint64_t n = 1;
    for (int a = 0; a < p.ndim && a < 3; ++a) n *= (uint64_t)(p.shape[a] > 0 ? p.shape[a] : 0);
    return n;
}

}  // namespace

extern "C" {

dq_status dq_batch_graph_create(const dq_batch_field* fields, uint64_t n, int branches, dq_batch_graph** graph) {
    if (!fields || n == 0 || !graph || branches < 1 || branches > 16) return DQ_EINVAL;
    *graph = nullptr;
    for (uint64_t i = 0; i < n; ++i) {
        const dq_status st = dq_validate(&fields[i].p);
        if (st != DQ_OK) return st;
    }
    dq_batch_graph* g = new dq_batch_graph();
    const int nb = (int)std::min<uint64_t>((uint64_t)branches, n);
    for (int k = 0; k <= nb; ++k) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            release(g);
            return DQ_EDEVICE;
        }
        g->streams.push_back(s);
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            release(g);
            return DQ_EDEVICE;
        }
        g->events.push_back(e);
    }
    // largest fields first, each to the least loaded branch
    std::vector<uint64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint64_t a, uint64_t b) { return cells(fields[a].p) > cells(fields[b].p); });
    std::vector<uint64_t> load(nb, 0);
    std::vector<int> branch_of(n, 0);
    for (uint64_t i : order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        branch_of[i] = b;
        load[b] += cells(fields[i].p);
    }

    hipStream_t origin = g->streams[0];
    if (hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed) != hipSuccess) {
        release(g);
        return DQ_EDEVICE;
    }
    dq_status st = DQ_OK;
    bool ok = hipEventRecord(g->events[0], origin) == hipSuccess;
    for (int b = 0; ok && b < nb; ++b) ok = hipStreamWaitEvent(g->streams[1 + b], g->events[0], 0) == hipSuccess;
    if (!ok) st = DQ_EDEVICE;
    for (uint64_t i : order) {
        if (st != DQ_OK) break;
        const dq_batch_field& f = fields[i];
        void* s = g->streams[1 + branch_of[i]];
        st = dq_compress(&f.p, f.x, f.codes, f.out_idx, f.out_val, f.out_cap, f.pads, f.cres, f.cws, f.cws_bytes, s,
                         nullptr);
        if (st == DQ_OK && f.x_hat)
            st = dq_decompress_dev(&f.p, f.cres, f.out_cap, f.codes, f.out_idx, f.out_val, f.pads, f.x_hat, f.dres,
                                   f.dws, f.dws_bytes, s, nullptr);
    }
    for (int b = 0; st == DQ_OK && b < nb; ++b) {
        if (hipEventRecord(g->events[1 + b], g->streams[1 + b]) != hipSuccess ||
            hipStreamWaitEvent(origin, g->events[1 + b], 0) != hipSuccess)
            st = DQ_EDEVICE;
    }
    hipGraph_t captured = nullptr;
    const bool ended = hipStreamEndCapture(origin, &captured) == hipSuccess;
    g->graph = captured;
    if (st == DQ_OK && !ended) st = DQ_EDEVICE;
    if (st == DQ_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) st = DQ_EDEVICE;
    if (st != DQ_OK) {
        (void)hipGetLastError();
        release(g);
        return st;
    }
    *graph = g;
    return DQ_OK;
}

dq_status dq_batch_graph_launch(dq_batch_graph* graph, void* hip_stream) {
    if (!graph || !graph->exec) return DQ_EINVAL;
    return hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(hip_stream)) == hipSuccess ? DQ_OK
                                                                                                  : DQ_EDEVICE;
}

dq_status dq_batch_graph_destroy(dq_batch_graph* graph) {
    if (!graph) return DQ_EINVAL;
    release(graph);
    return DQ_OK;
}

}  // extern "C"
