// A batch of searches as one captured HIP graph.
//
// Every request of the batch that fits the asynchronous search (one class
// batch, nothing read back: search_async) is queued, during a stream capture,
// on one of `slots` streams, each with a context of its own; the streams fork
// from the caller's stream and join back to it, so the whole batch is one
// graph, launched with one call and replayed as long as the requests stay the
// same (same buffers, sizes and options).  Requests are placed on the slots
// by the greedy arg-min of the load-balancing algorithm (Alg. 3: largest
// first, to the slot with the fewest pairs so far), and each slot's
// workspaces are sized for its largest request before the capture, so
// nothing is allocated inside it.
#include "asci_internal.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>

namespace asci {

GraphBatch::~GraphBatch()
{
    release_graph();
    if (main) (void)hipStreamDestroy(main);
    if (order) (void)hipEventDestroy(order);
    for (auto s : streams)
        if (s) (void)hipStreamDestroy(s);
    for (auto e : events)
        if (e) (void)hipEventDestroy(e);
    if (d_res) (void)hipFree(d_res);
}

void GraphBatch::release_graph()
{
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
}

namespace {

// the request fields a captured graph depends on
void fingerprint(const asci_request &r, std::vector<uint64_t> &key)
{
    const uint64_t w[] = {(uint64_t)(uintptr_t)r.h, (uint64_t)(uintptr_t)r.eri, (uint64_t)r.norb,
                          (uint64_t)r.nalpha, (uint64_t)r.nbeta, (uint64_t)(uintptr_t)r.dets,
                          (uint64_t)(uintptr_t)r.coeffs, (uint64_t)r.ndets, 0, (uint64_t)r.k,
                          (uint64_t)(uintptr_t)r.out_dets, (uint64_t)(uintptr_t)r.out_scores};
    key.insert(key.end(), w, w + sizeof(w) / sizeof(w[0]));
    uint64_t e;
    std::memcpy(&e, &r.E0, 8);
    key[key.size() - 4] = e;
    uint64_t ob[(sizeof(asci_options) + 7) / 8] = {0};
    std::memcpy(ob, &r.opt, sizeof(asci_options));
    key.insert(key.end(), ob, ob + sizeof(ob) / sizeof(ob[0]));
}

SearchArgs args_of(const asci_request &r)
{
    return SearchArgs{r.h, r.eri, r.norb, r.nalpha, r.nbeta, r.dets, r.coeffs, r.ndets, r.E0, resolve(&r.opt)};
}

}  // namespace

size_t graph_request_bytes(const asci_request &r, int finish_cap, bool spin_tables)
{
    return search_async_bytes(args_of(r), r.k, finish_cap, spin_tables);
}

void graph_batch_launch(GraphBatch &gb, int device, const asci_request *reqs, const std::vector<int> &idx, int slots,
                        int finish_cap, int spin_tables, hipStream_t stream)
{
    slots = std::max(1, std::min(slots, (int)std::max<size_t>(idx.size(), 1)));
    std::vector<uint64_t> key{(uint64_t)slots, (uint64_t)finish_cap, (uint64_t)spin_tables};
    for (int i : idx) fingerprint(reqs[i], key);
    ASCI_HIP(hipSetDevice(device));
    gb.device = device;
    // the graph is captured on and launched from a stream of its own (the
    // caller's may be the null stream, which cannot be captured), ordered after
    // the work queued on the caller's stream, which in turn waits for the graph
    if (!gb.main) ASCI_HIP(hipStreamCreateWithFlags(&gb.main, hipStreamNonBlocking));
    if (!gb.order) ASCI_HIP(hipEventCreateWithFlags(&gb.order, hipEventDisableTiming));
    ASCI_HIP(hipEventRecord(gb.order, stream));
    ASCI_HIP(hipStreamWaitEvent(gb.main, gb.order, 0));
    auto done = [&]() {
        ASCI_HIP(hipEventRecord(gb.order, gb.main));
        ASCI_HIP(hipStreamWaitEvent(stream, gb.order, 0));
    };
    if (gb.exec && key == gb.key) {
        ASCI_HIP(hipGraphLaunch(gb.exec, gb.main));
        done();
        return;
    }
    gb.release_graph();
    // slots: a context and a stream each, plus fork / join events
    while ((int)gb.ctxs.size() < slots) {
        auto c = std::make_unique<asci_ctx>();
        c->device = device;
        gb.ctxs.push_back(std::move(c));
        hipStream_t s = nullptr;
        ASCI_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        gb.streams.push_back(s);
    }
    while (gb.events.size() < (size_t)slots + 1) {
        hipEvent_t e = nullptr;
        ASCI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        gb.events.push_back(e);
    }
    if (gb.nres < idx.size()) {
        if (gb.d_res) (void)hipFree(gb.d_res);
        gb.d_res = nullptr;
        gb.nres = 0;
        ASCI_HIP(hipMalloc((void **)&gb.d_res, std::max<size_t>(idx.size(), 1) * sizeof(asci_async_result)));
        gb.nres = idx.size();
    }
    // placement: largest first, each to the slot with the fewest pairs so far
    std::vector<int> order(idx.size());
    for (size_t j = 0; j < idx.size(); ++j) order[j] = (int)j;
    std::vector<uint64_t> pairs(idx.size());
    for (size_t j = 0; j < idx.size(); ++j) pairs[j] = search_pairs(args_of(reqs[idx[j]]));
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pairs[a] > pairs[b]; });
    std::vector<std::vector<int>> plan((size_t)slots);
    std::vector<uint64_t> load((size_t)slots, 0);
    for (int j : order) {
        size_t q = 0;
        for (size_t p = 1; p < (size_t)slots; ++p)
            if (load[p] < load[q]) q = p;
        plan[q].push_back(j);
        load[q] += pairs[j];
    }
    // workspaces sized before the capture (nothing is allocated inside it)
    for (int q = 0; q < slots; ++q) {
        asci_ctx *c = gb.ctxs[(size_t)q].get();
        c->finish_cap = finish_cap;
        c->spin_tables = spin_tables;
        for (int j : plan[(size_t)q]) {
            const asci_request &r = reqs[idx[(size_t)j]];
            search_async(c, args_of(r), r.k, r.out_dets, r.out_scores, gb.d_res + j, gb.streams[(size_t)q], true);
        }
    }
    hipStream_t cs = gb.main;
    ASCI_HIP(hipStreamSynchronize(cs));
    ASCI_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    try {
        ASCI_HIP(hipEventRecord(gb.events[0], cs));
        for (int q = 0; q < slots; ++q) {
            hipStream_t s = gb.streams[(size_t)q];
            ASCI_HIP(hipStreamWaitEvent(s, gb.events[0], 0));
            asci_ctx *c = gb.ctxs[(size_t)q].get();
            for (int j : plan[(size_t)q]) {
                const asci_request &r = reqs[idx[(size_t)j]];
                search_async(c, args_of(r), r.k, r.out_dets, r.out_scores, gb.d_res + j, s, false);
            }
            ASCI_HIP(hipEventRecord(gb.events[(size_t)q + 1], s));
            ASCI_HIP(hipStreamWaitEvent(cs, gb.events[(size_t)q + 1], 0));
        }
        ASCI_HIP(hipStreamEndCapture(cs, &gb.graph));
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        throw;
    }
    ASCI_HIP(hipGraphInstantiate(&gb.exec, gb.graph, nullptr, nullptr, 0));
    gb.key = key;
    ASCI_HIP(hipGraphLaunch(gb.exec, cs));
    done();
}

void graph_batch_results(GraphBatch &gb, size_t count, std::vector<asci_async_result> &out)
{
    out.resize(count);
    if (count) ASCI_HIP(hipMemcpy(out.data(), gb.d_res, count * sizeof(asci_async_result), hipMemcpyDeviceToHost));
}

}  // namespace asci
