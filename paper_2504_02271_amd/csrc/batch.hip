// Many independent hypergraphs counted in one persistent launch.
//
// Every graph is normalised and its hyperwedges built separately; the
// closure work items of all graphs go into one queue (each item names its
// graph) and one launch of the closure kernel drains it, flushing its lane
// counters into the graph's counts whenever it moves to another graph.  The
// launch (counter reset + kernel) is captured once in a HIP graph per
// schedule and replayed.  The schedule (LDS chunk size, partners per item,
// item order) is chosen by timing the candidates.
#include <algorithm>
#include <memory>
#include <numeric>

#include "internal.hpp"

namespace htri {
namespace {

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_copy_items(const Item *src, int64_t n, Item *dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

struct Plan {
    htri_schedule sched{};
    DBuf<Item> items, witems;            // block items, single-owner items
    int64_t nitems = 0, nwitems = 0;
    int nblocks = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

}  // namespace
}  // namespace htri

struct htri_batch {
    htri::Allocator al;
    hipStream_t stream = nullptr;        // created by the batch (graph capture needs a real stream)
    std::vector<std::unique_ptr<htri::Graph>> graphs;
    htri::DBuf<htri::GraphDesc> descs;
    htri::DBuf<uint8_t> lut;
    htri::DBuf<unsigned long long> ctr;  // [0] queue, [1] probes, [2..] counts[g][21], then the wave queue
    std::vector<std::unique_ptr<htri::Plan>> plans;
    std::string err;
    ~htri_batch() {
        plans.clear();
        graphs.clear();
        descs.reset();
        lut.reset();
        ctr.reset();
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace htri {
namespace {

bool same_sched(const htri_schedule &a, const htri_schedule &b) {
    return a.chunk == b.chunk && a.partners == b.partners && a.order == b.order;
}

Plan &plan_for(htri_batch &B, const htri_schedule &sc) {
    for (auto &p : B.plans)
        if (same_sched(p->sched, sc)) return *p;
    CloseConfig cfg;
    cfg.cap = sc.chunk;
    cfg.jp = sc.partners;
    if (!valid_config(cfg) || (sc.order != 0 && sc.order != 1))
        fail(HTRI_E_INVALID, "schedule: chunk 256|512, partners 128|256, order 0|1");
    auto plan = std::make_unique<Plan>();
    plan->sched = sc;
    const int n = (int)B.graphs.size();
    // graph order in the queue; the queue is drained from its end, so order 1
    // puts the graphs with the most hyperwedges last (they start first)
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    if (sc.order == 1)
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int b) { return B.graphs[a]->nw < B.graphs[b]->nw; });
    std::vector<ItemLists> parts(n);
    int64_t total = 0, wtotal = 0;
    for (int q = 0; q < n; q++) {
        const int gi = ord[q];
        build_items(*B.graphs[gi], gi, cfg, parts[q], B.graphs[gi]->m);
        total += parts[q].nblock;
        wtotal += parts[q].nwave;
    }
    plan->items.alloc(B.al, total);
    plan->witems.alloc(B.al, wtotal);
    int64_t off = 0, woff = 0;
    for (int q = 0; q < n; q++) {
        if (parts[q].nblock) {
            hipLaunchKernelGGL(k_copy_items, dim3(grid_for(parts[q].nblock, 256, 4096)), dim3(256), 0, B.stream,
                               parts[q].block.p, parts[q].nblock, plan->items.p + off);
            HTRI_LAUNCH_CHECK();
        }
        if (parts[q].nwave) {
            hipLaunchKernelGGL(k_copy_items, dim3(grid_for(parts[q].nwave, 256, 4096)), dim3(256), 0, B.stream,
                               parts[q].wave.p, parts[q].nwave, plan->witems.p + woff);
            HTRI_LAUNCH_CHECK();
        }
        off += parts[q].nblock;
        woff += parts[q].nwave;
    }
    HTRI_HIP(hipStreamSynchronize(B.stream));
    plan->nitems = total;
    plan->nwitems = wtotal;
    plan->nblocks = device_cu_count() * close_blocks_per_cu(cfg, false, false);
    if ((int64_t)plan->nblocks > total + wtotal) plan->nblocks = (int)std::max<int64_t>(total + wtotal, 1);
    B.plans.push_back(std::move(plan));
    return *B.plans.back();
}

CloseArgs batch_args(htri_batch &B, const Plan &P) {
    CloseArgs a{};
    a.items = P.items.p;
    a.nitems = P.nitems;
    a.queue = (unsigned int *)B.ctr.p;
    a.witems = P.witems.p;
    a.nwitems = P.nwitems;
    a.wqueue = (unsigned int *)(B.ctr.p + 2 + 21 * (int64_t)B.graphs.size());
    a.graphs = B.descs.p;
    a.emask = 0x1FFFFEu;
    a.lut = B.lut.p;
    a.counts = B.ctr.p + 2;
    a.probes = B.ctr.p + 1;
    return a;
}

void enqueue_batch(htri_batch &B, const Plan &P) {
    const int64_t nctr = 3 + 21 * (int64_t)B.graphs.size();
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(nctr, 256, 1024)), dim3(256), 0, B.stream, B.ctr.p, nctr);
    HTRI_LAUNCH_CHECK();
    CloseConfig cfg;
    cfg.cap = P.sched.chunk;
    cfg.jp = P.sched.partners;
    launch_close_kernel(cfg, false, false, batch_args(B, P), P.nblocks, B.stream);
}

double run_plan(htri_batch &B, Plan &P, bool use_graph) {
    hipEvent_t e0, e1;
    HTRI_HIP(hipEventCreate(&e0));
    HTRI_HIP(hipEventCreate(&e1));
    if (use_graph && !P.exec) {
        HTRI_HIP(hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_batch(B, P);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(B.stream, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            throw;
        }
        HTRI_HIP(hipStreamEndCapture(B.stream, &P.graph));
        HTRI_HIP(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
    }
    HTRI_HIP(hipEventRecord(e0, B.stream));
    if (use_graph) HTRI_HIP(hipGraphLaunch(P.exec, B.stream));
    else enqueue_batch(B, P);
    HTRI_HIP(hipEventRecord(e1, B.stream));
    HTRI_HIP(hipEventSynchronize(e1));
    float ms = 0;
    HTRI_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

void read_counts(htri_batch &B, int64_t *counts) {
    const int n = (int)B.graphs.size();
    std::vector<unsigned long long> h(2 + 21 * (size_t)n);
    HTRI_HIP(hipMemcpyAsync(h.data(), B.ctr.p, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, B.stream));
    HTRI_HIP(hipStreamSynchronize(B.stream));
    for (int g = 0; g < n; g++) {
        int64_t tot = 0;
        for (int p = 1; p <= 20; p++) {
            counts[g * 21 + p] = (int64_t)h[2 + 21 * g + p];
            tot += counts[g * 21 + p];
        }
        counts[g * 21] = tot;
    }
}

template <typename F>
htri_status run_b(htri_batch *b, F &&fn) {
    try {
        fn();
        return HTRI_OK;
    } catch (const htri::Error &e) {
        if (b) b->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        return HTRI_E_OOM;
    }
}

}  // namespace
}  // namespace htri

using namespace htri;

extern "C" {

htri_status htri_batch_load(int32_t count, const int64_t *const *edge_offsets, const int64_t *num_edges,
                            const int32_t *const *members, const int32_t *num_vertices, uint32_t flags,
                            htri_batch **out) {
    if (!out || count < 0 || (count > 0 && (!edge_offsets || !num_edges || !members || !num_vertices)))
        return HTRI_E_INVALID;
    if (flags & ~HTRI_DEDUPE_EDGES) return HTRI_E_INVALID;
    *out = nullptr;
    htri_batch *B = new (std::nothrow) htri_batch();
    if (!B) return HTRI_E_OOM;
    htri_status st = run_b(B, [&] {
        HTRI_HIP(hipStreamCreate(&B->stream));
        B->al.stream = B->stream;
        for (int32_t g = 0; g < count; g++) {
            auto G = std::make_unique<Graph>();
            G->stream = B->stream;
            G->al.stream = B->stream;
            try {
                graph_load(*G, edge_offsets[g], num_edges[g], members[g], num_vertices[g], flags);
                build_wedges(*G);
            } catch (const Error &e) {
                throw Error{e.code, "graph " + std::to_string(g) + ": " + e.msg};
            }
            B->graphs.push_back(std::move(G));
        }
        std::vector<GraphDesc> d;
        for (auto &G : B->graphs) d.push_back(graph_desc(*G));
        B->descs.alloc(B->al, std::max<size_t>(d.size(), 1));
        if (!d.empty())
            HTRI_HIP(hipMemcpyAsync(B->descs.p, d.data(), sizeof(GraphDesc) * d.size(), hipMemcpyHostToDevice, B->stream));
        B->lut.alloc(B->al, 128);
        HTRI_HIP(hipMemcpyAsync(B->lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, B->stream));
        B->ctr.alloc(B->al, 3 + 21 * (size_t)count);
        HTRI_HIP(hipStreamSynchronize(B->stream));
    });
    if (st != HTRI_OK) {
        set_load_error(B->err);
        delete B;
        return st;
    }
    *out = B;
    return HTRI_OK;
}

htri_status htri_batch_info(const htri_batch *b, int64_t *wedges_per_graph) {
    if (!b || (!wedges_per_graph && !b->graphs.empty())) return HTRI_E_INVALID;
    for (size_t g = 0; g < b->graphs.size(); g++) wedges_per_graph[g] = b->graphs[g]->nw;
    return HTRI_OK;
}

htri_status htri_batch_count(htri_batch *b, const htri_schedule *sched, int32_t use_graph, int64_t *counts,
                             double *time_ms) {
    if (!b || !sched || !counts) return HTRI_E_INVALID;
    return run_b(b, [&] {
        Plan &P = plan_for(*b, *sched);
        const double ms = run_plan(*b, P, use_graph != 0);
        read_counts(*b, counts);
        if (time_ms) *time_ms = ms;
    });
}

htri_status htri_batch_autotune(htri_batch *b, int32_t repeats, htri_schedule *best, double *best_ms) {
    if (!b || !best) return HTRI_E_INVALID;
    return run_b(b, [&] {
        const int chunks[2] = {256, 512}, partners[2] = {128, 256};
        double bms = 1e300;
        htri_schedule bs{512, 256, 0};
        for (int c : chunks)
            for (int p : partners)
                for (int o = 0; o < 2; o++) {
                    htri_schedule sc{c, p, o};
                    Plan &P = plan_for(*b, sc);
                    (void)run_plan(*b, P, true);  // warm-up (and capture)
                    double t = 1e300;
                    for (int r = 0; r < std::max(1, (int)repeats); r++) t = std::min(t, run_plan(*b, P, true));
                    if (t < bms) {
                        bms = t;
                        bs = sc;
                    }
                }
        *best = bs;
        if (best_ms) *best_ms = bms;
    });
}

htri_status htri_batch_count_per_graph(htri_batch *b, const htri_schedule *sched, int64_t *counts, double *time_ms) {
    if (!b || !sched || !counts) return HTRI_E_INVALID;
    return run_b(b, [&] {
        CloseConfig cfg;
        cfg.cap = sched->chunk;
        cfg.jp = sched->partners;
        if (!valid_config(cfg)) fail(HTRI_E_INVALID, "schedule: chunk 256|512, partners 128|256");
        const int n = (int)b->graphs.size();
        // items of each graph (graph index 0 in its own one-graph launch)
        std::vector<ItemLists> items(n);
        std::vector<DBuf<GraphDesc>> desc(n);
        for (int g = 0; g < n; g++) {
            build_items(*b->graphs[g], 0, cfg, items[g], b->graphs[g]->m);
            desc[g].alloc(b->al, 1);
            GraphDesc d = graph_desc(*b->graphs[g]);
            HTRI_HIP(hipMemcpyAsync(desc[g].p, &d, sizeof(d), hipMemcpyHostToDevice, b->stream));
        }
        DBuf<unsigned long long> ctr(b->al, (size_t)n * 24);   // per graph: queue, probes, counts[21], wave queue
        HTRI_HIP(hipStreamSynchronize(b->stream));
        const int per_cu = close_blocks_per_cu(cfg, false, false);
        hipEvent_t e0, e1;
        HTRI_HIP(hipEventCreate(&e0));
        HTRI_HIP(hipEventCreate(&e1));
        HTRI_HIP(hipEventRecord(e0, b->stream));
        for (int g = 0; g < n; g++) {
            unsigned long long *c = ctr.p + 24 * (int64_t)g;
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, b->stream, c, (int64_t)24);
            HTRI_LAUNCH_CHECK();
            CloseArgs a{};
            a.items = items[g].block.p;
            a.nitems = items[g].nblock;
            a.queue = (unsigned int *)c;
            a.witems = items[g].wave.p;
            a.nwitems = items[g].nwave;
            a.wqueue = (unsigned int *)(c + 23);
            a.graphs = desc[g].p;
            a.emask = 0x1FFFFEu;
            a.lut = b->lut.p;
            a.counts = c + 2;
            a.probes = c + 1;
            int nb = device_cu_count() * per_cu;
            const int64_t ni = items[g].nblock + items[g].nwave;
            if ((int64_t)nb > ni) nb = (int)std::max<int64_t>(ni, 1);
            launch_close_kernel(cfg, false, false, a, nb, b->stream);
        }
        HTRI_HIP(hipEventRecord(e1, b->stream));
        HTRI_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HTRI_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::vector<unsigned long long> h((size_t)n * 24);
        HTRI_HIP(hipMemcpy(h.data(), ctr.p, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
        for (int g = 0; g < n; g++) {
            int64_t tot = 0;
            for (int p = 1; p <= 20; p++) {
                counts[g * 21 + p] = (int64_t)h[24 * (size_t)g + 2 + p];
                tot += counts[g * 21 + p];
            }
            counts[g * 21] = tot;
        }
        if (time_ms) *time_ms = ms;
    });
}

const char *htri_batch_last_error(const htri_batch *b) { return b ? b->err.c_str() : ""; }

void htri_batch_free(htri_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
}

}  // extern "C"
