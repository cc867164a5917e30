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
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <numeric>
#include <string>

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

// The closure of a set of graphs (members) under one schedule: their work
// items in one queue, drained by one persistent launch.
struct Plan {
    htri_schedule sched{};
    std::vector<int> members;            // graph indices, ascending
    DBuf<Item> items, witems;            // block items, single-owner items
    DBuf<unsigned long long> q;          // [0] block queue, [1] wave queue
    int64_t nitems = 0, nwitems = 0;
    int nblocks = 1;
};

// Plans replayed together: the counters cleared once, then each plan's
// launch, captured as one HIP graph.
struct Group {
    std::vector<Plan *> plans;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Group() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Size classes of the per-class schedules: by hyperwedges per graph.
constexpr int kSizeClasses = 3;
constexpr int64_t kClassMaxWedges[kSizeClasses - 1] = {(int64_t)1 << 18, (int64_t)1 << 21};
int size_class(int64_t nw) {
    int c = 0;
    while (c < kSizeClasses - 1 && nw >= kClassMaxWedges[c]) c++;
    return c;
}

// Step 1, the work items and the closure of every graph, captured once
// into one HIP graph: a record pass runs the per-graph host code eagerly
// (keeping its readbacks and sizing its allocations), then the same code is
// captured with every buffer taken from one arena that the plan owns.  A
// replay rebuilds every graph's hyperwedges from its loaded hypergraph and
// counts them; the graph's own descriptors and counters live in the arena
// too, so the plan is independent of the batch's other plans.
constexpr int kSideStreams = 8;
struct FullPlan {
    htri_schedule sched{};
    Replay rec;
    Allocator arena_al;                  // the arena's own allocator (it knows no arena)
    DBuf<char> arena;
    unsigned long long *ctr = nullptr;   // [0] queue, [1] probes, [2..] counts[g][21], then the wave queue
    int64_t nitems = 0, nwitems = 0;
    int nblocks = 1;
    // the graphs' step 1 runs on kSideStreams streams forked from the batch's
    // stream (default priority), so the captured graph has that many
    // independent branches
    std::vector<hipStream_t> side;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~FullPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipStream_t s : side) (void)hipStreamDestroy(s);
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
    std::vector<std::unique_ptr<htri::Group>> groups;
    std::vector<std::unique_ptr<htri::FullPlan>> full_plans;
    std::string err;
    ~htri_batch() {
        groups.clear();
        plans.clear();
        graphs.clear();      // the graphs' arena buffers are released as no-ops ...
        full_plans.clear();  // ... before the arenas themselves
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

std::vector<int> all_members(const htri_batch &B) {
    std::vector<int> m(B.graphs.size());
    std::iota(m.begin(), m.end(), 0);
    return m;
}

Plan &plan_for(htri_batch &B, const htri_schedule &sc, const std::vector<int> &members) {
    for (auto &p : B.plans)
        if (same_sched(p->sched, sc) && p->members == members) return *p;
    CloseConfig cfg;
    cfg.cap = sc.chunk;
    cfg.jp = sc.partners;
    if (!valid_config(cfg) || (sc.order != 0 && sc.order != 1))
        fail(HTRI_E_INVALID, "schedule: chunk 256|512, partners 128|256, order 0|1");
    auto plan = std::make_unique<Plan>();
    plan->sched = sc;
    plan->members = members;
    plan->q.alloc(B.al, 2);
    const int n = (int)members.size();
    // graph order in the queue; the queue is drained from its end, so order 1
    // puts the graphs with the most hyperwedges last (they start first)
    std::vector<int> ord(members);
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
    a.queue = (unsigned int *)P.q.p;
    a.witems = P.witems.p;
    a.nwitems = P.nwitems;
    a.wqueue = (unsigned int *)(P.q.p + 1);
    a.graphs = B.descs.p;
    a.emask = 0x1FFFFEu;
    a.lut = B.lut.p;
    a.counts = B.ctr.p + 2;
    a.probes = B.ctr.p + 1;
    return a;
}

void enqueue_group(htri_batch &B, const Group &G) {
    const int64_t nctr = 3 + 21 * (int64_t)B.graphs.size();
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(nctr, 256, 1024)), dim3(256), 0, B.stream, B.ctr.p, nctr);
    HTRI_LAUNCH_CHECK();
    for (const Plan *P : G.plans) {
        if (P->nitems + P->nwitems == 0) continue;
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, B.stream, P->q.p, (int64_t)2);
        HTRI_LAUNCH_CHECK();
        CloseConfig cfg;
        cfg.cap = P->sched.chunk;
        cfg.jp = P->sched.partners;
        launch_close_kernel(cfg, false, false, batch_args(B, *P), P->nblocks, B.stream);
    }
}

Group &group_for(htri_batch &B, const std::vector<Plan *> &plans) {
    for (auto &g : B.groups)
        if (g->plans == plans) return *g;
    auto g = std::make_unique<Group>();
    g->plans = plans;
    B.groups.push_back(std::move(g));
    return *B.groups.back();
}

double run_group(htri_batch &B, Group &P, bool use_graph) {
    hipEvent_t e0, e1;
    HTRI_HIP(hipEventCreate(&e0));
    HTRI_HIP(hipEventCreate(&e1));
    if (use_graph && !P.exec) {
        HTRI_HIP(hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_group(B, P);
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
    else enqueue_group(B, P);
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

// Release a graph's step-1 state (outside any capture).
void drop_step1(Graph &g) {
    g.fptr.reset();
    g.fadj.reset();
    g.mptr.reset();
    g.fmask.reset();
    g.indeg.reset();
    g.incl_pos.reset();
    g.incl_pairs.reset();
    g.n_incl_pairs = 0;
    g.have_incl = false;
    g.have_wedges = false;
}

// The per-graph host code of the full pipeline, in queue order: step 1 and
// the work items of each graph, the combined item lists, the graphs'
// descriptors, the counters, and the closure launch.
void enqueue_full(htri_batch &B, FullPlan &F, const CloseConfig &cfg, const std::vector<int> &ord) {
    hipStream_t s = B.stream;
    const int n = (int)B.graphs.size();
    std::vector<ItemLists> parts(n);
    int64_t total = 0, wtotal = 0;
    // fork: every side stream waits for the work already on the batch stream
    const int K = (int)F.side.size();
    std::vector<hipEvent_t> ev(K + 1, nullptr);
    for (auto &e : ev) HTRI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    struct EventsOut {
        std::vector<hipEvent_t> &v;
        ~EventsOut() {
            for (hipEvent_t e : v)
                if (e) (void)hipEventDestroy(e);
        }
    } events_out{ev};
    HTRI_HIP(hipEventRecord(ev[K], s));
    for (int k = 0; k < K; k++) HTRI_HIP(hipStreamWaitEvent(F.side[k], ev[K], 0));
    for (int q = 0; q < n; q++) {
        Graph &G = *B.graphs[ord[q]];
        hipStream_t gs = K > 0 ? F.side[q % K] : s;
        G.stream = gs;
        G.al.stream = gs;
        try {
            build_wedges(G);
            G.have_wedges = true;
            build_items(G, ord[q], cfg, parts[q], G.m);
        } catch (...) {
            G.stream = s;
            G.al.stream = s;
            throw;
        }
        G.stream = s;
        G.al.stream = s;
        total += parts[q].nblock;
        wtotal += parts[q].nwave;
    }
    // join
    for (int k = 0; k < K; k++) {
        HTRI_HIP(hipEventRecord(ev[k], F.side[k]));
        HTRI_HIP(hipStreamWaitEvent(s, ev[k], 0));
    }
    DBuf<Item> items(B.al, total), witems(B.al, wtotal);
    int64_t off = 0, woff = 0;
    for (int q = 0; q < n; q++) {
        if (parts[q].nblock) {
            hipLaunchKernelGGL(k_copy_items, dim3(grid_for(parts[q].nblock, 256, 4096)), dim3(256), 0, s,
                               parts[q].block.p, parts[q].nblock, items.p + off);
            HTRI_LAUNCH_CHECK();
        }
        if (parts[q].nwave) {
            hipLaunchKernelGGL(k_copy_items, dim3(grid_for(parts[q].nwave, 256, 4096)), dim3(256), 0, s,
                               parts[q].wave.p, parts[q].nwave, witems.p + woff);
            HTRI_LAUNCH_CHECK();
        }
        off += parts[q].nblock;
        woff += parts[q].nwave;
    }
    std::vector<GraphDesc> d;
    for (auto &G : B.graphs) d.push_back(graph_desc(*G));
    DBuf<GraphDesc> descs(B.al, std::max<size_t>(d.size(), 1));
    if (!d.empty())
        HTRI_HIP(hipMemcpyAsync(descs.p, persist_host(d.data(), sizeof(GraphDesc) * d.size()),
                                sizeof(GraphDesc) * d.size(), hipMemcpyHostToDevice, s));
    DBuf<unsigned long long> ctr(B.al, 3 + 21 * (size_t)n);
    const int64_t nctr = 3 + 21 * (int64_t)n;
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(nctr, 256, 1024)), dim3(256), 0, s, ctr.p, nctr);
    HTRI_LAUNCH_CHECK();
    F.nitems = total;
    F.nwitems = wtotal;
    F.nblocks = device_cu_count() * close_blocks_per_cu(cfg, false, false);
    if ((int64_t)F.nblocks > total + wtotal) F.nblocks = (int)std::max<int64_t>(total + wtotal, 1);
    CloseArgs a{};
    a.items = items.p;
    a.nitems = total;
    a.queue = (unsigned int *)ctr.p;
    a.witems = witems.p;
    a.nwitems = wtotal;
    a.wqueue = (unsigned int *)(ctr.p + 2 + 21 * (int64_t)n);
    a.graphs = descs.p;
    a.emask = 0x1FFFFEu;
    a.lut = B.lut.p;
    a.counts = ctr.p + 2;
    a.probes = ctr.p + 1;
    if (total + wtotal > 0) launch_close_kernel(cfg, false, false, a, F.nblocks, s);
    F.ctr = replay_capturing() ? ctr.p : nullptr;
}

FullPlan &full_plan_for(htri_batch &B, const htri_schedule &sc) {
    for (auto &p : B.full_plans)
        if (same_sched(p->sched, sc)) return *p;
    CloseConfig cfg;
    cfg.cap = sc.chunk;
    cfg.jp = sc.partners;
    if (!valid_config(cfg) || (sc.order != 0 && sc.order != 1))
        fail(HTRI_E_INVALID, "schedule: chunk 256|512, partners 128|256, order 0|1");
    const int n = (int)B.graphs.size();
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    if (sc.order == 1)
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return B.graphs[a]->nw < B.graphs[b]->nw; });
    auto F = std::make_unique<FullPlan>();
    F->sched = sc;
    for (int k = 0; k < kSideStreams && k < n; k++) {
        hipStream_t t = nullptr;
        HTRI_HIP(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
        F->side.push_back(t);
    }
    struct Scope {   // the thread's replay, cleared on every exit
        Scope(Replay *r) { tl_replay = r; }
        ~Scope() { tl_replay = nullptr; }
    };
    // record: eager, real allocations
    for (auto &G : B.graphs) drop_step1(*G);
    {
        Scope sc_rec(&F->rec);
        F->rec.mode = Replay::kRecord;
        enqueue_full(B, *F, cfg, ord);
        HTRI_HIP(hipStreamSynchronize(B.stream));
    }
    // capture: the same host code, buffers from the arena
    const size_t arena_bytes = F->rec.arena_bytes + ((size_t)1 << 20);
    F->arena_al.stream = B.stream;
    F->arena.alloc(F->arena_al, arena_bytes);
    const std::pair<const char *, const char *> range(F->arena.p, F->arena.p + arena_bytes);
    B.al.arenas.push_back(range);
    for (auto &G : B.graphs) {
        G->al.arenas.push_back(range);
        drop_step1(*G);
    }
    F->rec.mode = Replay::kCapture;
    F->rec.next = 0;
    F->rec.arena = F->arena.p;
    F->rec.arena_size = arena_bytes;
    F->rec.arena_off = 0;
    {
        Scope sc_cap(&F->rec);
        HTRI_HIP(hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_full(B, *F, cfg, ord);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(B.stream, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            throw;
        }
        HTRI_HIP(hipStreamEndCapture(B.stream, &F->graph));
    }
    if (F->rec.next != F->rec.vals.size()) fail(HTRI_E_STATE, "the captured pass read fewer values than recorded");
    HTRI_HIP(hipGraphInstantiate(&F->exec, F->graph, nullptr, nullptr, 0));
    // one replay fills every graph's step-1 state (the graphs now point into the arena)
    HTRI_HIP(hipGraphLaunch(F->exec, B.stream));
    HTRI_HIP(hipStreamSynchronize(B.stream));
    B.full_plans.push_back(std::move(F));
    // the batch's own descriptors follow the graphs' new buffers
    std::vector<GraphDesc> d;
    for (auto &G : B.graphs) d.push_back(graph_desc(*G));
    if (!d.empty())
        HTRI_HIP(hipMemcpyAsync(B.descs.p, d.data(), sizeof(GraphDesc) * d.size(), hipMemcpyHostToDevice, B.stream));
    HTRI_HIP(hipStreamSynchronize(B.stream));
    return *B.full_plans.back();
}

void read_counts_from(htri_batch &B, const unsigned long long *ctr, int64_t *counts) {
    const int n = (int)B.graphs.size();
    std::vector<unsigned long long> h(2 + 21 * (size_t)n);
    HTRI_HIP(hipMemcpyAsync(h.data(), ctr, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, B.stream));
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

std::vector<int> class_members(const htri_batch &B, int c) {
    std::vector<int> m;
    for (size_t g = 0; g < B.graphs.size(); g++)
        if (size_class(B.graphs[g]->nw) == c) m.push_back((int)g);
    return m;
}

std::string device_arch(int &cus) {
    int dev = 0;
    HTRI_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HTRI_HIP(hipGetDeviceProperties(&prop, dev));
    cus = prop.multiProcessorCount;
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// The schedule cache, a JSON file written by this library:
//   {"format": "htri-batch-schedules", "version": 1, "arch": "gfx950", "cus": 256,
//    "classes": [
//     {"class": 0, "max_wedges": 262144, "chunk": 512, "partners": 256, "order": 1, "ms": 1.5},
//     ...]}
// one class object per line.  A cache for another architecture or compute
// unit count is ignored.
bool json_int(const std::string &t, const std::string &key, size_t from, size_t to, long long &v) {
    const std::string k = "\"" + key + "\":";
    const size_t at = t.find(k, from);
    if (at == std::string::npos || at >= to) return false;
    size_t i = at + k.size();
    while (i < t.size() && t[i] == ' ') i++;
    char *end = nullptr;
    v = std::strtoll(t.c_str() + i, &end, 10);
    return end != t.c_str() + i;
}

bool read_schedule_cache(const char *path, const std::string &arch, int cus, htri_schedule out[kSizeClasses],
                         bool have[kSizeClasses]) {
    for (int c = 0; c < kSizeClasses; c++) have[c] = false;
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    std::string t;
    char buf[1024];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0 && t.size() < (1 << 20)) t.append(buf, got);
    std::fclose(f);
    if (t.find("\"htri-batch-schedules\"") == std::string::npos) return false;
    if (t.find("\"arch\": \"" + arch + "\"") == std::string::npos) return false;
    long long c0 = 0;
    if (!json_int(t, "cus", 0, t.size(), c0) || c0 != cus) return false;
    size_t at = 0;
    while ((at = t.find("{\"class\":", at)) != std::string::npos) {
        const size_t end = t.find('}', at);
        if (end == std::string::npos) break;
        long long c, ch, pa, od;
        if (json_int(t, "class", at, end, c) && json_int(t, "chunk", at, end, ch) &&
            json_int(t, "partners", at, end, pa) && json_int(t, "order", at, end, od) && c >= 0 &&
            c < kSizeClasses) {
            CloseConfig cfg;
            cfg.cap = (int)ch;
            cfg.jp = (int)pa;
            if (valid_config(cfg) && (od == 0 || od == 1)) {
                out[c] = htri_schedule{(int32_t)ch, (int32_t)pa, (int32_t)od};
                have[c] = true;
            }
        }
        at = end;
    }
    return true;
}

void write_schedule_cache(const char *path, const std::string &arch, int cus, const htri_schedule s[kSizeClasses],
                          const double ms[kSizeClasses]) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) fail(HTRI_E_INVALID, "cannot write the schedule cache " + tmp);
    std::fprintf(f, "{\"format\": \"htri-batch-schedules\", \"version\": 1, \"arch\": \"%s\", \"cus\": %d,\n",
                 arch.c_str(), cus);
    std::fprintf(f, " \"classes\": [\n");
    for (int c = 0; c < kSizeClasses; c++) {
        const long long mx = c < kSizeClasses - 1 ? (long long)kClassMaxWedges[c] : -1;
        std::fprintf(f, "  {\"class\": %d, \"max_wedges\": %lld, \"chunk\": %d, \"partners\": %d, \"order\": %d, "
                        "\"ms\": %.4f}%s\n",
                     c, mx, s[c].chunk, s[c].partners, s[c].order, ms[c], c + 1 < kSizeClasses ? "," : "");
    }
    std::fprintf(f, " ]}\n");
    if (std::fclose(f) != 0) fail(HTRI_E_INVALID, "cannot write the schedule cache " + tmp);
    if (std::rename(tmp.c_str(), path) != 0) fail(HTRI_E_INVALID, std::string("cannot replace ") + path);
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
        Plan &P = plan_for(*b, *sched, all_members(*b));
        const double ms = run_group(*b, group_for(*b, {&P}), use_graph != 0);
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
                    Group &G = group_for(*b, {&plan_for(*b, sc, all_members(*b))});
                    (void)run_group(*b, G, true);  // warm-up (and capture)
                    double t = 1e300;
                    for (int r = 0; r < std::max(1, (int)repeats); r++) t = std::min(t, run_group(*b, G, true));
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

htri_status htri_batch_autotune_classes(htri_batch *b, int32_t repeats, const char *cache_path, htri_schedule *best,
                                        double *best_ms, int32_t *from_cache) {
    if (!b || !best) return HTRI_E_INVALID;
    return run_b(b, [&] {
        int cus = 0;
        const std::string arch = device_arch(cus);
        htri_schedule sc[kSizeClasses];
        double ms[kSizeClasses];
        bool have[kSizeClasses];
        std::vector<int> mem[kSizeClasses];
        for (int c = 0; c < kSizeClasses; c++) {
            mem[c] = class_members(*b, c);
            sc[c] = htri_schedule{512, 256, 1};
            ms[c] = 0.0;
        }
        bool hit = false;
        if (cache_path && read_schedule_cache(cache_path, arch, cus, sc, have)) {
            hit = true;
            for (int c = 0; c < kSizeClasses; c++)
                if (!mem[c].empty() && !have[c]) hit = false;
        }
        if (!hit) {
            const int chunks[2] = {256, 512}, partners[2] = {128, 256};
            for (int c = 0; c < kSizeClasses; c++) {
                if (mem[c].empty()) continue;
                double bms = 1e300;
                for (int ch : chunks)
                    for (int pa : partners)
                        for (int o = 0; o < 2; o++) {
                            const htri_schedule cand{ch, pa, o};
                            Group &G = group_for(*b, {&plan_for(*b, cand, mem[c])});
                            (void)run_group(*b, G, true);
                            double t = 1e300;
                            for (int r = 0; r < std::max(1, (int)repeats); r++) t = std::min(t, run_group(*b, G, true));
                            if (t < bms) {
                                bms = t;
                                sc[c] = cand;
                            }
                        }
                ms[c] = bms;
            }
            if (cache_path) write_schedule_cache(cache_path, arch, cus, sc, ms);
        }
        for (int c = 0; c < kSizeClasses; c++) {
            best[c] = sc[c];
            if (best_ms) best_ms[c] = ms[c];
        }
        if (from_cache) *from_cache = hit ? 1 : 0;
    });
}

htri_status htri_batch_count_classes(htri_batch *b, const htri_schedule *sched, int32_t use_graph, int64_t *counts,
                                     double *time_ms) {
    if (!b || !sched || !counts) return HTRI_E_INVALID;
    return run_b(b, [&] {
        std::vector<Plan *> plans;
        for (int c = 0; c < kSizeClasses; c++) {
            const std::vector<int> m = class_members(*b, c);
            if (!m.empty()) plans.push_back(&plan_for(*b, sched[c], m));
        }
        const double ms = run_group(*b, group_for(*b, plans), use_graph != 0);
        read_counts(*b, counts);
        if (time_ms) *time_ms = ms;
    });
}

htri_status htri_batch_size_classes(const htri_batch *b, int32_t *class_of_graph) {
    if (!b || (!class_of_graph && !b->graphs.empty())) return HTRI_E_INVALID;
    for (size_t g = 0; g < b->graphs.size(); g++) class_of_graph[g] = size_class(b->graphs[g]->nw);
    return HTRI_OK;
}

htri_status htri_batch_count_full(htri_batch *b, const htri_schedule *sched, int64_t *counts, double *time_ms) {
    if (!b || !sched || !counts) return HTRI_E_INVALID;
    return run_b(b, [&] {
        FullPlan &F = full_plan_for(*b, *sched);
        hipEvent_t e0, e1;
        HTRI_HIP(hipEventCreate(&e0));
        HTRI_HIP(hipEventCreate(&e1));
        HTRI_HIP(hipEventRecord(e0, b->stream));
        HTRI_HIP(hipGraphLaunch(F.exec, b->stream));
        HTRI_HIP(hipEventRecord(e1, b->stream));
        HTRI_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HTRI_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        read_counts_from(*b, F.ctr, counts);
        if (time_ms) *time_ms = ms;
    });
}

htri_status htri_batch_count_full_per_graph(htri_batch *b, const htri_schedule *sched, int64_t *counts,
                                            double *time_ms) {
    if (!b || !sched || !counts) return HTRI_E_INVALID;
    return run_b(b, [&] {
        CloseConfig cfg;
        cfg.cap = sched->chunk;
        cfg.jp = sched->partners;
        if (!valid_config(cfg)) fail(HTRI_E_INVALID, "schedule: chunk 256|512, partners 128|256");
        const int n = (int)b->graphs.size();
        DBuf<unsigned long long> ctr(b->al, (size_t)n * 24);
        DBuf<GraphDesc> desc(b->al, (size_t)std::max(n, 1));
        HTRI_HIP(hipStreamSynchronize(b->stream));
        const int per_cu = close_blocks_per_cu(cfg, false, false);
        const auto t0 = std::chrono::steady_clock::now();
        for (int g = 0; g < n; g++) {
            Graph &G = *b->graphs[g];
            drop_step1(G);
            build_wedges(G);
            G.have_wedges = true;
            ItemLists items;
            build_items(G, 0, cfg, items, G.m);
            GraphDesc d = graph_desc(G);
            HTRI_HIP(hipMemcpyAsync(desc.p + g, &d, sizeof(d), hipMemcpyHostToDevice, b->stream));
            unsigned long long *c = ctr.p + 24 * (int64_t)g;
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, b->stream, c, (int64_t)24);
            HTRI_LAUNCH_CHECK();
            CloseArgs a{};
            a.items = items.block.p;
            a.nitems = items.nblock;
            a.queue = (unsigned int *)c;
            a.witems = items.wave.p;
            a.nwitems = items.nwave;
            a.wqueue = (unsigned int *)(c + 23);
            a.graphs = desc.p + g;
            a.emask = 0x1FFFFEu;
            a.lut = b->lut.p;
            a.counts = c + 2;
            a.probes = c + 1;
            int nb = device_cu_count() * per_cu;
            const int64_t ni = items.nblock + items.nwave;
            if ((int64_t)nb > ni) nb = (int)std::max<int64_t>(ni, 1);
            if (ni > 0) launch_close_kernel(cfg, false, false, a, nb, b->stream);
            // the items are freed on return; keep them until the launch is done
            HTRI_HIP(hipStreamSynchronize(b->stream));
        }
        const auto t1 = std::chrono::steady_clock::now();
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
        // the batch's descriptors follow the graphs' rebuilt buffers
        std::vector<GraphDesc> d;
        for (auto &G : b->graphs) d.push_back(graph_desc(*G));
        if (!d.empty())
            HTRI_HIP(hipMemcpyAsync(b->descs.p, d.data(), sizeof(GraphDesc) * d.size(), hipMemcpyHostToDevice,
                                    b->stream));
        HTRI_HIP(hipStreamSynchronize(b->stream));
        if (time_ms) *time_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    });
}

const char *htri_batch_last_error(const htri_batch *b) { return b ? b->err.c_str() : ""; }

void htri_batch_free(htri_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
}

}  // extern "C"
