// Internal declarations of the htri HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "htri.h"

namespace htri {

constexpr int kWave = 64;

// Status carried through the host code; converted to htri_status at the ABI.
struct Error {
    htri_status code;
    std::string msg;
};

#define HTRI_HIP(expr)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw ::htri::Error{HTRI_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define HTRI_LAUNCH_CHECK() HTRI_HIP(hipGetLastError())

inline void fail(htri_status code, const std::string &msg) { throw Error{code, msg}; }

// A data-dependent launch sequence (step 1 and the work items of a graph)
// replayed from a captured HIP graph.  The sequence first runs eagerly in
// record mode, which keeps every value the host reads back from the device
// and adds up every allocation; in capture mode the same host code takes
// those values from the record (no device-to-host copy, no stream
// synchronisation: the stream is being captured) and its buffers from one
// arena that is never reused, so every captured kernel keeps its buffers.
// Host arrays that captured copies read are kept in the record too.
struct Replay {
    enum Mode { kRecord, kCapture } mode = kRecord;
    std::vector<int64_t> vals;          // host readbacks, in order
    size_t next = 0;
    std::vector<std::vector<uint8_t>> host_srcs;
    size_t arena_bytes = 0;             // record: sum of the (aligned) allocations
    char *arena = nullptr;
    size_t arena_size = 0, arena_off = 0;
    bool capturing() const { return mode == kCapture; }
};
// the replay the calling thread is recording or capturing (nullptr: none)
extern thread_local Replay *tl_replay;

inline bool replay_capturing() { return tl_replay && tl_replay->mode == Replay::kCapture; }

// stream synchronisation, skipped while a replay is being captured
inline void stream_sync(hipStream_t s) {
    if (replay_capturing()) return;
    HTRI_HIP(hipStreamSynchronize(s));
}

// n 64-bit values read back from the device (recorded, or replayed)
inline void host_read_words(const void *dev, int64_t n, void *host, hipStream_t s) {
    if (n <= 0) return;
    if (replay_capturing()) {
        Replay &r = *tl_replay;
        if (r.next + (size_t)n > r.vals.size()) fail(HTRI_E_STATE, "replay ran past its recorded values");
        std::memcpy(host, r.vals.data() + r.next, sizeof(int64_t) * (size_t)n);
        r.next += (size_t)n;
        return;
    }
    HTRI_HIP(hipMemcpyAsync(host, dev, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    if (tl_replay) {
        const int64_t *h = (const int64_t *)host;
        tl_replay->vals.insert(tl_replay->vals.end(), h, h + n);
    }
}

template <typename T>
T host_read(const T *dev, hipStream_t s) {
    static_assert(sizeof(T) <= 8, "one word");
    int64_t w = 0;
    if (replay_capturing()) {
        host_read_words(dev, 1, &w, s);
    } else {
        T h{};
        HTRI_HIP(hipMemcpyAsync(&h, dev, sizeof(T), hipMemcpyDeviceToHost, s));
        HTRI_HIP(hipStreamSynchronize(s));
        std::memcpy(&w, &h, sizeof(T));
        if (tl_replay) tl_replay->vals.push_back(w);
    }
    T out{};
    std::memcpy(&out, &w, sizeof(T));
    return out;
}

// host data a captured host-to-device copy reads at every replay: kept in
// the record while capturing
inline const void *persist_host(const void *p, size_t bytes) {
    if (!replay_capturing() || bytes == 0) return p;
    tl_replay->host_srcs.emplace_back((const uint8_t *)p, (const uint8_t *)p + bytes);
    return tl_replay->host_srcs.back().data();
}

// Device memory through the caller's allocator (or hipMallocAsync/hipMalloc).
struct Allocator {
    htri_allocator user{};
    bool has_user = false;
    hipStream_t stream = nullptr;
    // replay arenas whose pieces this allocator handed out while capturing;
    // releasing them is a no-op (each arena's owner frees it whole)
    std::vector<std::pair<const char *, const char *>> arenas;
    bool in_arena(const void *p) const {
        for (const auto &a : arenas)
            if ((const char *)p >= a.first && (const char *)p < a.second) return true;
        return false;
    }

    void *alloc(size_t bytes) {
        if (bytes == 0) bytes = 256;
        const size_t aligned = (bytes + 255) & ~(size_t)255;
        if (replay_capturing()) {
            Replay &r = *tl_replay;
            if (r.arena_off + aligned > r.arena_size) fail(HTRI_E_STATE, "replay arena exhausted");
            void *q = r.arena + r.arena_off;
            r.arena_off += aligned;
            return q;
        }
        if (tl_replay) tl_replay->arena_bytes += aligned;
        void *p = nullptr;
        if (has_user) {
            p = user.alloc(bytes, (void *)stream, user.ctx);
            if (!p) fail(HTRI_E_OOM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
        } else {
            hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                fail(HTRI_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
            }
        }
        return p;
    }
    void release(void *p) {
        if (!p) return;
        if (!arenas.empty() && in_arena(p)) return;   // owned by a replay arena
        if (has_user)
            user.free(p, (void *)stream, user.ctx);
        else
            (void)hipFree(p);
    }
};

// A device buffer owned by its scope.
template <typename T>
struct DBuf {
    Allocator *a = nullptr;
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(Allocator &al, size_t count) : a(&al), n(count) { p = (T *)al.alloc(sizeof(T) * (count ? count : 1)); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : a(o.a), p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { reset(); a = o.a; p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { reset(); }
    void reset() {
        if (p && a) a->release(p);
        p = nullptr;
        n = 0;
    }
    void alloc(Allocator &al, size_t count) {
        reset();
        a = &al;
        n = count;
        p = (T *)al.alloc(sizeof(T) * (count ? count : 1));
    }
    T *get() const { return p; }
};

inline int bits_for(uint64_t maxval) {  // bits to represent values 0..maxval
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) b++;
    return b == 0 ? 1 : b;
}

inline unsigned grid_for(int64_t n, int block, int64_t cap = 1 << 20) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// ---------------------------------------------------------------- primitives
// (prims.hip)
// Exclusive prefix sum of n values; out may alias in.  total (may be NULL)
// receives the sum on the device.
void scan_exclusive_i64(Allocator &a, const int64_t *in, int64_t *out, int64_t n, int64_t *total,
                        hipStream_t s);
void scan_exclusive_u32(Allocator &a, const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                        hipStream_t s);
// Stable LSD radix sort of 64-bit keys on bits [0, key_bits), optional
// 32-bit payload, in place.
void radix_sort_u64(Allocator &a, uint64_t *keys, uint32_t *vals, int64_t n, int key_bits,
                    hipStream_t s);
// Fill n values with v (kernel, safe inside graph capture).
void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
void fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
int device_cu_count();

// ---------------------------------------------------------------- graph state

struct Timings {
    float wedges_ms = 0, schedule_ms = 0, closure_ms = 0, reduce_ms = 0, window_ms = 0, probe_ms = 0;
};

struct Graph {
    Allocator al;
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    std::string err;

    int64_t m = 0;          // hyperedges after dedupe
    int64_t removed = 0;
    int64_t nnz = 0;        // memberships after removing repeated ids
    int32_t n = 0;          // vertices
    int32_t max_size = 0;
    int32_t min_size = 0;       // smallest hyperedge size (0 for an empty graph)

    // normalised-id CSR (input order of survivors)
    DBuf<int64_t> eptr_n;
    DBuf<int32_t> emem_n;
    std::vector<int64_t> norm_to_input;  // host

    // internal (prec-order) CSR: rank r holds normalised hyperedge norm_of_rank[r]
    DBuf<int32_t> norm_of_rank;
    DBuf<int32_t> rank_of_norm;
    DBuf<int64_t> eptr;
    DBuf<int32_t> emem;
    DBuf<int32_t> esize;
    DBuf<int32_t> edge_of_mem;  // membership index -> rank
    DBuf<int64_t> vptr;         // E_v lists, ascending rank
    DBuf<int32_t> vadj;
    DBuf<int32_t> vpos;         // membership -> its position inside E_v


    // step 1: forward adjacency N+(r), sorted by rank
    bool have_wedges = false;
    int64_t nw = 0;
    int wbits = 0;              // low bits of a packed entry hold omega
    int rbits = 0;
    DBuf<int64_t> fptr;         // m+1
    DBuf<uint32_t> fadj;        // packed (dst << wbits) | omega
    DBuf<int64_t> mptr;         // m+1, offsets (in 32-bit words) of Omega masks
    DBuf<uint32_t> fmask;
    DBuf<uint32_t> indeg;       // earlier neighbours of each hyperedge
    int64_t summary[6] = {0, 0, 0, 0, 0, 0};
    // inclusion hyperwedges for the class-split sampler (built on first use):
    // their positions ascending, and (end, other end) pairs of ranks, both
    // ways, sorted
    bool have_incl = false;
    DBuf<int64_t> incl_pos;
    DBuf<int2> incl_pairs;
    int64_t n_incl_pairs = 0;

    Timings tm;
    int64_t cstats[16] = {0};
    int64_t stats_owner_end = 0;   // window start of the last count (for the S census)
};

// The dense window's possible starts: m minus a power of two of rows from
// kWindowRowsMax down to kWindowRowsMax >> (kWindowStarts - 1), or 0 (the
// whole graph).
constexpr int64_t kWindowRowsMax = 131072;
constexpr int kWindowStarts = 8;
inline int64_t window_start(int64_t m, int s) {
    const int64_t w = m - (kWindowRowsMax >> s);
    return w > 0 ? w : 0;
}

// api.hip: message for htri_last_error(NULL)
void set_load_error(const std::string &msg);

// load.hip
void graph_load(Graph &g, const int64_t *off, int64_t m_in, const int32_t *mem, int32_t n,
                uint32_t flags);
// wedges.hip
void build_wedges(Graph &g);
// closure.hip
// Read-only view of one graph's step-1 state, as the closure kernel sees it.
struct GraphDesc {
    const int64_t *fptr;
    const uint32_t *fadj;
    const int64_t *mptr;
    const uint32_t *fmask;
    const int32_t *esize;
    const int64_t *eptr;
    const int32_t *emem;
    // middle-centric closure only (null otherwise): the in-list of each
    // middle hyperedge j, i.e. the hyperwedges (r, j) of the owners probed
    const uint4 *inl;           // per entry: InEntry below
    const int64_t *iptr;        // m+1: in-list of j at [iptr[j], iptr[j+1])
    int32_t wbits;
    int32_t pad;
};
// A closure work item: graph g, owner r, chunk [cb, ce) of N+(r), partner
// positions [jb, je) of N+(r).  Middle-centric items: r is the middle j,
// [cb, ce) a chunk of N+(j) and [jb, je) positions in j's in-list.
struct Item {
    int32_t g, r, cb, ce, jb, je;
};
// Chunk capacity (entries of N+(r) in LDS) and partners per item.
struct CloseConfig {
    int cap = 512;
    int jp = 256;
};
struct CloseArgs {
    const Item *items;              // block items (one block each)
    int64_t nitems;
    unsigned int *queue;            // block-item counter, zero before the launch
    const Item *witems;             // single-owner items (one wave each), taken after the block items
    int64_t nwitems;
    unsigned int *wqueue;           // single-owner item counter, zero before the launch
    const GraphDesc *graphs;
    uint32_t emask;                 // patterns counted into per-edge counts
    const uint8_t *lut;             // 128-entry region table
    uint32_t *cwj;                  // per-wedge j-role count, all patterns (single graph)
    uint32_t *cwjm;                 // per-wedge j-role count, masked
    uint32_t *cwkm;                 // per-wedge k-role count, masked
    unsigned long long *counts;     // [graphs][21]; [g][0] unused (total formed on the host)
    unsigned long long *probes;     // entries probed
    unsigned long long *staged;     // hashed entries staged (null: not counted)
    unsigned long long *tedge;      // middle-centric with per-edge counts: per-hyperedge totals by
                                    // rank, to which each item adds its middle's j-role counts and
                                    // its hashed entries' k-role counts (cwkm is left to the window)
    unsigned long long *tp = nullptr;          // SparseTTT counting with per-pattern per-hyperedge
                                               // counts: rows of 21 by rank, three atomics per hit
    unsigned long long *wave_part = nullptr;   // single-graph launches: each wave's pattern counts,
                                               // [waves][21], summed afterwards in a fixed order
                                               // (null: each wave adds its counts per graph)
};
// counts[p] += sum over i of part[i][p], p = 1..20, in a fixed order (one
// block per pattern, no atomics)
void sum_pattern_parts(const unsigned long long *part, int64_t n, unsigned long long *counts, hipStream_t s);
// Owners with at most kWaveOwnerMax forward entries whose partner lists hold
// at most kWaveStreamMax entries in total are closed by one wave each.
constexpr int kWaveOwnerMax = 64;
// Middle-centric single-middle items: up to kWaveMidHashMax entries of N+(j)
// (and at most kWaveOwnerMax in-list entries) when e_j needs at most one
// Omega word.
constexpr int kWaveMidHashMax = 128;
constexpr int64_t kWaveStreamMax = 1 << 16;
struct ItemLists {
    DBuf<Item> block, wave;
    int64_t nblock = 0, nwave = 0;
};
GraphDesc graph_desc(const Graph &g);
// The in-list of the middle-centric closure: every hyperwedge (r, j) with
// r < owner_end, grouped by j (the transpose of the forward adjacency's
// prefix; no order inside a group).
// One entry, 16 bytes, for the hyperwedge (r, j) at forward index i:
//   x = i; y = (len << wbits) | omega_rj with len = |N+(r)| - 1 - (position
//   of j in N+(r)), the entries after j; z = the one shared vertex when
//   omega_rj = 1 and e_r has a stored mask, else kInNoVertex; w = (r << wbits)
//   | |e_r|.  Both packings fit as the forward entries do.
constexpr uint32_t kInNoVertex = 0xFFFFFFFFu;
struct InList {
    DBuf<uint4> inl;
    DBuf<int64_t> iptr;
    int64_t n = 0;
};
// transpose.hip: the later ends' side of the forward adjacency, bucketed by
// rank (no device atomic per hyperwedge).  It takes graphs of at most 2^28
// hyperedges and fewer than 2^32 hyperwedges (n: those of the owners
// covered).
bool transpose_fits(int64_t m, int64_t n);
// indeg[j] += earlier neighbours of j over all n hyperwedges; n_incl and
// max_omega receive the inclusion count and the largest omega
void count_later_ends(Graph &g, int64_t n, unsigned int *indeg, unsigned long long *n_incl,
                      unsigned int *max_omega);
// device bytes build_inlist needs at its peak
int64_t inlist_bytes(Graph &g, int64_t owner_end);
// HTRI_E_UNSUPPORTED beyond transpose_fits()
void build_inlist(Graph &g, int64_t owner_end, InList &out);
// middle-centric work items of one graph
void build_items_mid(Graph &g, int32_t gid, const CloseConfig &cfg, const InList &in, ItemLists &out);
// work items of one graph (graph index gid) for a configuration; owners at
// ranks >= owner_end get none (the dense window closes them)
void build_items(Graph &g, int32_t gid, const CloseConfig &cfg, ItemLists &out, int64_t owner_end);
// The dense window: owners [w0, m) closed by bitmap intersection.
struct WindowPlan {
    int64_t w0 = 0;
    int nrows = 0, nwords = 0;
    int64_t wedges = 0;
};
WindowPlan choose_window(Graph &g, uint32_t flags);
void close_window(Graph &g, const WindowPlan &w, uint32_t emask, const uint8_t *lut_dev, unsigned long long *counts,
                  unsigned long long *stats, uint32_t *cwj, uint32_t *cwjm, uint32_t *cwkm,
                  unsigned long long *tp = nullptr);
// mid: middle-centric items (default configuration only)
int close_blocks_per_cu(const CloseConfig &cfg, bool pe, bool pw, bool mid = false);
void launch_close_kernel(const CloseConfig &cfg, bool pe, bool pw, const CloseArgs &a, int nblocks, hipStream_t s,
                         bool mid = false);
bool valid_config(const CloseConfig &cfg);
// patterns 1-8 only, by searching around the inclusion hyperwedges; with
// dev_out, also the triangles of pattern target (sorted normalised triples)
void count_inclusion_classes(Graph &g, uint32_t mask, int64_t counts[21], uint64_t *t_dev /*m or null*/,
                             int target = 0, int64_t capacity = 0, int32_t *dev_out = nullptr,
                             unsigned long long *dev_found = nullptr,
                             unsigned long long *tp_rank = nullptr /* m*21, rank order, accumulated */);
// every hyperwedge closed, the triangles of pattern target listed
void enumerate_all_wedges(Graph &g, int target, int64_t capacity, int32_t *dev_out, unsigned long long *dev_found);
// tp_rank (SparseTTT only, or null): per-pattern counts of every hyperedge,
// rows of 21 by rank, added to
void count_patterns(Graph &g, uint32_t mask, uint32_t flags, int64_t counts[21], uint64_t *t_dev /*m or null*/,
                    uint32_t *cw_dev /*nw or null*/, unsigned long long *tp_rank = nullptr);
// fill the S entries of the last count's census (run on request)
void closure_stream_stats(Graph &g);
// subgraph.hip: the sub-hypergraph of sigma-sampling (kept: normalised ids
// in g of the kept hyperedges, ascending); out must carry g's stream and
// allocator
int64_t subgraph_fixed_size(int64_t m, double sigma);
double subgraph_triangle_scale(int64_t m, int64_t n, double sigma, int mode);
void subgraph_select(Graph &g, double sigma, uint64_t seed, int mode, Graph &out, std::vector<int32_t> &kept);
// sample.hip: closure of explicit wedges (per-sample counts) and weighted
// sums over uniform (mode 1) or pool (mode 2) draws
void close_wedge_list_counts(Graph &g, const int64_t *dev_idx, int64_t n, int64_t *dev_out);
void sample_sums(Graph &g, int mode, int64_t n, uint64_t seed, const int64_t *pool, const double *cdf,
                 int64_t pool_n, double scale, long long c[21], double y[21], double y2[21],
                 bool skip_inclusion = false);
// positions (forward-adjacency indices) of every inclusion hyperwedge
int64_t list_inclusion_wedges(Graph &g, DBuf<int64_t> &out);
// sample.hip: the learned proposal's training target of every hyperwedge
void wedge_importance_all(Graph &g, const double scale[21], double live, float *dev_out);
// dense.hip: DenseTTT counts (patterns 9-16, or 9 alone) into counts[21];
// tp_rank (m*21, rank order, accumulated): per-hyperedge counts of 10-16
void count_dense_ttt(Graph &g, bool rest, int64_t counts[21], float *ms,
                     unsigned long long *tp_rank = nullptr);
// perpattern.hip: per-hyperedge counts of every pattern (normalised ids,
// m*21 int64 on the device, [x][0] = all patterns) and the counts
void count_per_edge_patterns(Graph &g, int64_t counts[21], int64_t *dev_out);
// local clustering coefficients (normalised ids, device double[m])
void local_clustering(Graph &g, const double eps[21], double *dev_cc);
// advanced.hip: Appro-adv's draw split (alpha1..alpha4) and its estimate
void adv_split(int64_t n_inter, int64_t n_incl, int64_t alpha, int64_t out[4]);
void adv_estimate(Graph &g, int64_t alpha, uint64_t seed, double est[21], double se[21], int64_t alphas[4]);
// closure sums over draws from one hyperwedge type (advanced.hip's sampler)
void class_sample_sums(Graph &g, int kind, int64_t n, uint64_t seed, uint32_t stream, const int64_t *inc_pos,
                       int64_t n_inc, int64_t list_size, uint32_t keep_mask, long long c[21], double y[21],
                       double y2[21]);
void draw_pool(Graph &g, uint64_t seed, int64_t pool_n, int64_t *dev_pool);
void scan_inclusive_f64(Allocator &a, const double *in, double *out, int64_t n, hipStream_t s);

}  // namespace htri

// ABI handles
struct htri_graph {
    htri::Graph g;
};
struct htri_model;

namespace htri {

// mlp.hip: proposal features and scores
void wedge_features_all(Graph &g, float *dev_out);
// predicted closure count of each listed wedge (null list: wedges 0..n-1)
void score_wedges(Graph &g, const htri_model *model, const int64_t *dev_wedges, int64_t n, double *dev_score);

// Pattern of each 7-bit region-emptiness mask (bit 0 a .. bit 6 g), built
// on the host by region rules; 0 for masks that are not hyper-triangles.
const uint8_t *pattern_lut();

}  // namespace htri
