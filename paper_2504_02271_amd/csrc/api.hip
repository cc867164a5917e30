// C ABI of libhtri: argument checks, status codes, host <-> device copies.
#include <mutex>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace {

std::mutex g_err_mu;
std::string g_load_err;

template <typename F>
htri_status run(htri::Graph *g, F &&fn) {
    try {
        fn();
        return HTRI_OK;
    } catch (const htri::Error &e) {
        if (g) g->err = e.msg;
        else {
            std::lock_guard<std::mutex> lk(g_err_mu);
            g_load_err = e.msg;
        }
        return e.code;
    } catch (const std::bad_alloc &) {
        if (g) g->err = "host allocation failed";
        return HTRI_E_OOM;
    } catch (const std::exception &e) {
        if (g) g->err = e.what();
        return HTRI_E_INVALID;
    }
}

}  // namespace

namespace htri {
void set_load_error(const std::string &msg) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_load_err = msg;
}
}  // namespace htri

extern "C" {

const char *htri_status_string(htri_status s) {
    switch (s) {
        case HTRI_OK: return "ok";
        case HTRI_E_INVALID: return "invalid argument";
        case HTRI_E_RANGE: return "vertex id out of range";
        case HTRI_E_EMPTY_EDGE: return "empty hyperedge";
        case HTRI_E_DUPLICATE_EDGE: return "duplicate hyperedge";
        case HTRI_E_OOM: return "out of device memory";
        case HTRI_E_DEVICE: return "HIP runtime error";
        case HTRI_E_OVERFLOW: return "count overflow";
        case HTRI_E_STATE: return "call order";
        case HTRI_E_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

const char *htri_last_error(const htri_graph *h) {
    if (h) return h->g.err.c_str();
    std::lock_guard<std::mutex> lk(g_err_mu);
    return g_load_err.c_str();
}

htri_status htri_graph_load(const int64_t *edge_offsets, int64_t num_edges, const int32_t *members,
                            int32_t num_vertices, uint32_t flags, const htri_allocator *alloc, void *stream,
                            htri_graph **out) {
    if (!out) return HTRI_E_INVALID;
    *out = nullptr;
    if (!edge_offsets || num_edges < 0 || num_vertices < 0 || (!members && num_edges > 0)) {
        std::lock_guard<std::mutex> lk(g_err_mu);
        g_load_err = "null pointer or negative size";
        return HTRI_E_INVALID;
    }
    if (flags & ~(HTRI_DEDUPE_EDGES | HTRI_INPUT_ON_DEVICE | HTRI_ORDER_INPUT | HTRI_WIDE_TILE_KEYS)) {
        std::lock_guard<std::mutex> lk(g_err_mu);
        g_load_err = "unknown flag";
        return HTRI_E_INVALID;
    }
    if (alloc && (!alloc->alloc || !alloc->free)) {
        std::lock_guard<std::mutex> lk(g_err_mu);
        g_load_err = "allocator without alloc/free";
        return HTRI_E_INVALID;
    }
    htri_graph *h = nullptr;
    try {
        h = new htri_graph();
    } catch (...) {
        return HTRI_E_OOM;
    }
    h->g.stream = (hipStream_t)stream;
    h->g.al.stream = (hipStream_t)stream;
    if (alloc) {
        h->g.al.user = *alloc;
        h->g.al.has_user = true;
    }
    htri_status st = run(nullptr, [&] {
        htri::graph_load(h->g, edge_offsets, num_edges, members, num_vertices, flags);
    });
    if (st != HTRI_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        delete h;
        return st;
    }
    *out = h;
    return HTRI_OK;
}

htri_status htri_graph_info(const htri_graph *h, int64_t out[4]) {
    if (!h || !out) return HTRI_E_INVALID;
    out[0] = h->g.m;
    out[1] = h->g.removed;
    out[2] = h->g.nnz;
    out[3] = h->g.n;
    return HTRI_OK;
}

htri_status htri_graph_edge_map(const htri_graph *h, int64_t *new_to_input) {
    if (!h || (!new_to_input && h->g.m > 0)) return HTRI_E_INVALID;
    if (h->g.m) std::memcpy(new_to_input, h->g.norm_to_input.data(), sizeof(int64_t) * h->g.m);
    return HTRI_OK;
}

htri_status htri_graph_csr(const htri_graph *hc, int64_t *offsets, int32_t *members) {
    htri_graph *h = const_cast<htri_graph *>(hc);
    if (!h || !offsets || (!members && h->g.nnz > 0)) return HTRI_E_INVALID;
    return run(&h->g, [&] {
        htri::Graph &g = h->g;
        HTRI_HIP(hipMemcpyAsync(offsets, g.eptr_n.p, sizeof(int64_t) * (g.m + 1), hipMemcpyDeviceToHost, g.stream));
        if (g.nnz)
            HTRI_HIP(hipMemcpyAsync(members, g.emem_n.p, sizeof(int32_t) * g.nnz, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
    });
}

htri_status htri_subgraph(htri_graph *h, double sigma, uint64_t seed, int32_t mode, htri_graph **out,
                          int32_t *kept_ids, int64_t *num_kept, double *triangle_scale) {
    if (!out) return HTRI_E_INVALID;
    *out = nullptr;
    if (!h || !(sigma > 0.0 && sigma <= 1.0) || (mode != 0 && mode != 1)) return HTRI_E_INVALID;
    htri_graph *sub = nullptr;
    try {
        sub = new htri_graph();
    } catch (...) {
        return HTRI_E_OOM;
    }
    sub->g.stream = h->g.stream;
    sub->g.al = h->g.al;
    std::vector<int32_t> kept;
    htri_status st = run(&h->g, [&] { htri::subgraph_select(h->g, sigma, seed, mode, sub->g, kept); });
    if (st != HTRI_OK) {
        (void)hipStreamSynchronize(h->g.stream);
        delete sub;
        return st;
    }
    const int64_t n = (int64_t)kept.size();
    if (kept_ids && n) std::memcpy(kept_ids, kept.data(), sizeof(int32_t) * n);
    if (num_kept) *num_kept = n;
    if (triangle_scale) *triangle_scale = htri::subgraph_triangle_scale(h->g.m, n, sigma, mode);
    *out = sub;
    return HTRI_OK;
}

htri_status htri_build_wedges(htri_graph *h, int64_t summary[6]) {
    if (!h) return HTRI_E_INVALID;
    htri_status st = HTRI_OK;
    if (!h->g.have_wedges) st = run(&h->g, [&] { htri::build_wedges(h->g); });
    if (st == HTRI_OK && summary) std::memcpy(summary, h->g.summary, sizeof(int64_t) * 6);
    return st;
}

htri_status htri_clear_wedges(htri_graph *h) {
    if (!h) return HTRI_E_INVALID;
    return run(&h->g, [&] {
        htri::Graph &g = h->g;
        HTRI_HIP(hipStreamSynchronize(g.stream));
        g.fptr.reset();
        g.fadj.reset();
        g.mptr.reset();
        g.fmask.reset();
        g.indeg.reset();
        g.incl_pos.reset();
        g.incl_pairs.reset();
        g.n_incl_pairs = 0;
        g.have_incl = false;
        g.nw = 0;
        g.have_wedges = false;
    });
}

htri_status htri_clustering_coefficient(const int64_t counts[21], int64_t connected_triples,
                                        const double epsilon[21], double *cc) {
    if (!counts || !cc || connected_triples < 0) return HTRI_E_INVALID;
    double num = 0.0;
    for (int p = 1; p <= 20; p++) {
        const double e = epsilon ? epsilon[p] : 1.0;
        if (!(e >= 0.0 && e <= 1.0) || counts[p] < 0) return HTRI_E_INVALID;
        num += e * (double)counts[p];
    }
    *cc = connected_triples > 0 ? 3.0 * num / (double)connected_triples : 0.0;
    return HTRI_OK;
}

htri_status htri_enumerate(htri_graph *h, int32_t pattern, int64_t capacity, int32_t *out, int64_t *found,
                           uint32_t out_flags) {
    if (!h || !found || pattern < 1 || pattern > 20 || capacity < 0 || (capacity > 0 && !out)) return HTRI_E_INVALID;
    if (out_flags & ~HTRI_OUTPUT_ON_DEVICE) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    return run(&h->g, [&] {
        htri::Graph &g = h->g;
        const bool dev = out_flags & HTRI_OUTPUT_ON_DEVICE;
        htri::DBuf<int32_t> tmp;
        int32_t *dout = out;
        if (!dev && capacity > 0) {
            tmp.alloc(g.al, capacity * 3);
            dout = tmp.p;
        }
        htri::DBuf<unsigned long long> cnt(g.al, 1);
        htri::fill_u64((uint64_t *)cnt.p, 1, 0, g.stream);
        if (pattern <= 8) {
            int64_t c[21];
            htri::count_inclusion_classes(g, 0x1FFFFEu, c, nullptr, pattern, capacity, dout, cnt.p);
        } else {
            htri::enumerate_all_wedges(g, pattern, capacity, dout, cnt.p);
        }
        unsigned long long n = 0;
        HTRI_HIP(hipMemcpyAsync(&n, cnt.p, sizeof(n), hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
        *found = (int64_t)n;
        const int64_t w = std::min<int64_t>((int64_t)n, capacity);
        if (!dev && w > 0)
            HTRI_HIP(hipMemcpyAsync(out, dout, sizeof(int32_t) * 3 * w, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
    });
}

htri_status htri_closure_stats(const htri_graph *hc, int64_t out[16]) {
    if (!hc || !out) return HTRI_E_INVALID;
    htri_graph *h = const_cast<htri_graph *>(hc);
    return run(&h->g, [&] {
        htri::closure_stream_stats(h->g);
        std::memcpy(out, h->g.cstats, sizeof(int64_t) * 16);
    });
}

htri_status htri_get_wedges(const htri_graph *hc, int32_t *src, int32_t *dst, int32_t *omega) {
    htri_graph *h = const_cast<htri_graph *>(hc);
    if (!h || (h->g.nw > 0 && (!src || !dst))) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    return run(&h->g, [&] {
        htri::Graph &g = h->g;
        std::vector<int64_t> fptr((size_t)g.m + 1);
        std::vector<uint32_t> fadj((size_t)g.nw);
        std::vector<int32_t> nor((size_t)g.m);
        HTRI_HIP(hipMemcpyAsync(fptr.data(), g.fptr.p, sizeof(int64_t) * (g.m + 1), hipMemcpyDeviceToHost, g.stream));
        if (g.nw) HTRI_HIP(hipMemcpyAsync(fadj.data(), g.fadj.p, sizeof(uint32_t) * g.nw, hipMemcpyDeviceToHost, g.stream));
        if (g.m) HTRI_HIP(hipMemcpyAsync(nor.data(), g.norm_of_rank.p, sizeof(int32_t) * g.m, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
        const uint32_t wmask = (1u << g.wbits) - 1;
        for (int64_t r = 0; r < g.m; r++)
            for (int64_t e = fptr[r]; e < fptr[r + 1]; e++) {
                src[e] = nor[r];
                dst[e] = nor[fadj[e] >> g.wbits];
                if (omega) omega[e] = (int32_t)(fadj[e] & wmask);
            }
    });
}

namespace {
// endpoints and omega of listed hyperwedges (owner by binary search in fptr)
__global__ void k_wedge_list(const int64_t *fptr, const uint32_t *fadj, const int32_t *norm_of_rank, int64_t m,
                             int wbits, const int64_t *idx, int64_t n, int32_t *out) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = idx[t];
        int64_t lo = 0, hi = m;                  // largest r with fptr[r] <= e
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (fptr[mid] <= e) lo = mid; else hi = mid;
        }
        const uint32_t ent = fadj[e];
        out[t * 3 + 0] = norm_of_rank[lo];
        out[t * 3 + 1] = norm_of_rank[ent >> wbits];
        out[t * 3 + 2] = (int32_t)(ent & ((1u << wbits) - 1));
    }
}
}  // namespace

htri_status htri_get_wedge_list(const htri_graph *hc, const int64_t *wedge_idx, int64_t n, int32_t *src,
                                int32_t *dst, int32_t *omega) {
    htri_graph *h = const_cast<htri_graph *>(hc);
    if (!h || n < 0 || (n > 0 && (!wedge_idx || !src || !dst))) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    for (int64_t t = 0; t < n; t++)
        if (wedge_idx[t] < 0 || wedge_idx[t] >= h->g.nw) {
            h->g.err = "wedge index out of range";
            return HTRI_E_INVALID;
        }
    return run(&h->g, [&] {
        htri::Graph &g = h->g;
        if (n == 0) return;
        htri::DBuf<int64_t> idx(g.al, n);
        htri::DBuf<int32_t> out(g.al, n * 3);
        HTRI_HIP(hipMemcpyAsync(idx.p, wedge_idx, sizeof(int64_t) * n, hipMemcpyHostToDevice, g.stream));
        hipLaunchKernelGGL(k_wedge_list, dim3(htri::grid_for(n, 256)), dim3(256), 0, g.stream, g.fptr.p, g.fadj.p,
                           g.norm_of_rank.p, g.m, g.wbits, idx.p, n, out.p);
        HTRI_LAUNCH_CHECK();
        std::vector<int32_t> h3((size_t)n * 3);
        HTRI_HIP(hipMemcpyAsync(h3.data(), out.p, sizeof(int32_t) * n * 3, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
        for (int64_t t = 0; t < n; t++) {
            src[t] = h3[(size_t)t * 3];
            dst[t] = h3[(size_t)t * 3 + 1];
            if (omega) omega[t] = h3[(size_t)t * 3 + 2];
        }
    });
}

htri_status htri_count_patterns(htri_graph *h, uint32_t per_edge_pattern_mask, int64_t counts[21],
                                int64_t *per_edge, int32_t *per_wedge, uint32_t out_flags) {
    if (!h || !counts) return HTRI_E_INVALID;
    constexpr uint32_t kModes = HTRI_COUNT_NO_WINDOW | HTRI_COUNT_WINDOW_ALWAYS | HTRI_COUNT_INCLUSION_CLASSES |
                                HTRI_COUNT_DENSE_TTT | HTRI_COUNT_COMMON_VERTEX | HTRI_COUNT_SPARSE_TTT;
    if (out_flags & ~(HTRI_OUTPUT_ON_DEVICE | HTRI_COUNT_OWNER_PROBE | kModes)) return HTRI_E_INVALID;
    {
        const uint32_t modes = out_flags & kModes;
        if (modes & (modes - 1)) return HTRI_E_INVALID;        // at most one mode
    }
    if ((out_flags & (HTRI_COUNT_INCLUSION_CLASSES | HTRI_COUNT_SPARSE_TTT)) && per_wedge) return HTRI_E_INVALID;
    if ((out_flags & (HTRI_COUNT_DENSE_TTT | HTRI_COUNT_COMMON_VERTEX)) && (per_edge || per_wedge))
        return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    uint32_t mask = per_edge_pattern_mask ? (per_edge_pattern_mask & 0x1FFFFEu) : 0x1FFFFEu;
    return run(&h->g, [&] {
        htri::Graph &g = h->g;
        const bool dev = out_flags & HTRI_OUTPUT_ON_DEVICE;
        htri::DBuf<int64_t> t_tmp;
        htri::DBuf<uint32_t> cw_tmp;
        uint64_t *t_dev = nullptr;
        uint32_t *cw_dev = nullptr;
        if (per_edge) {
            if (dev) t_dev = (uint64_t *)per_edge;
            else { t_tmp.alloc(g.al, g.m); t_dev = (uint64_t *)t_tmp.p; }
        }
        if (per_wedge) {
            if (dev) cw_dev = (uint32_t *)per_wedge;
            else { cw_tmp.alloc(g.al, g.nw); cw_dev = cw_tmp.p; }
        }
        int64_t c[21];
        if (out_flags & HTRI_COUNT_INCLUSION_CLASSES) {
            htri::count_inclusion_classes(g, mask, c, t_dev);
        } else if (out_flags & (HTRI_COUNT_DENSE_TTT | HTRI_COUNT_COMMON_VERTEX)) {
            float ms = 0;
            htri::count_dense_ttt(g, (out_flags & HTRI_COUNT_DENSE_TTT) != 0, c, &ms);
            g.tm = htri::Timings{};
            g.tm.closure_ms = ms;
        } else {
            htri::count_patterns(g, mask, out_flags, c, t_dev, cw_dev);
        }
        if (per_edge && !dev && g.m)
            HTRI_HIP(hipMemcpyAsync(per_edge, t_dev, sizeof(int64_t) * g.m, hipMemcpyDeviceToHost, g.stream));
        if (per_wedge && !dev && g.nw)
            HTRI_HIP(hipMemcpyAsync(per_wedge, cw_dev, sizeof(int32_t) * g.nw, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
        std::memcpy(counts, c, sizeof(c));
    });
}

htri_status htri_count_per_edge_patterns(htri_graph *h, int64_t counts[21], int64_t *per_edge_patterns,
                                         uint32_t out_flags) {
    if (!h || !counts || !per_edge_patterns || (out_flags & ~HTRI_OUTPUT_ON_DEVICE)) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    return run(&h->g, [&] {
        htri::Graph &g = h->g;
        const bool dev = out_flags & HTRI_OUTPUT_ON_DEVICE;
        htri::DBuf<int64_t> tmp;
        int64_t *out = per_edge_patterns;
        if (!dev) {
            tmp.alloc(g.al, std::max<int64_t>(g.m * 21, 1));
            out = tmp.p;
        }
        int64_t c[21];
        htri::count_per_edge_patterns(g, c, out);
        if (!dev && g.m)
            HTRI_HIP(hipMemcpyAsync(per_edge_patterns, out, sizeof(int64_t) * g.m * 21, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
        std::memcpy(counts, c, sizeof(c));
    });
}

htri_status htri_local_clustering(htri_graph *h, const double epsilon[21], double *cc, uint32_t out_flags) {
    if (!h || !cc || (out_flags & ~HTRI_OUTPUT_ON_DEVICE)) return HTRI_E_INVALID;
    if (epsilon)
        for (int p = 1; p <= 20; p++)
            if (!(epsilon[p] >= 0.0 && epsilon[p] <= 1.0)) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    return run(&h->g, [&] {
        htri::Graph &g = h->g;
        if (g.m == 0) return;
        const bool dev = out_flags & HTRI_OUTPUT_ON_DEVICE;
        htri::DBuf<double> tmp;
        double *out = cc;
        if (!dev) {
            tmp.alloc(g.al, g.m);
            out = tmp.p;
        }
        htri::local_clustering(g, epsilon, out);
        if (!dev) HTRI_HIP(hipMemcpyAsync(cc, out, sizeof(double) * g.m, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
    });
}

htri_status htri_last_timings(const htri_graph *h, double ms[6]) {
    if (!h || !ms) return HTRI_E_INVALID;
    ms[0] = h->g.tm.wedges_ms;
    ms[1] = h->g.tm.schedule_ms;
    ms[2] = h->g.tm.closure_ms;
    ms[3] = h->g.tm.reduce_ms;
    ms[4] = h->g.tm.window_ms;
    ms[5] = h->g.tm.probe_ms;
    return HTRI_OK;
}

void htri_graph_free(htri_graph *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->g.stream);
    delete h;
}

}  // extern "C"
