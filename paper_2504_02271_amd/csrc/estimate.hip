// Hyperwedge-sampling estimators behind htri_estimate: the uniform estimator
// of Algorithm 6 (sigma = 1) and importance sampling from a learned
// proposal, optionally over a uniform candidate pool.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace htri {
namespace {

// CDF of the mixed proposal over the pool, from the inclusive scan of the
// scores: cdf_u = (1 - lambda) * raw_u / raw_total + lambda * (u + 1) / P
__global__ void k_mix_cdf(double *cdf, int64_t P, double lambda) {
    const double tot = cdf[P - 1];
    const double a = tot > 0 ? (1.0 - lambda) / tot : 0.0;
    const double b = tot > 0 ? lambda / (double)P : 1.0 / (double)P;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < P; u += (int64_t)gridDim.x * blockDim.x)
        cdf[u] = a * cdf[u] + b * (double)(u + 1);
}

}  // namespace
}  // namespace htri

using namespace htri;

namespace {
template <typename F>
htri_status run_g(htri_graph *h, F &&fn) {
    try {
        fn();
        return HTRI_OK;
    } catch (const htri::Error &e) {
        h->g.err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        h->g.err = "host allocation failed";
        return HTRI_E_OOM;
    }
}
}  // namespace

extern "C" {

htri_status htri_estimate(htri_graph *h, const htri_sample_params *p, double est[21], double stderr_[21],
                          double *time_ms) {
    if (!h || !p || !est) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    if (p->proposal != 0 && p->proposal != 1 && p->proposal != 2) {
        h->g.err = "proposal must be 0 (uniform), 1 (learned) or 2 (split by hyperwedge type)";
        return HTRI_E_INVALID;
    }
    if (p->proposal == 2 && (p->flags & HTRI_SAMPLE_EXACT_INCLUSION)) {
        h->g.err = "the split by hyperwedge type samples the inclusion hyperwedges itself";
        return HTRI_E_INVALID;
    }
    if (p->proposal == 1 && !p->model) {
        h->g.err = "the learned proposal needs a model";
        return HTRI_E_INVALID;
    }
    if (p->defensive_mix < 0 || p->defensive_mix > 1 || !(p->budget_fraction >= 0)) {
        h->g.err = "defensive_mix must lie in [0, 1] and budget_fraction >= 0";
        return HTRI_E_INVALID;
    }
    // The network's score is clamped at zero, so without the uniform floor a
    // hyperwedge scored at or below zero could never be drawn and the
    // importance weights would no longer cover every closure: unbiasedness
    // needs a positive draw probability on every hyperwedge.
    if (p->proposal == 1 && !(p->defensive_mix > 0)) {
        h->g.err = "the learned proposal needs defensive_mix > 0 (a positive draw probability everywhere)";
        return HTRI_E_INVALID;
    }
    return run_g(h, [&] {
        Graph &g = h->g;
        hipStream_t s = g.stream;
        const int64_t nw = g.nw;
        double e[21] = {0}, se[21] = {0};
        if (nw == 0) {
            std::memcpy(est, e, sizeof(e));
            if (stderr_) std::memcpy(stderr_, se, sizeof(se));
            if (time_ms) *time_ms = 0;
            return;
        }
        int64_t n = p->num_samples > 0 ? p->num_samples : (int64_t)std::llround(p->budget_fraction * (double)nw);
        if (n < 1) n = 1;
        if (p->proposal == 2) {
            hipEvent_t a0, a1;
            HTRI_HIP(hipEventCreate(&a0));
            HTRI_HIP(hipEventCreate(&a1));
            HTRI_HIP(hipEventRecord(a0, s));
            int64_t alphas[4];
            adv_estimate(g, n, p->seed, e, se, alphas);
            HTRI_HIP(hipEventRecord(a1, s));
            HTRI_HIP(hipEventSynchronize(a1));
            float ms = 0;
            HTRI_HIP(hipEventElapsedTime(&ms, a0, a1));
            (void)hipEventDestroy(a0);
            (void)hipEventDestroy(a1);
            std::memcpy(est, e, sizeof(e));
            if (stderr_) std::memcpy(stderr_, se, sizeof(se));
            if (time_ms) *time_ms = ms;
            return;
        }
        hipEvent_t e0, e1;
        HTRI_HIP(hipEventCreate(&e0));
        HTRI_HIP(hipEventCreate(&e1));
        HTRI_HIP(hipEventRecord(e0, s));
        long long c[21];
        double y[21], y2[21];
        // the inclusion stratum closed exactly: its closures are summed and
        // the sampled part counts only intersection-type hyperwedges
        const bool strat = (p->flags & HTRI_SAMPLE_EXACT_INCLUSION) != 0;
        double exact[21] = {0};
        if (strat && g.summary[2] > 0) {
            DBuf<int64_t> idx;
            const int64_t nc = list_inclusion_wedges(g, idx);
            DBuf<int64_t> cl(g.al, nc * 21);
            close_wedge_list_counts(g, idx.p, nc, cl.p);
            std::vector<int64_t> hc((size_t)nc * 21);
            HTRI_HIP(hipMemcpyAsync(hc.data(), cl.p, sizeof(int64_t) * nc * 21, hipMemcpyDeviceToHost, s));
            HTRI_HIP(hipStreamSynchronize(s));
            for (int64_t w = 0; w < nc; w++)
                for (int q = 0; q < 21; q++) exact[q] += (double)hc[(size_t)w * 21 + q];
        }
        if (p->proposal == 0) {
            sample_sums(g, 1, n, p->seed, nullptr, nullptr, 0, (double)nw, c, y, y2, strat);
            HTRI_HIP(hipEventRecord(e1, s));
            for (int q = 0; q < 21; q++) e[q] = (double)c[q] * (double)nw / (double)n;
        } else {
            int64_t P = nw;
            DBuf<int64_t> pool;
            if (p->pool_factor > 0) {
                P = (int64_t)std::llround(p->pool_factor * (double)n);
                P = std::max<int64_t>(P, 1);
                pool.alloc(g.al, P);
                draw_pool(g, p->seed, P, pool.p);
            }
            DBuf<double> score(g.al, P), cdf(g.al, P);
            score_wedges(g, p->model, pool.p, P, score.p);
            scan_inclusive_f64(g.al, score.p, cdf.p, P, s);
            hipLaunchKernelGGL(k_mix_cdf, dim3(grid_for(P, 256, 8192)), dim3(256), 0, s, cdf.p, P, p->defensive_mix);
            HTRI_LAUNCH_CHECK();
            sample_sums(g, 2, n, p->seed, pool.p, cdf.p, P, (double)nw / (double)P, c, y, y2, strat);
            HTRI_HIP(hipEventRecord(e1, s));
            for (int q = 0; q < 21; q++) e[q] = y[q] / (double)n;
        }
        HTRI_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HTRI_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        for (int q = 0; q < 21; q++) {
            const double var = (y2[q] - (double)n * e[q] * e[q]) / ((double)n * (double)std::max<int64_t>(n - 1, 1));
            se[q] = std::sqrt(std::max(var, 0.0));
            e[q] += exact[q];
        }
        std::memcpy(est, e, sizeof(e));
        if (stderr_) std::memcpy(stderr_, se, sizeof(se));
        if (time_ms) *time_ms = ms;
    });
}

htri_status htri_adv_split(int64_t n_inter, int64_t n_incl, int64_t alpha, int64_t out[4]) {
    if (!out || n_inter < 0 || n_incl < 0 || alpha < 0) return HTRI_E_INVALID;
    adv_split(n_inter, n_incl, alpha, out);
    return HTRI_OK;
}

htri_status htri_close_wedges(htri_graph *h, const int64_t *wedge_idx, int64_t n, int64_t *out) {
    if (!h || n < 0 || (n > 0 && (!wedge_idx || !out))) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    for (int64_t t = 0; t < n; t++)
        if (wedge_idx[t] < 0 || wedge_idx[t] >= h->g.nw) {
            h->g.err = "wedge index out of range";
            return HTRI_E_INVALID;
        }
    return run_g(h, [&] {
        Graph &g = h->g;
        if (n == 0) return;
        DBuf<int64_t> idx(g.al, n), o(g.al, n * 21);
        HTRI_HIP(hipMemcpyAsync(idx.p, wedge_idx, sizeof(int64_t) * n, hipMemcpyHostToDevice, g.stream));
        close_wedge_list_counts(g, idx.p, n, o.p);
        HTRI_HIP(hipMemcpyAsync(out, o.p, sizeof(int64_t) * n * 21, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
    });
}

htri_status htri_proposal_scores(htri_graph *h, const htri_model *model, const int64_t *wedge_idx, int64_t n,
                                 double *out) {
    if (!h || !model || n < 0 || (n > 0 && !out)) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    if (wedge_idx) {
        for (int64_t t = 0; t < n; t++)
            if (wedge_idx[t] < 0 || wedge_idx[t] >= h->g.nw) {
                h->g.err = "wedge index out of range";
                return HTRI_E_INVALID;
            }
    } else if (n != h->g.nw) {
        h->g.err = "without a wedge list n must equal the number of hyperwedges";
        return HTRI_E_INVALID;
    }
    return run_g(h, [&] {
        Graph &g = h->g;
        if (n == 0) return;
        DBuf<int64_t> idx;
        if (wedge_idx) {
            idx.alloc(g.al, n);
            HTRI_HIP(hipMemcpyAsync(idx.p, wedge_idx, sizeof(int64_t) * n, hipMemcpyHostToDevice, g.stream));
        }
        DBuf<double> sc(g.al, n);
        score_wedges(g, model, idx.p, n, sc.p);
        HTRI_HIP(hipMemcpyAsync(out, sc.p, sizeof(double) * n, hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
    });
}

htri_status htri_wedge_importance(htri_graph *h, const int64_t counts[21], uint32_t flags, float *dev_out) {
    if (!h || !counts || !dev_out || (flags & ~HTRI_IMPORTANCE_TOTAL)) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    return run_g(h, [&] {
        Graph &g = h->g;
        double scale[21] = {0};
        double live = 0;
        for (int p = 1; p <= 20; p++)
            if (counts[p] > 0) {
                scale[p] = (double)g.nw / (double)counts[p];
                live += 1;
            }
        if ((flags & HTRI_IMPORTANCE_TOTAL) && counts[0] > 0) {
            scale[0] = (double)g.nw / (double)counts[0];
            live += 1;
        }
        if (live == 0) live = 1;
        wedge_importance_all(g, scale, live, dev_out);
    });
}

htri_status htri_wedge_features(htri_graph *h, float *dev_features) {
    if (!h || !dev_features) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    return run_g(h, [&] {
        wedge_features_all(h->g, dev_features);
        HTRI_HIP(hipStreamSynchronize(h->g.stream));
    });
}

}  // extern "C"
