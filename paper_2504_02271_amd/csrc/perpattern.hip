// Per-hyperedge counts of every pattern, and local clustering coefficients
// (the hyperedge-level quantities of the fine-grained clustering
// coefficient, Def. 5.1 of Section 5).
//
// One call assembles t[x][p], the hyper-triangles of pattern p containing
// hyperedge x, from the searches that enumerate each class cheaply:
//   * all patterns together: the full count's per-hyperedge counts;
//   * patterns 1-8: the search around the inclusion hyperwedges (Count-CCC,
//     Count-TCC, Count-TTC), one atomic per hyperedge of each triangle;
//   * patterns 10-16: the thick-pair scan of Count-DenseTTT, the same way;
//   * patterns 17-20: one SparseTTT closure, each hit without a common
//     vertex adding to its three hyperedges' counts of its pattern;
//   * pattern 9, the common-vertex pattern that holds most triangles: the
//     remainder, all patterns minus the other nineteen.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace htri {
namespace {

// out[x][p] (normalised ids) from the rank-ordered partial counts and the
// all-pattern counts (normalised ids): pattern 9 is the remainder
__global__ void k_assemble(const unsigned long long *tr, const int64_t *t_all, const int32_t *norm_of_rank,
                           int64_t m, int64_t *out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = norm_of_rank[r];
        int64_t *o = out + x * 21;
        const unsigned long long *q = tr + r * 21;
        int64_t rest = 0;
        for (int p = 1; p <= 20; p++) {
            if (p == 9) continue;
            o[p] = (int64_t)q[p];
            rest += o[p];
        }
        o[0] = t_all[x];
        o[9] = t_all[x] - rest;
    }
}

// cc_x = sum_p eps[p] t[x][p] / C(deg_x, 2) (0 when deg_x < 2); with no
// per-pattern counts, t_all[x] / C(deg_x, 2)
__global__ void k_local_cc(const int64_t *fptr, const uint32_t *indeg, const int32_t *norm_of_rank, int64_t m,
                           const int64_t *tp, const int64_t *t_all, const double *eps, double *cc) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = norm_of_rank[r];
        const double d = (double)(fptr[r + 1] - fptr[r]) + (double)indeg[r];
        double num = 0.0;
        if (tp) {
            for (int p = 1; p <= 20; p++) num += eps[p] * (double)tp[x * 21 + p];
        } else {
            num = (double)t_all[x];
        }
        cc[x] = d >= 2.0 ? num / (d * (d - 1.0) / 2.0) : 0.0;
    }
}

}  // namespace

void count_per_edge_patterns(Graph &g, int64_t counts[21], int64_t *dev_out) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    DBuf<int64_t> t_all(A, std::max<int64_t>(m, 1));
    int64_t c[21];
    count_patterns(g, 0x1FFFFEu, 0, c, (uint64_t *)t_all.p, nullptr);
    DBuf<unsigned long long> tr(A, std::max<int64_t>(m * 21, 1));
    fill_u64((uint64_t *)tr.p, m * 21, 0, s);
    bool any18 = false, any1016 = false;
    for (int p = 1; p <= 8; p++) any18 |= c[p] > 0;
    for (int p = 10; p <= 16; p++) any1016 |= c[p] > 0;
    int64_t tmp[21];
    if (any18) count_inclusion_classes(g, 0x1FEu, tmp, nullptr, 0, 0, nullptr, nullptr, tr.p);
    if (any1016) count_dense_ttt(g, true, tmp, nullptr, tr.p);
    bool any1720 = false;
    for (int p = 17; p <= 20; p++) any1720 |= c[p] > 0;
    if (any1720) count_patterns(g, 0x1E0000u, HTRI_COUNT_SPARSE_TTT, tmp, nullptr, nullptr, tr.p);
    if (m > 0) {
        hipLaunchKernelGGL(k_assemble, dim3(grid_for(m, 256)), dim3(256), 0, s, tr.p, t_all.p, g.norm_of_rank.p, m,
                           dev_out);
        HTRI_LAUNCH_CHECK();
    }
    HTRI_HIP(hipStreamSynchronize(s));
    std::copy(c, c + 21, counts);
}

void local_clustering(Graph &g, const double eps[21], double *dev_cc) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    if (m == 0) return;
    DBuf<int64_t> tp, t_all;
    DBuf<double> e;
    int64_t c[21];
    if (eps) {
        tp.alloc(A, m * 21);
        count_per_edge_patterns(g, c, tp.p);
        e.alloc(A, 21);
        HTRI_HIP(hipMemcpyAsync(e.p, eps, sizeof(double) * 21, hipMemcpyHostToDevice, s));
    } else {
        t_all.alloc(A, m);
        count_patterns(g, 0x1FFFFEu, 0, c, (uint64_t *)t_all.p, nullptr);
    }
    hipLaunchKernelGGL(k_local_cc, dim3(grid_for(m, 256)), dim3(256), 0, s, g.fptr.p, g.indeg.p, g.norm_of_rank.p, m,
                       tp.p, t_all.p, e.p, dev_cc);
    HTRI_LAUNCH_CHECK();
    HTRI_HIP(hipStreamSynchronize(s));
}

}  // namespace htri
