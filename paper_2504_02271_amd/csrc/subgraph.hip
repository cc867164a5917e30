// Sub-hypergraph for sigma-sampling (Appro-bs, Algorithm 6, with sigma < 1):
// a random subset of the hyperedges and the hypergraph they induce, on which
// the hyperwedge sampler (or the exact count) runs; the result is scaled by
// the inverse of the probability that a hyper-triangle keeps all three of its
// hyperedges.
//
// Selection, by the Philox-4x32-10 word number x of stream kSubStream under
// the caller's seed (x = the hyperedge's normalised id):
//   mode 0: hyperedge x is kept when its word is below floor(sigma * 2^64)
//           (independently with probability sigma; a triangle survives with
//           probability sigma^3);
//   mode 1: exactly n = floor(sigma * m + 1/2) hyperedges, those with the n
//           smallest words (ties by id): a uniform n-subset, which a triangle
//           survives with probability n(n-1)(n-2) / (m(m-1)(m-2)).
#include <cmath>

#include "internal.hpp"
#include "philox.hpp"

namespace htri {

namespace {

constexpr uint32_t kSubStream = 4u;

__global__ void k_sub_bernoulli(int64_t m, uint64_t seed, uint64_t thr, bool all, uint32_t *keep) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += (int64_t)gridDim.x * blockDim.x)
        keep[x] = (all || philox_u64(seed, kSubStream, (uint64_t)x) < thr) ? 1u : 0u;
}

__global__ void k_sub_keys(int64_t m, uint64_t seed, uint64_t *key, uint32_t *id) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += (int64_t)gridDim.x * blockDim.x) {
        key[x] = philox_u64(seed, kSubStream, (uint64_t)x);
        id[x] = (uint32_t)x;
    }
}

// keep the first n ids of the (word, id) order
__global__ void k_sub_mark(const uint32_t *id, int64_t n, uint32_t *keep) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        keep[id[t]] = 1u;
}

// per hyperedge: 1 if kept (for the new ids) and its size if kept (for the
// new member offsets)
__global__ void k_sub_counts(const int64_t *eptr, const uint32_t *keep, int64_t m, int64_t *one, int64_t *size) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += (int64_t)gridDim.x * blockDim.x) {
        one[x] = keep[x] ? 1 : 0;
        size[x] = keep[x] ? eptr[x + 1] - eptr[x] : 0;
    }
}

// copy the kept hyperedges, in id order: one wave per hyperedge
__global__ void k_sub_fill(const int64_t *eptr, const int32_t *emem, const uint32_t *keep, const int64_t *pos,
                           const int64_t *moff, int64_t m, int64_t *new_off, int32_t *new_mem, int32_t *kept) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t x = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; x < m; x += nwaves) {
        if (!keep[x]) continue;
        const int64_t b = eptr[x], len = eptr[x + 1] - b, o = moff[x];
        if (lane == 0) {
            new_off[pos[x]] = o;
            kept[pos[x]] = (int32_t)x;
        }
        for (int64_t t = lane; t < len; t += kWave) new_mem[o + t] = emem[b + t];
    }
}

int64_t read_i64_at(const int64_t *p, hipStream_t s) {
    int64_t v = 0;
    HTRI_HIP(hipMemcpyAsync(&v, p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    return v;
}

}  // namespace

int64_t subgraph_fixed_size(int64_t m, double sigma) {
    const double n = std::floor(sigma * (double)m + 0.5);
    return n < 0 ? 0 : (n > (double)m ? m : (int64_t)n);
}

double subgraph_triangle_scale(int64_t m, int64_t n, double sigma, int mode) {
    if (mode == 0) return 1.0 / (sigma * sigma * sigma);
    if (n < 3) return 0.0;
    const double M = (double)m, N = (double)n;
    return (M * (M - 1.0) * (M - 2.0)) / (N * (N - 1.0) * (N - 2.0));
}

void subgraph_select(Graph &g, double sigma, uint64_t seed, int mode, Graph &out, std::vector<int32_t> &kept) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    DBuf<uint32_t> keep(A, m);
    if (mode == 0) {
        const bool all = sigma >= 1.0;
        const uint64_t thr = all ? 0 : (uint64_t)(sigma * 18446744073709551616.0);
        if (m > 0) {
            hipLaunchKernelGGL(k_sub_bernoulli, dim3(grid_for(m, 256)), dim3(256), 0, s, m, seed, thr, all, keep.p);
            HTRI_LAUNCH_CHECK();
        }
    } else {
        const int64_t n = subgraph_fixed_size(m, sigma);
        fill_u32(keep.p, m, 0u, s);
        if (m > 0) {
            DBuf<uint64_t> key(A, m);
            DBuf<uint32_t> id(A, m);
            hipLaunchKernelGGL(k_sub_keys, dim3(grid_for(m, 256)), dim3(256), 0, s, m, seed, key.p, id.p);
            HTRI_LAUNCH_CHECK();
            radix_sort_u64(A, key.p, id.p, m, 64, s);   // stable: ties stay in id order
            if (n > 0) {
                hipLaunchKernelGGL(k_sub_mark, dim3(grid_for(n, 256)), dim3(256), 0, s, id.p, n, keep.p);
                HTRI_LAUNCH_CHECK();
            }
        }
    }
    DBuf<int64_t> pos(A, m + 1), moff(A, m + 1);
    if (m > 0) {
        hipLaunchKernelGGL(k_sub_counts, dim3(grid_for(m, 256)), dim3(256), 0, s, g.eptr_n.p, keep.p, m, pos.p,
                           moff.p);
        HTRI_LAUNCH_CHECK();
    }
    scan_exclusive_i64(A, pos.p, pos.p, m, pos.p + m, s);
    scan_exclusive_i64(A, moff.p, moff.p, m, moff.p + m, s);
    const int64_t n = read_i64_at(pos.p + m, s);
    const int64_t nnz = read_i64_at(moff.p + m, s);
    DBuf<int64_t> new_off(A, n + 1);
    DBuf<int32_t> new_mem(A, nnz);
    DBuf<int32_t> kept_dev(A, n);
    if (m > 0) {
        hipLaunchKernelGGL(k_sub_fill, dim3(grid_for(m * kWave, 256, 16384)), dim3(256), 0, s, g.eptr_n.p, g.emem_n.p,
                           keep.p, pos.p, moff.p, m, new_off.p, new_mem.p, kept_dev.p);
        HTRI_LAUNCH_CHECK();
    }
    HTRI_HIP(hipMemcpyAsync(new_off.p + n, &nnz, sizeof(int64_t), hipMemcpyHostToDevice, s));
    kept.assign((size_t)n, 0);
    if (n > 0)
        HTRI_HIP(hipMemcpyAsync(kept.data(), kept_dev.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    // the kept hyperedges are distinct sets already; their order is the
    // subgraph's input order
    const uint32_t flags =
        HTRI_DEDUPE_EDGES | HTRI_INPUT_ON_DEVICE | (g.flags & (HTRI_ORDER_INPUT | HTRI_WIDE_TILE_KEYS));
    graph_load(out, new_off.p, n, new_mem.p, g.n, flags);
}

}  // namespace htri
