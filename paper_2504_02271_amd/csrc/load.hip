// Loading a hypergraph: validation, per-hyperedge sort + dedupe of vertex
// ids (Def. 2.1: a hyperedge is a vertex set), removal of duplicate
// hyperedges (the distinct-hyperedge assumption of Section 2), the
// processing order prec, and the vertex->hyperedge lists E_v ascending in
// that order (Algorithm 2, first step).  All on the device.
#include "internal.hpp"

namespace htri {

namespace {

enum : uint32_t { kErrOffsets = 1, kErrRange = 2, kErrEmpty = 4 };

__global__ void k_validate_offsets(const int64_t *off, int64_t m, uint32_t *err) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m;
         x += (int64_t)gridDim.x * blockDim.x) {
        int64_t a = off[x], b = off[x + 1];
        if (x == 0 && a != 0) atomicOr(err, kErrOffsets);
        if (b < a) atomicOr(err, kErrOffsets);
        if (b == a) atomicOr(err, kErrEmpty);
    }
}

__global__ void k_validate_members(const int32_t *mem, int64_t nnz, int32_t n, uint32_t *err) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = mem[t];
        if (v < 0 || v >= n) atomicOr(err, kErrRange);
    }
}

// key = (hyperedge << vbits) | vertex, one thread per hyperedge
__global__ void k_member_keys(const int64_t *off, int64_t m, const int32_t *mem, int vbits,
                              uint64_t *keys) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m;
         x += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t t = off[x]; t < off[x + 1]; t++)
            keys[t] = ((uint64_t)x << vbits) | (uint32_t)mem[t];
    }
}

// keep the first of equal keys; count survivors per hyperedge
__global__ void k_unique_flags(const uint64_t *keys, int64_t nnz, int vbits, int64_t *flag,
                               int32_t *size) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x) {
        bool first = t == 0 || keys[t] != keys[t - 1];
        flag[t] = first ? 1 : 0;
        if (first) atomicAdd(&size[keys[t] >> vbits], 1);
    }
}

__global__ void k_unique_scatter(const uint64_t *keys, int64_t nnz, int vbits, const int64_t *pos,
                                 int32_t *out) {
    const uint64_t vmask = (vbits >= 64) ? ~0ull : ((1ull << vbits) - 1);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x) {
        bool first = t == 0 || keys[t] != keys[t - 1];
        if (first) out[pos[t]] = (int32_t)(keys[t] & vmask);
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // splitmix64 finaliser
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// 64-bit hash of each hyperedge's sorted member list
__global__ void k_edge_hash(const int64_t *off, int64_t m, const int32_t *mem, uint64_t *h,
                            uint32_t *id) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m;
         x += (int64_t)gridDim.x * blockDim.x) {
        uint64_t acc = mix64((uint64_t)(off[x + 1] - off[x]));
        for (int64_t t = off[x]; t < off[x + 1]; t++) acc = mix64(acc ^ (uint32_t)mem[t]);
        h[x] = acc;
        id[x] = (uint32_t)x;
    }
}

// In hash order (ties in input order), a hyperedge equal to an earlier one
// of the same hash run is a later duplicate.
__global__ void k_find_dups(const uint64_t *h, const uint32_t *id, int64_t m, const int64_t *off,
                            const int32_t *mem, int32_t *keep, unsigned long long *removed) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
         q += (int64_t)gridDim.x * blockDim.x) {
        uint32_t x = id[q];
        keep[x] = 1;
        int64_t lx = off[x + 1] - off[x];
        for (int64_t r = q - 1; r >= 0 && h[r] == h[q]; r--) {
            uint32_t y = id[r];
            if (off[y + 1] - off[y] != lx) continue;
            bool eq = true;
            for (int64_t t = 0; t < lx && eq; t++) eq = mem[off[x] + t] == mem[off[y] + t];
            if (eq) {
                keep[x] = 0;
                atomicAdd(removed, 1ull);
                break;
            }
        }
    }
}

__global__ void k_keep_to_i64(const int32_t *keep, const int32_t *size, int64_t m, int64_t *flag,
                              int64_t *ksize) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m;
         x += (int64_t)gridDim.x * blockDim.x) {
        flag[x] = keep[x];
        ksize[x] = keep[x] ? size[x] : 0;
    }
}

// survivors, renumbered in input order
__global__ void k_compact_edges(const int32_t *keep, const int64_t *newid, int64_t m_in,
                                const int64_t *off1, const int32_t *mem1, const int64_t *eptr_n,
                                int32_t *emem_n, int64_t *n2i) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m_in;
         x += (int64_t)gridDim.x * blockDim.x) {
        if (!keep[x]) continue;
        int64_t y = newid[x];
        n2i[y] = x;
        int64_t d = eptr_n[y];
        for (int64_t t = off1[x]; t < off1[x + 1]; t++) emem_n[d++] = mem1[t];
    }
}

__global__ void k_scatter_eptr(const int32_t *keep, const int64_t *newid, const int64_t *kpre,
                               int64_t m_in, int64_t *eptr_n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m_in;
         x += (int64_t)gridDim.x * blockDim.x)
        if (keep[x]) eptr_n[newid[x]] = kpre[x];
}

__global__ void k_vertex_degree(const int32_t *mem, int64_t nnz, int64_t *dv) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd((unsigned long long *)&dv[mem[t]], 1ull);
}

// delta_x = sum over v in e_x of (|E_v| - 1); sort key with x as payload
__global__ void k_delta(const int64_t *eptr, const int32_t *emem, int64_t m, const int64_t *dv,
                        uint64_t *key, uint32_t *val, int32_t *size, unsigned int *maxsize) {
    // every lane of a wave runs the same iterations (the wave reductions
    // below read all 64 lanes); lanes past m contribute the identities
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        const int64_t x = base + threadIdx.x;
        unsigned int hi = 0u, lo = 0xFFFFFFFFu;
        if (x < m) {
            uint64_t d = 0;
            for (int64_t t = eptr[x]; t < eptr[x + 1]; t++) d += (uint64_t)(dv[emem[t]] - 1);
            key[x] = d;
            val[x] = (uint32_t)x;
            const int32_t s = (int32_t)(eptr[x + 1] - eptr[x]);
            size[x] = s;
            hi = lo = (unsigned int)s;
        }
        // largest and smallest size: one atomic of each per wave
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            hi = max(hi, (unsigned int)__shfl_xor((int)hi, o, 64));
            lo = min(lo, (unsigned int)__shfl_xor((int)lo, o, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            if (hi) atomicMax(&maxsize[0], hi);
            if (lo != 0xFFFFFFFFu) atomicMin(&maxsize[1], lo);
        }
    }
}

__global__ void k_rank_maps(const uint32_t *sorted_ids, int64_t m, int32_t *norm_of_rank,
                            int32_t *rank_of_norm, const int32_t *size_n, int32_t *esize,
                            int64_t *esize64) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x) {
        int32_t y = (int32_t)sorted_ids[r];
        norm_of_rank[r] = y;
        rank_of_norm[y] = (int32_t)r;
        esize[r] = size_n[y];
        esize64[r] = size_n[y];
    }
}

__global__ void k_rank_csr(const int32_t *norm_of_rank, int64_t m, const int64_t *eptr_n,
                           const int32_t *emem_n, const int64_t *eptr, int32_t *emem,
                           int32_t *edge_of_mem, uint64_t *vkey, uint32_t *vval) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t s = eptr_n[norm_of_rank[r]];
        int64_t b = eptr[r], e = eptr[r + 1];
        for (int64_t t = b; t < e; t++) {
            int32_t v = emem_n[s + (t - b)];
            emem[t] = v;
            edge_of_mem[t] = (int32_t)r;
            vkey[t] = (uint32_t)v;
            vval[t] = (uint32_t)t;
        }
    }
}

__global__ void k_transpose_fill(const uint64_t *vkey, const uint32_t *vval, int64_t nnz,
                                 const int64_t *vptr, const int32_t *edge_of_mem, int32_t *vadj,
                                 int32_t *vpos) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nnz;
         s += (int64_t)gridDim.x * blockDim.x) {
        uint32_t t = vval[s];
        int64_t v = (int64_t)vkey[s];
        vadj[s] = edge_of_mem[t];
        vpos[t] = (int32_t)(s - vptr[v]);
    }
}

template <typename T>
T read_scalar(const T *dev, hipStream_t s) {
    T h{};
    HTRI_HIP(hipMemcpyAsync(&h, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    return h;
}

}  // namespace

void graph_load(Graph &g, const int64_t *off_in, int64_t m_in, const int32_t *mem_in, int32_t n,
                uint32_t flags) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    if (m_in < 0 || n < 0) fail(HTRI_E_INVALID, "negative size");
    if (m_in >= (int64_t)INT32_MAX) fail(HTRI_E_UNSUPPORTED, "more than 2^31-1 hyperedges");
    g.n = n;
    g.flags = flags;
    const bool on_dev = flags & HTRI_INPUT_ON_DEVICE;

    // offsets on the device
    DBuf<int64_t> off(A, m_in + 1);
    if (on_dev)
        HTRI_HIP(hipMemcpyAsync(off.p, off_in, sizeof(int64_t) * (m_in + 1), hipMemcpyDeviceToDevice, s));
    else
        HTRI_HIP(hipMemcpyAsync(off.p, off_in, sizeof(int64_t) * (m_in + 1), hipMemcpyHostToDevice, s));
    DBuf<uint32_t> err(A, 1);
    fill_u32(err.p, 1, 0, s);
    if (m_in > 0) {
        hipLaunchKernelGGL(k_validate_offsets, dim3(grid_for(m_in, 256)), dim3(256), 0, s, off.p, m_in,
                           err.p);
        HTRI_LAUNCH_CHECK();
    }
    uint32_t e0 = read_scalar(err.p, s);
    if (e0 & kErrOffsets) fail(HTRI_E_INVALID, "edge_offsets must start at 0 and not decrease");
    int64_t nnz_in = 0;
    HTRI_HIP(hipMemcpyAsync(&nnz_in, off.p + m_in, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    if (m_in == 0 && nnz_in != 0) fail(HTRI_E_INVALID, "edge_offsets[0] must be 0");
    if (nnz_in >= (int64_t)UINT32_MAX) fail(HTRI_E_UNSUPPORTED, "more than 2^32 memberships");

    DBuf<int32_t> mem(A, nnz_in);
    if (nnz_in > 0) {
        if (on_dev)
            HTRI_HIP(hipMemcpyAsync(mem.p, mem_in, sizeof(int32_t) * nnz_in, hipMemcpyDeviceToDevice, s));
        else
            HTRI_HIP(hipMemcpyAsync(mem.p, mem_in, sizeof(int32_t) * nnz_in, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_validate_members, dim3(grid_for(nnz_in, 256)), dim3(256), 0, s, mem.p, nnz_in,
                           n, err.p);
        HTRI_LAUNCH_CHECK();
    }
    uint32_t e1 = read_scalar(err.p, s);
    if (e1 & kErrRange) fail(HTRI_E_RANGE, "a vertex id lies outside [0, num_vertices)");
    if (e1 & kErrEmpty) fail(HTRI_E_EMPTY_EDGE, "a hyperedge has no vertex (Def. 2.1)");

    // 1. sort members inside each hyperedge, drop repeated ids
    const int vbits = bits_for(n > 0 ? (uint64_t)(n - 1) : 0);
    const int ebits = bits_for(m_in > 0 ? (uint64_t)(m_in - 1) : 0);
    DBuf<int64_t> off1(A, m_in + 1);
    DBuf<int32_t> mem1(A, nnz_in);
    DBuf<int32_t> size1(A, m_in);
    int64_t nnz1 = 0;
    {
        DBuf<uint64_t> keys(A, nnz_in);
        if (m_in > 0) {
            hipLaunchKernelGGL(k_member_keys, dim3(grid_for(m_in, 256)), dim3(256), 0, s, off.p, m_in,
                               mem.p, vbits, keys.p);
            HTRI_LAUNCH_CHECK();
        }
        radix_sort_u64(A, keys.p, nullptr, nnz_in, ebits + vbits, s);
        DBuf<int64_t> flag(A, nnz_in + 1);
        fill_u32((uint32_t *)size1.p, m_in, 0, s);
        if (nnz_in > 0) {
            hipLaunchKernelGGL(k_unique_flags, dim3(grid_for(nnz_in, 256)), dim3(256), 0, s, keys.p, nnz_in,
                               vbits, flag.p, size1.p);
            HTRI_LAUNCH_CHECK();
        }
        DBuf<int64_t> total(A, 1);
        scan_exclusive_i64(A, flag.p, flag.p, nnz_in, total.p, s);
        nnz1 = read_scalar(total.p, s);
        mem1.alloc(A, nnz1);
        if (nnz_in > 0) {
            hipLaunchKernelGGL(k_unique_scatter, dim3(grid_for(nnz_in, 256)), dim3(256), 0, s, keys.p,
                               nnz_in, vbits, flag.p, mem1.p);
            HTRI_LAUNCH_CHECK();
        }
        // offsets of the deduplicated member lists
        DBuf<int64_t> sz64(A, m_in + 1);
        DBuf<int32_t> ones(A, m_in);
        fill_u32((uint32_t *)ones.p, m_in, 1, s);
        if (m_in > 0) {
            hipLaunchKernelGGL(k_keep_to_i64, dim3(grid_for(m_in, 256)), dim3(256), 0, s, ones.p, size1.p,
                               m_in, off1.p, sz64.p);
            HTRI_LAUNCH_CHECK();
        }
        scan_exclusive_i64(A, sz64.p, off1.p, m_in, off1.p + m_in, s);
    }
    mem.reset();

    // 2. duplicate hyperedges: hash, sort by hash (stable), compare runs
    DBuf<int32_t> keep(A, m_in);
    int64_t removed = 0;
    if (m_in > 0) {
        DBuf<uint64_t> h(A, m_in);
        DBuf<uint32_t> id(A, m_in);
        hipLaunchKernelGGL(k_edge_hash, dim3(grid_for(m_in, 256)), dim3(256), 0, s, off1.p, m_in, mem1.p,
                           h.p, id.p);
        HTRI_LAUNCH_CHECK();
        radix_sort_u64(A, h.p, id.p, m_in, 64, s);
        DBuf<unsigned long long> rem(A, 1);
        fill_u64((uint64_t *)rem.p, 1, 0, s);
        hipLaunchKernelGGL(k_find_dups, dim3(grid_for(m_in, 256)), dim3(256), 0, s, h.p, id.p, m_in,
                           off1.p, mem1.p, keep.p, rem.p);
        HTRI_LAUNCH_CHECK();
        removed = (int64_t)read_scalar(rem.p, s);
    }
    if (removed > 0 && !(flags & HTRI_DEDUPE_EDGES))
        fail(HTRI_E_DUPLICATE_EDGE, std::to_string(removed) +
                                        " duplicate hyperedge(s); pass HTRI_DEDUPE_EDGES to drop them");
    g.removed = removed;
    const int64_t m = m_in - removed;
    g.m = m;

    // 3. survivors renumbered in input order: normalised CSR
    g.eptr_n.alloc(A, m + 1);
    DBuf<int64_t> n2i(A, m);
    {
        DBuf<int64_t> flag(A, m_in + 1), ksize(A, m_in + 1);
        if (m_in > 0) {
            hipLaunchKernelGGL(k_keep_to_i64, dim3(grid_for(m_in, 256)), dim3(256), 0, s, keep.p, size1.p,
                               m_in, flag.p, ksize.p);
            HTRI_LAUNCH_CHECK();
        }
        scan_exclusive_i64(A, flag.p, flag.p, m_in, nullptr, s);
        // sizes of survivors, compacted: scan the masked sizes, then gather
        DBuf<int64_t> kpre(A, m_in + 1);
        scan_exclusive_i64(A, ksize.p, kpre.p, m_in, kpre.p + m_in, s);
        // eptr_n[y] = kpre[x] for survivor x -> y; eptr_n[m] = total
        g.nnz = read_scalar(kpre.p + m_in, s);
        g.emem_n.alloc(A, g.nnz);
        // build eptr_n by scattering kpre of survivors
        if (m_in > 0) {
            hipLaunchKernelGGL(k_scatter_eptr, dim3(grid_for(m_in, 256)), dim3(256), 0, s, keep.p, flag.p,
                               kpre.p, m_in, g.eptr_n.p);
            HTRI_LAUNCH_CHECK();
        }
        HTRI_HIP(hipMemcpyAsync(g.eptr_n.p + m, kpre.p + m_in, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        if (m_in > 0) {
            hipLaunchKernelGGL(k_compact_edges, dim3(grid_for(m_in, 256)), dim3(256), 0, s, keep.p, flag.p,
                               m_in, off1.p, mem1.p, g.eptr_n.p, g.emem_n.p, n2i.p);
            HTRI_LAUNCH_CHECK();
        }
    }
    g.norm_to_input.assign((size_t)m, 0);
    if (m > 0)
        HTRI_HIP(hipMemcpyAsync(g.norm_to_input.data(), n2i.p, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    off1.reset();
    mem1.reset();
    size1.reset();
    keep.reset();

    // 4. processing order prec: (delta_x, x) ascending
    DBuf<int64_t> dv(A, (size_t)n + 1);
    fill_u64((uint64_t *)dv.p, n, 0, s);
    if (g.nnz > 0) {
        hipLaunchKernelGGL(k_vertex_degree, dim3(grid_for(g.nnz, 256)), dim3(256), 0, s, g.emem_n.p, g.nnz,
                           dv.p);
        HTRI_LAUNCH_CHECK();
    }
    g.norm_of_rank.alloc(A, m);
    g.rank_of_norm.alloc(A, m);
    g.esize.alloc(A, m);
    DBuf<int64_t> esize64(A, m + 1);
    {
        DBuf<uint64_t> key(A, m);
        DBuf<uint32_t> val(A, m);
        DBuf<int32_t> size_n(A, m);
        DBuf<unsigned int> mx(A, 2);              // largest, smallest size
        fill_u32(mx.p, 1, 0, s);
        fill_u32(mx.p + 1, 1, 0xFFFFFFFFu, s);
        if (m > 0) {
            hipLaunchKernelGGL(k_delta, dim3(grid_for(m, 256)), dim3(256), 0, s, g.eptr_n.p, g.emem_n.p, m,
                               dv.p, key.p, val.p, size_n.p, mx.p);
            HTRI_LAUNCH_CHECK();
        }
        if (!(flags & HTRI_ORDER_INPUT)) {
            // delta <= nnz * max size: sort only the bits that can be set
            radix_sort_u64(A, key.p, val.p, m, bits_for((uint64_t)g.nnz), s);
        }
        g.max_size = (int32_t)read_scalar(mx.p, s);
        g.min_size = m > 0 ? (int32_t)read_scalar(mx.p + 1, s) : 0;
        if (m > 0) {
            hipLaunchKernelGGL(k_rank_maps, dim3(grid_for(m, 256)), dim3(256), 0, s, val.p, m,
                               g.norm_of_rank.p, g.rank_of_norm.p, size_n.p, g.esize.p, esize64.p);
            HTRI_LAUNCH_CHECK();
        }
    }

    // 5. internal CSR in prec order and E_v (stable sort by vertex)
    g.eptr.alloc(A, m + 1);
    scan_exclusive_i64(A, esize64.p, g.eptr.p, m, g.eptr.p + m, s);
    g.emem.alloc(A, g.nnz);
    g.edge_of_mem.alloc(A, g.nnz);
    g.vptr.alloc(A, (size_t)n + 1);
    g.vadj.alloc(A, g.nnz);
    g.vpos.alloc(A, g.nnz);
    {
        DBuf<uint64_t> vkey(A, g.nnz);
        DBuf<uint32_t> vval(A, g.nnz);
        if (m > 0) {
            hipLaunchKernelGGL(k_rank_csr, dim3(grid_for(m, 256)), dim3(256), 0, s, g.norm_of_rank.p, m,
                               g.eptr_n.p, g.emem_n.p, g.eptr.p, g.emem.p, g.edge_of_mem.p, vkey.p, vval.p);
            HTRI_LAUNCH_CHECK();
        }
        radix_sort_u64(A, vkey.p, vval.p, g.nnz, vbits, s);
        scan_exclusive_i64(A, dv.p, g.vptr.p, n, g.vptr.p + n, s);
        if (g.nnz > 0) {
            hipLaunchKernelGGL(k_transpose_fill, dim3(grid_for(g.nnz, 256)), dim3(256), 0, s, vkey.p, vval.p,
                               g.nnz, g.vptr.p, g.edge_of_mem.p, g.vadj.p, g.vpos.p);
            HTRI_LAUNCH_CHECK();
        }
        HTRI_HIP(hipStreamSynchronize(s));
    }
}

}  // namespace htri
