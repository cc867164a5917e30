// The later ends' side of the forward adjacency (Algorithm 2's hyperwedges
// seen from j): in-degrees, and the in-list that the closure around the
// middle hyperedge reads, built without a device atomic per hyperwedge.
//
// Later ends are grouped in buckets of 2^shift consecutive ranks.
//   1. hist: the owners are dealt to waves (one wave per owner, in turn);
//      each block counts its hyperwedges per bucket in LDS.  Lanes of a wave
//      hold consecutive entries of one sorted forward list, so their buckets
//      form runs and each run adds to its bucket once.
//   2. an exclusive scan of the block counts, bucket-major, gives every
//      block one contiguous run in every bucket.
//   3. scatter: the same blocks visit the same hyperwedges again and write,
//      run by run, the later end's offset inside its bucket (16 bits) and,
//      for the in-list, the 16-byte entry.
//   4. per chunk of one bucket (about n/1024 entries, 4,096 to 262,144): an
//      LDS histogram of the offsets, added to each later end's count with one
//      atomic per (chunk, later end).
//   5. in-list only: a scan of the counts gives each later end's range; each
//      chunk of 65,536 entries reserves its share of every later end's range
//      with one atomic and places its entries with LDS counters.
// No order is kept inside a later end's group.
#include <algorithm>

#include "internal.hpp"

namespace htri {
namespace {

// hist and scatter: 512 blocks of 1024 threads at most.  Each block keeps one
// partly written line per bucket (two for the in-list) open in its XCD's L2;
// fewer, larger blocks keep fewer open lines, so more of them fill before
// they are written back.
constexpr int kTrBlock = 1024, kTrGridMax = 512;
constexpr int kTrCountBlock = 1024;   // counting and placing blocks hold 64-128 KB of LDS: 16 waves each
// entries of one bucket per counting block (fewer on a small graph, so that
// its few buckets still spread over many blocks), and per placing block: a placing
// block reserves its share of each later end's range with one atomic, so it
// takes enough entries per later end to amortise them, while the 16-byte
// entries it scatters stay within a footprint the L2 can combine
constexpr uint32_t kChunkCountMax = 262144, kChunkCountMin = 4096, kChunkPlace = 65536;
// ranks per bucket: 2^15 for the in-degrees (the scatter writes 2-byte
// offsets only; fewer buckets give longer runs per block), 2^14 for the
// in-list (its placing blocks hold 2^shift LDS counters)
constexpr int kShiftIndeg = 15, kShiftInlist = 14, kShiftMax = 15;   // LDS counters: at most 128 KB
constexpr int kBucketsMax = 8192;
constexpr int kMaskWordsTr = 4;

__device__ __forceinline__ int tr_mask_words(int size) {
    return size <= 32 * kMaskWordsTr ? (size + 31) / 32 : 0;
}

struct Buckets {
    int shift = kShiftIndeg;
    int64_t nb = 1;
};

Buckets buckets_for(int64_t m, int shift_min) {
    Buckets b;
    const int bits = bits_for((uint64_t)(m > 0 ? m - 1 : 0));
    // a graph of fewer than 2^shift_min hyperedges is one bucket of its own
    // width (the counting blocks clear only that many LDS counters)
    b.shift = std::max(std::min(shift_min, bits), bits - 13);
    b.nb = ((m > 0 ? m : 1) + ((int64_t)1 << b.shift) - 1) >> b.shift;
    return b;
}

// lanes [0, nvalid) of the wave hold entries in bucket order (non-decreasing
// bucket ids); returns, for this lane, the lane that heads its run, and sets
// len on a head to the run's length
__device__ __forceinline__ int run_head(uint32_t bkt, bool valid, int lane, int nvalid, int *len) {
    const uint32_t prev = __shfl_up(bkt, 1, kWave);
    const bool head = valid && (lane == 0 || prev != bkt);
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    if (head) {
        const uint64_t after = heads & ~upto;
        const int nxt = after ? __ffsll((unsigned long long)after) - 1 : nvalid;
        *len = nxt - lane;
    }
    return 63 - __clzll((long long)(heads & upto));
}

// 1: per-block bucket counts of the hyperwedges of owners [0, owner_end);
// with STATS also the inclusion count and the largest omega (as the wedge
// summary needs them)
template <bool STATS>
__global__ __launch_bounds__(kTrBlock) void k_tr_hist(const int64_t *fptr, const uint32_t *fadj,
                                                      const int32_t *esize, int64_t owner_end, int wbits,
                                                      int shift, int nb, int min_size, uint32_t *hist,
                                                      unsigned long long *n_incl, unsigned int *max_omega) {
    extern __shared__ uint32_t sh[];
    for (int b = threadIdx.x; b < nb; b += blockDim.x) sh[b] = 0;
    __syncthreads();
    const uint32_t wmask = (1u << wbits) - 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long inc = 0;
    unsigned int mx = 0;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < owner_end; r += nwaves) {
        const int64_t b0 = fptr[r], e = fptr[r + 1];
        const int32_t sr = STATS ? esize[r] : 0;
        for (int64_t q0 = b0; q0 < e; q0 += kWave) {
            const int64_t q = q0 + lane;
            const bool valid = q < e;
            const int nvalid = (int)min<int64_t>(e - q0, (int64_t)kWave);
            uint32_t bkt = 0xFFFFFFFFu;
            if (valid) {
                const uint32_t ent = fadj[q];
                const uint32_t j = ent >> wbits;
                bkt = j >> shift;
                if (STATS) {
                    const uint32_t om = ent & wmask;
                    // inclusion: omega = min(|e_r|, |e_j|); omega = |e_r|
                    // decides it alone, omega below the smallest size rules
                    // it out, so |e_j| is read only in between
                    if ((int32_t)om == sr) {
                        inc++;
                    } else if ((int32_t)om >= min_size && (int32_t)om == esize[j]) {
                        inc++;
                    }
                    if (om > mx) mx = om;
                }
            }
            int len = 0;
            const int h = run_head(bkt, valid, lane, nvalid, &len);
            if (valid && h == lane) atomicAdd(&sh[bkt], (uint32_t)len);
        }
    }
    __shared__ unsigned long long s_inc;
    __shared__ unsigned int s_mx;
    if (STATS) {
        if (threadIdx.x == 0) {
            s_inc = 0;
            s_mx = 0;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            inc += __shfl_xor(inc, o, 64);
            const unsigned int x = __shfl_xor(mx, o, 64);
            mx = x > mx ? x : mx;
        }
    }
    __syncthreads();
    if (STATS) {
        // one pair of device atomics per block, not per wave
        if (lane == 0) {
            if (inc) atomicAdd(&s_inc, inc);
            if (mx) atomicMax(&s_mx, mx);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_inc) atomicAdd(n_incl, s_inc);
            if (s_mx) atomicMax(max_omega, s_mx);
        }
    }
    for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[(int64_t)b * gridDim.x + blockIdx.x] = sh[b];
}

// 3: the same owners, dealt the same way: each hyperwedge's later-end offset
// in its bucket to its block's run, and with PAYLOAD its in-list entry
template <bool PAYLOAD>
__global__ __launch_bounds__(kTrBlock) void k_tr_scatter(const int64_t *fptr, const uint32_t *fadj,
                                                         int64_t owner_end, int wbits, int shift, int nb,
                                                         const uint32_t *off, const int32_t *esize,
                                                         const int64_t *eptr, const int32_t *emem,
                                                         const int64_t *mptr, const uint32_t *fmask,
                                                         uint16_t *tj, uint4 *te) {
    extern __shared__ uint32_t sh[];
    for (int b = threadIdx.x; b < nb; b += blockDim.x) sh[b] = off[(int64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const uint32_t wmask = (1u << wbits) - 1;
    const uint32_t lmask = (1u << shift) - 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < owner_end; r += nwaves) {
        const int64_t b0 = fptr[r], e = fptr[r + 1];
        int sr = 0, Wr = 0;
        int64_t mb = 0, rb = 0;
        if (PAYLOAD) {
            sr = esize[r];
            Wr = tr_mask_words(sr);
            mb = mptr[r];
            rb = eptr[r];
        }
        for (int64_t q0 = b0; q0 < e; q0 += kWave) {
            const int64_t q = q0 + lane;
            const bool valid = q < e;
            const int nvalid = (int)min<int64_t>(e - q0, (int64_t)kWave);
            uint32_t ent = 0, bkt = 0xFFFFFFFFu;
            if (valid) {
                ent = fadj[q];
                bkt = (ent >> wbits) >> shift;
            }
            int len = 0;
            const int h = run_head(bkt, valid, lane, nvalid, &len);
            uint32_t base = 0;
            if (valid && h == lane) base = atomicAdd(&sh[bkt], (uint32_t)len);
            base = __shfl(base, h, kWave);
            if (valid) {
                const uint32_t pos = base + (uint32_t)(lane - h);
                const uint32_t j = ent >> wbits;
                tj[pos] = (uint16_t)(j & lmask);
                if (PAYLOAD) {
                    const uint32_t om = ent & wmask;
                    uint32_t v = kInNoVertex;
                    if (om == 1u && Wr > 0) {
                        const int64_t mo = mb + (q - b0) * Wr;
                        for (int w = 0; w < Wr; w++) {
                            const uint32_t x = fmask[mo + w];
                            if (x) v = (uint32_t)emem[rb + w * 32 + __ffs(x) - 1];
                        }
                    }
                    te[pos] = make_uint4((uint32_t)q, ((uint32_t)(e - q - 1) << wbits) | om, v,
                                         ((uint32_t)r << wbits) | (uint32_t)sr);
                }
            }
        }
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// chunk c of the bucketed entries: its bucket and range [lo, hi)
__device__ __forceinline__ bool chunk_range(int c, const uint32_t *cst, int nb, const uint32_t *bo, uint32_t chunk,
                                            int *bucket, uint32_t *lo, uint32_t *hi) {
    if ((uint32_t)c >= cst[nb]) return false;
    int a = 0, z = nb;  // last bucket with cst[b] <= c
    while (z - a > 1) {
        const int mid = (a + z) >> 1;
        if (cst[mid] <= (uint32_t)c) a = mid;
        else z = mid;
    }
    *bucket = a;
    const uint32_t s = bo[a] + (uint32_t)(c - cst[a]) * chunk;
    const uint32_t e = bo[a + 1];
    *lo = s;
    *hi = e - s > chunk ? s + chunk : e;
    return true;
}

// chunks per bucket (0 for an empty one)
__global__ void k_tr_chunks(const uint32_t *bo, int nb, uint32_t chunk, uint32_t *cst) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
        const uint64_t n = bo[b + 1] - bo[b];
        cst[b] = (uint32_t)((n + chunk - 1) / chunk);
    }
}

// bucket starts from the block runs: bo[b] = off[b * G]; bo[nb] = n
__global__ void k_tr_bucket_starts(const uint32_t *off, int nb, int G, uint32_t n, uint32_t *bo) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nb; b += gridDim.x * blockDim.x)
        bo[b] = b < nb ? off[(int64_t)b * G] : n;
}

// 4: per chunk, LDS counts of its later ends, added to cnt (uint32 or u64)
template <typename C>
__global__ __launch_bounds__(kTrCountBlock) void k_tr_count(const uint16_t *tj, const uint32_t *cst, int nb,
                                                       const uint32_t *bo, uint32_t chunk, int shift, int64_t m,
                                                       C *cnt) {
    extern __shared__ uint32_t sh[];
    int b;
    uint32_t lo, hi;
    if (!chunk_range(blockIdx.x, cst, nb, bo, chunk, &b, &lo, &hi)) return;
    const int width = 1 << shift;
    for (int i = threadIdx.x; i < width; i += blockDim.x) sh[i] = 0;
    __syncthreads();
    for (uint32_t p = lo + threadIdx.x; p < hi; p += blockDim.x) atomicAdd(&sh[tj[p]], 1u);
    __syncthreads();
    const int64_t j0 = (int64_t)b << shift;
    for (int i = threadIdx.x; i < width; i += blockDim.x) {
        const uint32_t c = sh[i];
        if (c && j0 + i < m) atomicAdd(&cnt[j0 + i], (C)c);
    }
}

// 5: per chunk, its share of each later end's in-list range, then every
// entry to its slot
__global__ __launch_bounds__(kTrCountBlock) void k_tr_place(const uint16_t *tj, const uint4 *te, const uint32_t *cst,
                                                       int nb, const uint32_t *bo, int shift, int64_t m,
                                                       const int64_t *iptr, uint32_t *cursor, uint4 *inl,
                                                       unsigned int *bad) {
    extern __shared__ uint32_t sh[];
    int b;
    uint32_t lo, hi;
    if (!chunk_range(blockIdx.x, cst, nb, bo, kChunkPlace, &b, &lo, &hi)) return;
    const int width = 1 << shift;
    for (int i = threadIdx.x; i < width; i += blockDim.x) sh[i] = 0;
    __syncthreads();
    for (uint32_t p = lo + threadIdx.x; p < hi; p += blockDim.x) atomicAdd(&sh[tj[p]], 1u);
    __syncthreads();
    const int64_t j0 = (int64_t)b << shift;
    for (int i = threadIdx.x; i < width; i += blockDim.x) {
        const uint32_t c = sh[i];
        if (c) {
            if (j0 + i < m) {
                sh[i] = (uint32_t)iptr[j0 + i] + atomicAdd(&cursor[j0 + i], c);
            } else {
                atomicOr(bad, 1u);
                sh[i] = 0;
            }
        }
    }
    __syncthreads();
    // the chunk's offsets and entries are not read again: non-temporal loads (the kernel ran
    // about 4% faster with them than with plain loads, at the same HBM traffic and L2 hit rate)
    for (uint32_t p = lo + threadIdx.x; p < hi; p += blockDim.x) {
        const uint16_t jl = __builtin_nontemporal_load(tj + p);
        const int64_t j = j0 + jl;
        if (j >= m) continue;
        const uint32_t slot = atomicAdd(&sh[jl], 1u);
        if ((int64_t)slot < iptr[j + 1]) {
            const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(te + p));
            inl[slot] = make_uint4(x.x, x.y, x.z, x.w);
        } else {
            atomicOr(bad, 1u);
        }
    }
}

// steps 1-3 and the chunk table; returns the chunk count (host)
struct Bucketed {
    Buckets bk;
    int G = 0;
    DBuf<uint32_t> bo, cst_count, cst_place;
    DBuf<uint16_t> tj;
    DBuf<uint4> te;
    uint32_t ncount = 0, nplace = 0;   // grid bounds: at most one partial chunk per bucket
    uint32_t chunk_count = kChunkCountMax;
};

// entries per counting block: about n / 1024, a power of two in [4096, 262144]
uint32_t count_chunk(int64_t n) {
    uint32_t c = kChunkCountMin;
    while (c < kChunkCountMax && (int64_t)c * 1024 < n) c <<= 1;
    return c;
}

// chunk table: chunks of at most `chunk` entries per bucket, scanned
void chunk_table(Allocator &A, const Bucketed &bw, uint32_t chunk, int64_t n, DBuf<uint32_t> &cst, uint32_t *bound,
                 hipStream_t s) {
    const int nb = (int)bw.bk.nb;
    cst.alloc(A, nb + 1);
    hipLaunchKernelGGL(k_tr_chunks, dim3(grid_for(nb, 256)), dim3(256), 0, s, bw.bo.p, nb, chunk, cst.p);
    HTRI_LAUNCH_CHECK();
    scan_exclusive_u32(A, cst.p, cst.p, nb, cst.p + nb, s);
    *bound = (uint32_t)(nb + n / chunk + 1);
}

template <bool PAYLOAD, bool STATS>
void bucket_hyperwedges(Graph &g, int64_t owner_end, int64_t n, int shift_min, Bucketed &out,
                        unsigned long long *n_incl, unsigned int *max_omega) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    out.bk = buckets_for(g.m, shift_min);
    const int nb = (int)out.bk.nb;
    const int G = (int)grid_for(owner_end * kWave, kTrBlock,
                                std::max<int64_t>(256, std::min<int64_t>(kTrGridMax, (1 << 22) / nb)));
    out.G = G;
    const size_t lds = sizeof(uint32_t) * (size_t)nb;
    DBuf<uint32_t> hist(A, (size_t)nb * G);
    hipLaunchKernelGGL((k_tr_hist<STATS>), dim3(G), dim3(kTrBlock), lds, s, g.fptr.p, g.fadj.p, g.esize.p, owner_end,
                       g.wbits, out.bk.shift, nb, (int)g.min_size, hist.p, n_incl, max_omega);
    HTRI_LAUNCH_CHECK();
    scan_exclusive_u32(A, hist.p, hist.p, (int64_t)nb * G, nullptr, s);
    out.bo.alloc(A, nb + 1);
    hipLaunchKernelGGL(k_tr_bucket_starts, dim3(grid_for(nb + 1, 256)), dim3(256), 0, s, hist.p, nb, G, (uint32_t)n,
                       out.bo.p);
    HTRI_LAUNCH_CHECK();
    out.tj.alloc(A, n);
    if (PAYLOAD) out.te.alloc(A, n);
    hipLaunchKernelGGL((k_tr_scatter<PAYLOAD>), dim3(G), dim3(kTrBlock), lds, s, g.fptr.p, g.fadj.p, owner_end,
                       g.wbits, out.bk.shift, nb, hist.p, g.esize.p, g.eptr.p, g.emem.p, g.mptr.p, g.fmask.p,
                       out.tj.p, out.te.p);
    HTRI_LAUNCH_CHECK();
    hist.reset();
    out.chunk_count = count_chunk(n);
    chunk_table(A, out, out.chunk_count, n, out.cst_count, &out.ncount, s);
    if (PAYLOAD) chunk_table(A, out, kChunkPlace, n, out.cst_place, &out.nplace, s);
}

bool fits_shift(int64_t m, int shift_min) {
    const Buckets b = buckets_for(m, shift_min);
    return b.shift <= kShiftMax && b.nb <= kBucketsMax;
}

}  // namespace

bool transpose_fits(int64_t m, int64_t n) {
    return m > 0 && n > 0 && n < (int64_t)UINT32_MAX && fits_shift(m, kShiftIndeg) && fits_shift(m, kShiftInlist);
}

void count_later_ends(Graph &g, int64_t n, unsigned int *indeg, unsigned long long *n_incl,
                      unsigned int *max_omega) {
    if (!transpose_fits(g.m, n)) fail(HTRI_E_UNSUPPORTED, "later-end transpose beyond its limits");
    Bucketed bw;
    bucket_hyperwedges<false, true>(g, g.m, n, kShiftIndeg, bw, n_incl, max_omega);
    const int nb = (int)bw.bk.nb;
    hipLaunchKernelGGL((k_tr_count<unsigned int>), dim3(bw.ncount), dim3(kTrCountBlock),
                       sizeof(uint32_t) << bw.bk.shift, g.stream, bw.tj.p, bw.cst_count.p, nb, bw.bo.p,
                       bw.chunk_count, bw.bk.shift, g.m, indeg);
    HTRI_LAUNCH_CHECK();
    stream_sync(g.stream);
}

int64_t inlist_bytes(Graph &g, int64_t owner_end) {
    int64_t n = 0;
    if (owner_end > 0) {
        HTRI_HIP(hipMemcpyAsync(&n, g.fptr.p + owner_end, sizeof(int64_t), hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
    }
    // the entries twice (bucketed, then placed), the bucket offsets, the
    // counts, offsets and cursors, the item counts
    return n * 34 + (g.m + 1) * 60 + (int64_t)buckets_for(g.m, kShiftInlist).nb * 2048 * 4;
}

// The in-list for owners below owner_end.
void build_inlist(Graph &g, int64_t owner_end, InList &out) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    int64_t n = 0;
    if (owner_end > 0) {
        HTRI_HIP(hipMemcpyAsync(&n, g.fptr.p + owner_end, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HTRI_HIP(hipStreamSynchronize(s));
    }
    if (2 * g.wbits > 32) fail(HTRI_E_UNSUPPORTED, "in-list packing needs hyperedge sizes below 2^16");
    out.n = n;
    out.iptr.alloc(A, m + 1);
    if (n == 0) {
        fill_u64((uint64_t *)out.iptr.p, m + 1, 0, s);
        out.inl.alloc(A, 0);
        stream_sync(s);
        return;
    }
    if (!transpose_fits(m, n)) fail(HTRI_E_UNSUPPORTED, "in-list beyond the transpose's limits");
    Bucketed bw;
    bucket_hyperwedges<true, false>(g, owner_end, n, kShiftInlist, bw, nullptr, nullptr);
    const int nb = (int)bw.bk.nb;
    const size_t lds = sizeof(uint32_t) << bw.bk.shift;
    {
        DBuf<unsigned long long> cnt(A, m + 1);
        fill_u64((uint64_t *)cnt.p, m + 1, 0, s);
        hipLaunchKernelGGL((k_tr_count<unsigned long long>), dim3(bw.ncount), dim3(kTrCountBlock), lds, s, bw.tj.p,
                           bw.cst_count.p, nb, bw.bo.p, bw.chunk_count, bw.bk.shift, m, cnt.p);
        HTRI_LAUNCH_CHECK();
        scan_exclusive_i64(A, (const int64_t *)cnt.p, out.iptr.p, m, out.iptr.p + m, s);
    }
    int64_t total = 0;
    HTRI_HIP(hipMemcpyAsync(&total, out.iptr.p + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    if (total != n) fail(HTRI_E_DEVICE, "in-list counts do not add up to the hyperwedges");
    out.inl.alloc(A, n);
    DBuf<uint32_t> cursor(A, m);
    DBuf<unsigned int> bad(A, 1);
    fill_u32(cursor.p, m, 0, s);
    fill_u32(bad.p, 1, 0, s);
    hipLaunchKernelGGL(k_tr_place, dim3(bw.nplace), dim3(kTrCountBlock), lds, s, bw.tj.p, bw.te.p, bw.cst_place.p, nb,
                       bw.bo.p, bw.bk.shift, m, out.iptr.p, cursor.p, out.inl.p, bad.p);
    HTRI_LAUNCH_CHECK();
    unsigned int hb = 0;
    HTRI_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(hb), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    if (hb) fail(HTRI_E_DEVICE, "in-list slot outside its middle's range");
}

}  // namespace htri
