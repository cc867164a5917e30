// Hyperwedge sampling (Algorithm 6 with sigma = 1; unbiased by Lemma 4.1)
// and its importance-sampling form with a learned proposal.
//
// A drawn hyperwedge (r, j) is closed exactly like in the exact count: the
// third hyperedges k after j that lie in N+(r) and N+(j).  One wave closes
// one sample by a tile merge of the two sorted lists (64 entries of each per
// step, membership found by a 6-step shuffle search inside the other tile);
// per-pattern counts are aggregated across the wave and kept in the lane
// whose index is the pattern.  Samples are assigned to waves round-robin so
// that every floating-point sum has a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"
#include "philox.hpp"

namespace htri {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaskWordsMax = 4;

__host__ __device__ __forceinline__ int mask_words(int size) {
    return size <= 32 * kMaskWordsMax ? (size + 31) / 32 : 0;
}

__device__ int triple_common_s(const int64_t *eptr, const int32_t *emem, int32_t r, int32_t j, int32_t k) {
    int64_t a = eptr[r], ae = eptr[r + 1], b = eptr[j], be = eptr[j + 1], c = eptr[k], ce = eptr[k + 1];
    int cnt = 0;
    while (a < ae && b < be && c < ce) {
        int32_t x = emem[a], y = emem[b], z = emem[c];
        if (x == y && y == z) { cnt++; a++; b++; c++; continue; }
        int32_t mx = x > y ? x : y;
        mx = mx > z ? mx : z;
        if (x < mx) a++;
        if (y < mx) b++;
        if (z < mx) c++;
    }
    return cnt;
}

__device__ __forceinline__ uint32_t region_mask_s(int si, int sj, int sk, int wij, int wik, int wjk, int g) {
    int a = si - wij - wik + g, b = sj - wij - wjk + g, c = sk - wik - wjk + g;
    int d = wij - g, e = wjk - g, f = wik - g;
    return (uint32_t)(a > 0) | ((uint32_t)(b > 0) << 1) | ((uint32_t)(c > 0) << 2) | ((uint32_t)(d > 0) << 3) |
           ((uint32_t)(e > 0) << 4) | ((uint32_t)(f > 0) << 5) | ((uint32_t)(g > 0) << 6);
}

struct SampleArgs {
    const int64_t *fptr;
    const uint32_t *fadj;
    const int64_t *mptr;
    const uint32_t *fmask;
    const int32_t *esize;
    const int64_t *eptr;
    const int32_t *emem;
    int64_t m;
    int64_t nw;
    int wbits;
    const uint8_t *lut;
    int64_t n;                  // samples
    // mode 0: explicit wedge list, per-sample counts out
    const int64_t *idx;
    int64_t *out_counts;        // n x 21
    // mode 1: uniform draws (Philox stream 0); mode 2: pool draws by CDF
    uint64_t seed;
    const int64_t *pool;        // pool index -> wedge
    const double *cdf;          // inclusive CDF over the pool
    int64_t pool_n;
    double scale;               // multiplies every closure (mode 1: |wedges|; mode 2: |wedges|/pool)
    int skip_inclusion;         // drawn inclusion hyperwedges close nothing (their stratum is exact)
    // mode 3: draws from one hyperwedge type (Philox stream cls_stream): the
    // cls_n inclusion hyperwedges at the sorted positions cls_pos (cls_kind
    // 1), or the intersection ones, every other position (cls_kind 0); only
    // the patterns in keep_mask are counted
    const int64_t *cls_pos;
    int64_t cls_npos;           // number of inclusion positions in cls_pos
    int64_t cls_n;              // size of the drawn type's list
    int cls_kind;
    uint32_t cls_stream;
    uint32_t keep_mask;
    // accumulation: per wave [21] x (int64 sum c, double sum y, double sum y^2)
    long long *acc_c;
    double *acc_y;
    double *acc_y2;
};

// owner of wedge e: largest r with fptr[r] <= e
__device__ __forceinline__ int64_t owner_of(const int64_t *fptr, int64_t m, int64_t e) {
    int64_t lo = 0, hi = m;  // answer in [0, m-1]
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (fptr[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// Close wedge e (global index into the forward adjacency).  Returns, in lane
// p (1..20), the number of closing third hyperedges of pattern p and, in lane
// 0, their total; other lanes return 0.
// on_hit(r, j, k, pattern) is called by each lane that finds a third
// hyperedge k (ranks).
template <typename OnHit>
__device__ long long wave_close_f(const SampleArgs &A, const uint8_t *lut, int64_t e, const OnHit &on_hit) {
    const int lane = __lane_id();
    const uint32_t wmask = (1u << A.wbits) - 1;
    const int64_t r = owner_of(A.fptr, A.m, e);
    const int64_t rb = A.fptr[r];
    const int64_t pos = e - rb;
    const uint32_t jent = A.fadj[e];
    const uint32_t j = jent >> A.wbits;
    const int wrj = (int)(jent & wmask);
    const int si = A.esize[r], sj = A.esize[j];
    if (A.skip_inclusion && wrj == (si < sj ? si : sj)) return 0;
    const int W = mask_words(si);
    const int64_t mbase = A.mptr[r];
    uint32_t mj[kMaskWordsMax];
#pragma unroll
    for (int w = 0; w < kMaskWordsMax; w++) mj[w] = w < W ? A.fmask[mbase + pos * W + w] : 0u;

    int64_t a0 = e + 1, a1 = A.fptr[r + 1];         // N+(r) after j
    int64_t b0 = A.fptr[j], b1 = A.fptr[j + 1];     // N+(j)
    long long cnt = 0;
    while (a0 < a1 && b0 < b1) {
        const int64_t ia = a0 + lane, ib = b0 + lane;
        const bool va = ia < a1, vb = ib < b1;
        const uint32_t ae = va ? A.fadj[ia] : 0u;
        const uint32_t be = vb ? A.fadj[ib] : 0u;
        const uint32_t ak = va ? (ae >> A.wbits) : 0xFFFFFFFFu;
        const uint32_t bk = vb ? (be >> A.wbits) : 0xFFFFFFFFu;
        // position of ak among the b tile: number of b keys < ak
        int p = 0;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            uint32_t v = __shfl(bk, p + s - 1, kWave);
            if (v < ak) p += s;
        }
        const int pc = p < kWave ? p : kWave - 1;
        const uint32_t bk_at = __shfl(bk, pc, kWave);
        const uint32_t be_at = __shfl(be, pc, kWave);
        const bool hit = va && p < kWave && bk_at == ak;
        int pat = 0;
        if (hit) {
            const uint32_t k = ak;
            const int wrk = (int)(ae & wmask);
            const int wjk = (int)(be_at & wmask);
            const int sk = A.esize[k];
            int g;
            if (W > 0) {
                const int64_t posk = ia - rb;
                g = 0;
#pragma unroll
                for (int w = 0; w < kMaskWordsMax; w++)
                    if (w < W) g += __popc(mj[w] & A.fmask[mbase + posk * W + w]);
            } else {
                g = triple_common_s(A.eptr, A.emem, (int32_t)r, (int32_t)j, (int32_t)k);
            }
            pat = lut[region_mask_s(si, sj, sk, wrj, wrk, wjk, g)];
            on_hit((int32_t)r, (int32_t)j, (int32_t)k, pat);
        }
        uint64_t pend = __ballot(hit);
        if (lane == 0) cnt += __popcll(pend);
        while (pend) {
            const int src = __ffsll((unsigned long long)pend) - 1;
            const int p0 = __shfl(pat, src, kWave);
            const uint64_t mm = __ballot(hit && pat == p0);
            if (lane == p0) cnt += __popcll(mm);
            pend &= ~mm;
        }
        // advance the tile whose largest key is smaller (both if equal)
        const int la = (int)((a1 - a0) < kWave ? (a1 - a0) : kWave) - 1;
        const int lb = (int)((b1 - b0) < kWave ? (b1 - b0) : kWave) - 1;
        const uint32_t amax = __shfl(ak, la, kWave);
        const uint32_t bmax = __shfl(bk, lb, kWave);
        if (amax <= bmax) a0 += kWave;
        if (bmax <= amax) b0 += kWave;
    }
    return cnt;
}

__device__ __forceinline__ long long wave_close(const SampleArgs &A, const uint8_t *lut, int64_t e) {
    return wave_close_f(A, lut, e, [](int32_t, int32_t, int32_t, int) {});
}

// Every hyperwedge closed by one wave; the hyper-triangles of pattern
// `target` are written as sorted triples of normalised ids while room lasts
// (found counts them all).
__global__ __launch_bounds__(kBlock) void k_enumerate(SampleArgs A, int target, const int32_t *norm_of_rank,
                                                      int64_t capacity, int32_t *out,
                                                      unsigned long long *found) {
    __shared__ uint8_t lut[128];
    if (threadIdx.x < 128) lut[threadIdx.x] = A.lut[threadIdx.x];
    __syncthreads();
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    auto emit = [&](int32_t r, int32_t j, int32_t k, int pat) {
        if (pat != target) return;
        const unsigned long long at = atomicAdd(found, 1ull);
        if ((int64_t)at < capacity) {
            int32_t a = norm_of_rank[r], b = norm_of_rank[j], c = norm_of_rank[k];
            if (a > b) { const int32_t x = a; a = b; b = x; }
            if (b > c) { const int32_t x = b; b = c; c = x; }
            if (a > b) { const int32_t x = a; a = b; b = x; }
            out[at * 3 + 0] = a;
            out[at * 3 + 1] = b;
            out[at * 3 + 2] = c;
        }
    };
    for (int64_t e = wave; e < A.nw; e += nwaves) (void)wave_close_f(A, lut, e, emit);
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_sample_close(SampleArgs A) {
    __shared__ uint8_t lut[128];
    if (threadIdx.x < 128) lut[threadIdx.x] = A.lut[threadIdx.x];
    __syncthreads();
    const int lane = __lane_id();
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    long long sc = 0;
    double sy = 0, sy2 = 0;
    for (int64_t t = wave; t < A.n; t += nwaves) {
        int64_t e;
        double wgt = A.scale;
        if (MODE == 0) {
            e = A.idx[t];
        } else if (MODE == 1) {
            e = (int64_t)philox_index(A.seed, 0u, (uint64_t)t, (uint64_t)A.nw);
        } else if (MODE == 3) {
            const int64_t u = (int64_t)philox_index(A.seed, A.cls_stream, (uint64_t)t, (uint64_t)A.cls_n);
            if (A.cls_kind == 1) {
                e = A.cls_pos[u];
            } else {
                // the u-th position that holds no inclusion hyperwedge: u plus
                // the number of inclusion positions p_i with p_i - i <= u
                int64_t lo = 0, hi = A.cls_npos;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (A.cls_pos[mid] - mid <= u) lo = mid + 1; else hi = mid;
                }
                e = u + lo;
            }
        } else {
            // inverse CDF over the pool: first u with cdf[u] > U * total
            const double total = A.cdf[A.pool_n - 1];
            const double U = philox_unit(A.seed, 2u, (uint64_t)t) * total;
            int64_t lo = 0, hi = A.pool_n - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (A.cdf[mid] > U) hi = mid; else lo = mid + 1;
            }
            const double q = (A.cdf[lo] - (lo > 0 ? A.cdf[lo - 1] : 0.0)) / total;
            e = A.pool ? A.pool[lo] : lo;
            wgt = A.scale / q;
        }
        long long c = wave_close(A, lut, e);
        if (MODE == 3) c = ((A.keep_mask >> lane) & 1u) ? c : 0;
        if (MODE == 0) {
            if (lane < 21) A.out_counts[t * 21 + lane] = c;
        } else {
            sc += c;
            const double y = (double)c * wgt;
            sy += y;
            sy2 += y * y;
        }
    }
    if (MODE != 0 && lane < 21) {
        A.acc_c[wave * 21 + lane] = sc;
        A.acc_y[wave * 21 + lane] = sy;
        A.acc_y2[wave * 21 + lane] = sy2;
    }
}

// Fixed-order reduction of the per-wave accumulators: block p reduces
// pattern p; thread t sums waves t, t + 256, ... in order, then the block
// adds the 256 partial sums pairwise in a fixed tree.
constexpr int kReduceThreads = 256;
__global__ __launch_bounds__(kReduceThreads) void k_sample_reduce(const long long *acc_c, const double *acc_y,
                                                                  const double *acc_y2, int64_t nwaves, long long *c,
                                                                  double *y, double *y2) {
    __shared__ long long sc[kReduceThreads];
    __shared__ double sy[kReduceThreads], sy2[kReduceThreads];
    const int p = blockIdx.x, t = threadIdx.x;
    long long s = 0;
    double a = 0, b = 0;
    for (int64_t w = t; w < nwaves; w += kReduceThreads) {
        s += acc_c[w * 21 + p];
        a += acc_y[w * 21 + p];
        b += acc_y2[w * 21 + p];
    }
    sc[t] = s;
    sy[t] = a;
    sy2[t] = b;
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
            sc[t] += sc[t + o];
            sy[t] += sy[t + o];
            sy2[t] += sy2[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        c[p] = sc[0];
        y[p] = sy[0];
        y2[p] = sy2[0];
    }
}

// Training target of the learned proposal for every hyperwedge e:
// log1p(sqrt(sum_p (c_p(e) * scale[p])^2) / live), c_p(e) the forward closure
// of e in pattern p, scale[p] = |wedges| / H_p for the patterns present (0
// otherwise); scale[0] weighs the total closure (0: left out).  One wave per
// hyperwedge.
__global__ __launch_bounds__(kBlock) void k_wedge_importance(SampleArgs A, const double *scale, double live,
                                                             float *out) {
    __shared__ uint8_t lut[128];
    if (threadIdx.x < 128) lut[threadIdx.x] = A.lut[threadIdx.x];
    __syncthreads();
    const int lane = __lane_id();
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    const double sc = lane < 21 ? scale[lane] : 0.0;
    for (int64_t e = wave; e < A.nw; e += nwaves) {
        const long long c = wave_close(A, lut, e);
        double y = (double)c * sc;
        y = y * y;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) y += __shfl_xor(y, o, kWave);
        if (lane == 0) out[e] = (float)log1p(sqrt(y) / live);
    }
}

__global__ void k_pool_draw(uint64_t seed, int64_t pool_n, int64_t nw, int64_t *pool) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < pool_n;
         u += (int64_t)gridDim.x * blockDim.x)
        pool[u] = (int64_t)philox_index(seed, 1u, (uint64_t)u, (uint64_t)nw);
}

int sample_grid() { return device_cu_count() * 8; }

SampleArgs base_args(Graph &g, const uint8_t *lut) {
    SampleArgs a{};
    a.fptr = g.fptr.p;
    a.fadj = g.fadj.p;
    a.mptr = g.mptr.p;
    a.fmask = g.fmask.p;
    a.esize = g.esize.p;
    a.eptr = g.eptr.p;
    a.emem = g.emem.p;
    a.m = g.m;
    a.nw = g.nw;
    a.wbits = g.wbits;
    a.lut = lut;
    return a;
}

}  // namespace

void close_wedge_list_counts(Graph &g, const int64_t *dev_idx, int64_t n, int64_t *dev_out) {
    if (n <= 0) return;
    hipStream_t s = g.stream;
    DBuf<uint8_t> lut(g.al, 128);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    SampleArgs a = base_args(g, lut.p);
    a.n = n;
    a.idx = dev_idx;
    a.out_counts = dev_out;
    int grid = (int)std::min<int64_t>(sample_grid(), (n + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(k_sample_close<0>, dim3(std::max(grid, 1)), dim3(kBlock), 0, s, a);
    HTRI_LAUNCH_CHECK();
    HTRI_HIP(hipStreamSynchronize(s));
}

void enumerate_all_wedges(Graph &g, int target, int64_t capacity, int32_t *dev_out, unsigned long long *dev_found) {
    if (g.nw <= 0) return;
    hipStream_t s = g.stream;
    DBuf<uint8_t> lut(g.al, 128);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    SampleArgs a = base_args(g, lut.p);
    const int grid = (int)std::min<int64_t>(sample_grid(), (g.nw + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(k_enumerate, dim3(std::max(grid, 1)), dim3(kBlock), 0, s, a, target, g.norm_of_rank.p,
                       capacity, dev_out, dev_found);
    HTRI_LAUNCH_CHECK();
    HTRI_HIP(hipStreamSynchronize(s));
}

namespace {

// Launch the sampling closure and the fixed-order reduction of its per-wave
// sums into dc / dy / dy2 (21 each); the per-wave buffers hold
// grid * kWavesPerBlock * 21 entries.
void launch_sample_sums(Graph &g, int mode, int grid, int64_t n, uint64_t seed, const int64_t *pool,
                        const double *cdf, int64_t pool_n, double scale, bool skip_inclusion, const uint8_t *lut,
                        long long *ac, double *ay, double *ay2, long long *dc, double *dy, double *dy2) {
    hipStream_t s = g.stream;
    const int64_t nwaves = (int64_t)grid * kWavesPerBlock;
    SampleArgs a = base_args(g, lut);
    a.n = n;
    a.seed = seed;
    a.pool = pool;
    a.cdf = cdf;
    a.pool_n = pool_n;
    a.scale = scale;
    a.skip_inclusion = skip_inclusion ? 1 : 0;
    a.acc_c = ac;
    a.acc_y = ay;
    a.acc_y2 = ay2;
    if (mode == 1)
        hipLaunchKernelGGL(k_sample_close<1>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_sample_close<2>, dim3(grid), dim3(kBlock), 0, s, a);
    HTRI_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sample_reduce, dim3(21), dim3(kReduceThreads), 0, s, ac, ay, ay2, nwaves, dc, dy, dy2);
    HTRI_LAUNCH_CHECK();
}

}  // namespace

// Weighted closure sums over n draws.  mode 1: uniform (scale = |wedges|);
// mode 2: from a pool by its CDF (scale = |wedges| / pool size).
void sample_sums(Graph &g, int mode, int64_t n, uint64_t seed, const int64_t *pool, const double *cdf,
                 int64_t pool_n, double scale, long long c[21], double y[21], double y2[21], bool skip_inclusion) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    DBuf<uint8_t> lut(A, 128);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    const int grid = std::max(1, sample_grid());
    const int64_t nwaves = (int64_t)grid * kWavesPerBlock;
    DBuf<long long> ac(A, nwaves * 21);
    DBuf<double> ay(A, nwaves * 21), ay2(A, nwaves * 21);
    DBuf<long long> dc(A, 21);
    DBuf<double> dy(A, 21), dy2(A, 21);
    launch_sample_sums(g, mode, grid, n, seed, pool, cdf, pool_n, scale, skip_inclusion, lut.p, ac.p, ay.p, ay2.p,
                       dc.p, dy.p, dy2.p);
    HTRI_HIP(hipMemcpyAsync(c, dc.p, sizeof(long long) * 21, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipMemcpyAsync(y, dy.p, sizeof(double) * 21, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipMemcpyAsync(y2, dy2.p, sizeof(double) * 21, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
}

void wedge_importance_all(Graph &g, const double scale[21], double live, float *dev_out) {
    if (g.nw <= 0) return;
    hipStream_t s = g.stream;
    DBuf<uint8_t> lut(g.al, 128);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    DBuf<double> sc(g.al, 21);
    HTRI_HIP(hipMemcpyAsync(sc.p, scale, sizeof(double) * 21, hipMemcpyHostToDevice, s));
    SampleArgs a = base_args(g, lut.p);
    const int grid = (int)std::min<int64_t>(sample_grid(), (g.nw + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(k_wedge_importance, dim3(std::max(grid, 1)), dim3(kBlock), 0, s, a, sc.p, live, dev_out);
    HTRI_LAUNCH_CHECK();
    HTRI_HIP(hipStreamSynchronize(s));
}

// Closure sums over n draws from one hyperwedge type (Appro-adv): kind 1
// the inclusion list (sorted positions inc_pos, n_inc of them), kind 0 the
// intersection list (every other position); Philox stream `stream`; only the
// patterns of keep_mask are summed; every closure weighs list_size.
void class_sample_sums(Graph &g, int kind, int64_t n, uint64_t seed, uint32_t stream, const int64_t *inc_pos,
                       int64_t n_inc, int64_t list_size, uint32_t keep_mask, long long c[21], double y[21],
                       double y2[21]) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    DBuf<uint8_t> lut(A, 128);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    const int grid = std::max(1, sample_grid());
    const int64_t nwaves = (int64_t)grid * kWavesPerBlock;
    DBuf<long long> ac(A, nwaves * 21);
    DBuf<double> ay(A, nwaves * 21), ay2(A, nwaves * 21);
    DBuf<long long> dc(A, 21);
    DBuf<double> dy(A, 21), dy2(A, 21);
    SampleArgs a = base_args(g, lut.p);
    a.n = n;
    a.seed = seed;
    a.scale = (double)list_size;
    a.cls_pos = inc_pos;
    a.cls_npos = n_inc;
    a.cls_n = list_size;
    a.cls_kind = kind;
    a.cls_stream = stream;
    a.keep_mask = keep_mask;
    a.acc_c = ac.p;
    a.acc_y = ay.p;
    a.acc_y2 = ay2.p;
    hipLaunchKernelGGL(k_sample_close<3>, dim3(grid), dim3(kBlock), 0, s, a);
    HTRI_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sample_reduce, dim3(21), dim3(kReduceThreads), 0, s, ac.p, ay.p, ay2.p, nwaves, dc.p, dy.p,
                       dy2.p);
    HTRI_LAUNCH_CHECK();
    HTRI_HIP(hipMemcpyAsync(c, dc.p, sizeof(long long) * 21, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipMemcpyAsync(y, dy.p, sizeof(double) * 21, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipMemcpyAsync(y2, dy2.p, sizeof(double) * 21, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
}

void draw_pool(Graph &g, uint64_t seed, int64_t pool_n, int64_t *dev_pool) {
    if (pool_n <= 0) return;
    hipLaunchKernelGGL(k_pool_draw, dim3(grid_for(pool_n, 256, 8192)), dim3(256), 0, g.stream, seed, pool_n, g.nw,
                       dev_pool);
    HTRI_LAUNCH_CHECK();
}

}  // namespace htri

// ---------------------------------------------------------------- no-allocation uniform estimate
//
// htri_estimate_uniform_noalloc keeps every intermediate buffer of the
// uniform estimate (the pattern table, the per-wave partial sums and their
// reduction) in one file-scope device array instead of allocating.  The
// host code never passes the array's name to a kernel: it looks the array's
// device address up once per device (hipGetSymbolAddress) and passes that.

namespace htri {
namespace {

constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr size_t kScratchLutOff = 0;          // 128 B pattern table
constexpr size_t kScratchSumOff = 256;        // 21 x (int64 c, double y, double y2)
constexpr size_t kScratchWaveOff = 4096;      // per-wave sums, 3 x nwaves x 21 x 8 B

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
unsigned char *scratch_on_device() {
    int dev = 0;
    HTRI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(HTRI_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HTRI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) fail(HTRI_E_DEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    return (unsigned char *)g_scratch_ptr[dev];
}

struct LutArg {
    uint8_t v[128];
};

__global__ void k_put_lut(LutArg t, uint8_t *dst) {
    if (threadIdx.x < 128) dst[threadIdx.x] = t.v[threadIdx.x];
}

// est_q = c_q |wedges| / n and its standard error, as htri_estimate forms them
__global__ void k_uniform_finish(const long long *c, const double *y, const double *y2, int64_t n, int64_t nw,
                                 double *est, double *se) {
    const int q = threadIdx.x;
    if (q >= 21) return;
    if (n <= 0 || nw <= 0) {
        est[q] = 0.0;
        if (se) se[q] = 0.0;
        return;
    }
    const double e = (double)c[q] * (double)nw / (double)n;
    est[q] = e;
    if (se) {
        const double nn = (double)n, ne = nn * e;
        const double var = (y2[q] - ne * e) / (nn * (double)(n > 1 ? n - 1 : 1));
        se[q] = sqrt(var > 0.0 ? var : 0.0);
    }
}

}  // namespace

}  // namespace htri

using namespace htri;

extern "C" htri_status htri_estimate_uniform_noalloc(htri_graph *h, int64_t num_samples, uint64_t seed,
                                                     double *dev_est, double *dev_stderr) {
    if (!h || !dev_est || num_samples < 1) return HTRI_E_INVALID;
    if (!h->g.have_wedges) {
        h->g.err = "htri_build_wedges has not run";
        return HTRI_E_STATE;
    }
    try {
        Graph &g = h->g;
        hipStream_t s = g.stream;
        unsigned char *base = scratch_on_device();
        const int grid = std::max(1, sample_grid());
        const int64_t nwaves = (int64_t)grid * kWavesPerBlock;
        const size_t need = kScratchWaveOff + (size_t)3 * (size_t)nwaves * 21 * 8;
        if (need > kScratchBytes) {
            g.err = "this device needs " + std::to_string(need) + " bytes of sampling scratch; the static buffer holds " +
                    std::to_string(kScratchBytes);
            return HTRI_E_UNSUPPORTED;
        }
        uint8_t *lut = base + kScratchLutOff;
        long long *dc = (long long *)(base + kScratchSumOff);
        double *dy = (double *)(base + kScratchSumOff + 21 * 8);
        double *dy2 = (double *)(base + kScratchSumOff + 42 * 8);
        long long *ac = (long long *)(base + kScratchWaveOff);
        double *ay = (double *)(base + kScratchWaveOff + (size_t)nwaves * 21 * 8);
        double *ay2 = (double *)(base + kScratchWaveOff + (size_t)2 * nwaves * 21 * 8);
        if (g.nw > 0) {
            LutArg t;
            std::memcpy(t.v, pattern_lut(), 128);
            hipLaunchKernelGGL(k_put_lut, dim3(1), dim3(128), 0, s, t, lut);
            HTRI_LAUNCH_CHECK();
            // every wave writes its own partial sums, so nothing needs clearing
            launch_sample_sums(g, 1, grid, num_samples, seed, nullptr, nullptr, 0, (double)g.nw, false, lut, ac, ay,
                               ay2, dc, dy, dy2);
        }
        hipLaunchKernelGGL(k_uniform_finish, dim3(1), dim3(64), 0, s, dc, dy, dy2, g.nw > 0 ? num_samples : 0, g.nw,
                           dev_est, dev_stderr);
        HTRI_LAUNCH_CHECK();
        return HTRI_OK;
    } catch (const htri::Error &e) {
        h->g.err = e.msg;
        return e.code;
    }
}
