// Appro-adv (Algorithm 7, Section 4.2): hyperwedge sampling split by
// hyperwedge type.  A budget of alpha draws is divided by the type counts
// |T| (intersection) and |C| (inclusion): alpha1 = |T|^2 alpha / |W|^2
// draws from T estimate the class with three intersection hyperwedges
// (TTT, patterns 9-20), alpha2 = |C|^2 alpha / |W|^2 draws from C the class
// with three inclusion hyperwedges (CCC, pattern 1), and alpha3 = alpha4 =
// |T| |C| alpha / |W|^2 draws from T and from C the two mixed classes
// (TTC, patterns 6-8, two intersection hyperwedges; TCC, patterns 2-5, two
// inclusion hyperwedges).  Each draw counts the hyper-triangles of its class
// attributed to it -- the one whose earliest hyperwedge (in the hyperwedge
// order over rank pairs) of the drawn type it is -- so every class total is
// the mean over its draws times the size of the drawn type's list.
//
// TTT and CCC draws reuse the sampler's forward closure (a triangle's
// earliest hyperwedge is the one the forward closure attributes it to).
// TTC and TCC draws look only at the third hyperedges k joined to an end of
// the drawn hyperwedge by an inclusion hyperwedge: those lists are short
// (inclusion hyperwedges are rare), and every mixed triangle has one.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "philox.hpp"

namespace htri {
namespace {

constexpr int kAdvBlock = 256;

__device__ __forceinline__ int64_t owner_of_a(const int64_t *fptr, int64_t m, int64_t e) {
    int64_t lo = 0, hi = m;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (fptr[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// both ends (ranks) of the inclusion hyperwedges at the listed positions
__global__ void k_incl_ends(const int64_t *fptr, const uint32_t *fadj, int64_t m, int wbits, const int64_t *pos,
                            int64_t n, int2 *ends) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = pos[t];
        ends[t] = make_int2((int)owner_of_a(fptr, m, e), (int)(fadj[e] >> wbits));
    }
}

__device__ __forceinline__ int common2(const int64_t *eptr, const int32_t *emem, int32_t a, int32_t b) {
    int64_t x = eptr[a], xe = eptr[a + 1], y = eptr[b], ye = eptr[b + 1];
    int c = 0;
    while (x < xe && y < ye) {
        const int32_t u = emem[x], v = emem[y];
        if (u == v) {
            c++;
            x++;
            y++;
        } else if (u < v) {
            x++;
        } else {
            y++;
        }
    }
    return c;
}

__device__ __forceinline__ int common3(const int64_t *eptr, const int32_t *emem, int32_t a, int32_t b, int32_t k) {
    int64_t x = eptr[a], xe = eptr[a + 1], y = eptr[b], ye = eptr[b + 1], z = eptr[k], ze = eptr[k + 1];
    int c = 0;
    while (x < xe && y < ye && z < ze) {
        const int32_t u = emem[x], v = emem[y], w = emem[z];
        if (u == v && v == w) {
            c++;
            x++;
            y++;
            z++;
            continue;
        }
        const int32_t mx = max(u, max(v, w));
        if (u < mx) x++;
        if (v < mx) y++;
        if (w < mx) z++;
    }
    return c;
}

__device__ __forceinline__ uint32_t region_bits(int si, int sj, int sk, int wij, int wik, int wjk, int g) {
    const int a = si - wij - wik + g, b = sj - wij - wjk + g, c = sk - wik - wjk + g;
    const int d = wij - g, e = wjk - g, f = wik - g;
    return (uint32_t)(a > 0) | ((uint32_t)(b > 0) << 1) | ((uint32_t)(c > 0) << 2) | ((uint32_t)(d > 0) << 3) |
           ((uint32_t)(e > 0) << 4) | ((uint32_t)(f > 0) << 5) | ((uint32_t)(g > 0) << 6);
}

// first pair whose end is x (pairs sorted by end, then partner)
__device__ __forceinline__ int64_t first_pair(const int2 *pairs, int64_t n, int32_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (pairs[mid].x < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool has_pair(const int2 *pairs, int64_t n, int32_t x, int32_t y) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int2 p = pairs[mid];
        if (p.x < x || (p.x == x && p.y < y)) lo = mid + 1; else hi = mid;
    }
    return lo < n && pairs[lo].x == x && pairs[lo].y == y;
}

struct CrossArgs {
    const int64_t *fptr;
    const uint32_t *fadj;
    const int64_t *eptr;
    const int32_t *emem;
    const int32_t *esize;
    int64_t m;
    int wbits;
    const uint8_t *lut;
    const int64_t *inc_pos;   // sorted positions of the inclusion hyperwedges
    int64_t n_inc;
    const int2 *pairs;        // (end, other end) of every inclusion hyperwedge, both ways, sorted
    int64_t npairs;
    int kind;                 // 0: draws from T for TTC (patterns 6-8); 1: draws from C for TCC (2-5)
    int64_t list_size;        // |T| or |C|
    uint64_t seed;
    uint32_t stream;
    int64_t n;                // draws
    long long *part;          // per block: 4 sums of counts, then 4 sums of squared counts
};

// One thread per draw.  The drawn hyperwedge (r, j), r earlier than j; a
// third hyperedge k joined to r or j by an inclusion hyperwedge.  TTC from
// an intersection hyperwedge: k is joined to exactly one end by inclusion
// and meets the other; the triangle's two intersection hyperwedges are
// (r, j) and (j, k) [or (r, k)], and it counts when (r, j) is the earlier.
// TCC from an inclusion hyperwedge: k is joined to exactly one end by
// inclusion (three would be CCC) and meets the other; its two inclusion
// hyperwedges are (r, j) and (r, k) [or (j, k)], counted when (r, j) is the
// earlier.  With r < j in rank, (r, j) precedes (j, k) iff r < k, and
// precedes (r, k) iff j < k.
__global__ __launch_bounds__(kAdvBlock) void k_adv_cross(CrossArgs A) {
    __shared__ uint8_t lut[128];
    __shared__ long long red[kAdvBlock];
    if (threadIdx.x < 128) lut[threadIdx.x] = A.lut[threadIdx.x];
    __syncthreads();
    const uint32_t wmask = (1u << A.wbits) - 1;
    const int base = A.kind == 0 ? 6 : 2;
    const int npat = A.kind == 0 ? 3 : 4;
    long long cnt[4] = {0, 0, 0, 0}, sq[4] = {0, 0, 0, 0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < A.n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = (int64_t)philox_index(A.seed, A.stream, (uint64_t)t, (uint64_t)A.list_size);
        int64_t e;
        if (A.kind == 1) {
            e = A.inc_pos[u];
        } else {
            int64_t lo = 0, hi = A.n_inc;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (A.inc_pos[mid] - mid <= u) lo = mid + 1; else hi = mid;
            }
            e = u + lo;
        }
        const int32_t r = (int32_t)owner_of_a(A.fptr, A.m, e);
        const uint32_t ent = A.fadj[e];
        const int32_t j = (int32_t)(ent >> A.wbits);
        const int wrj = (int)(ent & wmask);
        const int sr = A.esize[r], sj = A.esize[j];
        int c[4] = {0, 0, 0, 0};
        for (int side = 0; side < 2; side++) {
            // side 0: k joined to r by inclusion; side 1: k joined to j
            const int32_t x = side == 0 ? r : j, y = side == 0 ? j : r;
            for (int64_t q = first_pair(A.pairs, A.npairs, x); q < A.npairs && A.pairs[q].x == x; q++) {
                const int32_t k = A.pairs[q].y;
                if (k == y) continue;
                if (has_pair(A.pairs, A.npairs, y, k)) continue;       // joined to both ends by inclusion
                const int sk = A.esize[k];
                const int wxk = sk < (side == 0 ? sr : sj) ? sk : (side == 0 ? sr : sj);
                const int wyk = common2(A.eptr, A.emem, y, k);
                if (wyk == 0) continue;                                // k misses the other end
                const bool counts = side == 0 ? (A.kind == 0 ? r < k : j < k) : (A.kind == 0 ? j < k : r < k);
                if (!counts) continue;
                const int g = common3(A.eptr, A.emem, r, j, k);
                const int wrk = side == 0 ? wxk : wyk;
                const int wjk = side == 0 ? wyk : wxk;
                const int p = lut[region_bits(sr, sj, sk, wrj, wrk, wjk, g)];
                if (p >= base && p < base + npat) c[p - base]++;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            cnt[i] += c[i];
            sq[i] += (long long)c[i] * c[i];
        }
    }
    // fixed-order block sums of the 8 accumulators
    for (int i = 0; i < 8; i++) {
        red[threadIdx.x] = i < 4 ? cnt[i] : sq[i - 4];
        __syncthreads();
        for (int o = kAdvBlock / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) A.part[(int64_t)blockIdx.x * 8 + i] = red[0];
        __syncthreads();
    }
}

// alpha_i of Algorithm 7: a / b * alpha rounded half up; at least 1 when the
// type list is not empty (the paper leaves the rounding open).
int64_t adv_share(double num, double den, int64_t alpha, bool nonempty) {
    if (!nonempty || den <= 0) return 0;
    const int64_t v = (int64_t)std::floor(num / den * (double)alpha + 0.5);
    return std::max<int64_t>(v, 1);
}

void ensure_incl_lists(Graph &g) {
    if (g.have_incl) return;
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    DBuf<int64_t> pos;
    const int64_t nc = list_inclusion_wedges(g, pos);
    // ascending positions (the listing kernel appends in no fixed order)
    g.incl_pos.alloc(A, nc);
    std::vector<int2> ends((size_t)nc);
    if (nc > 0) {
        DBuf<uint32_t> dummy(A, nc);
        fill_u32(dummy.p, nc, 0, s);
        radix_sort_u64(A, (uint64_t *)pos.p, dummy.p, nc, bits_for((uint64_t)g.nw), s);
        HTRI_HIP(hipMemcpyAsync(g.incl_pos.p, pos.p, sizeof(int64_t) * nc, hipMemcpyDeviceToDevice, s));
        DBuf<int2> dends(A, nc);
        hipLaunchKernelGGL(k_incl_ends, dim3(grid_for(nc, 256, 4096)), dim3(256), 0, s, g.fptr.p, g.fadj.p, g.m,
                           g.wbits, pos.p, nc, dends.p);
        HTRI_LAUNCH_CHECK();
        HTRI_HIP(hipMemcpyAsync(ends.data(), dends.p, sizeof(int2) * nc, hipMemcpyDeviceToHost, s));
        HTRI_HIP(hipStreamSynchronize(s));
    }
    std::vector<int2> pairs;
    pairs.reserve((size_t)nc * 2);
    for (const int2 &p : ends) {
        pairs.push_back(make_int2(p.x, p.y));
        pairs.push_back(make_int2(p.y, p.x));
    }
    std::sort(pairs.begin(), pairs.end(),
              [](const int2 &a, const int2 &b) { return a.x < b.x || (a.x == b.x && a.y < b.y); });
    g.incl_pairs.alloc(A, pairs.size());
    if (!pairs.empty())
        HTRI_HIP(hipMemcpyAsync(g.incl_pairs.p, pairs.data(), sizeof(int2) * pairs.size(), hipMemcpyHostToDevice, s));
    HTRI_HIP(hipStreamSynchronize(s));
    g.n_incl_pairs = (int64_t)pairs.size();
    g.have_incl = true;
}

// counts (sums over draws) and squared counts of the mixed class drawn from
// `kind`'s list, patterns base.. in c[0..3]
void cross_sums(Graph &g, int kind, int64_t n, uint64_t seed, uint32_t stream, long long c[4], long long c2[4]) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    for (int i = 0; i < 4; i++) c[i] = c2[i] = 0;
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + kAdvBlock - 1) / kAdvBlock, (int64_t)device_cu_count() * 4);
    DBuf<uint8_t> lut(A, 128);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    DBuf<long long> part(A, (size_t)grid * 8);
    CrossArgs a{};
    a.fptr = g.fptr.p;
    a.fadj = g.fadj.p;
    a.eptr = g.eptr.p;
    a.emem = g.emem.p;
    a.esize = g.esize.p;
    a.m = g.m;
    a.wbits = g.wbits;
    a.lut = lut.p;
    a.inc_pos = g.incl_pos.p;
    a.n_inc = g.summary[2];
    a.pairs = g.incl_pairs.p;
    a.npairs = g.n_incl_pairs;
    a.kind = kind;
    a.list_size = kind == 0 ? g.summary[1] : g.summary[2];
    a.seed = seed;
    a.stream = stream;
    a.n = n;
    a.part = part.p;
    hipLaunchKernelGGL(k_adv_cross, dim3(grid), dim3(kAdvBlock), 0, s, a);
    HTRI_LAUNCH_CHECK();
    std::vector<long long> h((size_t)grid * 8);
    HTRI_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(long long) * h.size(), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < grid; b++)
        for (int i = 0; i < 4; i++) {
            c[i] += h[(size_t)b * 8 + i];
            c2[i] += h[(size_t)b * 8 + 4 + i];
        }
}

}  // namespace

void adv_split(int64_t n_inter, int64_t n_incl, int64_t alpha, int64_t out[4]) {
    const double t = (double)n_inter, c = (double)n_incl, w = t + c;
    out[0] = adv_share(t * t, w * w, alpha, n_inter > 0);
    out[1] = adv_share(c * c, w * w, alpha, n_incl > 0);
    out[2] = adv_share(t * c, w * w, alpha, n_inter > 0 && n_incl > 0);
    out[3] = out[2];
}

// Appro-adv estimate on g (sigma = 1): est[21], stderr[21], the four draw
// counts.  Philox streams 8 (TTT), 9 (CCC), 10 (TTC), 11 (TCC).
void adv_estimate(Graph &g, int64_t alpha, uint64_t seed, double est[21], double se[21], int64_t alphas[4]) {
    for (int q = 0; q < 21; q++) est[q] = se[q] = 0.0;
    const int64_t nT = g.summary[1], nC = g.summary[2];
    adv_split(nT, nC, alpha, alphas);
    if (g.nw == 0) return;
    ensure_incl_lists(g);
    auto finish = [&](int p, long long sum, double y2, int64_t n, int64_t list) {
        const double e = (double)sum * (double)list / (double)n;
        est[p] = e;
        const double nn = (double)n;
        const double var = (y2 - nn * e * e) / (nn * (double)std::max<int64_t>(n - 1, 1));
        se[p] = std::sqrt(std::max(var, 0.0));
    };
    long long c[21];
    double y[21], y2[21];
    if (alphas[0] > 0) {   // TTT: patterns 9-20, forward closure of intersection hyperwedges
        class_sample_sums(g, 0, alphas[0], seed, 8u, g.incl_pos.p, nC, nT, 0x1FFE00u, c, y, y2);
        for (int p = 9; p <= 20; p++) finish(p, c[p], y2[p], alphas[0], nT);
    }
    if (alphas[1] > 0) {   // CCC: pattern 1, forward closure of inclusion hyperwedges
        class_sample_sums(g, 1, alphas[1], seed, 9u, g.incl_pos.p, nC, nC, 0x2u, c, y, y2);
        finish(1, c[1], y2[1], alphas[1], nC);
    }
    long long cc[4], cq[4];
    if (alphas[2] > 0) {   // TTC: patterns 6-8 from intersection hyperwedges
        cross_sums(g, 0, alphas[2], seed, 10u, cc, cq);
        for (int i = 0; i < 3; i++)
            finish(6 + i, cc[i], (double)cq[i] * (double)nT * (double)nT, alphas[2], nT);
    }
    if (alphas[3] > 0) {   // TCC: patterns 2-5 from inclusion hyperwedges
        cross_sums(g, 1, alphas[3], seed, 11u, cc, cq);
        for (int i = 0; i < 4; i++)
            finish(2 + i, cc[i], (double)cq[i] * (double)nC * (double)nC, alphas[3], nC);
    }
    double tot = 0.0, v = 0.0;
    for (int p = 1; p <= 20; p++) {
        tot += est[p];
        v += se[p] * se[p];
    }
    est[0] = tot;
    se[0] = std::sqrt(v);   // the classes are drawn independently; within a class patterns add their variances as an approximation
}

}  // namespace htri
