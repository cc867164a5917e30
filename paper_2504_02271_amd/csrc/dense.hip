// Class-targeted counting of the DenseTTT subclass (patterns 9-16: three
// intersection hyperwedges and a vertex common to all three hyperedges;
// Section 3.2, Count-DenseTTT with its vertex lists tau_v and Lemma 3.1).
//
// The GPU form splits the subclass by whether some pair of the three
// hyperedges shares more than the triple's common vertices:
//
//  * Pattern 9, the common-vertex pattern: the three pairwise
//    intersections are one vertex v, each hyperedge has a private vertex.
//    Every hyperedge of size >= 2 holding v meets every other one in v, so
//    all such hyperedges whose pairwise intersections are exactly {v}
//    form one group (Lemma 3.1: their hyperwedges share Omega = {v} and so
//    close with each other).  With d'_v the hyperedges of size >= 2 at v and
//    P_v the "thick" pairs among them (hyperwedges sharing v and at least
//    one more vertex), inclusion-exclusion over the triples of the group
//    gives the triangles whose pairwise intersections are exactly {v}:
//        sum_v C(d'_v, 3) - |P_v| (d'_v - 2)
//              + sum_x C(deg_{P_v}(x), 2) - triangles(P_v);
//    the common-vertex triangles whose shared set has two or more vertices
//    are triangles of P_v, checked one by one at the set's smallest vertex.
//    Only the thick hyperwedges are visited (a small fraction of all).
//  * Patterns 10-16 have a non-empty pair region, so at least one thick
//    pair.  Each thick hyperwedge (x, y) and each v in Omega_xy scans the
//    hyperedges c of E_v (the tau_v list of the paper, as hyperedges); the
//    triangle {x, y, c} is counted at its smallest triple-common vertex and
//    its earliest thick pair, and classified by its regions.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace htri {
namespace {

constexpr int kMaskWordsMax = 4;
constexpr int kDenseBlock = 256;

__host__ __device__ __forceinline__ int mask_words(int size) {
    return size <= 32 * kMaskWordsMax ? (size + 31) / 32 : 0;
}

__device__ __forceinline__ unsigned long long choose3(unsigned long long d) {
    return d < 3 ? 0ull : d * (d - 1) / 2 * (d - 2) / 3;
}

// fixed-order block reduction of one 64-bit value per thread into part[blockIdx.x]
__device__ void block_sum_u64(unsigned long long v, unsigned long long *red, unsigned long long *part) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
    __syncthreads();
}

// d'_v for every vertex, and per-block partial sums of C(d'_v, 3)
__global__ __launch_bounds__(kDenseBlock) void k_dprime(const int64_t *vptr, const int32_t *vadj, const int32_t *esize,
                                                        int64_t n, uint32_t *dp, unsigned long long *part) {
    __shared__ unsigned long long red[kDenseBlock];
    unsigned long long acc = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        uint32_t d = 0;
        for (int64_t t = vptr[v]; t < vptr[v + 1]; t++) d += esize[vadj[t]] >= 2;
        dp[v] = d;
        acc += choose3(d);
    }
    block_sum_u64(acc, red, part);
}

// Omega_rj as vertex ids, for the hyperwedge at position e of owner r
// (stored mask, or a merge of the two member lists)
template <typename F>
__device__ void omega_vertices(const int64_t *eptr, const int32_t *emem, const int64_t *mptr, const uint32_t *fmask,
                               int32_t r, int sr, int64_t pos, int32_t j, F &&visit) {
    const int W = mask_words(sr);
    const int64_t rb = eptr[r];
    if (W > 0) {
        const int64_t mo = mptr[r] + pos * W;
        for (int w = 0; w < W; w++) {
            uint32_t bits = fmask[mo + w];
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1;
                visit(emem[rb + w * 32 + b]);
            }
        }
    } else {
        int64_t a = rb, ae = eptr[r + 1], b = eptr[j], be = eptr[j + 1];
        while (a < ae && b < be) {
            const int32_t u = emem[a], v = emem[b];
            if (u == v) {
                visit(u);
                a++;
                b++;
            } else if (u < v) {
                a++;
            } else {
                b++;
            }
        }
    }
}

// per owner: records of its thick hyperwedges (2 per shared vertex)
__global__ void k_thick_count(const int64_t *fptr, const uint32_t *fadj, int64_t m, int wbits, int64_t *cnt) {
    const uint32_t wmask = (1u << wbits) - 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < m; r += nwaves) {
        unsigned long long c = 0;
        for (int64_t e = fptr[r] + lane; e < fptr[r + 1]; e += kWave) {
            const uint32_t om = fadj[e] & wmask;
            if (om >= 2) c += 2ull * om;
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
        if (lane == 0) cnt[r] = (int64_t)c;
    }
}

// records (v << rbits | x, y) and (v << rbits | y, x) for every thick
// hyperwedge (x, y) and every v in Omega_xy; owner r's records start at off[r]
__global__ void k_thick_fill(const int64_t *fptr, const uint32_t *fadj, const int64_t *eptr, const int32_t *emem,
                             const int64_t *mptr, const uint32_t *fmask, const int32_t *esize, int64_t m, int wbits,
                             int rbits, const int64_t *off, uint64_t *key, uint32_t *val) {
    const uint32_t wmask = (1u << wbits) - 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < m; r += nwaves) {
        int64_t at = off[r];
        const int sr = esize[r];
        const int64_t b0 = fptr[r];
        for (int64_t e0 = b0; e0 < fptr[r + 1]; e0 += kWave) {
            const int64_t e = e0 + lane;
            const bool ok = e < fptr[r + 1];
            const uint32_t ent = ok ? fadj[e] : 0u;
            const uint32_t om = ent & wmask;
            const int64_t mine = (ok && om >= 2) ? 2 * (int64_t)om : 0;
            int64_t incl = mine;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int64_t u = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += u;
            }
            const int64_t total = __shfl(incl, kWave - 1, kWave);
            if (mine) {
                int64_t w = at + incl - mine;
                const int32_t j = (int32_t)(ent >> wbits);
                omega_vertices(eptr, emem, mptr, fmask, (int32_t)r, sr, e - b0, j, [&](int32_t v) {
                    key[w] = ((uint64_t)(uint32_t)v << rbits) | (uint64_t)r;
                    val[w] = (uint32_t)j;
                    key[w + 1] = ((uint64_t)(uint32_t)v << rbits) | (uint64_t)j;
                    val[w + 1] = (uint32_t)r;
                    w += 2;
                });
            }
            at += total;
        }
    }
}

// start of each run of equal keys (flags), for the groups (v, x)
__global__ void k_key_runs(const uint64_t *key, int64_t n, int64_t *flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_run_starts(const int64_t *flag_scan, const uint64_t *key, int64_t n, int64_t *start) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (i == 0 || key[i] != key[i - 1]) start[flag_scan[i]] = i;
}

// every group's partners ascending (insertion sort; groups are short), and
// the per-block sums of C(group size, 2)
__global__ __launch_bounds__(kDenseBlock) void k_group_sort(const int64_t *start, int64_t ngroups, int64_t n,
                                                            uint32_t *val, unsigned long long *part) {
    __shared__ unsigned long long red[kDenseBlock];
    unsigned long long acc = 0;
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < ngroups;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = start[gi], b = gi + 1 < ngroups ? start[gi + 1] : n;
        for (int64_t i = a + 1; i < b; i++) {
            const uint32_t x = val[i];
            int64_t k = i - 1;
            while (k >= a && val[k] > x) {
                val[k + 1] = val[k];
                k--;
            }
            val[k + 1] = x;
        }
        const unsigned long long d = (unsigned long long)(b - a);
        acc += d * (d - 1) / 2;
    }
    block_sum_u64(acc, red, part);
}

__device__ __forceinline__ int64_t find_group(const uint64_t *key, const int64_t *start, int64_t ngroups, uint64_t k) {
    int64_t lo = 0, hi = ngroups;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[start[mid]] < k) lo = mid + 1; else hi = mid;
    }
    return (lo < ngroups && key[start[lo]] == k) ? lo : -1;
}

__device__ __forceinline__ int common_count(const int64_t *eptr, const int32_t *emem, int32_t a, int32_t b) {
    int64_t x = eptr[a], xe = eptr[a + 1], y = eptr[b], ye = eptr[b + 1];
    int c = 0;
    while (x < xe && y < ye) {
        if (emem[x] == emem[y]) { c++; x++; y++; } else if (emem[x] < emem[y]) x++; else y++;
    }
    return c;
}

// A triangle {x, y, z} of thick pairs at v is also of the common-vertex
// pattern when its three pairwise intersections are one and the same set
// (then all three share g >= 2 vertices and nothing else pairwise) and every
// hyperedge has a private vertex; it is counted at the set's smallest vertex.
__device__ bool shared_set_pattern(const int64_t *eptr, const int32_t *emem, const int32_t *esize, int32_t x,
                                   int32_t y, int32_t z, int32_t v) {
    int64_t a = eptr[x], ae = eptr[x + 1], b = eptr[y], be = eptr[y + 1], c = eptr[z], ce = eptr[z + 1];
    int g = 0;
    int32_t first = -1;
    while (a < ae && b < be && c < ce) {
        const int32_t p = emem[a], q = emem[b], r = emem[c];
        if (p == q && q == r) {
            if (g == 0) first = p;
            g++;
            a++;
            b++;
            c++;
            continue;
        }
        const int32_t mx = max(p, max(q, r));
        if (p < mx) a++;
        if (q < mx) b++;
        if (r < mx) c++;
    }
    if (first != v) return false;
    if (esize[x] <= g || esize[y] <= g || esize[z] <= g) return false;
    return common_count(eptr, emem, x, y) == g && common_count(eptr, emem, x, z) == g &&
           common_count(eptr, emem, y, z) == g;
}

// per record (v, x, y) with x < y: d'_v - 2 (one thick pair of the group at
// v), the triangles {x, y, z} of thick pairs at v with z > y, and those of
// them that are common-vertex triangles with a shared set of two or more
// vertices
__global__ __launch_bounds__(kDenseBlock) void k_thick_pairs(const uint64_t *key, const uint32_t *val,
                                                             const int64_t *start, int64_t ngroups, int64_t n,
                                                             int rbits, const uint32_t *dp, const int64_t *eptr,
                                                             const int32_t *emem, const int32_t *esize,
                                                             unsigned long long *part1, unsigned long long *part2,
                                                             unsigned long long *part3) {
    __shared__ unsigned long long red[kDenseBlock];
    unsigned long long s1 = 0, s2 = 0, s3 = 0;
    const uint64_t rmask = ((uint64_t)1 << rbits) - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[i];
        const uint32_t x = (uint32_t)(k & rmask), y = val[i];
        if (y <= x) continue;
        const uint64_t v = k >> rbits;
        s1 += (unsigned long long)dp[v] - 2ull;
        // partners of x at v (this record's group) and of y at v, both ascending
        const int64_t gx = find_group(key, start, ngroups, k);
        const int64_t gy = find_group(key, start, ngroups, (v << rbits) | (uint64_t)y);
        if (gx < 0 || gy < 0) continue;
        int64_t a = start[gx], ae = gx + 1 < ngroups ? start[gx + 1] : n;
        int64_t b = start[gy], be = gy + 1 < ngroups ? start[gy + 1] : n;
        while (a < ae && b < be) {
            const uint32_t p = val[a], q = val[b];
            if (p == q) {
                if (p > y) {
                    s2++;
                    s3 += shared_set_pattern(eptr, emem, esize, (int32_t)x, (int32_t)y, (int32_t)p, (int32_t)v);
                }
                a++;
                b++;
            } else if (p < q) {
                a++;
            } else {
                b++;
            }
        }
    }
    block_sum_u64(s1, red, part1);
    block_sum_u64(s2, red, part2);
    block_sum_u64(s3, red, part3);
}

__device__ __forceinline__ uint32_t region_bits(int si, int sj, int sk, int wij, int wik, int wjk, int g) {
    const int a = si - wij - wik + g, b = sj - wij - wjk + g, c = sk - wik - wjk + g;
    const int d = wij - g, e = wjk - g, f = wik - g;
    return (uint32_t)(a > 0) | ((uint32_t)(b > 0) << 1) | ((uint32_t)(c > 0) << 2) | ((uint32_t)(d > 0) << 3) |
           ((uint32_t)(e > 0) << 4) | ((uint32_t)(f > 0) << 5) | ((uint32_t)(g > 0) << 6);
}

// order this wave's earlier LDS accesses before its later ones, across lanes
__device__ __forceinline__ void wave_lds_sync_d() {
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

constexpr int kHashSlots = 512;              // per wave: vertices of e_x and e_y
constexpr int kDenseWaves = kDenseBlock / kWave;

__device__ __forceinline__ uint32_t vhash(uint32_t v) { return (v * 2654435761u) >> (32 - 9); }

// Patterns 10-16: one wave per record (v, x, y) with x < y; lanes over the
// hyperedges c of E_v.  The triangle {x, y, c} counts here when v is its
// smallest triple-common vertex and (x, y) its earliest thick pair (pairs
// ordered by their rank pairs).
__global__ __launch_bounds__(kDenseBlock) void k_dense_rest(const uint64_t *key, const uint32_t *val, int64_t n,
                                                            int rbits, const int64_t *vptr, const int32_t *vadj,
                                                            const int64_t *eptr, const int32_t *emem,
                                                            const int32_t *esize, const uint8_t *glut,
                                                            unsigned long long *part, unsigned long long *tp) {
    __shared__ uint2 tab[kDenseWaves][kHashSlots];   // (vertex + 1, bit 0: in x, bit 1: in y)
    __shared__ uint8_t lut[128];
    __shared__ unsigned long long red[kDenseBlock];
    if (threadIdx.x < 128) lut[threadIdx.x] = glut[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    uint2 *T = tab[wv];
    const uint64_t rmask = ((uint64_t)1 << rbits) - 1;
    unsigned long long cnt[7] = {0, 0, 0, 0, 0, 0, 0};
    const int64_t nwaves = (int64_t)gridDim.x * kDenseWaves;
    for (int64_t i = (int64_t)blockIdx.x * kDenseWaves + wv; i < n; i += nwaves) {
        const uint64_t k = key[i];
        const int32_t x = (int32_t)(k & rmask), y = (int32_t)val[i];
        if (y <= x) continue;                             // wave-uniform
        const int32_t v = (int32_t)(k >> rbits);
        const int sx = esize[x], sy = esize[y];
        const bool small = sx + sy <= kHashSlots / 2;
        if (small) {
            for (int t = lane; t < kHashSlots; t += kWave) T[t] = make_uint2(0u, 0u);
            wave_lds_sync_d();
            for (int t = lane; t < sx + sy; t += kWave) {
                const bool inx = t < sx;
                const uint32_t u = (uint32_t)emem[inx ? eptr[x] + t : eptr[y] + (t - sx)];
                uint32_t h = vhash(u);
                while (true) {
                    const uint32_t old = atomicCAS(&T[h].x, 0u, u + 1);
                    if (old == 0u || old == u + 1) break;
                    h = (h + 1) & (kHashSlots - 1);
                }
                atomicOr(&T[h].y, inx ? 1u : 2u);
            }
            wave_lds_sync_d();
        }
        int wxy = 0;
        {   // omega_xy (wave-uniform): vertices flagged in both
            int c = 0;
            if (small) {
                for (int t = lane; t < kHashSlots; t += kWave) c += T[t].y == 3u;
            } else if (lane == 0) {
                int64_t a = eptr[x], ae = eptr[x + 1], b = eptr[y], be = eptr[y + 1];
                while (a < ae && b < be) {
                    if (emem[a] == emem[b]) { c++; a++; b++; } else if (emem[a] < emem[b]) a++; else b++;
                }
            }
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
            wxy = c;
        }
        for (int64_t t = vptr[v] + lane; t < vptr[v + 1]; t += kWave) {
            const int32_t c = vadj[t];
            if (c == x || c == y) continue;
            int wxc = 0, wyc = 0, g = 0;
            int32_t gmin = 0x7FFFFFFF;
            for (int64_t q = eptr[c]; q < eptr[c + 1]; q++) {
                const uint32_t u = (uint32_t)emem[q];
                uint32_t fl = 0;
                if (small) {
                    uint32_t h = vhash(u);
                    while (true) {
                        const uint2 s = T[h];
                        if (s.x == 0u) break;
                        if (s.x == u + 1) { fl = s.y; break; }
                        h = (h + 1) & (kHashSlots - 1);
                    }
                } else {
                    int64_t lo = eptr[x], hi = eptr[x + 1];
                    while (lo < hi) { const int64_t md = (lo + hi) >> 1; if ((uint32_t)emem[md] < u) lo = md + 1; else hi = md; }
                    if (lo < eptr[x + 1] && (uint32_t)emem[lo] == u) fl |= 1u;
                    lo = eptr[y]; hi = eptr[y + 1];
                    while (lo < hi) { const int64_t md = (lo + hi) >> 1; if ((uint32_t)emem[md] < u) lo = md + 1; else hi = md; }
                    if (lo < eptr[y + 1] && (uint32_t)emem[lo] == u) fl |= 2u;
                }
                wxc += fl & 1u;
                wyc += (fl >> 1) & 1u;
                if (fl == 3u) {
                    g++;
                    if ((int32_t)u < gmin) gmin = (int32_t)u;
                }
            }
            if (gmin != v) continue;                                  // not the smallest common vertex
            if ((wxc >= 2 && c < y) || (wyc >= 2 && c < x)) continue; // an earlier thick pair counts it
            const int p = lut[region_bits(sx, sy, esize[c], wxy, wxc, wyc, g)];
            if (p >= 10 && p <= 16) {
                cnt[p - 10]++;
                if (tp) {   // per hyperedge and pattern (rank order, 21 per hyperedge)
                    atomicAdd(&tp[(int64_t)x * 21 + p], 1ull);
                    atomicAdd(&tp[(int64_t)y * 21 + p], 1ull);
                    atomicAdd(&tp[(int64_t)c * 21 + p], 1ull);
                }
            }
        }
    }
    for (int p = 0; p < 7; p++) block_sum_u64(cnt[p], red, part + (int64_t)p * gridDim.x);
}

template <typename T>
T read_back(const T *dev, hipStream_t s) {
    return host_read(dev, s);
}

unsigned long long sum_parts(const unsigned long long *dev, int n, hipStream_t s) {
    std::vector<unsigned long long> h((size_t)n);
    HTRI_HIP(hipMemcpyAsync(h.data(), dev, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    unsigned long long t = 0;
    for (unsigned long long x : h) t += x;
    return t;
}

}  // namespace

// DenseTTT counts: counts[9..16] (others 0).  rest: also patterns 10-16
// (false: pattern 9 alone).  ms: device time.
void count_dense_ttt(Graph &g, bool rest, int64_t counts[21], float *ms, unsigned long long *tp_rank) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    for (int p = 0; p < 21; p++) counts[p] = 0;
    const int64_t m = g.m, n = g.n;
    hipEvent_t e0, e1;
    HTRI_HIP(hipEventCreate(&e0));
    HTRI_HIP(hipEventCreate(&e1));
    HTRI_HIP(hipEventRecord(e0, s));
    // sum_v C(d'_v, 3)
    const int gb = (int)grid_for(std::max<int64_t>(n, 1), kDenseBlock, 4096);
    DBuf<uint32_t> dp(A, std::max<int64_t>(n, 1));
    DBuf<unsigned long long> p0(A, gb);
    hipLaunchKernelGGL(k_dprime, dim3(gb), dim3(kDenseBlock), 0, s, g.vptr.p, g.vadj.p, g.esize.p, n, dp.p, p0.p);
    HTRI_LAUNCH_CHECK();
    const unsigned long long S1 = sum_parts(p0.p, gb, s);
    // thick-hyperwedge records
    DBuf<int64_t> off(A, m + 1);
    if (m > 0) {
        hipLaunchKernelGGL(k_thick_count, dim3(grid_for(m * kWave, 256, 8192)), dim3(256), 0, s, g.fptr.p, g.fadj.p,
                           m, g.wbits, off.p);
        HTRI_LAUNCH_CHECK();
    }
    scan_exclusive_i64(A, off.p, off.p, m, off.p + m, s);
    const int64_t nrec = m > 0 ? read_back(off.p + m, s) : 0;
    unsigned long long Sterm = 0, Sc2 = 0, Stri = 0, E9 = 0;
    unsigned long long rest_cnt[7] = {0, 0, 0, 0, 0, 0, 0};
    if (nrec > 0) {
        if (nrec >= (int64_t)UINT32_MAX) fail(HTRI_E_UNSUPPORTED, "too many thick hyperwedge records");
        const int rbits = g.rbits;
        const int vbits = bits_for((uint64_t)std::max<int64_t>(n - 1, 1));
        if (rbits + vbits > 64) fail(HTRI_E_UNSUPPORTED, "vertex and rank bits exceed a 64-bit key");
        DBuf<uint64_t> key(A, nrec);
        DBuf<uint32_t> val(A, nrec);
        hipLaunchKernelGGL(k_thick_fill, dim3(grid_for(m * kWave, 256, 8192)), dim3(256), 0, s, g.fptr.p, g.fadj.p,
                           g.eptr.p, g.emem.p, g.mptr.p, g.fmask.p, g.esize.p, m, g.wbits, rbits, off.p, key.p,
                           val.p);
        HTRI_LAUNCH_CHECK();
        radix_sort_u64(A, key.p, val.p, nrec, rbits + vbits, s);
        DBuf<int64_t> flag(A, nrec + 1);
        hipLaunchKernelGGL(k_key_runs, dim3(grid_for(nrec, 256, 4096)), dim3(256), 0, s, key.p, nrec, flag.p);
        HTRI_LAUNCH_CHECK();
        scan_exclusive_i64(A, flag.p, flag.p, nrec, flag.p + nrec, s);
        const int64_t ng = read_back(flag.p + nrec, s);
        DBuf<int64_t> start(A, ng);
        hipLaunchKernelGGL(k_run_starts, dim3(grid_for(nrec, 256, 4096)), dim3(256), 0, s, flag.p, key.p, nrec,
                           start.p);
        HTRI_LAUNCH_CHECK();
        const int gg = (int)grid_for(ng, kDenseBlock, 4096);
        DBuf<unsigned long long> pc(A, gg);
        hipLaunchKernelGGL(k_group_sort, dim3(gg), dim3(kDenseBlock), 0, s, start.p, ng, nrec, val.p, pc.p);
        HTRI_LAUNCH_CHECK();
        Sc2 = sum_parts(pc.p, gg, s);
        const int gr = (int)grid_for(nrec, kDenseBlock, 4096);
        DBuf<unsigned long long> pa(A, gr), pb(A, gr), pe(A, gr);
        hipLaunchKernelGGL(k_thick_pairs, dim3(gr), dim3(kDenseBlock), 0, s, key.p, val.p, start.p, ng, nrec, rbits,
                           dp.p, g.eptr.p, g.emem.p, g.esize.p, pa.p, pb.p, pe.p);
        HTRI_LAUNCH_CHECK();
        Sterm = sum_parts(pa.p, gr, s);
        Stri = sum_parts(pb.p, gr, s);
        E9 = sum_parts(pe.p, gr, s);
        if (rest) {
            DBuf<uint8_t> lut(A, 128);
            HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
            const int gw = (int)std::min<int64_t>((nrec + kDenseWaves - 1) / kDenseWaves,
                                                  (int64_t)device_cu_count() * 16);
            DBuf<unsigned long long> pr(A, (size_t)gw * 7);
            hipLaunchKernelGGL(k_dense_rest, dim3(gw), dim3(kDenseBlock), 0, s, key.p, val.p, nrec, rbits, g.vptr.p,
                               g.vadj.p, g.eptr.p, g.emem.p, g.esize.p, lut.p, pr.p, tp_rank);
            HTRI_LAUNCH_CHECK();
            std::vector<unsigned long long> h((size_t)gw * 7);
            HTRI_HIP(hipMemcpyAsync(h.data(), pr.p, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, s));
            HTRI_HIP(hipStreamSynchronize(s));
            for (int p = 0; p < 7; p++)
                for (int b = 0; b < gw; b++) rest_cnt[p] += h[(size_t)p * gw + b];
        }
    }
    HTRI_HIP(hipEventRecord(e1, s));
    HTRI_HIP(hipEventSynchronize(e1));
    float t = 0;
    HTRI_HIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms) *ms = t;
    counts[9] = (int64_t)(S1 - Sterm + Sc2 - Stri + E9);
    for (int p = 10; p <= 16; p++) counts[p] = (int64_t)rest_cnt[p - 10];
    for (int p = 1; p <= 20; p++) counts[0] += counts[p];
}

}  // namespace htri
