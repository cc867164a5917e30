// Step 2 of the two-step framework: close every hyperwedge and classify the
// hyper-triangle (Algorithm 3 for the intersection-only class, Algorithm 5
// for the classes with inclusion hyperwedges, combined over all patterns as
// the paper's Exact-adv).
//
// Orientation: hyperedges are ranked by prec; the forward list N+(r) holds
// the later neighbours of r, sorted.  A triangle r < j < k is found exactly
// once, at its two earliest hyperedges: k lies in both N+(r) and N+(j).
//
// Two closures share the owners:
//  * the dense window (k_window_rows, k_close_window): the owners of the top
//    ranks get bitmap rows over the window; c(r, j) = |N+(r) & N+(j)| is an
//    AND + popcount, and the common-vertex pattern is counted in bulk per
//    (owner, shared vertex) class;
//  * probing (k_close) for the other owners, by default around the middle
//    hyperedge: an item is (middle j, a chunk of at most CAP entries of
//    N+(j), a piece of j's in-list); the chunk goes into an LDS
//    open-addressing hash and, for every hyperwedge (r, j) of the piece, the
//    entries of N+(r) after j are streamed from HBM with coalesced loads and
//    probed against it (HTRI_COUNT_OWNER_PROBE hashes the owner's chunk and
//    streams each partner's N+(j) instead).
// A hit is classified from the sizes, the three omegas and g =
// popcount(Omega & Omega) over the hashed hyperedge's member positions
// through a 128-entry region-emptiness table (the common-vertex pattern by a
// shortcut test).  Persistent blocks pull items from two queues (block items,
// then single-middle wave items).  Pattern counts live one per lane (lane p
// holds pattern p); in a single-graph launch each wave (each window block)
// writes them to its own slot when it finishes and a fixed-order reduction
// sums the slots, in a batched launch a wave adds them to its graph's counts
// when it moves to another graph or finishes.  Per-hyperedge counts come
// from per-wedge role counters and per-wave sums added to the hyperedges'
// totals during the closure.
#include <algorithm>

#include "internal.hpp"

namespace htri {

namespace {

constexpr int kBlock = 256;
constexpr int kMaskWordsMax = 4;
constexpr uint32_t kEmptyPos = 0xFFFFFFFFu;

__host__ __device__ __forceinline__ int mask_words(int size) {
    return size <= 32 * kMaskWordsMax ? (size + 31) / 32 : 0;
}

__device__ __forceinline__ uint32_t hslot(uint32_t k, int hbits) {
    // full-rate 24x24-bit multiply by a golden-ratio constant, top bits
    return (uint32_t)__umul24(k ^ (k >> 24), 0x9E3779u) >> (32 - hbits);   // __umul24 returns int
}

// Loads through the global address space (the graph's arrays reach the
// kernel through a descriptor, so the compiler cannot infer it).
template <typename T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}

// 16-byte loads through the global address space
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 gld(const uint4 *p) {
    const u32x4_t v = *(const __attribute__((address_space(1))) u32x4_t *)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}

// first index in [a, b) whose entry's rank is >= key
__device__ __forceinline__ int64_t lower_rank(const uint32_t *fadj, int64_t a, int64_t b, uint32_t key,
                                              int wbits) {
    while (a < b) {
        int64_t mid = a + ((b - a) >> 1);
        if ((gld(fadj + mid) >> wbits) < key) a = mid + 1; else b = mid;
    }
    return a;
}

// |e_r & e_j & e_k| by a three-way merge of sorted member lists (hyperedges
// too large for stored masks)
__device__ int triple_common(const int64_t *eptr, const int32_t *emem, int32_t r, int32_t j, int32_t k) {
    int64_t a = gld(eptr + r), ae = gld(eptr + r + 1), b = gld(eptr + j), be = gld(eptr + j + 1),
            c = gld(eptr + k), ce = gld(eptr + k + 1);
    int cnt = 0;
    while (a < ae && b < be && c < ce) {
        int32_t x = gld(emem + a), y = gld(emem + b), z = gld(emem + c);
        if (x == y && y == z) { cnt++; a++; b++; c++; continue; }
        int32_t mx = x > y ? x : y;
        mx = mx > z ? mx : z;
        if (x < mx) a++;
        if (y < mx) b++;
        if (z < mx) c++;
    }
    return cnt;
}

// Omega_jr over e_j's member positions for the hyperwedge (r, j) at position
// off of N+(r): each vertex of Omega_rj (over e_r's positions) located in
// e_j's sorted member list jm[0, sj) (LDS) by binary search, or a merge of
// the two member lists when e_r has no stored mask.
__device__ void middle_mask(const int64_t *eptr, const int32_t *emem, const int64_t *mptr, const uint32_t *fmask,
                            int32_t r, int sr, int64_t off, const int32_t *jm, int sj, uint32_t &o0, uint32_t &o1,
                            uint32_t &o2, uint32_t &o3) {
    o0 = o1 = o2 = o3 = 0u;
    auto set = [&](int q) {
        const uint32_t bit = 1u << (q & 31);
        const int w = q >> 5;
        o0 |= w == 0 ? bit : 0u;
        o1 |= w == 1 ? bit : 0u;
        o2 |= w == 2 ? bit : 0u;
        o3 |= w == 3 ? bit : 0u;
    };
    const int64_t rb = gld(eptr + r);
    const int Wr = mask_words(sr);
    if (Wr > 0) {
        const int64_t mo = gld(mptr + r) + off * Wr;
        for (int w = 0; w < Wr; w++) {
            uint32_t x = gld(fmask + mo + w);
            while (x) {
                const int b = __ffs(x) - 1;
                x &= x - 1;
                const int32_t v = gld(emem + rb + w * 32 + b);
                int lo = 0, hi = sj;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (jm[mid] < v) lo = mid + 1; else hi = mid;
                }
                if (lo < sj && jm[lo] == v) set(lo);
            }
        }
    } else {
        int a = 0, b = 0;
        while (a < sr && b < sj) {
            const int32_t va = gld(emem + rb + a), vb = jm[b];
            if (va == vb) {
                set(b);
                a++;
                b++;
            } else if (va < vb) {
                a++;
            } else {
                b++;
            }
        }
    }
}

// Omega_jr of an in-list entry: the shared vertex's position in jm (one
// bit), or middle_mask() when the entry holds no single vertex
__device__ __forceinline__ void entry_mask(const GraphDesc &G, const uint4 &E, int wbits, const int32_t *jm, int sj,
                                           uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3) {
    const uint32_t wmask = (1u << wbits) - 1;
    if (E.z != kInNoVertex) {
        const int32_t v = (int32_t)E.z;
        int lo = 0, hi = sj;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (jm[mid] < v) lo = mid + 1; else hi = mid;
        }
        const bool in = lo < sj && jm[lo] == v;
        const uint32_t bit = in ? 1u << (lo & 31) : 0u;
        const int w = lo >> 5;
        o0 = w == 0 ? bit : 0u;
        o1 = w == 1 ? bit : 0u;
        o2 = w == 2 ? bit : 0u;
        o3 = w == 3 ? bit : 0u;
    } else {
        const int32_t r = (int32_t)(E.w >> wbits);
        const int64_t off = (int64_t)E.x - gld(G.fptr + r);
        middle_mask(G.eptr, G.emem, G.mptr, G.fmask, r, (int)(E.w & wmask), off, jm, sj, o0, o1, o2, o3);
    }
}

__device__ __forceinline__ uint32_t region_mask(int si, int sj, int sk, int wij, int wik, int wjk, int g) {
    int a = si - wij - wik + g, b = sj - wij - wjk + g, c = sk - wik - wjk + g;
    int d = wij - g, e = wjk - g, f = wik - g;
    return (uint32_t)(a > 0) | ((uint32_t)(b > 0) << 1) | ((uint32_t)(c > 0) << 2) | ((uint32_t)(d > 0) << 3) |
           ((uint32_t)(e > 0) << 4) | ((uint32_t)(f > 0) << 5) | ((uint32_t)(g > 0) << 6);
}

// Emptiness mask of the common-vertex pattern: the three private regions and
// the triple region non-empty, the three pair-only regions empty.
constexpr uint32_t kMaskCommonVertex = 0x47;
constexpr uint32_t kPatternCommonVertex = 9;

// Each lane p (1..20) of a wave holds the wave's count of pattern p, and
// every lane a share of the common-vertex pattern's count; add them to
// counts[g] and clear.
__device__ __forceinline__ void flush_wave_counts(unsigned long long &wcnt, unsigned long long &c9,
                                                  unsigned long long *counts, int g, int lane) {
    unsigned long long s9 = c9;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s9 += __shfl_xor(s9, o, kWave);
    if (lane == (int)kPatternCommonVertex) wcnt += s9;
    if (lane >= 1 && lane < 21 && wcnt) atomicAdd(&counts[(int64_t)g * 21 + lane], wcnt);
    wcnt = 0;
    c9 = 0;
}

// Items a block or a wave claims from its queue with one atomic (one hot
// address: fewer round trips, and the claimed items run back to back).
constexpr unsigned int kBlockBatch = 4;
constexpr unsigned int kWaveBatch = 8;

// What a probe needs of the partner j: |e_j|, omega_rj, Omega_rj (mask
// words over the owner's members), whether the common-vertex shortcut can
// apply to j at all, and j's rank (for the member merge of owners without a
// stored mask).
struct JParams {
    int sj, wij;
    bool fast;
    uint32_t m0, m1, m2, m3;
    int32_t jr;
};

// U partner-list entries e[u] = (k, omega_jk) per lane (partner data
// for the shortcut test in fwij / fm0 / ffast, the rest from jparams) against the
// chunk of owner r staged in the bucketed open-addressing table (two
// (entry, position) slots per 16-byte bucket, buckets probed linearly; a
// bucket's second slot fills after its first).  The work goes in phases so
// that each phase's LDS reads are in flight together: the first buckets;
// slot selection; the rare continuation past a full bucket; size and mask
// word of each k found; the common-vertex shortcut (all three omegas equal
// omega_rj, Omega_rk = Omega_rj and every hyperedge larger than that: the
// triple shares exactly those vertices); region classification for the
// other hits.  hit[u]: entry u closes a hyper-triangle; mhit[u]: it counts
// towards the per-hyperedge counts; po[u]: its pattern unless it is the
// common-vertex one (counted in c9), else 0.
template <int U, bool PER_EDGE, bool TP, typename JF>
__device__ __forceinline__ void probe_tile(const uint2 *tab, int hbits, int wbits, uint32_t wmask,
                                           const uint32_t (&e)[U], const bool (&val)[U],
                                           const int (&fwij)[U], const uint32_t (&fm0)[U],
                                           const bool (&ffast)[U],
                                           const JF &jparams, const uint2 *ent_sm, const uint32_t *ent_mx,
                                           uint32_t *ent_ck, const uint8_t *lut, int W, int si, const GraphDesc &G,
                                           int32_t r, uint32_t emask, unsigned long long &c9,
                                           bool (&hit)[U], bool (&mhit)[U], uint32_t (&po)[U],
                                           unsigned long long *tp) {
    const uint4 *tq = reinterpret_cast<const uint4 *>(tab);
    const uint32_t nbm1 = (1u << (hbits - 1)) - 1;
    const uint32_t kmask = ~wmask;
    uint32_t b[U];
    uint4 B[U];
#pragma unroll
    for (int u = 0; u < U; u++) b[u] = hslot(e[u] >> wbits, hbits - 1);
#pragma unroll
    for (int u = 0; u < U; u++) B[u] = tq[b[u]];
    uint2 sl[U];
    bool cont[U];
    bool more = false;
#pragma unroll
    for (int u = 0; u < U; u++) {
        // an empty slot's entry word is 0 and a probed key k << wbits never is (k > j > r >= 0)
        const uint32_t kk = e[u] & kmask;
        const bool h0 = (B[u].x & kmask) == kk;
        const bool h1 = (B[u].z & kmask) == kk;
        hit[u] = val[u] & (h0 | h1);
        cont[u] = val[u] & !(h0 | h1) & (B[u].z != 0u);
        more |= cont[u];
        sl[u] = h0 ? make_uint2(B[u].x, B[u].y) : make_uint2(B[u].z, B[u].w);
    }
    if (more) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (cont[u]) {
                const uint32_t kk = e[u] & kmask;
                uint32_t bb = b[u];
                bool h0, h1;
                uint4 Bx;
                do {
                    bb = (bb + 1) & nbm1;
                    Bx = tq[bb];
                    h0 = (Bx.x & kmask) == kk;
                    h1 = (Bx.z & kmask) == kk;
                } while (!(h0 | h1 | (Bx.z == 0u)));
                hit[u] = h0 | h1;
                sl[u] = h0 ? make_uint2(Bx.x, Bx.y) : make_uint2(Bx.z, Bx.w);
            }
        }
    }
    uint2 sm[U];
#pragma unroll
    for (int u = 0; u < U; u++) sm[u] = ent_sm[hit[u] ? sl[u].y : 0u];
    // SparseTTT-only counting (emask bit 31): a triangle with a vertex common
    // to all three hyperedges is dropped as soon as g > 0 is known
    const bool sparse_only = (emask >> 31) & 1u;
    bool fast[U];
    bool slow = false;
    uint32_t n9 = 0;
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int wik = (int)(sl[u].x & wmask), wjk = (int)(e[u] & wmask);
        fast[u] = hit[u] & ffast[u] & (wik == fwij[u]) & (wjk == fwij[u]) & (sm[u].y == fm0[u]) &
                  ((int)sm[u].x > fwij[u]);
        if (sparse_only && fast[u]) {
            hit[u] = false;
            fast[u] = false;
        }
        n9 += fast[u];
        po[u] = 0u;
        slow |= hit[u] & !fast[u];
    }
    if (slow) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (hit[u] && !fast[u]) {
                const JParams J = jparams(u);
                const uint32_t pos = sl[u].y;
                const int wik = (int)(sl[u].x & wmask), wjk = (int)(e[u] & wmask);
                int g;
                if (W > 0) {
                    g = __popc(J.m0 & sm[u].y);
                    if (W > 1) {
                        const uint32_t *mx = ent_mx + pos * (kMaskWordsMax - 1);
                        g += __popc(J.m1 & mx[0]);
                        if (W > 2) g += __popc(J.m2 & mx[1]);
                        if (W > 3) g += __popc(J.m3 & mx[2]);
                    }
                } else {
                    g = triple_common(G.eptr, G.emem, r, J.jr, (int32_t)(e[u] >> wbits));
                }
                if (sparse_only && g > 0) {
                    hit[u] = false;
                    continue;
                }
                const uint32_t m7 = region_mask(si, J.sj, (int)sm[u].x, J.wij, wik, wjk, g);
                if (m7 != kMaskCommonVertex) po[u] = lut[m7];
                else n9++;
                if (TP) {
                    // per-hyperedge counts by pattern (rank-ordered rows of 21): the hashed
                    // hyperedge, the partner (segment) and the third one
                    const uint32_t p = m7 != kMaskCommonVertex ? (uint32_t)lut[m7] : kPatternCommonVertex;
                    atomicAdd(&tp[(int64_t)r * 21 + p], 1ull);
                    atomicAdd(&tp[(int64_t)J.jr * 21 + p], 1ull);
                    atomicAdd(&tp[(int64_t)(e[u] >> wbits) * 21 + p], 1ull);
                }
            }
        }
    }
    c9 += n9;
    if (PER_EDGE) {
        // every pattern counted per hyperedge (the default): a hit is a counted hit
        const bool all_patterns = (emask & 0x1FFFFEu) == 0x1FFFFEu;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t p = po[u] ? po[u] : kPatternCommonVertex;
            mhit[u] = hit[u] && (all_patterns || ((emask >> p) & 1u));
            if (mhit[u]) atomicAdd(&ent_ck[sl[u].y], 1u);
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; u++) mhit[u] = false;
    }
}

// Add the wave's other-pattern hits (po[u] != 0) into lane p's counter.
template <int U>
__device__ __forceinline__ void aggregate_other(const uint32_t *po, int lane, unsigned long long &wcnt) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        uint64_t pend = __ballot(po[u] != 0);
        while (pend) {
            const int srcl = __ffsll((unsigned long long)pend) - 1;
            const uint32_t p0 = (uint32_t)__shfl((int)po[u], srcl, kWave);
            const uint64_t mm = __ballot(po[u] == p0);
            if ((uint32_t)lane == p0) wcnt += (unsigned long long)__popcll(mm);
            pend &= ~mm;
        }
    }
}

// Shared memory of the closure kernel: the block layout (owner chunk and
// partner segments of a block item) or, once the block items are drained,
// one slice per wave for single-owner items.
template <int CAP, int JP, bool PE, bool PW>
struct CloseBlockLds {
    uint2 tab[4 * CAP];                                // slots (entry, position); buckets of two
    uint2 ent_sm[CAP];                                 // (|e_k|, Omega_rk word 0)
    uint32_t ent_mx[CAP * (kMaskWordsMax - 1)];        // Omega_rk words 1..3
    uint32_t ent_ck[PE ? CAP : 1];
    int64_t seg_pre[kBlock + 1];
    int64_t seg_src[JP];
    uint32_t seg_size[JP];
    uint32_t seg_om[JP];
    uint32_t seg_mask[JP * kMaskWordsMax];
    uint32_t seg_cj[PW ? JP : 1];
    uint32_t seg_cjm[PE ? JP : 1];
};
// Owner-centric wave items take the partner data from the chunk arrays
// (partner q is entry q of N+(r)); middle-centric ones keep it apart in
// p_sm / p_ent, with p_ent = (rank of r) << wbits | omega_jr.  Middle-centric
// wave items hash up to kWaveMidHashMax entries and have at most one Omega
// word (the item builder sends the others to block items), so their extra
// mask words are not kept.
template <bool MID>
struct CloseWaveLds {
    static constexpr int kHash = MID ? kWaveMidHashMax : kWaveOwnerMax;
    uint2 tab[4 * kHash];
    uint2 ent_sm[kHash];                               // (|e_k|, Omega word 0 of the hashed entry)
    uint32_t ent_mx[MID ? 4 : kWaveOwnerMax * (kMaskWordsMax - 1)];
    uint32_t ent_ck[kHash];
    int64_t src[kWaveOwnerMax];                        // partner segment start minus its stream offset
    uint32_t ent[kHash];                               // packed entry (rank, omega) of the hashed list
    int32_t incl[kWaveOwnerMax];                       // end of each partner segment in the stream
    uint32_t cj[kWaveOwnerMax];
    uint32_t cjm[kWaveOwnerMax];
    uint2 p_sm[MID ? kWaveOwnerMax : 2];               // (|e_r|, Omega_jr word 0)
    uint32_t p_mx[4];                                  // (no extra Omega words in wave items)
    uint32_t p_ent[MID ? kWaveOwnerMax : 4];
    int32_t jmem[MID ? 32 : 4];                        // e_j's members (at most 32 when stored)
};
template <int CAP, int JP, bool PE, bool PW, bool MID>
union CloseLds {
    CloseBlockLds<CAP, JP, PE, PW> b;
    CloseWaveLds<MID> w[kBlock / kWave];
};

// Order this wave's earlier LDS accesses before its later ones, across lanes
// (LDS executes one wave's instructions in order once they are issued).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// MID = false: owner-centric items (owner r hashed, each partner's N+(j)
// streamed).  MID = true: middle-centric items (the middle j's N+(j)
// hashed, the rest of N+(r) after j streamed for each hyperwedge (r, j) of
// j's in-list); a hit k closes r < j < k.  The classification is the same
// with the roles (r, j, k) read as (j, r, k): sizes |e_j|, |e_r|, |e_k|,
// omegas omega_jr (segment), omega_jk (hashed entry), omega_rk (streamed
// entry), and g = popcount(Omega_jr & Omega_jk) over e_j's member
// positions; the region table is invariant under relabelling.
template <int CAP, int JP, bool PER_EDGE, bool PER_WEDGE, bool MID, bool TP = false>
__global__ __launch_bounds__(kBlock, 4) void k_close(CloseArgs A) {
    static_assert(JP <= kBlock, "one thread per partner");
    // partner-list entries per lane per step: fewer registers for the short
    // middle-centric segments, more loads in flight for the long partner lists
    constexpr int kU = MID ? 2 : 4;
    constexpr int HMAX = 4 * CAP;
    static_assert(sizeof(CloseWaveLds<MID>) % 16 == 0, "wave slices keep the table 16-byte aligned");
    __shared__ __align__(16) CloseLds<CAP, JP, PER_EDGE, PER_WEDGE, MID> L;
    uint2 *tab = L.b.tab;
    uint2 *ent_sm = L.b.ent_sm;
    uint32_t *ent_mx = L.b.ent_mx;
    uint32_t *ent_ck = L.b.ent_ck;
    int64_t *seg_pre = L.b.seg_pre;
    int64_t *seg_src = L.b.seg_src;
    uint32_t *seg_size = L.b.seg_size;
    uint32_t *seg_om = L.b.seg_om;
    uint32_t *seg_mask = L.b.seg_mask;
    uint32_t *seg_cj = L.b.seg_cj;
    uint32_t *seg_cjm = L.b.seg_cjm;
    (void)HMAX;
    __shared__ uint8_t lut[128];
    __shared__ int32_t s_jmem[MID ? 32 * kMaskWordsMax : 1];   // the middle's members
    __shared__ int64_t sh_item;
    __shared__ int64_t sh_scan[kBlock / kWave + 1];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if (tid < 128) lut[tid] = A.lut[tid];
    unsigned long long wcnt = 0;     // lane p: this wave's count of pattern p (p != 9)
    unsigned long long c9 = 0;       // this lane's count of the common-vertex pattern
    unsigned long long all_probes = 0, all_staged = 0;
    int cur_g = -1;

    int64_t bnext = 0, bend = 0;     // claimed queue positions [bnext, bend), block-uniform
    for (;;) {
        __syncthreads();
        if (bnext >= bend) {
            if (tid == 0) sh_item = (int64_t)atomicAdd(A.queue, kBlockBatch);
            __syncthreads();
            bnext = sh_item;
            bend = bnext + kBlockBatch;
        }
        const int64_t c = bnext++;
        if (c >= A.nitems) break;
        const Item item = A.items[A.nitems - 1 - c];
        if (item.g != cur_g) {
            if (cur_g >= 0) flush_wave_counts(wcnt, c9, A.counts, cur_g, lane);
            cur_g = item.g;
        }
        const GraphDesc G = A.graphs[item.g];
        const uint32_t wmask = (1u << G.wbits) - 1;
        const int wbits = G.wbits;
        const int32_t r = item.r;
        const int64_t base = gld(G.fptr + r);
        const int32_t d = (int32_t)(gld(G.fptr + r + 1) - base);
        // whole_chunk: the chunk is all of the hashed list (no rank cut);
        // whole_in: the item holds every partner of the hashed list
        const bool whole_chunk = item.cb == 0 && item.ce == d;
        bool whole_in = item.jb == 0 && item.je == d - 1;
        int64_t ibase = 0;
        if (MID) {
            ibase = gld(G.iptr + r);
            whole_in = item.jb == 0 && (int64_t)item.je == gld(G.iptr + r + 1) - ibase;
        }
        const bool single = whole_chunk && whole_in;
        // rank of the hyperedge of partner segment q (the member merge of
        // hashed hyperedges without a stored mask)
        auto seg_rank = [&](int q) -> int32_t {
            if (MID) return (int32_t)(gld(G.inl + ibase + item.jb + q).w >> wbits);
            return (int32_t)(gld(G.fadj + base + item.jb + q) >> wbits);
        };
        const int si = gld(G.esize + r);
        const int W = mask_words(si);
        const int64_t mbase = gld(G.mptr + r);
        const int cl = item.ce - item.cb;
        int hbits = 6;
        while ((1 << hbits) < 4 * cl) hbits++;
        const int H = 1 << hbits;
        const uint32_t lo = gld(G.fadj + base + item.cb) >> wbits;
        const uint32_t hi = gld(G.fadj + base + item.ce - 1) >> wbits;

        for (int s = tid; s < H; s += kBlock) tab[s] = make_uint2(0u, kEmptyPos);
        if (MID && W > 0) {
            const int64_t jb0 = gld(G.eptr + r);
            for (int t = tid; t < si; t += kBlock) s_jmem[t] = gld(G.emem + jb0 + t);
        }
        __syncthreads();
        // stage the chunk
        for (int q = tid; q < cl; q += kBlock) {
            const uint32_t ent = gld(G.fadj + base + item.cb + q);
            const uint32_t k = ent >> wbits;
            const int64_t mo = mbase + (int64_t)(item.cb + q) * W;
            ent_sm[q] = make_uint2((uint32_t)gld(G.esize + k), W > 0 ? gld(G.fmask + mo) : 0u);
            for (int w = 1; w < W; w++) ent_mx[q * (kMaskWordsMax - 1) + (w - 1)] = gld(G.fmask + mo + w);
            if (PER_EDGE) ent_ck[q] = 0;
            // slot = (entry, position): claim the position word, then write the entry
            uint32_t slot = hslot(k, hbits - 1) * 2;
            while (atomicCAS(&tab[slot].y, kEmptyPos, (uint32_t)q) != kEmptyPos) slot = (slot + 1) & (H - 1);
            tab[slot].x = ent;
        }
        // partner segments: N+(j) cut to the chunk's rank range
        const int nseg = item.je - item.jb;
        int64_t len = 0;
        int64_t my_wedge = 0;          // MID: the hyperwedge (r, j) of this thread's segment
        if (MID && tid < nseg) {
            const uint4 E = gld(G.inl + ibase + item.jb + tid);
            const int64_t i = (int64_t)E.x;
            int64_t a = i + 1, b = a + (int64_t)(E.y >> wbits);
            if (!whole_chunk) {
                a = lower_rank(G.fadj, a, b, lo, wbits);
                b = lower_rank(G.fadj, a, b, hi + 1, wbits);
            }
            len = b - a;
            seg_src[tid] = a;
            const uint32_t om = E.y & wmask;
            const uint32_t sz = E.w & wmask;
            seg_size[tid] = sz;
            const bool fj = (W == 1) && ((uint32_t)si > om) && (sz > om);
            seg_om[tid] = om | (fj ? 0x80000000u : 0u);
            if (W > 0) {
                uint32_t o0, o1, o2, o3;
                entry_mask(G, E, wbits, s_jmem, si, o0, o1, o2, o3);
                seg_mask[tid * kMaskWordsMax + 0] = o0;
                if (W > 1) seg_mask[tid * kMaskWordsMax + 1] = o1;
                if (W > 2) seg_mask[tid * kMaskWordsMax + 2] = o2;
                if (W > 3) seg_mask[tid * kMaskWordsMax + 3] = o3;
            }
            if (PER_WEDGE) seg_cj[tid] = 0;
            if (PER_EDGE) seg_cjm[tid] = 0;
            my_wedge = i;
        }
        if (!MID && tid < nseg) {
            const int pj = item.jb + tid;
            const uint32_t jent = gld(G.fadj + base + pj);
            const uint32_t j = jent >> wbits;
            int64_t a = gld(G.fptr + j), b = gld(G.fptr + j + 1);
            if (!single) {
                a = lower_rank(G.fadj, a, b, lo, wbits);
                b = lower_rank(G.fadj, a, b, hi + 1, wbits);
            }
            len = b - a;
            seg_src[tid] = a;
            seg_size[tid] = (uint32_t)gld(G.esize + j);
            {
                const uint32_t om = jent & wmask;
                const uint32_t sz = (uint32_t)gld(G.esize + j);
                const bool fj = (W == 1) && ((uint32_t)si > om) && (sz > om);
                seg_om[tid] = om | (fj ? 0x80000000u : 0u);   // bit 31: the shortcut can apply to j
            }
            for (int w = 0; w < W; w++) seg_mask[tid * kMaskWordsMax + w] = gld(G.fmask + mbase + (int64_t)pj * W + w);
            if (PER_WEDGE) seg_cj[tid] = 0;
            if (PER_EDGE) seg_cjm[tid] = 0;
        }
        // exclusive scan of segment lengths
        {
            int64_t incl = len;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                int64_t u = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += u;
            }
            if (lane == kWave - 1) sh_scan[wave] = incl;
            __syncthreads();
            if (tid == 0) {
                int64_t run = 0;
                for (int w = 0; w < kBlock / kWave; w++) {
                    int64_t c = sh_scan[w];
                    sh_scan[w] = run;
                    run += c;
                }
                sh_scan[kBlock / kWave] = run;
            }
            __syncthreads();
            seg_pre[tid] = sh_scan[wave] + incl - len;
            if (tid == 0) seg_pre[kBlock] = sh_scan[kBlock / kWave];
        }
        __syncthreads();
        const int64_t total = seg_pre[kBlock];
        all_probes += (unsigned long long)total;
        all_staged += (unsigned long long)cl;

        // Partner-list entries go through probe_tile(); both loops below
        // keep the next tile's loads in flight while the current tile is
        // classified.
        if (total >= (int64_t)nseg * 256) {
            // Dense items (long partner segments): one wave per partner, the
            // partner's data wave-uniform, lanes striding over its segment.
            constexpr int TILE = kWave * kU;
            int qd = wave;
            while (qd < nseg && seg_pre[qd + 1] == seg_pre[qd]) qd += kBlock / kWave;
            int64_t i0 = 0;
            uint32_t entA[kU];
            bool valA[kU];
            if (qd < nseg) {
                const int64_t slen = seg_pre[qd + 1] - seg_pre[qd];
                const int64_t sbase = seg_src[qd];
#pragma unroll
                for (int u = 0; u < kU; u++) {
                    const int64_t i = u * kWave + lane;
                    valA[u] = i < slen;
                    entA[u] = valA[u] ? gld(G.fadj + sbase + i) : 0u;
                }
            }
            unsigned long long hits = 0, mhits = 0;     // wave-uniform, current segment
            while (qd < nseg) {
                // the tile after this one
                const int64_t slen = seg_pre[qd + 1] - seg_pre[qd];
                int qn = qd;
                int64_t in = i0 + TILE;
                if (in >= slen) {
                    qn = qd + kBlock / kWave;
                    while (qn < nseg && seg_pre[qn + 1] == seg_pre[qn]) qn += kBlock / kWave;
                    in = 0;
                }
                uint32_t entB[kU];
                bool valB[kU];
                if (qn < nseg) {
                    const int64_t nlen = seg_pre[qn + 1] - seg_pre[qn];
                    const int64_t nbase = seg_src[qn];
#pragma unroll
                    for (int u = 0; u < kU; u++) {
                        const int64_t i = in + u * kWave + lane;
                        valB[u] = i < nlen;
                        entB[u] = valB[u] ? gld(G.fadj + nbase + i) : 0u;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < kU; u++) {
                        valB[u] = false;
                        entB[u] = 0u;
                    }
                }
                // this tile
                const int sjd = __builtin_amdgcn_readfirstlane((int)seg_size[qd]);
                const int wd = __builtin_amdgcn_readfirstlane((int)(seg_om[qd] & 0x7FFFFFFFu));
                const uint32_t m0 = W > 0 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)seg_mask[qd * kMaskWordsMax]) : 0u;
                const uint32_t m1 = W > 1 ? seg_mask[qd * kMaskWordsMax + 1] : 0u;
                const uint32_t m2 = W > 2 ? seg_mask[qd * kMaskWordsMax + 2] : 0u;
                const uint32_t m3 = W > 3 ? seg_mask[qd * kMaskWordsMax + 3] : 0u;
                const bool fastd = (W == 1) && (si > wd) && (sjd > wd);
                const int32_t jr = (W == 0 || TP) ? seg_rank(qd) : 0;
                const JParams Jd{sjd, wd, fastd, m0, m1, m2, m3, jr};
                bool hit[kU], mhit[kU];
                uint32_t po[kU];
                int fwij[kU];
                uint32_t fm0[kU];
                bool ffast[kU];
#pragma unroll
                for (int u = 0; u < kU; u++) {
                    fwij[u] = wd;
                    fm0[u] = m0;
                    ffast[u] = fastd;
                }
                probe_tile<kU, PER_EDGE, TP>(tab, hbits, wbits, wmask, entA, valA, fwij, fm0, ffast, [&](int) { return Jd; },
                                     ent_sm, ent_mx, ent_ck, lut, W, si, G, r, A.emask, c9, hit, mhit, po, A.tp);
                bool other = false;
#pragma unroll
                for (int u = 0; u < kU; u++) {
                    other |= po[u] != 0;
                    if (PER_WEDGE) hits += (unsigned long long)__popcll(__ballot(hit[u]));
                    if (PER_EDGE) mhits += (unsigned long long)__popcll(__ballot(mhit[u]));
                }
                if (__ballot(other)) aggregate_other<kU>(po, lane, wcnt);
                if (qn != qd) {
                    if (lane == 0) {
                        if (PER_WEDGE) seg_cj[qd] = (uint32_t)hits;
                        if (PER_EDGE) seg_cjm[qd] = (uint32_t)mhits;
                    }
                    hits = mhits = 0;
                }
                qd = qn;
                i0 = in;
#pragma unroll
                for (int u = 0; u < kU; u++) {
                    entA[u] = entB[u];
                    valA[u] = valB[u];
                }
            }
        } else {
            // Flattened items: the partner segments laid end to end; each step
            // a wave takes 64*kU consecutive entries, kU per lane.
            // here total < nseg * 256 <= 65536: stream offsets fit in 32 bits
            const int total32 = (int)total;
            // Middle-centric (short segments): each wave takes its own
            // contiguous quarter of the stream (a multiple of 64*kU entries)
            // and a lane's segment cursor moves forward by a linear scan.
            // Owner-centric: the waves interleave steps over the whole stream
            // and a lane finds its segment by binary search.
            constexpr int kStep = kWave * kU;
            constexpr int kWaves = kBlock / kWave;
            const int per_wave = (total32 + kWaves * kStep - 1) / (kWaves * kStep) * kStep;
            const int f_hi = MID ? min(total32, (wave + 1) * per_wave) : total32;
            int qa = -1;                   // address cursor
            int qa_end = 0;
            int64_t srca = 0;
            int q = -1;                    // segment whose counters this lane holds
            uint32_t cj = 0, cjm = 0;
            const int stride = MID ? kStep : kBlock * kU;
            auto fetch = [&](int f0, uint32_t *ent, int *segu) {
#pragma unroll
                for (int u = 0; u < kU; u++) {
                    const int f = f0 + u;
                    segu[u] = -1;
                    int64_t addr = 0;
                    if (f < f_hi) {
                        if (f >= qa_end) {
                            int lo_s;
                            if (MID && qa >= 0) {
                                lo_s = qa + 1;
                                while ((int)seg_pre[lo_s + 1] <= f) lo_s++;   // stops below nseg: f < total
                            } else {
                                lo_s = qa < 0 ? 0 : qa + 1;
                                int hi_s = nseg;
                                while (lo_s < hi_s) {
                                    int mid = (lo_s + hi_s) >> 1;
                                    if ((int)seg_pre[mid + 1] <= f) lo_s = mid + 1; else hi_s = mid;
                                }
                            }
                            qa = lo_s;
                            qa_end = (int)seg_pre[qa + 1];
                            srca = seg_src[qa] - seg_pre[qa];
                        }
                        segu[u] = qa;
                        addr = srca + f;
                    }
                    ent[u] = segu[u] >= 0 ? gld(G.fadj + addr) : 0u;
                }
            };
            int fb = MID ? wave * per_wave : wave * kStep;
            uint32_t entA[kU];
            int seguA[kU];
            if (fb < f_hi) fetch(fb + lane * kU, entA, seguA);
            for (; fb < f_hi; fb += stride) {
                uint32_t entB[kU];
                int seguB[kU];
                const int fbn = fb + stride;
                if (fbn < f_hi) {
                    fetch(fbn + lane * kU, entB, seguB);
                } else {
#pragma unroll
                    for (int u = 0; u < kU; u++) {
                        entB[u] = 0u;
                        seguB[u] = -1;
                    }
                }
                bool valA[kU], hit[kU], mhit[kU];
                uint32_t po[kU];
#pragma unroll
                for (int u = 0; u < kU; u++) valA[u] = seguA[u] >= 0;
                // shortcut data per entry, reloaded only where the segment changes
                int fwij[kU];
                uint32_t fm0[kU];
                bool ffast[kU];
                {
                    int qc = -1, cw = 0;
                    uint32_t cm = 0u;
                    bool cf = false;
#pragma unroll
                    for (int u = 0; u < kU; u++) {
                        const int qq = seguA[u] < 0 ? 0 : seguA[u];
                        if (qq != qc) {
                            qc = qq;
                            const uint32_t om = seg_om[qq];
                            cw = (int)(om & 0x7FFFFFFFu);
                            cf = (om >> 31) != 0u;
                            cm = W > 0 ? seg_mask[qq * kMaskWordsMax + 0] : 0u;
                        }
                        fwij[u] = cw;
                        fm0[u] = cm;
                        ffast[u] = cf;
                    }
                }
                auto jf = [&](int u) {
                    const int qq = seguA[u] < 0 ? 0 : seguA[u];
                    JParams J;
                    J.sj = (int)seg_size[qq];
                    J.wij = (int)(seg_om[qq] & 0x7FFFFFFFu);
                    J.fast = (W == 1) && (si > J.wij) && (J.sj > J.wij);
                    J.m0 = W > 0 ? seg_mask[qq * kMaskWordsMax + 0] : 0u;
                    J.m1 = W > 1 ? seg_mask[qq * kMaskWordsMax + 1] : 0u;
                    J.m2 = W > 2 ? seg_mask[qq * kMaskWordsMax + 2] : 0u;
                    J.m3 = W > 3 ? seg_mask[qq * kMaskWordsMax + 3] : 0u;
                    J.jr = (W == 0 || TP) ? seg_rank(qq) : 0;
                    return J;
                };
                probe_tile<kU, PER_EDGE, TP>(tab, hbits, wbits, wmask, entA, valA, fwij, fm0, ffast, jf, ent_sm, ent_mx, ent_ck,
                                     lut, W, si, G, r, A.emask, c9, hit, mhit, po, A.tp);
                bool other = false;
#pragma unroll
                for (int u = 0; u < kU; u++) {
                    other |= po[u] != 0;
                    if (seguA[u] < 0) continue;
                    if (seguA[u] != q) {
                        if (q >= 0) {
                            if (PER_WEDGE && cj) atomicAdd(&seg_cj[q], cj);
                            if (PER_EDGE && cjm) atomicAdd(&seg_cjm[q], cjm);
                        }
                        cj = cjm = 0;
                        q = seguA[u];
                    }
                    cj += hit[u];
                    cjm += mhit[u];
                }
                if (__ballot(other)) aggregate_other<kU>(po, lane, wcnt);
#pragma unroll
                for (int u = 0; u < kU; u++) {
                    entA[u] = entB[u];
                    seguA[u] = seguB[u];
                }
            }
            if (q >= 0) {
                if (PER_WEDGE && cj) atomicAdd(&seg_cj[q], cj);
                if (PER_EDGE && cjm) atomicAdd(&seg_cjm[q], cjm);
            }
        }
        __syncthreads();
        // per-wedge counters (single-graph launches only)
        // A middle-centric segment (one hyperwedge) meets each chunk once;
        // an owner-centric partner meets every chunk of its owner.
        if (PER_WEDGE || PER_EDGE) {
            const bool seg_direct = MID ? whole_chunk : single;
            if (MID && PER_EDGE) {
                // the middle's j-role total of this item: one atomic per wave
                unsigned long long sj = tid < nseg ? (unsigned long long)seg_cjm[tid] : 0ull;
#pragma unroll
                for (int o = kWave / 2; o > 0; o >>= 1) sj += __shfl_xor(sj, o, kWave);
                if (lane == 0 && sj) atomicAdd(&A.tedge[r], sj);
            }
            if (tid < nseg) {
                const int64_t e = MID ? my_wedge : base + item.jb + tid;
                if (seg_direct) {
                    if (PER_WEDGE) A.cwj[e] = seg_cj[tid];
                    if (PER_EDGE) A.cwjm[e] = seg_cjm[tid];
                } else {
                    if (PER_WEDGE && seg_cj[tid]) atomicAdd(&A.cwj[e], seg_cj[tid]);
                    if (PER_EDGE && seg_cjm[tid]) atomicAdd(&A.cwjm[e], seg_cjm[tid]);
                }
            }
            if (PER_EDGE) {
                for (int qq = tid; qq < cl; qq += kBlock) {
                    const int64_t e = base + item.cb + qq;
                    if (MID) {
                        if (ent_ck[qq])
                            atomicAdd(&A.tedge[gld(G.fadj + e) >> wbits], (unsigned long long)ent_ck[qq]);
                    } else if (single) {
                        A.cwkm[e] = ent_ck[qq];
                    } else if (ent_ck[qq]) {
                        atomicAdd(&A.cwkm[e], ent_ck[qq]);
                    }
                }
            }
        }
    }
    if (tid == 0 && all_probes) atomicAdd(A.probes, all_probes);
    if (tid == 0 && all_staged && A.staged) atomicAdd(A.staged, all_staged);

    // Single-owner items, one wave each, in the wave's own LDS slice: the
    // block items are drained and every wave of the block has passed the
    // loop's last barrier, so the block layout is dead.  No block barrier
    // from here on.
    CloseWaveLds<MID> &Wl = L.w[wave];
    // partner data: the chunk's own entries (owner-centric) or the in-list's
    const uint2 *p_sm = MID ? Wl.p_sm : Wl.ent_sm;
    const uint32_t *p_ent = MID ? Wl.p_ent : Wl.ent;
    const uint32_t *p_mx = MID ? Wl.p_mx : Wl.ent_mx;
    unsigned long long wprobes = 0, wstaged = 0;
    int64_t wnext = 0, wend = 0;     // claimed queue positions [wnext, wend)
    for (;;) {
        if (wnext >= wend) {
            unsigned int c0 = 0;
            if (lane == 0) c0 = atomicAdd(A.wqueue, kWaveBatch);
            wnext = (unsigned int)__builtin_amdgcn_readfirstlane((int)c0);
            wend = wnext + kWaveBatch;
        }
        const int64_t c = wnext++;
        if (c >= A.nwitems) break;
        const Item item = A.witems[A.nwitems - 1 - c];
        if (item.g != cur_g) {
            if (cur_g >= 0) flush_wave_counts(wcnt, c9, A.counts, cur_g, lane);
            cur_g = item.g;
        }
        const GraphDesc G = A.graphs[item.g];
        const int wbits = G.wbits;
        const uint32_t wmask = (1u << wbits) - 1;
        const int32_t r = item.r;
        const int64_t base = gld(G.fptr + r);
        const int d = item.ce;                 // all of the hashed list N+(r)
        const int npart = MID ? item.je : d - 1;   // partners: in-list entries, or entries 0 .. d-2
        const int si = gld(G.esize + r);
        const int W = mask_words(si);
        const int64_t mbase = gld(G.mptr + r);
        int hbits = 6;
        while ((1 << hbits) < 4 * d) hbits++;
        const int H = 1 << hbits;              // <= 4 * CloseWaveLds<MID>::kHash
        wave_lds_sync();                       // the previous owner's reads are done
        for (int t = lane; t < H; t += kWave) Wl.tab[t] = make_uint2(0u, kEmptyPos);
        if (MID && W > 0) {
            const int64_t jb0 = gld(G.eptr + r);
            for (int t = lane; t < si; t += kWave) Wl.jmem[t] = gld(G.emem + jb0 + t);
        }
        wave_lds_sync();
        // lane q holds entry q of the hashed list (owner-centric: also the
        // partner j_q of the wedge (r, j_q)) and, middle-centric, entry q of
        // the in-list
        int64_t len = 0, a = 0;
        int64_t my_wedge = 0;
        Wl.cj[lane] = 0;
        Wl.cjm[lane] = 0;
        for (int t = lane; t < d; t += kWave) {
            const uint32_t ent = gld(G.fadj + base + t);
            const uint32_t k = ent >> wbits;
            const int64_t mo = mbase + (int64_t)t * W;
            Wl.ent_sm[t] = make_uint2((uint32_t)gld(G.esize + k), W > 0 ? gld(G.fmask + mo) : 0u);
            if (!MID)
                for (int w = 1; w < W; w++) Wl.ent_mx[t * (kMaskWordsMax - 1) + (w - 1)] = gld(G.fmask + mo + w);
            Wl.ent[t] = ent;
            if (PER_EDGE) Wl.ent_ck[t] = 0;
            uint32_t slot = hslot(k, hbits - 1) * 2;
            while (atomicCAS(&Wl.tab[slot].y, kEmptyPos, (uint32_t)t) != kEmptyPos) slot = (slot + 1) & (H - 1);
            Wl.tab[slot].x = ent;
            if (!MID && t < d - 1) {
                a = gld(G.fptr + k);
                len = gld(G.fptr + k + 1) - a;
            }
        }
        if (MID && lane < npart) {
            const uint4 E = gld(G.inl + gld(G.iptr + r) + lane);
            const int64_t i = (int64_t)E.x;
            a = i + 1;
            len = (int64_t)(E.y >> wbits);
            uint32_t o0 = 0u, o1 = 0u, o2 = 0u, o3 = 0u;
            if (W > 0) entry_mask(G, E, wbits, Wl.jmem, si, o0, o1, o2, o3);
            Wl.p_sm[lane] = make_uint2(E.w & wmask, o0);   // W <= 1: o1..o3 are 0
            Wl.p_ent[lane] = (E.w & ~wmask) | (E.y & wmask);   // (r << wbits) | omega_rj
            my_wedge = i;
        }
        int64_t incl = len;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int64_t u = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += u;
        }
        const int64_t total = __shfl(incl, kWave - 1, kWave);   // lanes >= npart add nothing
        if (lane < npart) {
            Wl.incl[lane] = (int32_t)incl;
            Wl.src[lane] = a - (incl - len);
        }
        wave_lds_sync();
        wprobes += (unsigned long long)total;
        wstaged += (unsigned long long)d;
        // the partner lists end to end, kU consecutive entries per lane
        int qa = 0;                            // search cursor (monotone per lane)
        int q = -1;                            // segment whose counters this lane holds
        uint32_t cj = 0, cjm = 0;
        const int wtotal = (int)total;          // <= kWaveStreamMax
        for (int fb = 0; fb < wtotal; fb += kWave * kU) {
            uint32_t ent4[kU];
            int seg4[kU];
#pragma unroll
            for (int u = 0; u < kU; u++) {
                const int f = fb + lane * kU + u;
                seg4[u] = -1;
                ent4[u] = 0u;
                if (f < wtotal) {
                    while (Wl.incl[qa] <= f) qa++;     // ends at a segment < npart since f < total
                    seg4[u] = qa;
                    ent4[u] = gld(G.fadj + Wl.src[qa] + f);
                }
            }
            bool val4[kU], hit[kU], mhit[kU];
            uint32_t po[kU];
#pragma unroll
            for (int u = 0; u < kU; u++) val4[u] = seg4[u] >= 0;
            int fwij[kU];
            uint32_t fm0[kU];
            bool ffast[kU];
            {
                int qc = -1, cw = 0;
                uint32_t cm = 0u;
                bool cf = false;
#pragma unroll
                for (int u = 0; u < kU; u++) {
                    const int qq = seg4[u] < 0 ? 0 : seg4[u];
                    if (qq != qc) {
                        qc = qq;
                        const uint2 jsm = p_sm[qq];
                        cw = (int)(p_ent[qq] & wmask);
                        cm = jsm.y;
                        cf = (W == 1) && (si > cw) && ((int)jsm.x > cw);
                    }
                    fwij[u] = cw;
                    fm0[u] = cm;
                    ffast[u] = cf;
                }
            }
            auto jf = [&](int u) {
                const int qq = seg4[u] < 0 ? 0 : seg4[u];
                const uint2 jsm = p_sm[qq];
                const uint32_t jent = p_ent[qq];
                JParams J;
                J.sj = (int)jsm.x;
                J.wij = (int)(jent & wmask);
                J.fast = (W == 1) && (si > J.wij) && (J.sj > J.wij);
                J.m0 = jsm.y;
                J.m1 = W > 1 ? p_mx[qq * (kMaskWordsMax - 1) + 0] : 0u;
                J.m2 = W > 2 ? p_mx[qq * (kMaskWordsMax - 1) + 1] : 0u;
                J.m3 = W > 3 ? p_mx[qq * (kMaskWordsMax - 1) + 2] : 0u;
                J.jr = (int32_t)(jent >> wbits);
                return J;
            };
            probe_tile<kU, PER_EDGE, TP>(Wl.tab, hbits, wbits, wmask, ent4, val4, fwij, fm0, ffast, jf, Wl.ent_sm, Wl.ent_mx,
                                 Wl.ent_ck, lut, W, si, G, r, A.emask, c9, hit, mhit, po, A.tp);
            bool other = false;
#pragma unroll
            for (int u = 0; u < kU; u++) {
                other |= po[u] != 0;
                if (seg4[u] < 0) continue;
                if (seg4[u] != q) {
                    if (q >= 0) {
                        if (PER_WEDGE && cj) atomicAdd(&Wl.cj[q], cj);
                        if (PER_EDGE && cjm) atomicAdd(&Wl.cjm[q], cjm);
                    }
                    cj = cjm = 0;
                    q = seg4[u];
                }
                cj += hit[u];
                cjm += mhit[u];
            }
            if (__ballot(other)) aggregate_other<kU>(po, lane, wcnt);
        }
        if (q >= 0) {
            if (PER_WEDGE && cj) atomicAdd(&Wl.cj[q], cj);
            if (PER_EDGE && cjm) atomicAdd(&Wl.cjm[q], cjm);
        }
        wave_lds_sync();
        if (PER_WEDGE || PER_EDGE) {
            if (lane < npart) {
                const int64_t e = MID ? my_wedge : base + lane;
                if (PER_WEDGE) A.cwj[e] = Wl.cj[lane];
                if (PER_EDGE) A.cwjm[e] = Wl.cjm[lane];
            }
            if (MID && PER_EDGE) {
                unsigned long long sj = Wl.cjm[lane];   // 0 beyond the item's partners
#pragma unroll
                for (int o = kWave / 2; o > 0; o >>= 1) sj += __shfl_xor(sj, o, kWave);
                if (lane == 0 && sj) atomicAdd(&A.tedge[r], sj);
            }
            if (PER_EDGE)
                for (int t = lane; t < d; t += kWave) {
                    if (!MID) A.cwkm[base + t] = Wl.ent_ck[t];
                    else if (Wl.ent_ck[t])
                        atomicAdd(&A.tedge[Wl.ent[t] >> wbits], (unsigned long long)Wl.ent_ck[t]);
                }
        }
    }
    if (lane == 0 && wprobes) atomicAdd(A.probes, wprobes);
    if (lane == 0 && wstaged && A.staged) atomicAdd(A.staged, wstaged);
    if (A.wave_part) {
        // one graph: every wave writes its 21 counts to its own slot (zeros
        // if it closed nothing); a fixed-order reduction adds them up
        unsigned long long s9 = c9;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s9 += __shfl_xor(s9, o, kWave);
        if (lane == (int)kPatternCommonVertex) wcnt += s9;
        const int64_t gw = (int64_t)blockIdx.x * (kBlock / kWave) + wave;
        if (lane < 21) A.wave_part[gw * 21 + lane] = lane >= 1 ? wcnt : 0ull;
    } else if (cur_g >= 0) {
        flush_wave_counts(wcnt, c9, A.counts, cur_g, lane);
    }
}

// counts[p] += sum_i part[i * 21 + p]: block p sums a strided share per
// thread, then a tree in shared memory (fixed order, no atomics)
__global__ __launch_bounds__(256) void k_sum_parts(const unsigned long long *part, int64_t n,
                                                   unsigned long long *counts) {
    __shared__ unsigned long long red[256];
    const int p = blockIdx.x + 1;
    unsigned long long v = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) v += part[i * 21 + p];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[p] += red[0];
}

// Work items per owner: block items in cnt, and wcnt = 1 for an owner closed
// by one wave (at most kWaveOwnerMax forward entries and at most
// kWaveStreamMax entries in its partners' lists; it then has no block item).
__global__ void k_item_counts(const int64_t *fptr, const uint32_t *fadj, int wbits, int64_t m, int64_t owner_end,
                              int cap, int jp, int64_t *cnt, int64_t *wcnt) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t base = fptr[r];
        const int64_t d = fptr[r + 1] - base;
        int64_t c = 0;
        bool wave = false;
        if (d >= 2 && r < owner_end) {
            if (d <= kWaveOwnerMax) {
                int64_t sz = 0;
                for (int64_t e = base; e < base + d - 1; e++) {
                    const uint32_t j = fadj[e] >> wbits;
                    sz += fptr[j + 1] - fptr[j];
                }
                wave = sz <= kWaveStreamMax;
            }
            if (!wave) {
                for (int64_t cb = 0; cb < d; cb += cap) {
                    int64_t ce = cb + cap < d ? cb + cap : d;
                    c += (ce - 1 + jp - 1) / jp;
                }
            }
        }
        cnt[r] = c;
        wcnt[r] = wave ? 1 : 0;
    }
}

__global__ void k_item_fill(const int64_t *fptr, int64_t m, int64_t owner_end, int cap, int jp, int32_t gid,
                            const int64_t *ioff, const int64_t *woff, Item *items, Item *witems) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = fptr[r + 1] - fptr[r];
        if (d < 2 || r >= owner_end) continue;
        if (woff[r + 1] != woff[r]) {
            Item it;
            it.g = gid;
            it.r = (int32_t)r;
            it.cb = 0;
            it.ce = (int32_t)d;
            it.jb = 0;
            it.je = (int32_t)(d - 1);
            witems[woff[r]] = it;
            continue;
        }
        int64_t o = ioff[r];
        for (int64_t cb = 0; cb < d; cb += cap) {
            int64_t ce = cb + cap < d ? cb + cap : d;
            int64_t jend = ce - 1;
            for (int64_t jb = 0; jb < jend; jb += jp) {
                Item it;
                it.g = gid;
                it.r = (int32_t)r;
                it.cb = (int32_t)cb;
                it.ce = (int32_t)ce;
                it.jb = (int32_t)jb;
                it.je = (int32_t)(jb + jp < jend ? jb + jp : jend);
                items[o++] = it;
            }
        }
    }
}

// S = sum over hyperwedges (r, j) of |N+(j)|; S[1] the same over the
// hyperwedges at positions < e_split (the owners before the dense window)
__global__ void k_stream_size(const int64_t *fptr, const uint32_t *fadj, int64_t nw, int64_t e_split, int wbits,
                              unsigned long long *S) {
    __shared__ unsigned long long sh[256], sh2[256];
    unsigned long long acc = 0, acc2 = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t j = fadj[e] >> wbits;
        const unsigned long long l = (unsigned long long)(fptr[j + 1] - fptr[j]);
        acc += l;
        if (e < e_split) acc2 += l;
    }
    sh[threadIdx.x] = acc;
    sh2[threadIdx.x] = acc2;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[threadIdx.x] += sh[threadIdx.x + o];
            sh2[threadIdx.x] += sh2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(S, sh[0]);
        atomicAdd(S + 1, sh2[0]);
    }
}

// per-hyperedge counts from the per-wedge role counters: the j- and k-role
// counts of hyperwedge (r, x), e0 <= position < nw, go to x (one thread per
// hyperwedge) ...
__global__ void k_edge_counts_roles(const uint32_t *fadj, int64_t e0, int64_t nw, int wbits, const uint32_t *cwjm,
                                    const uint32_t *cwkm, unsigned long long *t) {
    for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cwjm[e] + cwkm[e];
        if (c) atomicAdd(&t[fadj[e] >> wbits], (unsigned long long)c);
    }
}

// ... and the j-role counts of r's hyperwedges to r (one wave per owner)
__global__ void k_edge_counts_owner(const int64_t *fptr, int64_t m, const uint32_t *cwjm, unsigned long long *t) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < m; r += nwaves) {
        const int64_t b = fptr[r + 1];
        unsigned long long own = 0;
        for (int64_t e = fptr[r] + lane; e < b; e += kWave) own += cwjm[e];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) own += __shfl_xor(own, o, kWave);
        if (lane == 0 && own) atomicAdd(&t[r], own);
    }
}

__global__ void k_rank_to_norm_u64(const unsigned long long *t, const int32_t *norm_of_rank, int64_t m,
                                   int64_t *out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x)
        out[norm_of_rank[r]] = (int64_t)t[r];
}

template <int CAP, int JP, bool PE, bool PW, bool MID>
int occ_blocks() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_close<CAP, JP, PE, PW, MID>, kBlock, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

template <int CAP, int JP, bool MID>
struct CloseVariants {
    static int blocks(bool pe, bool pw) {
        return pe ? (pw ? occ_blocks<CAP, JP, true, true, MID>() : occ_blocks<CAP, JP, true, false, MID>())
                  : (pw ? occ_blocks<CAP, JP, false, true, MID>() : occ_blocks<CAP, JP, false, false, MID>());
    }
    static void launch(bool pe, bool pw, const CloseArgs &a, int nb, hipStream_t s) {
        if (a.tp) {
            // SparseTTT with per-pattern per-hyperedge counts: its own instance (default
            // configuration only), so that the other closures carry none of its code
            if constexpr (CAP == 512 && JP == 256) {
                if (pe || pw) fail(HTRI_E_INVALID, "per-pattern counts of the closure take no per-edge or per-wedge output");
                hipLaunchKernelGGL((k_close<CAP, JP, false, false, MID, true>), dim3(nb), dim3(kBlock), 0, s, a);
                HTRI_LAUNCH_CHECK();
            } else {
                fail(HTRI_E_INVALID, "per-pattern counts of the closure run the default configuration only");
            }
            return;
        }
        if (pe && pw) hipLaunchKernelGGL((k_close<CAP, JP, true, true, MID>), dim3(nb), dim3(kBlock), 0, s, a);
        else if (pe) hipLaunchKernelGGL((k_close<CAP, JP, true, false, MID>), dim3(nb), dim3(kBlock), 0, s, a);
        else if (pw) hipLaunchKernelGGL((k_close<CAP, JP, false, true, MID>), dim3(nb), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_close<CAP, JP, false, false, MID>), dim3(nb), dim3(kBlock), 0, s, a);
        HTRI_LAUNCH_CHECK();
    }
};

}  // namespace

void sum_pattern_parts(const unsigned long long *part, int64_t n, unsigned long long *counts, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sum_parts, dim3(20), dim3(256), 0, s, part, n, counts);
    HTRI_LAUNCH_CHECK();
}

bool valid_config(const CloseConfig &c) {
    return (c.cap == 256 || c.cap == 512) && (c.jp == 128 || c.jp == 256);
}

int close_blocks_per_cu(const CloseConfig &c, bool pe, bool pw, bool mid) {
    if (mid) {
        if (c.cap == 512 && c.jp == 256) return CloseVariants<512, 256, true>::blocks(pe, pw);
        fail(HTRI_E_INVALID, "middle-centric closure runs the default configuration only");
    }
    if (c.cap == 256 && c.jp == 128) return CloseVariants<256, 128, false>::blocks(pe, pw);
    if (c.cap == 256 && c.jp == 256) return CloseVariants<256, 256, false>::blocks(pe, pw);
    if (c.cap == 512 && c.jp == 128) return CloseVariants<512, 128, false>::blocks(pe, pw);
    if (c.cap == 512 && c.jp == 256) return CloseVariants<512, 256, false>::blocks(pe, pw);
    fail(HTRI_E_INVALID, "unsupported closure configuration");
    return 0;
}

void launch_close_kernel(const CloseConfig &c, bool pe, bool pw, const CloseArgs &a, int nb, hipStream_t s,
                         bool mid) {
    if (mid) {
        if (c.cap == 512 && c.jp == 256) return CloseVariants<512, 256, true>::launch(pe, pw, a, nb, s);
        fail(HTRI_E_INVALID, "middle-centric closure runs the default configuration only");
    }
    if (c.cap == 256 && c.jp == 128) return CloseVariants<256, 128, false>::launch(pe, pw, a, nb, s);
    if (c.cap == 256 && c.jp == 256) return CloseVariants<256, 256, false>::launch(pe, pw, a, nb, s);
    if (c.cap == 512 && c.jp == 128) return CloseVariants<512, 128, false>::launch(pe, pw, a, nb, s);
    if (c.cap == 512 && c.jp == 256) return CloseVariants<512, 256, false>::launch(pe, pw, a, nb, s);
    fail(HTRI_E_INVALID, "unsupported closure configuration");
}

GraphDesc graph_desc(const Graph &g) {
    GraphDesc d{};
    d.fptr = g.fptr.p;
    d.fadj = g.fadj.p;
    d.mptr = g.mptr.p;
    d.fmask = g.fmask.p;
    d.esize = g.esize.p;
    d.eptr = g.eptr.p;
    d.emem = g.emem.p;
    d.wbits = g.wbits;
    return d;
}

// ---------------------------------------------------------------- in-list

namespace {

// Middle-centric work items per middle j (at least one forward entry and one
// in-list entry): wcnt = 1 for a middle closed by one wave (at most
// kWaveMidHashMax forward entries, at most kWaveOwnerMax in-list entries, at
// most one Omega word, and at most kWaveStreamMax streamed entries), else
// one block item per chunk of N+(j) and piece of jp in-list entries.
__global__ void k_item_counts_mid(const int64_t *fptr, const int64_t *iptr, const uint4 *inl, const int32_t *esize,
                                  int wbits, int64_t m, int cap, int jp, int64_t *cnt, int64_t *wcnt) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = fptr[j + 1] - fptr[j];
        const int64_t nin = iptr[j + 1] - iptr[j];
        int64_t c = 0;
        bool wave = false;
        if (d >= 1 && nin >= 1) {
            if (d <= kWaveMidHashMax && nin <= kWaveOwnerMax && mask_words(esize[j]) <= 1) {
                int64_t sz = 0;
                for (int64_t p = iptr[j]; p < iptr[j + 1]; p++) sz += (int64_t)(inl[p].y >> wbits);
                wave = sz <= kWaveStreamMax;
            }
            if (!wave) c = ((d + cap - 1) / cap) * ((nin + jp - 1) / jp);
        }
        cnt[j] = c;
        wcnt[j] = wave ? 1 : 0;
    }
}

__global__ void k_item_fill_mid(const int64_t *fptr, const int64_t *iptr, int64_t m, int cap, int jp, int32_t gid,
                                const int64_t *ioff, const int64_t *woff, Item *items, Item *witems) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = fptr[j + 1] - fptr[j];
        const int64_t nin = iptr[j + 1] - iptr[j];
        if (d < 1 || nin < 1) continue;
        if (woff[j + 1] != woff[j]) {
            witems[woff[j]] = Item{gid, (int32_t)j, 0, (int32_t)d, 0, (int32_t)nin};
            continue;
        }
        int64_t o = ioff[j];
        for (int64_t cb = 0; cb < d; cb += cap) {
            const int64_t ce = cb + cap < d ? cb + cap : d;
            for (int64_t jb = 0; jb < nin; jb += jp)
                items[o++] = Item{gid, (int32_t)j, (int32_t)cb, (int32_t)ce, (int32_t)jb,
                                  (int32_t)(jb + jp < nin ? jb + jp : nin)};
        }
    }
}

int64_t read_i64(const int64_t *p, hipStream_t s) {
    int64_t v = 0;
    HTRI_HIP(hipMemcpyAsync(&v, p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    return v;
}

// scan the per-owner item counts, allocate the lists and let fill() write them
template <typename F>
void items_from_counts(Graph &g, DBuf<int64_t> &icnt, DBuf<int64_t> &wcnt, ItemLists &out, F fill) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    scan_exclusive_i64(A, icnt.p, icnt.p, m, icnt.p + m, s);
    scan_exclusive_i64(A, wcnt.p, wcnt.p, m, wcnt.p + m, s);
    int64_t tot[2] = {0, 0};
    tot[0] = host_read(icnt.p + m, s);
    tot[1] = host_read(wcnt.p + m, s);
    out.nblock = tot[0];
    out.nwave = tot[1];
    // the item counters are 32-bit and run past the end by one claim per block or wave
    const int64_t limit = (int64_t)UINT32_MAX - ((int64_t)1 << 24);
    if (out.nblock >= limit || out.nwave >= limit) fail(HTRI_E_UNSUPPORTED, "too many work items");
    out.block.alloc(A, out.nblock);
    out.wave.alloc(A, out.nwave);
    if (m > 0 && out.nblock + out.nwave > 0) fill();
    stream_sync(s);
}

}  // namespace

void build_items(Graph &g, int32_t gid, const CloseConfig &cfg, ItemLists &out, int64_t owner_end) {
    hipStream_t s = g.stream;
    const int64_t m = g.m;
    DBuf<int64_t> icnt(g.al, m + 1), wcnt(g.al, m + 1);
    if (m > 0) {
        hipLaunchKernelGGL(k_item_counts, dim3(grid_for(m, 256)), dim3(256), 0, s, g.fptr.p, g.fadj.p, g.wbits, m,
                           owner_end, cfg.cap, cfg.jp, icnt.p, wcnt.p);
        HTRI_LAUNCH_CHECK();
    }
    items_from_counts(g, icnt, wcnt, out, [&] {
        hipLaunchKernelGGL(k_item_fill, dim3(grid_for(m, 256)), dim3(256), 0, s, g.fptr.p, m, owner_end, cfg.cap,
                           cfg.jp, gid, icnt.p, wcnt.p, out.block.p, out.wave.p);
        HTRI_LAUNCH_CHECK();
    });
}

void build_items_mid(Graph &g, int32_t gid, const CloseConfig &cfg, const InList &in, ItemLists &out) {
    hipStream_t s = g.stream;
    const int64_t m = g.m;
    DBuf<int64_t> icnt(g.al, m + 1), wcnt(g.al, m + 1);
    if (m > 0) {
        hipLaunchKernelGGL(k_item_counts_mid, dim3(grid_for(m, 256)), dim3(256), 0, s, g.fptr.p, in.iptr.p, in.inl.p,
                           g.esize.p, g.wbits, m, cfg.cap, cfg.jp, icnt.p, wcnt.p);
        HTRI_LAUNCH_CHECK();
    }
    items_from_counts(g, icnt, wcnt, out, [&] {
        hipLaunchKernelGGL(k_item_fill_mid, dim3(grid_for(m, 256)), dim3(256), 0, s, g.fptr.p, in.iptr.p, m, cfg.cap,
                           cfg.jp, gid, icnt.p, wcnt.p, out.block.p, out.wave.p);
        HTRI_LAUNCH_CHECK();
    });
}

// ---------------------------------------------------------------- dense window

namespace {

// The owners of the top ranks [w0, m) are closed by bitmap intersection.
// Every forward neighbour of such an owner also lies in [w0, m), so each
// hyperedge x of the window gets a row bitmap over the window: BF_x =
// N+(x), BF1_x = its entries with omega = 1, and BI1_x = {j : x in N+(j),
// omega_jx = 1} (the transpose of BF1), plus exclusive popcount prefixes of
// BF_x per 32-bit word (position of an entry in N+(x)).  The closure of a
// hyperwedge (r, j) is then |BF_r & BF_j|.  The common-vertex pattern is
// counted in bulk: for a class K_v = {k in N+(r) : omega_rk = 1, Omega_rk =
// {v}, |e_k| > 1} (v one vertex of e_r), a partner j in K_v closes a
// common-vertex triangle with exactly the k in K_v with omega_jk = 1 (the
// three pairwise intersections are then all {v} and every hyperedge has a
// private vertex), i.e. |K_v & BF1_j|.  The owner's kWinClasses largest
// classes are counted this way; the other hits are enumerated bit by bit and
// classified by their regions like probed hits.
constexpr int kWinRowsMax = (int)kWindowRowsMax;
constexpr int kWinWordsMax = kWinRowsMax / 32;
constexpr int kWinClasses = 8;              // bulk-counted classes at most (fewer for wide windows)
constexpr int kWinLdsBudget = 60 * 1024;    // bytes of row bitmaps per block of k_close_window
constexpr int kEnumQ = 64;                  // queued hits per wave in k_close_window
constexpr int kWinPartners = 8;             // partners closed side by side per wave

// exclusive prefix of popcounts of x[0..n) into out (n up to kWinWordsMax),
// whole block, contiguous chunks per thread
__device__ __forceinline__ void block_popcount_prefix(const uint32_t *x, int n, int32_t *out, int32_t *wsum) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (n + nt - 1) / nt;
    const int a = tid * per, b = min(n, a + per);
    int own = 0;
    for (int w = a; w < b; w++) own += __popc(x[w]);
    int incl = own;
    const int lane = tid & (kWave - 1), wv = tid / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int u = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += u;
    }
    if (lane == kWave - 1) wsum[wv] = incl;
    __syncthreads();
    int run = incl - own;
    for (int q = 0; q < wv; q++) run += wsum[q];
    for (int w = a; w < b; w++) {
        out[w] = run;
        run += __popc(x[w]);
    }
    __syncthreads();
}

// one block per window row; dynamic shared memory: two rows of nwords words
// and their prefix
__global__ __launch_bounds__(256) void k_window_rows(const int64_t *fptr, const uint32_t *fadj, int wbits, int64_t w0,
                                                     int nwords, uint32_t *bf, uint32_t *bf1, uint32_t *pf) {
    extern __shared__ uint32_t dyn[];
    uint32_t *rf = dyn, *r1 = dyn + nwords;
    int32_t *pre = (int32_t *)(dyn + 2 * nwords);
    __shared__ int32_t wsum[256 / kWave];
    const int tid = threadIdx.x;
    const int row = blockIdx.x;
    const uint32_t wmask = (1u << wbits) - 1;
    for (int w = tid; w < nwords; w += blockDim.x) rf[w] = r1[w] = 0u;
    __syncthreads();
    const int64_t b = fptr[w0 + row], e = fptr[w0 + row + 1];
    for (int64_t i = b + tid; i < e; i += blockDim.x) {
        const uint32_t ent = fadj[i];
        const int kr = (int)((int64_t)(ent >> wbits) - w0);          // in (row, nrows)
        atomicOr(&rf[kr >> 5], 1u << (kr & 31));
        if ((ent & wmask) == 1u) atomicOr(&r1[kr >> 5], 1u << (kr & 31));
    }
    __syncthreads();
    block_popcount_prefix(rf, nwords, pre, wsum);
    const int64_t ro = (int64_t)row * nwords;
    for (int w = tid; w < nwords; w += blockDim.x) {
        bf[ro + w] = rf[w];
        bf1[ro + w] = r1[w];
        pf[ro + w] = (uint32_t)pre[w];
    }
}

// bi1, the transpose of bf1 as an nrows x nrows bit matrix: one wave per 64
// rows and 8 words (256 columns) of bf1; bit j of word J over the 64 rows is
// one ballot, whose halves are words 2X and 2X + 1 of bi1's row 32 J + j.
// Every word of bi1 is written once.
__global__ __launch_bounds__(256) void k_window_transpose(const uint32_t *bf1, int nrows, int nwords, uint32_t *bi1) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nx = (nrows + 63) / 64, nj = (nwords + 7) / 8;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; t < nx * nj; t += nw) {
        const int X = (int)(t / nj), J0 = (int)(t % nj) * 8;
        const int x = X * 64 + lane;
        uint32_t w[8];
#pragma unroll
        for (int jw = 0; jw < 8; jw++)
            w[jw] = (x < nrows && J0 + jw < nwords) ? bf1[(int64_t)x * nwords + J0 + jw] : 0u;
#pragma unroll
        for (int jw = 0; jw < 8; jw++) {
            uint32_t out = 0u;
#pragma unroll
            for (int j = 0; j < 32; j++) {
                const uint64_t b = __ballot((w[jw] >> j) & 1u);
                if ((lane & 31) == j) out = lane < 32 ? (uint32_t)b : (uint32_t)(b >> 32);
            }
            const int c = 32 * (J0 + jw) + (lane & 31), word = 2 * X + (lane >> 5);
            if (c < nrows && word < nwords) bi1[(int64_t)c * nwords + word] = out;
        }
    }
}

struct WinArgs {
    GraphDesc G;
    int64_t w0;
    int nrows, nwords;
    const uint32_t *bf, *bf1, *bi1;
    const uint32_t *pf;
    int max_classes;                // class bitmaps that fit the block's shared memory
    const uint8_t *lut;
    uint32_t emask;
    unsigned int *queue;
    unsigned long long *counts;     // [21]
    unsigned long long *block_part; // each block's pattern counts [blocks][21], summed afterwards
    unsigned long long *stats;      // [0] bitmap words read, [1] hits enumerated
    uint32_t *cwj, *cwjm, *cwkm;
    unsigned long long *tp;         // as CloseArgs::tp (null: not kept)
};

// dynamic shared memory: BR, PR and max_classes class rows of nwords words
template <bool PER_EDGE, bool PER_WEDGE>
__global__ __launch_bounds__(kBlock, 6) void k_close_window(WinArgs A) {
    extern __shared__ uint32_t dyn[];
    uint32_t *BR = dyn;
    int32_t *PR = (int32_t *)(dyn + A.nwords);
    uint32_t *BKbase = dyn + 2 * A.nwords;
    auto BK = [&](int c) { return BKbase + (int64_t)c * A.nwords; };
    __shared__ uint32_t cls[32 * kMaskWordsMax];
    __shared__ int32_t cslot[32 * kMaskWordsMax];  // class slot of member position v, or -1
    __shared__ int32_t wsum[kBlock / kWave];
    __shared__ unsigned long long cnt[21];
    __shared__ int sh_row, sh_nc;
    __shared__ uint64_t enumq[(kBlock / kWave) * kEnumQ];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const GraphDesc &G = A.G;
    const int wbits = G.wbits;
    const uint32_t wmask = (1u << wbits) - 1;
    const int nwords = A.nwords;
    const bool count9 = (A.emask >> kPatternCommonVertex) & 1u;
    if (tid < 21) cnt[tid] = 0ull;
    unsigned long long words_read = 0, enumerated = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const unsigned int c = atomicAdd(A.queue, 1u);
            sh_row = (int64_t)c < A.nrows ? (int)c : -1;
        }
        __syncthreads();
        const int row = sh_row;
        if (row < 0) break;
        const int32_t r = (int32_t)(A.w0 + row);
        const int64_t base = gld(G.fptr + r);
        const int d = (int)(gld(G.fptr + r + 1) - base);
        if (d < 2) continue;
        const int si = gld(G.esize + r);
        const int W = mask_words(si);
        const int64_t mbase = gld(G.mptr + r);
        for (int w = tid; w < nwords; w += kBlock) BR[w] = 0u;
        if (tid < 32 * kMaskWordsMax) cls[tid] = 0u;
        __syncthreads();
        const bool classes = (W >= 1) && (si >= 2);
        // member position of the single shared vertex of an omega = 1 entry
        auto single_pos = [&](int64_t q) -> int {
            for (int w = 0; w < W; w++) {
                const uint32_t x = gld(G.fmask + mbase + q * W + w);
                if (x) return 32 * w + __ffs(x) - 1;
            }
            return -1;
        };
        for (int q = tid; q < d; q += kBlock) {
            const uint32_t ent = gld(G.fadj + base + q);
            const int kr = (int)((int64_t)(ent >> wbits) - A.w0);
            atomicOr(&BR[kr >> 5], 1u << (kr & 31));
            if (classes && (ent & wmask) == 1u && gld(G.esize + (ent >> wbits)) > 1) {
                const int v = single_pos(q);
                if (v >= 0) atomicAdd(&cls[v], 1u);
            }
        }
        __syncthreads();
        if (tid == 0) {
            // the kWinClasses largest classes with at least two members
            int nc = 0;
            const int npos = 32 * W;
            for (int v = 0; v < 32 * kMaskWordsMax; v++) cslot[v] = -1;
            if (classes) {
                for (; nc < A.max_classes; nc++) {
                    int best = -1;
                    uint32_t bc = 1;
                    for (int v = 0; v < npos; v++)
                        if (cslot[v] < 0 && cls[v] > bc) { bc = cls[v]; best = v; }
                    if (best < 0) break;
                    cslot[best] = nc;
                }
            }
            sh_nc = nc;
        }
        // exclusive popcount prefix of BR (positions in N+(r)); ends with a barrier
        block_popcount_prefix(BR, nwords, PR, wsum);
        const int nc = sh_nc;
        for (int t = tid; t < nc * nwords; t += kBlock) BKbase[t] = 0u;
        __syncthreads();
        // class slot of an entry of N+(r), or -1
        auto class_of = [&](uint32_t ent, int64_t q) -> int {
            if (nc == 0 || (ent & wmask) != 1u || gld(G.esize + (ent >> wbits)) <= 1) return -1;
            const int v = single_pos(q);
            return v >= 0 ? cslot[v] : -1;
        };
        if (nc > 0) {
            for (int q = tid; q < d; q += kBlock) {
                const uint32_t ent = gld(G.fadj + base + q);
                const int c = class_of(ent, q);
                if (c >= 0) {
                    const int kr = (int)((int64_t)(ent >> wbits) - A.w0);
                    atomicOr(&BK(c)[kr >> 5], 1u << (kr & 31));
                }
            }
        }
        __syncthreads();
        // k-role of the common-vertex triangles: for k in class c, |K_c & BI1_k|
        // (8 lanes per entry, eight entries per wave: the word ranges are often short)
        if (PER_EDGE) {
            constexpr int kGroup = 8;
            const int sub = lane / kGroup, gl = lane % kGroup;
            for (int qb = wave * (kWave / kGroup); qb < d; qb += kBlock / kGroup) {
                const int q = qb + sub;
                uint32_t kf = 0;
                unsigned long long rg = 0;
                if (q < d) {
                    const uint32_t ent = gld(G.fadj + base + q);
                    const int kr = (int)((int64_t)(ent >> wbits) - A.w0);
                    const int c = count9 ? class_of(ent, q) : -1;
                    if (c >= 0) {
                        const uint32_t *bik = A.bi1 + (int64_t)kr * nwords;
                        for (int w = (row >> 5) + gl; w <= (kr >> 5); w += kGroup) kf += __popc(BK(c)[w] & gld(bik + w));
                        rg = (unsigned long long)((kr >> 5) - (row >> 5) + 1);
                    }
                }
#pragma unroll
                for (int o = kGroup / 2; o > 0; o >>= 1) kf += __shfl_xor(kf, o, kWave);
#pragma unroll
                for (int g2 = 0; g2 < kWave / kGroup; g2++) words_read += __shfl(rg, g2 * kGroup, kWave);
                if (gl == 0 && q < d) A.cwkm[base + q] = kf;
            }
            __threadfence();
            __syncthreads();
        }
        // Hits outside the bulk-counted classes, (position in N+(r), position
        // in N+(j), partner) with 17 bits each, wait in the wave's queue and
        // are classified one lane per hit when the queue fills and after the
        // last partner, so that their dependent loads run side by side.
        uint64_t *Q = enumq + wave * kEnumQ;
        int qn = 0;                                   // wave-uniform
        // classify one hit; returns whether it counts in the per-hyperedge
        // counts (its k-role is added here, its j-role by the caller)
        auto classify_hit = [&](int pr, int pj, int qq) -> bool {
            const uint32_t jent = gld(G.fadj + base + qq);
            const int32_t j = (int32_t)(jent >> wbits);
            const int wij = (int)(jent & wmask);
            const int sj = gld(G.esize + j);
            const int64_t jbase = gld(G.fptr + j);
            const uint32_t kent = gld(G.fadj + base + pr);
            const int32_t k = (int32_t)(kent >> wbits);
            const int wik = (int)(kent & wmask);
            const int wjk = (int)(gld(G.fadj + jbase + pj) & wmask);
            const int sk = gld(G.esize + k);
            int g;
            if (W > 0) {
                g = 0;
                for (int x = 0; x < W; x++)
                    g += __popc(gld(G.fmask + mbase + (int64_t)qq * W + x) & gld(G.fmask + mbase + (int64_t)pr * W + x));
            } else {
                g = triple_common(G.eptr, G.emem, r, j, k);
            }
            // SparseTTT-only counting (emask bit 31): a hit with a vertex
            // common to all three hyperedges is dropped
            if (((A.emask >> 31) & 1u) && g > 0) return false;
            const uint32_t p = A.lut[region_mask(si, sj, sk, wij, wik, wjk, g)];
            atomicAdd(&cnt[p], 1ull);
            if (A.tp) {
                atomicAdd(&A.tp[(int64_t)r * 21 + p], 1ull);
                atomicAdd(&A.tp[(int64_t)j * 21 + p], 1ull);
                atomicAdd(&A.tp[(int64_t)k * 21 + p], 1ull);
            }
            enumerated++;
            const bool counted = PER_EDGE && ((A.emask >> p) & 1u);
            if (counted) atomicAdd(&A.cwkm[base + pr], 1u);
            return counted;
        };
        // The queue is in partner order: the j-role counts of a run of equal
        // partners go out as one atomic, from the run's last lane.
        auto flush = [&]() {
            wave_lds_sync();
            int qq = -1;
            bool counted = false;
            if (lane < qn) {
                const uint64_t e = Q[lane];
                qq = (int)(e >> 34);
                counted = classify_hit((int)(e & 0x1FFFFu), (int)((e >> 17) & 0x1FFFFu), qq);
            }
            if (PER_EDGE) {
                const int qprev = __shfl_up(qq, 1, kWave);
                const int qnext = __shfl_down(qq, 1, kWave);
                const uint64_t starts = __ballot(lane < qn && (lane == 0 || qprev != qq));
                const uint64_t cm = __ballot(counted);
                if (lane < qn && (lane == qn - 1 || qnext != qq)) {
                    const uint64_t upto = (2ull << lane) - 1ull;   // lanes 0 .. lane (all 64 for lane 63)
                    const int s0 = 63 - __clzll(starts & upto);
                    const uint32_t n = (uint32_t)__popcll(cm & upto & ~((1ull << s0) - 1ull));
                    if (n) atomicAdd(&A.cwjm[base + qq], n);
                }
            }
            wave_lds_sync();
            qn = 0;
        };
        // partners: entries 0 .. d-2, kWinPartners per wave (kPG lanes each:
        // the partners' set-up loads overlap and short rows fill the lanes)
        constexpr int kPG = kWave / kWinPartners;
        const int psub = lane / kPG, pl = lane % kPG;
        for (int qb = wave * kWinPartners; qb < d - 1; qb += (kBlock / kWave) * kWinPartners) {
            const int q = qb + psub;
            const bool qv = q < d - 1;
            uint32_t jent = 0u;
            int jr = nwords * 32, cj = -1;
            if (qv) {
                jent = gld(G.fadj + base + q);
                jr = (int)((jent >> wbits) - (uint32_t)A.w0);
                cj = class_of(jent, q);
            }
            const bool dom = cj >= 0;
            const uint32_t *bfj = A.bf + (int64_t)(qv ? jr : 0) * nwords;
            const uint32_t *bf1j = A.bf1 + (int64_t)(qv ? jr : 0) * nwords;
            const uint32_t *pfj = A.pf + (int64_t)(qv ? jr : 0) * nwords;
            const int wfirst = qv ? (jr >> 5) : nwords;
            int wmin = wfirst;              // the wave's loop covers every group's row
#pragma unroll
            for (int g2 = 1; g2 < kWinPartners; g2++) wmin = min(wmin, __shfl(wfirst, g2 * kPG, kWave));
            const int span = nwords - __shfl(wmin, 0, kWave);
            uint32_t all = 0, fast = 0;
            for (int t0 = 0; t0 < span; t0 += kPG) {
                const int w = wfirst + t0 + pl;
                uint32_t bw = 0u, a = 0u, non = 0u;
                if (w < nwords) {
                    bw = gld(bfj + w);
                    a = BR[w] & bw;
                    all += __popc(a);
                    const uint32_t fs = dom ? (BK(cj)[w] & gld(bf1j + w)) : 0u;
                    fast += __popc(fs);
                    non = a & ~fs;
                }
                if (!__ballot(non != 0u)) continue;
                const int c = __popc(non);
                int incl = c;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const int t = __shfl_up(incl, o, kWave);
                    if (lane >= o) incl += t;
                }
                const int total = __shfl(incl, kWave - 1, kWave);
                if (qn + total > kEnumQ) flush();
                if (total <= kEnumQ) {
                    int slot = qn + incl - c;
                    if (non) {
                        const int pr0 = PR[w];
                        const uint32_t brw = BR[w];
                        const int pj0 = (int)gld(pfj + w);
                        while (non) {
                            const int bpos = __ffs(non) - 1;
                            non &= non - 1;
                            const uint32_t below = (1u << bpos) - 1u;
                            const uint64_t pr = (uint64_t)(pr0 + __popc(brw & below));   // position of k in N+(r)
                            const uint64_t pj = (uint64_t)(pj0 + __popc(bw & below));    // position of k in N+(j)
                            Q[slot++] = pr | (pj << 17) | ((uint64_t)q << 34);
                        }
                    }
                    qn += total;
                } else {
                    // more hits in this step than the queue holds: classify them in place
                    while (non) {
                        const int bpos = __ffs(non) - 1;
                        non &= non - 1;
                        const uint32_t below = (1u << bpos) - 1u;
                        if (classify_hit(PR[w] + __popc(BR[w] & below), (int)gld(pfj + w) + __popc(bw & below), q))
                            atomicAdd(&A.cwjm[base + q], 1u);
                    }
                }
            }
            const unsigned long long rg = qv ? (unsigned long long)(nwords - (jr >> 5)) * (dom ? 2u : 1u) : 0ull;
#pragma unroll
            for (int g2 = 0; g2 < kWinPartners; g2++) words_read += __shfl(rg, g2 * kPG, kWave);
#pragma unroll
            for (int o = kPG / 2; o > 0; o >>= 1) {
                all += __shfl_xor(all, o, kWave);
                fast += __shfl_xor(fast, o, kWave);
            }
            if (pl == 0 && qv) {
                if (fast && !((A.emask >> 31) & 1u)) atomicAdd(&cnt[kPatternCommonVertex], (unsigned long long)fast);
                if (PER_WEDGE) A.cwj[base + q] = all;
                // the enumerated hits add theirs when they are classified
                if (PER_EDGE && count9 && fast) atomicAdd(&A.cwjm[base + q], fast);
            }
        }
        if (qn > 0) flush();
    }
    __syncthreads();
    if (tid < 21) A.block_part[(int64_t)blockIdx.x * 21 + tid] = tid >= 1 ? cnt[tid] : 0ull;
    // words_read is per wave (lane 0's copy counts); enumerated is per lane
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) enumerated += __shfl_xor(enumerated, o, kWave);
    if (lane == 0) {
        atomicAdd(&A.stats[0], words_read);
        atomicAdd(&A.stats[1], enumerated);
    }
}

}  // namespace

WindowPlan choose_window(Graph &g, uint32_t flags) {
    WindowPlan w;
    w.w0 = g.m;
    if ((flags & HTRI_COUNT_NO_WINDOW) || g.m < 3 || g.nw == 0) return w;
    auto fptr_at = [&](int64_t i) {
        int64_t v = 0;
        HTRI_HIP(hipMemcpyAsync(&v, g.fptr.p + i, sizeof(int64_t), hipMemcpyDeviceToHost, g.stream));
        HTRI_HIP(hipStreamSynchronize(g.stream));
        return v;
    };
    const int64_t e_end = fptr_at(g.m);
    // candidates: the whole graph (or the largest window), then every power of
    // two below it down to 1024 rows (the starts window_start() lists)
    std::vector<int64_t> cands{std::min<int64_t>(g.m, kWinRowsMax)};
    for (int s = 0; s < kWindowStarts; s++) {
        const int64_t c = kWindowRowsMax >> s;
        if (c < cands[0]) cands.push_back(c);
    }
    for (const int64_t n : cands) {
        const int64_t w0 = g.m - n;
        const int64_t inside = e_end - fptr_at(w0);
        if (inside == 0) continue;
        const double density = (double)inside / (0.5 * (double)n * (double)n);
        if ((flags & HTRI_COUNT_WINDOW_ALWAYS) || density >= 1.0 / 8.0) {
            w.w0 = w0;
            w.nrows = (int)n;
            w.nwords = (int)((n + 31) / 32);
            w.wedges = inside;
            return w;
        }
    }
    return w;
}

void close_window(Graph &g, const WindowPlan &w, uint32_t emask, const uint8_t *lut_dev, unsigned long long *counts,
                  unsigned long long *stats, uint32_t *cwj, uint32_t *cwjm, uint32_t *cwkm, unsigned long long *tp) {
    if (w.nrows == 0) return;
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t cells = (int64_t)w.nrows * w.nwords;
    DBuf<uint32_t> bf(A, cells), bf1(A, cells), bi1(A, cells);
    DBuf<uint32_t> pf(A, cells);
    DBuf<unsigned int> queue(A, 1);
    fill_u32(queue.p, 1, 0, s);
    hipLaunchKernelGGL(k_window_rows, dim3(w.nrows), dim3(256), (size_t)3 * w.nwords * sizeof(uint32_t), s, g.fptr.p,
                       g.fadj.p, g.wbits, w.w0, w.nwords, bf.p, bf1.p, pf.p);
    HTRI_LAUNCH_CHECK();
    {
        const int64_t tasks = (int64_t)((w.nrows + 63) / 64) * ((w.nwords + 7) / 8);
        hipLaunchKernelGGL(k_window_transpose, dim3(grid_for(tasks * kWave, 256, 8192)), dim3(256), 0, s, bf1.p,
                           w.nrows, w.nwords, bi1.p);
        HTRI_LAUNCH_CHECK();
    }
    WinArgs a;
    a.G = graph_desc(g);
    a.w0 = w.w0;
    a.nrows = w.nrows;
    a.nwords = w.nwords;
    a.bf = bf.p;
    a.bf1 = bf1.p;
    a.bi1 = bi1.p;
    a.pf = pf.p;
    a.max_classes = std::max(0, std::min(kWinClasses, kWinLdsBudget / (4 * w.nwords) - 2));
    const size_t shmem = (size_t)(2 + a.max_classes) * w.nwords * sizeof(uint32_t);
    a.lut = lut_dev;
    a.emask = emask;
    a.queue = queue.p;
    a.counts = counts;
    a.stats = stats;
    a.cwj = cwj;
    a.cwjm = cwjm;
    a.cwkm = cwkm;
    a.tp = tp;
    const bool pe = cwjm != nullptr, pw = cwj != nullptr;
    int nb = 0;
    hipError_t oe;
    if (pe && pw) oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_close_window<true, true>, kBlock, shmem);
    else if (pe) oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_close_window<true, false>, kBlock, shmem);
    else if (pw) oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_close_window<false, true>, kBlock, shmem);
    else oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_close_window<false, false>, kBlock, shmem);
    if (oe != hipSuccess || nb < 1) nb = 1;
    const int grid = (int)std::min<int64_t>((int64_t)device_cu_count() * nb, w.nrows);
    DBuf<unsigned long long> bpart(g.al, (int64_t)grid * 21);
    a.block_part = bpart.p;
    if (pe && pw) hipLaunchKernelGGL((k_close_window<true, true>), dim3(grid), dim3(kBlock), shmem, s, a);
    else if (pe) hipLaunchKernelGGL((k_close_window<true, false>), dim3(grid), dim3(kBlock), shmem, s, a);
    else if (pw) hipLaunchKernelGGL((k_close_window<false, true>), dim3(grid), dim3(kBlock), shmem, s, a);
    else hipLaunchKernelGGL((k_close_window<false, false>), dim3(grid), dim3(kBlock), shmem, s, a);
    HTRI_LAUNCH_CHECK();
    sum_pattern_parts(bpart.p, grid, counts, s);
    // the bitmaps are freed when this returns: wait for the kernels
    HTRI_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- inclusion classes

namespace {

// Every hyper-triangle of the classes CCC, TCC and TTC (patterns 1-8) holds
// at least one inclusion hyperwedge (Def. 2.3), and those are few, so these
// classes are counted by searching around the inclusion hyperwedges only
// (the approach of Count-CCC, Count-TCC and Count-TTC, Section 3.1).  For an
// inclusion hyperwedge e_s < e_L (e_s a proper subset of e_L) the third
// hyperedges are the other hyperedges meeting e_s (a vertex of e_s is a
// vertex of e_L), with omega_sk = |e_s & e_k| = g and omega_Lk from a
// merge of member lists.  A triangle with several inclusion hyperwedges is
// counted at the least of them (pairs ordered by (smaller rank, larger rank));
// a candidate k is taken once, at its smallest common vertex with e_s.

// inclusion hyperwedges as (owner, partner) rank pairs; one wave per owner
__global__ void k_incl_pairs(const int64_t *fptr, const uint32_t *fadj, const int32_t *esize, int64_t m, int wbits,
                             unsigned long long *n, int2 *pairs) {
    const uint32_t wmask = (1u << wbits) - 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < m; r += nwaves) {
        const int32_t sr = esize[r];
        for (int64_t e = fptr[r] + lane; e < fptr[r + 1]; e += kWave) {
            const uint32_t ent = fadj[e];
            const int32_t j = (int32_t)(ent >> wbits);
            const int32_t sj = esize[j];
            if ((int32_t)(ent & wmask) == (sr < sj ? sr : sj)) {
                const unsigned long long at = atomicAdd(n, 1ull);
                pairs[at] = make_int2((int32_t)r, j);
            }
        }
    }
}

// forward-adjacency positions of the inclusion hyperwedges; one wave per owner
__global__ void k_incl_index(const int64_t *fptr, const uint32_t *fadj, const int32_t *esize, int64_t m, int wbits,
                             unsigned long long *n, int64_t cap, int64_t *idx) {
    const uint32_t wmask = (1u << wbits) - 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < m; r += nwaves) {
        const int32_t sr = esize[r];
        for (int64_t e = fptr[r] + lane; e < fptr[r + 1]; e += kWave) {
            const uint32_t ent = fadj[e];
            const int32_t sj = esize[ent >> wbits];
            if ((int32_t)(ent & wmask) == (sr < sj ? sr : sj)) {
                const unsigned long long at = atomicAdd(n, 1ull);
                if ((int64_t)at < cap) idx[at] = e;
            }
        }
    }
}

// |e_a & e_b| of two sorted member lists, and their smallest common vertex (or -1)
__device__ __forceinline__ int common_members(const int64_t *eptr, const int32_t *emem, int32_t a, int32_t b,
                                              int32_t &first) {
    int64_t x = eptr[a], xe = eptr[a + 1], y = eptr[b], ye = eptr[b + 1];
    int c = 0;
    first = -1;
    while (x < xe && y < ye) {
        const int32_t u = emem[x], v = emem[y];
        if (u < v) x++;
        else if (v < u) y++;
        else {
            if (c == 0) first = u;
            c++;
            x++;
            y++;
        }
    }
    return c;
}

__device__ __forceinline__ uint64_t pair_key(int32_t a, int32_t b) {
    const uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return ((uint64_t)lo << 32) | hi;
}

// one block per inclusion hyperwedge
// (with out: the triangles of pattern `target` written as sorted triples of
// normalised ids while room lasts, found counting them all)
__global__ __launch_bounds__(kBlock) void k_incl_count(const int2 *pairs, const int64_t *eptr, const int32_t *emem,
                                                       const int32_t *esize, const int64_t *vptr,
                                                       const int32_t *vadj, const uint8_t *lut_g, uint32_t emask,
                                                       unsigned long long *counts, unsigned long long *t,
                                                       int target, const int32_t *norm_of_rank, int64_t capacity,
                                                       int32_t *out, unsigned long long *found,
                                                       unsigned long long *tp) {
    __shared__ unsigned long long cnt[21];
    __shared__ uint8_t lut[128];
    const int tid = threadIdx.x;
    if (tid < 21) cnt[tid] = 0ull;
    if (tid < 128) lut[tid] = lut_g[tid];
    __syncthreads();
    const int2 pr = pairs[blockIdx.x];
    const bool first_small = esize[pr.x] < esize[pr.y];
    const int32_t sv = first_small ? pr.x : pr.y, Lv = first_small ? pr.y : pr.x;   // e_s inside e_L
    const int ss = esize[sv], sL = esize[Lv];
    const uint64_t key_sL = pair_key(sv, Lv);
    for (int64_t q = eptr[sv]; q < eptr[sv + 1]; q++) {
        const int32_t v = emem[q];
        for (int64_t x = vptr[v] + tid; x < vptr[v + 1]; x += kBlock) {
            const int32_t k = vadj[x];
            if (k == sv || k == Lv) continue;
            int32_t first;
            const int wsk = common_members(eptr, emem, sv, k, first);
            if (first != v) continue;                       // k is taken at its smallest common vertex
            int32_t f2;
            const int wLk = common_members(eptr, emem, Lv, k, f2);
            const int sk = esize[k];
            // count at the least inclusion hyperwedge of the triangle
            if (wsk == (ss < sk ? ss : sk) && pair_key(sv, k) < key_sL) continue;
            if (wLk == (sL < sk ? sL : sk) && pair_key(Lv, k) < key_sL) continue;
            const uint32_t p = lut[region_mask(ss, sL, sk, ss, wsk, wLk, wsk)];
            atomicAdd(&cnt[p], 1ull);
            if (out && (int)p == target) {
                const unsigned long long at = atomicAdd(found, 1ull);
                if ((int64_t)at < capacity) {
                    int32_t a = norm_of_rank[sv], b = norm_of_rank[Lv], c = norm_of_rank[k];
                    if (a > b) { const int32_t x = a; a = b; b = x; }
                    if (b > c) { const int32_t x = b; b = c; c = x; }
                    if (a > b) { const int32_t x = a; a = b; b = x; }
                    out[at * 3 + 0] = a;
                    out[at * 3 + 1] = b;
                    out[at * 3 + 2] = c;
                }
            }
            if (t && ((emask >> p) & 1u)) {
                atomicAdd(&t[sv], 1ull);
                atomicAdd(&t[Lv], 1ull);
                atomicAdd(&t[k], 1ull);
            }
            if (tp) {   // per hyperedge and pattern (rank order, 21 per hyperedge)
                atomicAdd(&tp[(int64_t)sv * 21 + p], 1ull);
                atomicAdd(&tp[(int64_t)Lv * 21 + p], 1ull);
                atomicAdd(&tp[(int64_t)k * 21 + p], 1ull);
            }
        }
    }
    __syncthreads();
    if (tid >= 1 && tid < 21 && cnt[tid]) atomicAdd(&counts[tid], cnt[tid]);
}

}  // namespace

int64_t list_inclusion_wedges(Graph &g, DBuf<int64_t> &out) {
    hipStream_t s = g.stream;
    const int64_t nc = g.summary[2];
    out.alloc(g.al, nc);
    DBuf<unsigned long long> n(g.al, 1);
    fill_u64((uint64_t *)n.p, 1, 0, s);
    if (g.m > 0 && nc > 0) {
        hipLaunchKernelGGL(k_incl_index, dim3(grid_for(g.m * kWave, 256, 8192)), dim3(256), 0, s, g.fptr.p, g.fadj.p,
                           g.esize.p, g.m, g.wbits, n.p, nc, out.p);
        HTRI_LAUNCH_CHECK();
    }
    unsigned long long found = 0;
    HTRI_HIP(hipMemcpyAsync(&found, n.p, sizeof(found), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    if ((int64_t)found != nc) fail(HTRI_E_DEVICE, "inclusion hyperwedge count differs from step 1");
    return nc;
}

void count_inclusion_classes(Graph &g, uint32_t mask, int64_t counts[21], uint64_t *t_dev, int target,
                             int64_t capacity, int32_t *dev_out, unsigned long long *dev_found,
                             unsigned long long *tp_rank) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    hipEvent_t e0, e1, e2;
    HTRI_HIP(hipEventCreate(&e0));
    HTRI_HIP(hipEventCreate(&e1));
    HTRI_HIP(hipEventCreate(&e2));
    HTRI_HIP(hipEventRecord(e0, s));
    const int64_t nc = g.summary[2];                  // inclusion hyperwedges (step 1)
    DBuf<int2> pairs(A, nc);
    DBuf<unsigned long long> ctr(A, 22);              // [0] pair count, [1..21] pattern counts
    DBuf<uint8_t> lut(A, 128);
    fill_u64((uint64_t *)ctr.p, 22, 0, s);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    DBuf<unsigned long long> t;
    if (t_dev) {
        t.alloc(A, m);
        fill_u64((uint64_t *)t.p, m, 0, s);
    }
    if (m > 0 && nc > 0) {
        hipLaunchKernelGGL(k_incl_pairs, dim3(grid_for(m * kWave, 256, 8192)), dim3(256), 0, s, g.fptr.p, g.fadj.p,
                           g.esize.p, m, g.wbits, ctr.p, pairs.p);
        HTRI_LAUNCH_CHECK();
    }
    HTRI_HIP(hipEventRecord(e1, s));
    unsigned long long found = 0;
    HTRI_HIP(hipMemcpyAsync(&found, ctr.p, sizeof(found), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    if ((int64_t)found != nc) fail(HTRI_E_DEVICE, "inclusion hyperwedge count differs from step 1");
    if (nc > 0) {
        hipLaunchKernelGGL(k_incl_count, dim3((unsigned)nc), dim3(kBlock), 0, s, pairs.p, g.eptr.p, g.emem.p,
                           g.esize.p, g.vptr.p, g.vadj.p, lut.p, mask, ctr.p + 1, t_dev ? t.p : nullptr, target,
                           g.norm_of_rank.p, capacity, dev_out, dev_found, tp_rank);
        HTRI_LAUNCH_CHECK();
    }
    HTRI_HIP(hipEventRecord(e2, s));
    if (t_dev && m > 0) {
        hipLaunchKernelGGL(k_rank_to_norm_u64, dim3(grid_for(m, 256)), dim3(256), 0, s, t.p, g.norm_of_rank.p, m,
                           (int64_t *)t_dev);
        HTRI_LAUNCH_CHECK();
    }
    unsigned long long hc[22];
    HTRI_HIP(hipMemcpyAsync(hc, ctr.p, sizeof(hc), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    counts[0] = 0;
    for (int p = 1; p <= 20; p++) {
        counts[p] = p <= 8 ? (int64_t)hc[1 + p] : 0;
        counts[0] += counts[p];
    }
    g.tm.schedule_ms = 0;
    HTRI_HIP(hipEventElapsedTime(&g.tm.schedule_ms, e0, e1));
    HTRI_HIP(hipEventElapsedTime(&g.tm.closure_ms, e1, e2));
    g.tm.reduce_ms = g.tm.window_ms = 0;
    g.tm.probe_ms = g.tm.closure_ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
}

// ---------------------------------------------------------------- LUT

namespace {
struct LutBuilder {
    uint8_t lut[128];
    LutBuilder() {
        // regions: bit 0 a (i only), 1 b (j only), 2 c (k only), 3 d (i&j),
        // 4 e (j&k), 5 f (k&i), 6 g (i&j&k)
        const int single[3] = {0, 1, 2};
        auto pair = [](int x, int y) {
            int lo = x < y ? x : y, hi = x < y ? y : x;
            if (lo == 0 && hi == 1) return 3;
            if (lo == 1 && hi == 2) return 4;
            return 5;
        };
        for (int msk = 0; msk < 128; msk++) {
            auto on = [&](int bit) { return (msk >> bit) & 1; };
            lut[msk] = 0;
            if (!((on(3) || on(6)) && (on(4) || on(6)) && (on(5) || on(6)))) continue;
            // set of non-empty regions inside hyperedge x
            auto regions_of = [&](int x) {
                int s = 0;
                for (int b = 0; b < 7; b++) {
                    bool in = (b == single[x]) || b == 6 || (b >= 3 && b <= 5 &&
                              ((b == 3 && (x == 0 || x == 1)) || (b == 4 && (x == 1 || x == 2)) ||
                               (b == 5 && (x == 0 || x == 2))));
                    if (in && on(b)) s |= 1 << b;
                }
                return s;
            };
            int R[3] = {regions_of(0), regions_of(1), regions_of(2)};
            if (R[0] == R[1] || R[1] == R[2] || R[0] == R[2]) continue;  // equal hyperedges
            auto sub = [&](int x, int y) { return (R[x] & ~R[y]) == 0; };
            bool C[3][3] = {};
            int nc = 0;
            for (int x = 0; x < 3; x++)
                for (int y = x + 1; y < 3; y++) {
                    C[x][y] = C[y][x] = sub(x, y) || sub(y, x);
                    nc += C[x][y];
                }
            int p = 0;
            if (nc == 3) {
                p = 1;
            } else if (nc == 2) {
                int x = 0;
                for (int c = 0; c < 3; c++)
                    if (C[c][(c + 1) % 3] && C[c][(c + 2) % 3]) x = c;
                int y = (x + 1) % 3, z = (x + 2) % 3;
                if (sub(x, y)) p = on(pair(y, z)) ? 3 : 2;   // x inside both
                else p = on(single[x]) ? 5 : 4;               // x contains both
            } else if (nc == 1) {
                int L = 0, S = 0, X = 0;
                for (int x = 0; x < 3; x++)
                    for (int y = 0; y < 3; y++)
                        if (x != y && C[x][y] && sub(y, x)) { L = x; S = y; X = 3 - x - y; }
                if (!on(pair(L, X))) p = 6;       // X meets L only inside S
                else if (!on(single[L])) p = 7;   // L has no private vertex
                else p = 8;
            } else {
                int s = on(0) + on(1) + on(2), q = on(3) + on(4) + on(5);
                if (!on(6)) p = 17 + s;
                else if (q == 0) p = 9;
                else if (q == 1) p = 10;
                else if (q == 2) p = (s == 2) ? 11 : 12;
                else p = 13 + s;
            }
            lut[msk] = (uint8_t)p;
        }
    }
};
}  // namespace

const uint8_t *pattern_lut() {
    static LutBuilder b;
    return b.lut;
}

// ---------------------------------------------------------------- driver

// S and S outside the window of the last count (cstats[0] and [7]), out of
// the count's own time
void closure_stream_stats(Graph &g) {
    if (g.cstats[0] >= 0 || !g.have_wedges) return;
    hipStream_t s = g.stream;
    DBuf<unsigned long long> S(g.al, 2);
    fill_u64((uint64_t *)S.p, 2, 0, s);
    if (g.nw > 0) {
        const int64_t e_split = g.stats_owner_end < g.m ? read_i64(g.fptr.p + g.stats_owner_end, s) : g.nw;
        hipLaunchKernelGGL(k_stream_size, dim3(grid_for(g.nw, 256, 2048)), dim3(256), 0, s, g.fptr.p, g.fadj.p, g.nw,
                           e_split, g.wbits, S.p);
        HTRI_LAUNCH_CHECK();
    }
    unsigned long long h[2] = {0, 0};
    HTRI_HIP(hipMemcpyAsync(h, S.p, sizeof(h), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    g.cstats[0] = (int64_t)h[0];
    g.cstats[7] = (int64_t)h[1];
}

void count_patterns(Graph &g, uint32_t mask, uint32_t flags, int64_t counts[21], uint64_t *t_dev, uint32_t *cw_dev,
                    unsigned long long *tp_rank) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    const CloseConfig cfg;  // 512-entry chunks, 256 partners per item
    hipEvent_t e0, e1, e2, e3, ew;
    HTRI_HIP(hipEventCreate(&e0));
    HTRI_HIP(hipEventCreate(&e1));
    HTRI_HIP(hipEventCreate(&e2));
    HTRI_HIP(hipEventCreate(&e3));
    HTRI_HIP(hipEventCreate(&ew));
    HTRI_HIP(hipEventRecord(e0, s));

    const WindowPlan win = choose_window(g, flags);
    const int64_t owner_end = win.nrows ? win.w0 : m;
    // probing direction: around the middle hyperedge unless asked otherwise
    // or its in-list does not fit (then around the owner)
    bool mid = !(flags & HTRI_COUNT_OWNER_PROBE) && owner_end > 0;
    int64_t mid_wedges = 0;   // hyperwedges of the owners before owner_end (the in-list)
    if (mid) {
        size_t free_b = 0, total_b = 0;
        const int64_t n_in = read_i64(g.fptr.p + owner_end, s);
        mid_wedges = n_in;
        if (n_in > 0 && !transpose_fits(m, n_in)) mid = false;
        else if (hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
                 (double)inlist_bytes(g, owner_end) > 0.9 * (double)free_b)
            mid = false;
    }
    InList in;
    ItemLists items;
    if (mid) {
        try {
            build_inlist(g, owner_end, in);
            build_items_mid(g, 0, cfg, in, items);
        } catch (const Error &e) {
            if (e.code != HTRI_E_OOM) throw;
            HTRI_HIP(hipStreamSynchronize(s));
            in = InList();
            items = ItemLists();
            mid = false;
        }
    }
    if (!mid) build_items(g, 0, cfg, items, owner_end);
    const int64_t nitems = items.nblock + items.nwave;
    DBuf<uint8_t> lut(A, 128);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    DBuf<GraphDesc> desc(A, 1);
    GraphDesc hd = graph_desc(g);
    if (mid) {
        hd.inl = in.inl.p;
        hd.iptr = in.iptr.p;
    }
    HTRI_HIP(hipMemcpyAsync(desc.p, &hd, sizeof(GraphDesc), hipMemcpyHostToDevice, s));
    // counters: [0] block queue, [1..21] pattern counts, [22] probes,
    // [23] wave queue, [24] S, [25] S before the window, [26..27] window
    // stats, [28] hashed entries staged
    DBuf<unsigned long long> ctr(A, 29);
    fill_u64((uint64_t *)ctr.p, 29, 0, s);

    const bool pe = t_dev != nullptr;
    const bool pw = cw_dev != nullptr;
    DBuf<uint32_t> cwjm, cwkm;
    // per-hyperedge totals by rank; middle-centric items add to them during
    // the closure, and the role reduce adds the hyperwedges from e_roles on
    // (the window's, or all of them when probing around the owner)
    DBuf<unsigned long long> tsum;
    const int64_t e_roles = mid ? mid_wedges : 0;
    if (pe) {
        cwjm.alloc(A, g.nw);
        cwkm.alloc(A, g.nw);
        tsum.alloc(A, m);
        fill_u32(cwjm.p, g.nw, 0, s);
        fill_u32(cwkm.p, g.nw, 0, s);
        fill_u64((uint64_t *)tsum.p, m, 0, s);
    }
    if (pw) fill_u32(cw_dev, g.nw, 0, s);

    int nblocks = device_cu_count() * close_blocks_per_cu(cfg, pe, pw, mid);
    if ((int64_t)nblocks > nitems) nblocks = (int)std::max<int64_t>(nitems, 1);
    HTRI_HIP(hipStreamSynchronize(s));
    HTRI_HIP(hipEventRecord(e1, s));

    CloseArgs a;
    a.items = items.block.p;
    a.nitems = items.nblock;
    a.queue = (unsigned int *)ctr.p;
    a.witems = items.wave.p;
    a.nwitems = items.nwave;
    a.wqueue = (unsigned int *)(ctr.p + 23);
    a.graphs = desc.p;
    // SparseTTT-only counting: bit 31 tells the probe to drop every hit with
    // a vertex common to all three hyperedges
    a.emask = (flags & HTRI_COUNT_SPARSE_TTT) ? ((mask & 0x1E0000u) | 0x80000000u) : mask;
    a.lut = lut.p;
    a.cwj = cw_dev;
    a.cwjm = cwjm.p;
    a.cwkm = cwkm.p;
    a.counts = ctr.p + 1;
    a.probes = ctr.p + 22;
    a.staged = ctr.p + 28;
    a.tedge = mid && pe ? tsum.p : nullptr;
    DBuf<unsigned long long> wpart(A, (int64_t)nblocks * (kBlock / kWave) * 21);
    a.wave_part = wpart.p;
    // per-pattern per-hyperedge counts are kept for SparseTTT counting only
    a.tp = (flags & HTRI_COUNT_SPARSE_TTT) ? tp_rank : nullptr;
    close_window(g, win, a.emask, lut.p, ctr.p + 1, ctr.p + 26, cw_dev, pe ? cwjm.p : nullptr, pe ? cwkm.p : nullptr,
                 a.tp);
    HTRI_HIP(hipEventRecord(ew, s));
    launch_close_kernel(cfg, pe, pw, a, nblocks, s, mid);
    HTRI_HIP(hipEventRecord(e2, s));
    sum_pattern_parts(wpart.p, (int64_t)nblocks * (kBlock / kWave), a.counts, s);

    if (pe) {
        DBuf<unsigned long long> &t = tsum;
        if (m > 0) {
            if (g.nw > e_roles) {
                hipLaunchKernelGGL(k_edge_counts_roles, dim3(grid_for(g.nw - e_roles, 256, 16384)), dim3(256), 0, s,
                                   g.fadj.p, e_roles, g.nw, g.wbits, cwjm.p, cwkm.p, t.p);
                HTRI_LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(k_edge_counts_owner, dim3(grid_for(m * kWave, 256, 8192)), dim3(256), 0, s, g.fptr.p, m,
                               cwjm.p, t.p);
            HTRI_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_rank_to_norm_u64, dim3(grid_for(m, 256)), dim3(256), 0, s, t.p, g.norm_of_rank.p, m,
                               (int64_t *)t_dev);
            HTRI_LAUNCH_CHECK();
        }
        HTRI_HIP(hipEventRecord(e3, s));
        HTRI_HIP(hipStreamSynchronize(s));
    } else {
        HTRI_HIP(hipEventRecord(e3, s));
    }
    unsigned long long hc[29];
    HTRI_HIP(hipMemcpyAsync(hc, ctr.p, sizeof(hc), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    int64_t tot = 0;
    counts[0] = 0;
    for (int p = 1; p <= 20; p++) {
        counts[p] = (int64_t)hc[1 + p];
        tot += counts[p];
    }
    counts[0] = tot;
    int64_t mask_words_total = 0, mask_words_before = 0, wedges_before = g.nw;
    HTRI_HIP(hipMemcpyAsync(&mask_words_total, g.mptr.p + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (win.nrows) {
        HTRI_HIP(hipMemcpyAsync(&mask_words_before, g.mptr.p + win.w0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HTRI_HIP(hipMemcpyAsync(&wedges_before, g.fptr.p + win.w0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    HTRI_HIP(hipStreamSynchronize(s));
    if (!win.nrows) mask_words_before = mask_words_total;
    g.cstats[0] = -1;                 // S: computed on request (closure_stream_stats)
    g.cstats[1] = (int64_t)hc[22];
    g.cstats[2] = nitems;
    g.cstats[3] = mask_words_total;
    g.cstats[4] = nblocks;
    g.cstats[5] = win.nrows;
    g.cstats[6] = win.wedges;
    g.cstats[7] = -1;
    g.stats_owner_end = owner_end;
    g.cstats[8] = wedges_before;
    g.cstats[9] = mask_words_before;
    g.cstats[10] = (int64_t)hc[26];
    g.cstats[11] = (int64_t)hc[27];
    g.cstats[12] = mid ? 1 : 0;
    g.cstats[13] = mid ? in.n : 0;
    g.cstats[14] = 0;
    g.cstats[15] = (int64_t)hc[28];
    HTRI_HIP(hipEventElapsedTime(&g.tm.schedule_ms, e0, e1));
    HTRI_HIP(hipEventElapsedTime(&g.tm.closure_ms, e1, e2));
    HTRI_HIP(hipEventElapsedTime(&g.tm.window_ms, e1, ew));
    HTRI_HIP(hipEventElapsedTime(&g.tm.probe_ms, ew, e2));
    HTRI_HIP(hipEventElapsedTime(&g.tm.reduce_ms, e2, e3));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    (void)hipEventDestroy(e3);
    (void)hipEventDestroy(ew);
}

}  // namespace htri
