// Step 2 of the two-step framework: close every hyperwedge and classify the
// hyper-triangle (Algorithm 3 for the intersection-only class, Algorithm 5
// for the classes with inclusion hyperwedges, combined over all patterns as
// the paper's Exact-adv).
//
// Orientation: hyperedges are ranked by prec; the forward list N+(r) holds
// the later neighbours of r, sorted.  A triangle r < j < k is found exactly
// once, by owner r, as a k that lies in both N+(r) and N+(j).
//
// Work decomposition (MI355X): an item is (owner r, a chunk of at most CAP
// consecutive entries of N+(r), a piece of at most 256 partners j of r).
// The chunk goes into an LDS open-addressing hash; every partner's N+(j),
// restricted to the chunk's rank range, is streamed from HBM with coalesced
// loads and probed against the hash.  A hit is classified from the sizes,
// the three omegas and g = popcount(Omega_rj & Omega_rk) (both masks are
// over e_r's member positions) through a 128-entry region-emptiness table.
// Persistent blocks pull items from a queue; pattern counts stay in per-lane
// LDS counters and leave the kernel as one partial per block.
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

constexpr int kUnroll = 4;   // partner-list entries per lane per step

// Find the slot of key kk = (k << wbits) in the bucketed open-addressing
// table (two (entry, position) slots per 16-byte bucket, buckets probed
// linearly; a bucket's second slot fills after its first).  Returns whether
// it is present; slot in out.
__device__ __forceinline__ bool lookup(const uint2 *tab, uint32_t kk, uint32_t kmask, int wbits, int hbits,
                                       uint2 &out) {
    const uint4 *tq = reinterpret_cast<const uint4 *>(tab);
    const uint32_t nbm1 = (1u << (hbits - 1)) - 1;
    uint32_t b = hslot(kk >> wbits, hbits - 1);
    uint4 B = tq[b];
    bool h0 = ((B.x & kmask) == kk) & (B.y != kEmptyPos);
    bool h1 = ((B.z & kmask) == kk) & (B.w != kEmptyPos);
    while (!(h0 | h1 | (B.w == kEmptyPos))) {      // full bucket without the key: next one
        b = (b + 1) & nbm1;
        B = tq[b];
        h0 = ((B.x & kmask) == kk) & (B.y != kEmptyPos);
        h1 = ((B.z & kmask) == kk) & (B.w != kEmptyPos);
    }
    out = h0 ? make_uint2(B.x, B.y) : make_uint2(B.z, B.w);
    return h0 | h1;
}

// One partner-list entry e = (k, omega_jk) of partner j against the staged
// chunk of owner r.  hit: k lies in the chunk (a hyper-triangle r, j, k);
// mhit: its pattern is counted into the per-hyperedge counts.  Returns the
// pattern when it is not the common-vertex one (counted in c9), else 0.
template <bool PER_EDGE>
__device__ __forceinline__ uint32_t probe_entry(const uint2 *tab, int hbits, int wbits, uint32_t wmask, uint32_t e,
                                                const uint2 *ent_sm, const uint32_t *ent_mx, uint32_t *ent_ck,
                                                const uint8_t *lut, int W, int si, int sj, int wij, bool fast_j,
                                                uint32_t m0, uint32_t m1, uint32_t m2, uint32_t m3,
                                                const GraphDesc &G, int32_t r, int32_t jr, uint32_t emask,
                                                unsigned long long &c9, bool &hit, bool &mhit) {
    uint2 sl;
    if (!lookup(tab, e & ~wmask, ~wmask, wbits, hbits, sl)) return 0u;
    hit = true;
    const uint32_t pos = sl.y;
    const int wik = (int)(sl.x & wmask);
    const int wjk = (int)(e & wmask);
    const uint2 sm = ent_sm[pos];
    // Omega_rk = Omega_rj and all three omegas equal: the triple shares
    // exactly those vertices and nothing else
    const bool fast = fast_j & (wik == wij) & (wjk == wij) & (sm.y == m0) & ((int)sm.x > wij);
    uint32_t p = kPatternCommonVertex, other = 0u;
    if (!fast) {
        const uint32_t k = e >> wbits;
        int g;
        if (W > 0) {
            g = __popc(m0 & sm.y);
            if (W > 1) {
                const uint32_t *mx = ent_mx + pos * (kMaskWordsMax - 1);
                g += __popc(m1 & mx[0]);
                if (W > 2) g += __popc(m2 & mx[1]);
                if (W > 3) g += __popc(m3 & mx[2]);
            }
        } else {
            g = triple_common(G.eptr, G.emem, r, jr, (int32_t)k);
        }
        const uint32_t m7 = region_mask(si, sj, (int)sm.x, wij, wik, wjk, g);
        if (m7 != kMaskCommonVertex) {
            p = lut[m7];
            other = p;
        }
    }
    c9 += (other == 0u);
    if (PER_EDGE && ((emask >> p) & 1u)) {
        mhit = true;
        atomicAdd(&ent_ck[pos], 1u);
    }
    return other;
}

// Add the wave's other-pattern hits (po[u] != 0) into lane p's counter.
__device__ __forceinline__ void aggregate_other(const uint32_t *po, int lane, unsigned long long &wcnt) {
#pragma unroll
    for (int u = 0; u < kUnroll; u++) {
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

template <int CAP, int JP, bool PER_EDGE, bool PER_WEDGE>
__global__ __launch_bounds__(kBlock, 4) void k_close(CloseArgs A) {
    static_assert(JP <= kBlock, "one thread per partner");
    constexpr int HMAX = 4 * CAP;
    __shared__ __align__(16) uint2 tab[HMAX];        // slots (entry, position); buckets of two
    __shared__ uint2 ent_sm[CAP];                         // (|e_k|, Omega_rk word 0)
    __shared__ uint32_t ent_mx[CAP * (kMaskWordsMax - 1)];  // Omega_rk words 1..3
    __shared__ uint32_t ent_ck[PER_EDGE ? CAP : 1];
    __shared__ int64_t seg_pre[kBlock + 1];
    __shared__ int64_t seg_src[JP];
    __shared__ uint32_t seg_size[JP];
    __shared__ uint32_t seg_om[JP];
    __shared__ uint32_t seg_mask[JP * kMaskWordsMax];
    __shared__ uint32_t seg_cj[PER_WEDGE ? JP : 1];
    __shared__ uint32_t seg_cjm[PER_EDGE ? JP : 1];
    __shared__ uint8_t lut[128];
    __shared__ int64_t sh_item;
    __shared__ int64_t sh_scan[kBlock / kWave + 1];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if (tid < 128) lut[tid] = A.lut[tid];
    unsigned long long wcnt = 0;     // lane p: this wave's count of pattern p (p != 9)
    unsigned long long c9 = 0;       // this lane's count of the common-vertex pattern
    unsigned long long all_probes = 0;
    int cur_g = -1;

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            unsigned int c = atomicAdd(A.queue, 1u);
            sh_item = (int64_t)c < A.nitems ? A.nitems - 1 - (int64_t)c : -1;
        }
        __syncthreads();
        const int64_t it = sh_item;
        if (it < 0) break;
        const Item item = A.items[it];
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
        const bool single = item.cb == 0 && item.ce == d && item.jb == 0 && item.je == d - 1;
        const int si = gld(G.esize + r);
        const int W = mask_words(si);
        const int64_t mbase = gld(G.mptr + r);
        const int cl = item.ce - item.cb;
        int hbits = 6;
        while ((1 << hbits) < 4 * cl) hbits++;
        const int H = 1 << hbits;
        const uint32_t lo = gld(G.fadj + base + item.cb) >> wbits;
        const uint32_t hi = gld(G.fadj + base + item.ce - 1) >> wbits;

        for (int s = tid; s < H; s += kBlock) tab[s] = make_uint2(0xFFFFFFFFu, kEmptyPos);
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
        if (tid < nseg) {
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
            seg_om[tid] = jent & wmask;
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

        // Partner-list entries go through probe_entry(); both loops below
        // keep the next tile's loads in flight while the current tile is
        // classified.
        if (total >= (int64_t)nseg * 64) {
            // Dense items (long partner segments): one wave per partner, the
            // partner's data wave-uniform, lanes striding over its segment.
            constexpr int TILE = kWave * kUnroll;
            int qd = wave;
            while (qd < nseg && seg_pre[qd + 1] == seg_pre[qd]) qd += kBlock / kWave;
            int64_t i0 = 0;
            uint32_t entA[kUnroll];
            bool valA[kUnroll];
            if (qd < nseg) {
                const int64_t slen = seg_pre[qd + 1] - seg_pre[qd];
                const int64_t sbase = seg_src[qd];
#pragma unroll
                for (int u = 0; u < kUnroll; u++) {
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
                uint32_t entB[kUnroll];
                bool valB[kUnroll];
                if (qn < nseg) {
                    const int64_t nlen = seg_pre[qn + 1] - seg_pre[qn];
                    const int64_t nbase = seg_src[qn];
#pragma unroll
                    for (int u = 0; u < kUnroll; u++) {
                        const int64_t i = in + u * kWave + lane;
                        valB[u] = i < nlen;
                        entB[u] = valB[u] ? gld(G.fadj + nbase + i) : 0u;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < kUnroll; u++) {
                        valB[u] = false;
                        entB[u] = 0u;
                    }
                }
                // this tile
                const int sjd = __builtin_amdgcn_readfirstlane((int)seg_size[qd]);
                const int wd = __builtin_amdgcn_readfirstlane((int)seg_om[qd]);
                const uint32_t m0 = W > 0 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)seg_mask[qd * kMaskWordsMax]) : 0u;
                const uint32_t m1 = W > 1 ? seg_mask[qd * kMaskWordsMax + 1] : 0u;
                const uint32_t m2 = W > 2 ? seg_mask[qd * kMaskWordsMax + 2] : 0u;
                const uint32_t m3 = W > 3 ? seg_mask[qd * kMaskWordsMax + 3] : 0u;
                const bool fastd = (W == 1) && (si > wd) && (sjd > wd);
                const int32_t jr = (W == 0) ? (int32_t)(gld(G.fadj + base + item.jb + qd) >> wbits) : 0;
                uint32_t po[kUnroll];
                bool other = false;
#pragma unroll
                for (int u = 0; u < kUnroll; u++) {
                    bool hit = false, mhit = false;
                    po[u] = valA[u] ? probe_entry<PER_EDGE>(tab, hbits, wbits, wmask, entA[u], ent_sm, ent_mx, ent_ck,
                                                            lut, W, si, sjd, wd, fastd, m0, m1, m2, m3, G, r, jr,
                                                            A.emask, c9, hit, mhit)
                                    : 0u;
                    other |= po[u] != 0;
                    if (PER_WEDGE) hits += (unsigned long long)__popcll(__ballot(hit));
                    if (PER_EDGE) mhits += (unsigned long long)__popcll(__ballot(mhit));
                }
                if (__ballot(other)) aggregate_other(po, lane, wcnt);
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
                for (int u = 0; u < kUnroll; u++) {
                    entA[u] = entB[u];
                    valA[u] = valB[u];
                }
            }
        } else {
            // Flattened items: the partner segments laid end to end; each step
            // a wave takes 64*kUnroll consecutive entries, kUnroll per lane.
            int qa = -1;                   // address cursor
            int64_t qa_end = 0, srca = 0;
            int q = -1;                    // processing cursor
            int sj = 0, wij = 0;
            uint32_t mj0 = 0, mj1 = 0, mj2 = 0, mj3 = 0;
            bool fast_j = false;
            uint32_t cj = 0, cjm = 0;
            int32_t jrank = 0;
            const int64_t stride = (int64_t)kBlock * kUnroll;
            auto fetch = [&](int64_t f0, uint32_t *ent, int *segu) {
#pragma unroll
                for (int u = 0; u < kUnroll; u++) {
                    const int64_t f = f0 + u;
                    segu[u] = -1;
                    int64_t addr = 0;
                    if (f < total) {
                        if (f >= qa_end) {
                            int lo_s = qa < 0 ? 0 : qa + 1, hi_s = nseg;
                            while (lo_s < hi_s) {
                                int mid = (lo_s + hi_s) >> 1;
                                if (seg_pre[mid + 1] <= f) lo_s = mid + 1; else hi_s = mid;
                            }
                            qa = lo_s;
                            qa_end = seg_pre[qa + 1];
                            srca = seg_src[qa] - seg_pre[qa];
                        }
                        segu[u] = qa;
                        addr = srca + f;
                    }
                    ent[u] = segu[u] >= 0 ? gld(G.fadj + addr) : 0u;
                }
            };
            int64_t fb = (int64_t)wave * kWave * kUnroll;
            uint32_t entA[kUnroll];
            int seguA[kUnroll];
            if (fb < total) fetch(fb + (int64_t)lane * kUnroll, entA, seguA);
            for (; fb < total; fb += stride) {
                uint32_t entB[kUnroll];
                int seguB[kUnroll];
                const int64_t fbn = fb + stride;
                if (fbn < total) {
                    fetch(fbn + (int64_t)lane * kUnroll, entB, seguB);
                } else {
#pragma unroll
                    for (int u = 0; u < kUnroll; u++) {
                        entB[u] = 0u;
                        seguB[u] = -1;
                    }
                }
                uint32_t po[kUnroll];
                bool other = false;
#pragma unroll
                for (int u = 0; u < kUnroll; u++) {
                    po[u] = 0;
                    if (seguA[u] < 0) continue;
                    if (seguA[u] != q) {
                        if (q >= 0) {
                            if (PER_WEDGE && cj) atomicAdd(&seg_cj[q], cj);
                            if (PER_EDGE && cjm) atomicAdd(&seg_cjm[q], cjm);
                        }
                        cj = cjm = 0;
                        q = seguA[u];
                        sj = (int)seg_size[q];
                        wij = (int)seg_om[q];
                        fast_j = (W == 1) && (si > wij) && (sj > wij);
                        mj0 = W > 0 ? seg_mask[q * kMaskWordsMax + 0] : 0u;
                        mj1 = W > 1 ? seg_mask[q * kMaskWordsMax + 1] : 0u;
                        mj2 = W > 2 ? seg_mask[q * kMaskWordsMax + 2] : 0u;
                        mj3 = W > 3 ? seg_mask[q * kMaskWordsMax + 3] : 0u;
                        if (W == 0) jrank = (int32_t)(gld(G.fadj + base + item.jb + q) >> wbits);
                    }
                    bool hit = false, mhit = false;
                    po[u] = probe_entry<PER_EDGE>(tab, hbits, wbits, wmask, entA[u], ent_sm, ent_mx, ent_ck, lut, W,
                                                  si, sj, wij, fast_j, mj0, mj1, mj2, mj3, G, r, jrank, A.emask, c9,
                                                  hit, mhit);
                    other |= po[u] != 0;
                    cj += hit;
                    cjm += mhit;
                }
                if (__ballot(other)) aggregate_other(po, lane, wcnt);
#pragma unroll
                for (int u = 0; u < kUnroll; u++) {
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
        if (PER_WEDGE || PER_EDGE) {
            if (tid < nseg) {
                const int64_t e = base + item.jb + tid;
                if (single) {
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
                    if (single) A.cwkm[e] = ent_ck[qq];
                    else if (ent_ck[qq]) atomicAdd(&A.cwkm[e], ent_ck[qq]);
                }
            }
        }
    }
    if (cur_g >= 0) flush_wave_counts(wcnt, c9, A.counts, cur_g, lane);
    if (tid == 0 && all_probes) atomicAdd(A.probes, all_probes);
}

// number of items per owner
__global__ void k_item_counts(const int64_t *fptr, int64_t m, int cap, int jp, int64_t *cnt) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = fptr[r + 1] - fptr[r];
        int64_t c = 0;
        if (d >= 2) {
            for (int64_t cb = 0; cb < d; cb += cap) {
                int64_t ce = cb + cap < d ? cb + cap : d;
                c += (ce - 1 + jp - 1) / jp;
            }
        }
        cnt[r] = c;
    }
}

__global__ void k_item_fill(const int64_t *fptr, int64_t m, int cap, int jp, int32_t gid, const int64_t *ioff,
                            Item *items) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = fptr[r + 1] - fptr[r];
        if (d < 2) continue;
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

// S = sum over hyperwedges (r, j) of |N+(j)|
__global__ void k_stream_size(const int64_t *fptr, const uint32_t *fadj, int64_t nw, int wbits,
                              unsigned long long *S) {
    __shared__ unsigned long long sh[256];
    unsigned long long acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t j = fadj[e] >> wbits;
        acc += (unsigned long long)(fptr[j + 1] - fptr[j]);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(S, sh[0]);
}

// per-hyperedge counts from the per-wedge role counters
__global__ void k_edge_counts(const int64_t *fptr, const uint32_t *fadj, int64_t m, int wbits,
                              const uint32_t *cwjm, const uint32_t *cwkm, unsigned long long *t) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long own = 0;
        for (int64_t e = fptr[r]; e < fptr[r + 1]; e++) {
            uint32_t x = fadj[e] >> wbits;
            uint32_t c = cwjm[e] + cwkm[e];
            if (c) atomicAdd(&t[x], (unsigned long long)c);
            own += cwjm[e];
        }
        if (own) atomicAdd(&t[r], own);
    }
}

__global__ void k_rank_to_norm_u64(const unsigned long long *t, const int32_t *norm_of_rank, int64_t m,
                                   int64_t *out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x)
        out[norm_of_rank[r]] = (int64_t)t[r];
}

template <int CAP, int JP, bool PE, bool PW>
int occ_blocks() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_close<CAP, JP, PE, PW>, kBlock, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

template <int CAP, int JP>
struct CloseVariants {
    static int blocks(bool pe, bool pw) {
        return pe ? (pw ? occ_blocks<CAP, JP, true, true>() : occ_blocks<CAP, JP, true, false>())
                  : (pw ? occ_blocks<CAP, JP, false, true>() : occ_blocks<CAP, JP, false, false>());
    }
    static void launch(bool pe, bool pw, const CloseArgs &a, int nb, hipStream_t s) {
        if (pe && pw) hipLaunchKernelGGL((k_close<CAP, JP, true, true>), dim3(nb), dim3(kBlock), 0, s, a);
        else if (pe) hipLaunchKernelGGL((k_close<CAP, JP, true, false>), dim3(nb), dim3(kBlock), 0, s, a);
        else if (pw) hipLaunchKernelGGL((k_close<CAP, JP, false, true>), dim3(nb), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_close<CAP, JP, false, false>), dim3(nb), dim3(kBlock), 0, s, a);
        HTRI_LAUNCH_CHECK();
    }
};

}  // namespace

bool valid_config(const CloseConfig &c) {
    return (c.cap == 256 || c.cap == 512) && (c.jp == 128 || c.jp == 256);
}

int close_blocks_per_cu(const CloseConfig &c, bool pe, bool pw) {
    if (c.cap == 256 && c.jp == 128) return CloseVariants<256, 128>::blocks(pe, pw);
    if (c.cap == 256 && c.jp == 256) return CloseVariants<256, 256>::blocks(pe, pw);
    if (c.cap == 512 && c.jp == 128) return CloseVariants<512, 128>::blocks(pe, pw);
    if (c.cap == 512 && c.jp == 256) return CloseVariants<512, 256>::blocks(pe, pw);
    fail(HTRI_E_INVALID, "unsupported closure configuration");
    return 0;
}

void launch_close_kernel(const CloseConfig &c, bool pe, bool pw, const CloseArgs &a, int nb, hipStream_t s) {
    if (c.cap == 256 && c.jp == 128) return CloseVariants<256, 128>::launch(pe, pw, a, nb, s);
    if (c.cap == 256 && c.jp == 256) return CloseVariants<256, 256>::launch(pe, pw, a, nb, s);
    if (c.cap == 512 && c.jp == 128) return CloseVariants<512, 128>::launch(pe, pw, a, nb, s);
    if (c.cap == 512 && c.jp == 256) return CloseVariants<512, 256>::launch(pe, pw, a, nb, s);
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

int64_t build_items(Graph &g, int32_t gid, const CloseConfig &cfg, DBuf<Item> &out) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    DBuf<int64_t> icnt(A, m + 1);
    if (m > 0) {
        hipLaunchKernelGGL(k_item_counts, dim3(grid_for(m, 256)), dim3(256), 0, s, g.fptr.p, m, cfg.cap, cfg.jp,
                           icnt.p);
        HTRI_LAUNCH_CHECK();
    }
    scan_exclusive_i64(A, icnt.p, icnt.p, m, icnt.p + m, s);
    int64_t nitems = 0;
    HTRI_HIP(hipMemcpyAsync(&nitems, icnt.p + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    if (nitems >= (int64_t)UINT32_MAX) fail(HTRI_E_UNSUPPORTED, "too many work items");
    out.alloc(A, nitems);
    if (m > 0 && nitems > 0) {
        hipLaunchKernelGGL(k_item_fill, dim3(grid_for(m, 256)), dim3(256), 0, s, g.fptr.p, m, cfg.cap, cfg.jp, gid,
                           icnt.p, out.p);
        HTRI_LAUNCH_CHECK();
    }
    HTRI_HIP(hipStreamSynchronize(s));
    return nitems;
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

void count_patterns(Graph &g, uint32_t mask, int64_t counts[21], uint64_t *t_dev, uint32_t *cw_dev) {
    hipStream_t s = g.stream;
    Allocator &A = g.al;
    const int64_t m = g.m;
    const CloseConfig cfg;  // 512-entry chunks, 256 partners per item
    hipEvent_t e0, e1, e2, e3;
    HTRI_HIP(hipEventCreate(&e0));
    HTRI_HIP(hipEventCreate(&e1));
    HTRI_HIP(hipEventCreate(&e2));
    HTRI_HIP(hipEventCreate(&e3));
    HTRI_HIP(hipEventRecord(e0, s));

    DBuf<Item> items;
    const int64_t nitems = build_items(g, 0, cfg, items);
    DBuf<uint8_t> lut(A, 128);
    HTRI_HIP(hipMemcpyAsync(lut.p, pattern_lut(), 128, hipMemcpyHostToDevice, s));
    DBuf<GraphDesc> desc(A, 1);
    GraphDesc hd = graph_desc(g);
    HTRI_HIP(hipMemcpyAsync(desc.p, &hd, sizeof(GraphDesc), hipMemcpyHostToDevice, s));
    // counters: queue (1), pattern counts (21), probes (1), S (1)
    DBuf<unsigned long long> ctr(A, 24);
    fill_u64((uint64_t *)ctr.p, 24, 0, s);

    const bool pe = t_dev != nullptr;
    const bool pw = cw_dev != nullptr;
    DBuf<uint32_t> cwjm, cwkm;
    if (pe) {
        cwjm.alloc(A, g.nw);
        cwkm.alloc(A, g.nw);
        fill_u32(cwjm.p, g.nw, 0, s);
        fill_u32(cwkm.p, g.nw, 0, s);
    }
    if (pw) fill_u32(cw_dev, g.nw, 0, s);

    int nblocks = device_cu_count() * close_blocks_per_cu(cfg, pe, pw);
    if ((int64_t)nblocks > nitems) nblocks = (int)std::max<int64_t>(nitems, 1);
    HTRI_HIP(hipStreamSynchronize(s));
    HTRI_HIP(hipEventRecord(e1, s));

    CloseArgs a;
    a.items = items.p;
    a.nitems = nitems;
    a.queue = (unsigned int *)ctr.p;
    a.graphs = desc.p;
    a.emask = mask;
    a.lut = lut.p;
    a.cwj = cw_dev;
    a.cwjm = cwjm.p;
    a.cwkm = cwkm.p;
    a.counts = ctr.p + 1;
    a.probes = ctr.p + 22;
    launch_close_kernel(cfg, pe, pw, a, nblocks, s);
    HTRI_HIP(hipEventRecord(e2, s));

    if (g.nw > 0) {
        hipLaunchKernelGGL(k_stream_size, dim3(grid_for(g.nw, 256, 2048)), dim3(256), 0, s, g.fptr.p, g.fadj.p, g.nw,
                           g.wbits, ctr.p + 23);
        HTRI_LAUNCH_CHECK();
    }
    if (pe) {
        DBuf<unsigned long long> t(A, m);
        fill_u64((uint64_t *)t.p, m, 0, s);
        if (m > 0) {
            hipLaunchKernelGGL(k_edge_counts, dim3(grid_for(m, 256)), dim3(256), 0, s, g.fptr.p, g.fadj.p, m, g.wbits,
                               cwjm.p, cwkm.p, t.p);
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
    unsigned long long hc[24];
    HTRI_HIP(hipMemcpyAsync(hc, ctr.p, sizeof(hc), hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    int64_t tot = 0;
    counts[0] = 0;
    for (int p = 1; p <= 20; p++) {
        counts[p] = (int64_t)hc[1 + p];
        tot += counts[p];
    }
    counts[0] = tot;
    int64_t mask_words_total = 0;
    HTRI_HIP(hipMemcpy(&mask_words_total, g.mptr.p + m, sizeof(int64_t), hipMemcpyDeviceToHost));
    g.cstats[0] = (int64_t)hc[23];
    g.cstats[1] = (int64_t)hc[22];
    g.cstats[2] = nitems;
    g.cstats[3] = mask_words_total;
    g.cstats[4] = nblocks;
    HTRI_HIP(hipEventElapsedTime(&g.tm.schedule_ms, e0, e1));
    HTRI_HIP(hipEventElapsedTime(&g.tm.closure_ms, e1, e2));
    HTRI_HIP(hipEventElapsedTime(&g.tm.reduce_ms, e2, e3));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    (void)hipEventDestroy(e3);
}

}  // namespace htri
