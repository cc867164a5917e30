/*
 * htri -- hyper-triangle counting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the HIP library libhtri.so.  Plain pointers and sizes only.
 *
 * The library implements the two-step method of Yin et al., "Efficient
 * Computation of Hyper-triangles on Hypergraphs" (PVLDB 18(3), 2024):
 *
 *   htri_graph_load      normalise a hypergraph (Def. 2.1: a hyperedge is a
 *                        non-empty vertex set; Section 2: no two hyperedges
 *                        hold the same set) and build the vertex->hyperedge
 *                        lists E_v (Algorithm 2, first step).
 *   htri_build_wedges    step 1 (Algorithm 2): every hyperwedge (pair of
 *                        hyperedges sharing a vertex, Def. 2.2) with its
 *                        common-vertex count omega and common-vertex set
 *                        Omega; its type (Def. 2.3) follows from omega.
 *   htri_count_patterns  step 2 (Algorithms 3 and 5, combined as the paper's
 *                        Exact-adv): close every hyperwedge with each third
 *                        hyperedge adjacent to both, classify the triple into
 *                        one of the 20 patterns by which of its seven regions
 *                        (Section 2, after Def. 2.4) are empty, and reduce
 *                        per-pattern counts (H of Table 1) and per-hyperedge
 *                        counts (input of the clustering coefficient,
 *                        Def. 5.1).
 *   htri_estimate        hyperwedge sampling (Algorithm 6 with sigma = 1,
 *                        unbiased by Lemma 4.1), with a uniform proposal or a
 *                        learned importance proposal.
 *   htri_model_*         the proposal network (16 -> 64 -> 64 -> 1, ReLU) and
 *                        its training kernels.
 *   htri_batch_*         many independent hypergraphs counted in one launch.
 *
 * Conventions shared by every entry point
 *  - Every function returns an htri_status; no C++ exception crosses the ABI.
 *    On error the outputs are left unchanged and the handle stays usable;
 *    htri_last_error() describes the failure.
 *  - Device work runs on the stream given at load time (NULL = the default
 *    stream).  Functions that fill host arrays synchronise that stream before
 *    returning.
 *  - Internal order: hyperedges are processed in the order "prec" defined by
 *    (delta_x, x) ascending, delta_x = sum over v in e_x of (|E_v| - 1), x the
 *    normalised id (HTRI_ORDER_INPUT selects plain id order instead).  A
 *    hyperwedge is stored once, oriented from the earlier to the later
 *    hyperedge in this order; each hyper-triangle is found exactly once, at
 *    its two earliest hyperedges (the role of the hyperwedge order O of
 *    Section 2).  Pattern and per-hyperedge counts do not depend on the order;
 *    per-wedge closure counts do, and are reported together with the
 *    orientation (htri_get_wedges).
 *  - Normalised ids: surviving hyperedges renumbered 0..m-1 in input order
 *    (later duplicates dropped).  Per-hyperedge outputs use normalised ids.
 *  - Pattern numbering: 1 (CCC), 2-5 (TCC), 6-8 (TTC), 9-16 (DenseTTT),
 *    17-20 (SparseTTT).  Counts arrays have 21 entries: [0] = total,
 *    [p] = pattern p.
 *  - Not re-entrant on one handle; distinct handles may be used from
 *    distinct threads.
 */
#ifndef HTRI_H
#define HTRI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HTRI_OK = 0,
    HTRI_E_INVALID = -1,          /* bad argument or malformed CSR            */
    HTRI_E_RANGE = -2,            /* vertex id outside [0, num_vertices)      */
    HTRI_E_EMPTY_EDGE = -3,       /* a hyperedge with no vertex (Def. 2.1)    */
    HTRI_E_DUPLICATE_EDGE = -4,   /* two equal hyperedges, dedupe not asked   */
    HTRI_E_OOM = -5,              /* device allocation failed                 */
    HTRI_E_DEVICE = -6,           /* a HIP runtime error                      */
    HTRI_E_OVERFLOW = -7,         /* counts could exceed int64                */
    HTRI_E_STATE = -8,            /* call order (e.g. count before wedges)    */
    HTRI_E_UNSUPPORTED = -9       /* size beyond what the library handles     */
} htri_status;

typedef struct htri_graph htri_graph;

/* Optional device allocator (e.g. a framework's caching allocator).
 * alloc returns a device pointer of at least `bytes` bytes usable on
 * `stream`, or NULL; free releases it.  NULL allocator = hipMalloc/hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} htri_allocator;

#define HTRI_DEDUPE_EDGES 1u      /* drop later duplicate hyperedges          */
#define HTRI_INPUT_ON_DEVICE 2u   /* offsets/members are device pointers      */
#define HTRI_OUTPUT_ON_DEVICE 4u  /* per_edge / per_wedge are device pointers */
#define HTRI_ORDER_INPUT 8u       /* orient by normalised id, not by delta    */
/* Hyperwedge build with 64-bit sort keys in its LDS tiles, the form graphs
 * of 2^24 or more hyperedges need (smaller graphs use 32-bit keys); the
 * hyperwedges are the same either way. */
#define HTRI_WIDE_TILE_KEYS 256u
/* htri_count_patterns flags (with HTRI_OUTPUT_ON_DEVICE) */
#define HTRI_COUNT_NO_WINDOW 16u     /* close every owner by probing           */
#define HTRI_COUNT_WINDOW_ALWAYS 32u /* use the dense window whenever it holds */
                                     /* a hyperwedge (else: when dense enough) */
#define HTRI_COUNT_INCLUSION_CLASSES 64u /* count only patterns 1-8 (classes    */
                                         /* CCC, TCC, TTC), around the inclusion */
                                         /* hyperwedges; per_wedge must be NULL  */
#define HTRI_COUNT_OWNER_PROBE 128u  /* probe every partner's whole forward    */
                                     /* list against its owner's (instead of   */
                                     /* each owner's rest against the middle)  */
/* Class-targeted counts of the intersection-only class (Section 3.2): */
#define HTRI_COUNT_DENSE_TTT 512u    /* patterns 9-16 only (DenseTTT)          */
#define HTRI_COUNT_COMMON_VERTEX 1024u /* pattern 9 only                       */
#define HTRI_COUNT_SPARSE_TTT 2048u  /* patterns 17-20 only (SparseTTT)        */

/* Load and normalise a hypergraph (Def. 2.1 and the distinct-hyperedge
 * assumption of Section 2), build E_v (Algorithm 2).
 *   edge_offsets  int64[num_edges+1], edge_offsets[0] == 0, non-decreasing;
 *                 hyperedge x holds members[edge_offsets[x] .. edge_offsets[x+1]).
 *   members       int32[edge_offsets[num_edges]], ids in [0, num_vertices);
 *                 any order; a repeated id inside one hyperedge counts once.
 *   flags         HTRI_DEDUPE_EDGES | HTRI_INPUT_ON_DEVICE | HTRI_ORDER_INPUT |
 *                 HTRI_WIDE_TILE_KEYS (kept for htri_build_wedges).
 *   alloc         NULL or an allocator used for every device buffer.
 *   stream        hipStream_t (NULL = default stream).
 *   out           receives the handle; caller frees it with htri_graph_free.
 * The input arrays are only read during the call and remain the caller's.
 * Errors: HTRI_E_INVALID, HTRI_E_RANGE, HTRI_E_EMPTY_EDGE,
 * HTRI_E_DUPLICATE_EDGE, HTRI_E_OOM, HTRI_E_DEVICE, HTRI_E_UNSUPPORTED.
 * On error *out is NULL and htri_last_error(NULL) describes the failure. */
htri_status htri_graph_load(const int64_t *edge_offsets, int64_t num_edges, const int32_t *members,
                            int32_t num_vertices, uint32_t flags, const htri_allocator *alloc,
                            void *stream, htri_graph **out);

/* Normalised sizes: out[0] = m (hyperedges kept), out[1] = duplicates removed,
 * out[2] = nnz after removing repeated vertex ids, out[3] = num_vertices. */
htri_status htri_graph_info(const htri_graph *g, int64_t out[4]);

/* Normalised id -> input index, int64[m] host array. */
htri_status htri_graph_edge_map(const htri_graph *g, int64_t *new_to_input);

/* Normalised CSR (members sorted ascending within each hyperedge), host
 * arrays int64[m+1] and int32[nnz]. */
htri_status htri_graph_csr(const htri_graph *g, int64_t *offsets, int32_t *members);

/* Step 1 (Algorithm 2): build every hyperwedge with omega and Omega.
 *   summary (may be NULL) int64[6]: |wedges|, |intersection-type|,
 *   |inclusion-type|, W = sum_x C(deg_x, 2) with deg_x = |N_{e_x}| (the
 *   connected triples), max omega, m.
 * Errors: HTRI_E_OOM, HTRI_E_DEVICE, HTRI_E_OVERFLOW (W beyond int64),
 * HTRI_E_UNSUPPORTED (m or omega too large for the packed adjacency). */
htri_status htri_build_wedges(htri_graph *g, int64_t summary[6]);

/* Release the step-1 state (hyperwedges, masks) so that htri_build_wedges
 * runs again; the loaded hypergraph stays.  Used to time step 1 repeatedly
 * and to free device memory between counts. */
htri_status htri_clear_wedges(htri_graph *g);

/* Wedges in the library's internal order, oriented src -> dst (src earlier
 * in prec), normalised ids, host arrays of |wedges| entries; omega may be
 * NULL.  This is the order of per_wedge in htri_count_patterns. */
htri_status htri_get_wedges(const htri_graph *g, int32_t *src, int32_t *dst, int32_t *omega);

/* The same for listed hyperwedges only (indices into the htri_get_wedges
 * order, host arrays of n entries; omega may be NULL): for hypergraphs whose
 * whole wedge list is too large to copy. */
htri_status htri_get_wedge_list(const htri_graph *g, const int64_t *wedge_idx, int64_t n, int32_t *src,
                                int32_t *dst, int32_t *omega);

/* Step 2 (Algorithms 3 and 5 as Exact-adv): exact count of every pattern.
 *   per_edge_pattern_mask  bit p (1..20) set: triangles of pattern p count
 *                          in per_edge.  0 is taken as "all patterns".
 *   counts      int64[21] host array: [0] total, [p] pattern p.
 *   per_edge    NULL or int64[m]: per normalised hyperedge, the number of
 *               masked triangles containing it (host or device array, see
 *               HTRI_OUTPUT_ON_DEVICE in out_flags).
 *   per_wedge   NULL or int32[|wedges|]: per hyperwedge (htri_get_wedges
 *               order), the number of third hyperedges that close it and
 *               come after dst in prec (all patterns).
 *   out_flags   HTRI_OUTPUT_ON_DEVICE, HTRI_COUNT_OWNER_PROBE, and at
 *               most one of HTRI_COUNT_NO_WINDOW / HTRI_COUNT_WINDOW_ALWAYS /
 *               HTRI_COUNT_INCLUSION_CLASSES / HTRI_COUNT_DENSE_TTT /
 *               HTRI_COUNT_COMMON_VERTEX / HTRI_COUNT_SPARSE_TTT.
 *               DENSE_TTT counts patterns 9-16 without closing every
 *               hyperwedge (Count-DenseTTT, Section 3.2, Lemma 3.1): pattern
 *               9 for each vertex v from the hyperedges of size >= 2 holding
 *               v and the "thick" pairs among them (sharing v and more),
 *               by inclusion-exclusion over the triples; patterns 10-16,
 *               which all have a thick pair, by scanning E_v from every
 *               thick hyperwedge.  COMMON_VERTEX counts pattern 9 alone
 *               that way.  Both need per_edge and per_wedge NULL; counts[p]
 *               outside the class are 0.  SPARSE_TTT counts patterns 17-20
 *               (Count-SparseTTT: the closure with every hit that has a
 *               vertex common to all three hyperedges dropped as soon as
 *               g > 0 is known; the dense window, where chosen, enumerates
 *               its hits the same way and skips its bulk counting of the
 *               common-vertex pattern); per_edge counts the
 *               masked patterns among 17-20, per_wedge must be NULL.  The last counts only the
 *               classes whose hyper-triangles hold an inclusion hyperwedge
 *               (patterns 1-8; Count-CCC, Count-TCC and Count-TTC of
 *               Section 3.1 search only around those hyperwedges): counts[p]
 *               for p > 8 are 0, per_edge counts the masked triangles of
 *               patterns 1-8.  By default the owners of the top ranks (the
 *               whole graph or a power of two of them, up to 131072) are
 *               closed by bitmap intersection when the hyperwedges among
 *               them fill at least 1/8 of all pairs (the largest such set);
 *               the counts do not depend on the choice.  The other owners
 *               are closed by hash probing, by default around the middle
 *               hyperedge: for each hyperwedge (r, j), the entries of N+(r)
 *               after j are probed against N+(j).  HTRI_COUNT_OWNER_PROBE
 *               probes each partner's whole N+(j) against N+(r) instead; it
 *               is also taken when the middle-side lists (about 40 bytes
 *               per hyperwedge) do not fit in free device memory or hold
 *               2^32 hyperwedges or more.
 * Errors: HTRI_E_STATE (no wedges yet), HTRI_E_INVALID (unknown flag),
 * HTRI_E_OOM, HTRI_E_DEVICE. */
htri_status htri_count_patterns(htri_graph *g, uint32_t per_edge_pattern_mask, int64_t counts[21],
                                int64_t *per_edge, int32_t *per_wedge, uint32_t out_flags);

/* Fine-grained hypergraph clustering coefficient (Def. 5.1):
 * 3 * sum_p epsilon[p] * counts[p] / connected_triples, with epsilon[p] in
 * [0, 1] for p = 1..20 (epsilon[0] unused; NULL = all 1, the classical
 * coefficient) and connected_triples = W from htri_build_wedges (summary[3],
 * the pairs of hyperedges meeting a common one: the denominator read as
 * the connected triples, which keeps the value in [0, 1]).  0 when W = 0.
 * Host arithmetic only.  Errors: HTRI_E_INVALID (NULL, negative, epsilon
 * outside [0, 1]). */
htri_status htri_clustering_coefficient(const int64_t counts[21], int64_t connected_triples,
                                        const double epsilon[21], double *cc);

/* Per-hyperedge counts of every pattern in one call (the hyperedge-level
 * counts of the fine-grained clustering coefficient, Def. 5.1):
 * per_edge_patterns int64[m][21] (normalised ids; [x][0] all patterns,
 * [x][p] the hyper-triangles of pattern p holding x; host, or device with
 * HTRI_OUTPUT_ON_DEVICE), counts int64[21] as htri_count_patterns.  Built
 * from the full count's per-hyperedge counts, the search around the
 * inclusion hyperwedges (patterns 1-8), the thick-pair scan of
 * Count-DenseTTT (10-16) and one SparseTTT closure (17-20), each adding
 * a hyper-triangle to its three hyperedges' counts of its pattern; pattern 9
 * is the remainder.  Errors: HTRI_E_INVALID, HTRI_E_STATE,
 * HTRI_E_OOM, HTRI_E_DEVICE. */
htri_status htri_count_per_edge_patterns(htri_graph *g, int64_t counts[21], int64_t *per_edge_patterns,
                                         uint32_t out_flags);

/* Local clustering coefficient of every hyperedge (normalised ids, double[m],
 * host or device with HTRI_OUTPUT_ON_DEVICE): cc_x = sum_p epsilon[p]
 * t[x][p] / C(deg_x, 2), deg_x = |N_{e_x}|, 0 when deg_x < 2; epsilon NULL
 * weighs every pattern 1 (then cc_x = t_x / C(deg_x, 2), in [0, 1]), else
 * each epsilon[p] in [0, 1] (Def. 5.1's weights applied per hyperedge).
 * Errors: HTRI_E_INVALID, HTRI_E_STATE, HTRI_E_OOM, HTRI_E_DEVICE. */
htri_status htri_local_clustering(htri_graph *g, const double epsilon[21], double *cc, uint32_t out_flags);

/* List the hyper-triangles of one pattern (the enumeration half of the
 * problem statement, Section 2): pattern 1..20; out receives up to capacity
 * triples of normalised hyperedge ids, each sorted ascending, in no fixed
 * order (host array int32[3*capacity], or device with HTRI_OUTPUT_ON_DEVICE
 * in out_flags); found = the number of hyper-triangles of the pattern, which
 * may exceed capacity (then an unspecified capacity of them are written).
 * Patterns 1-8 are searched around the inclusion hyperwedges; the others by
 * closing every hyperwedge.
 * Errors: HTRI_E_INVALID, HTRI_E_STATE (no wedges yet), HTRI_E_OOM,
 * HTRI_E_DEVICE. */
htri_status htri_enumerate(htri_graph *g, int32_t pattern, int64_t capacity, int32_t *out, int64_t *found,
                           uint32_t out_flags);

/* Device time of the stages of the last htri_build_wedges +
 * htri_count_patterns, milliseconds: [0] wedge build, [1] schedule,
 * [2] closure (window and probing), [3] reduce, [4] the dense window
 * (bitmaps and their closure), [5] the probing closure kernel.  Measured
 * with HIP events on the handle's stream. */
htri_status htri_last_timings(const htri_graph *g, double ms[6]);

/* Work census of the last htri_count_patterns: out[0] = S, the closure
 * stream sum over hyperwedges (r, j) of |N+(j)|; out[1] = entries the
 * probing kernel probed (owner-centric: the partners' lists cut to each
 * chunk's rank range; middle-centric: the entries of N+(r) after j);
 * out[2] = work items; out[3] = 32-bit Omega mask words stored; out[4] =
 * closure blocks launched; out[5] = rows of the dense window (0: none);
 * out[6] = hyperwedges owned inside it; out[7] = S over the owners outside
 * it; out[8] = hyperwedges owned outside it; out[9] = mask words of those;
 * out[10] = 32-bit bitmap words the window closure read; out[11] = window
 * hits enumerated one by one (all but the bulk-counted common-vertex ones);
 * out[12] = 1 if the probing ran middle-centric, 0 if owner-centric;
 * out[13] = hyperwedges in the middle-side in-list; out[14] = its mask
 * words; out[15] = hashed entries the probing kernel staged in LDS. */
htri_status htri_closure_stats(const htri_graph *g, int64_t out[16]);

/* ---------------------------------------------------------------- sampling */

typedef struct htri_model htri_model;

/* Sampling flag: close every inclusion hyperwedge exactly (a small stratum)
 * and sample only the intersection-type ones, whose sampled closures carry
 * the estimate of the rest (separate sampling of the two hyperwedge types,
 * as in Appro-adv, Algorithm 7, with the inclusion stratum exhausted). */
#define HTRI_SAMPLE_EXACT_INCLUSION 1

typedef struct {
    double budget_fraction;   /* samples = budget_fraction * |wedges| ...      */
    int64_t num_samples;      /* ... unless num_samples > 0                    */
    uint64_t seed;            /* Philox-4x32-10 key                            */
    int32_t proposal;         /* 0 = uniform, 1 = learned, 2 = split by type   */
    int32_t flags;            /* HTRI_SAMPLE_EXACT_INCLUSION or 0              */
    const htri_model *model;  /* required for proposal 1                       */
    double defensive_mix;     /* lambda: q = (1-lambda) q_model + lambda/|pool| */
                              /* (proposal 1 needs lambda > 0: the network's   */
                              /* score can be 0, and unbiasedness needs q > 0  */
                              /* on every hyperwedge; lambda <= 0 is refused)  */
    double pool_factor;       /* learned: candidate pool = pool_factor*samples  */
                              /* (<= 0: the pool is every wedge)                */
} htri_sample_params;

/* Hyperwedge-sampling estimate (Algorithm 6, sigma = 1; unbiased by Lemma
 * 4.1, and for any positive proposal by importance weighting; proposal 2 is
 * Algorithm 7, Appro-adv).
 *   proposal 0 (uniform): n draws w_t = floor(u_t * |wedges| / 2^64) with u_t
 *     the 64-bit word t of Philox stream 0 under `seed`;
 *     est_p = (|wedges| / n) * sum_t c_p(w_t), c_p(w) = the third hyperedges
 *     after w's later end that close w in pattern p.
 *   proposal 1 (learned): a pool of P = round(pool_factor * n) hyperwedges
 *     drawn uniformly (Philox stream 1; every hyperwedge when pool_factor <=
 *     0, P = |wedges|), scored s_u (htri_proposal_scores), the float64 CDF
 *     C_u = (1 - lambda) * S_u / S_P + lambda * (u + 1) / P over the inclusive
 *     sums S_u of the scores; draw t takes the first u with C_u > U_t * C_P,
 *     U_t = (word t of Philox stream 2 >> 11) * 2^-53, with the realised
 *     probability q_u = (C_u - C_{u-1}) / C_P, and
 *     est_p = (|wedges| / P) * (1/n) * sum_t c_p(pool[u_t]) / q_{u_t}.
 *   proposal 2 (Appro-adv, Algorithm 7, Section 4.2): the budget of n draws
 *     is split by the hyperwedge types (htri_adv_split): alpha1 draws from
 *     the |T| intersection hyperwedges (Philox stream 8) estimate patterns
 *     9-20 (TTT), alpha2 from the |C| inclusion ones (stream 9) pattern 1
 *     (CCC), alpha3 from T (stream 10) patterns 6-8 (TTC) and alpha4 from C
 *     (stream 11) patterns 2-5 (TCC).  Draw t of a list takes its element
 *     floor(u_t * size / 2^64) (T: the positions of htri_get_wedges that
 *     hold no inclusion hyperwedge, in order; C: those that do).  A draw
 *     counts the hyper-triangles of its class for which it is the earliest
 *     hyperwedge of its type (hyperwedges ordered by their rank pairs), and
 *     est_p = (list size / alpha_i) * sum of the draws' counts.  stderr_[p]
 *     per pattern; stderr_[0] adds the per-pattern variances (the classes
 *     are independent; within a class the covariance is left out).
 *     Not combinable with HTRI_SAMPLE_EXACT_INCLUSION.
 *   With HTRI_SAMPLE_EXACT_INCLUSION, drawn inclusion hyperwedges close
 *   nothing and the exact closures of all inclusion hyperwedges are added.
 *   est       double[21] host array: estimated H, [0] = total.
 *   stderr_   NULL or double[21]: standard error of each estimate.
 *   time_ms   NULL or double: device time of the estimate.
 * Errors: HTRI_E_STATE, HTRI_E_INVALID (also lambda outside [0, 1], or
 * lambda <= 0 with proposal 1), HTRI_E_OOM, HTRI_E_DEVICE. */
htri_status htri_estimate(htri_graph *g, const htri_sample_params *p, double est[21],
                          double stderr_[21], double *time_ms);

/* Appro-adv's split of a budget of alpha draws by hyperwedge type
 * (Algorithm 7, line 4): out[0] = alpha1 = |T|^2 alpha / |W|^2 (TTT),
 * out[1] = alpha2 = |C|^2 alpha / |W|^2 (CCC), out[2] = alpha3 and out[3] =
 * alpha4 = |T| |C| alpha / |W|^2 (TTC, TCC), with |W| = |T| + |C|, each
 * rounded half up and at least 1 when its lists are non-empty (the paper
 * leaves the rounding open), 0 otherwise.  Host arithmetic only. */
htri_status htri_adv_split(int64_t n_inter, int64_t n_incl, int64_t alpha, int64_t out[4]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * uniform estimate of htri_estimate (proposal 0, no flags, num_samples
 * draws under `seed`), computed without any allocation.  Its intermediate
 * buffers (the pattern table, per-wave partial sums and their reduction,
 * about 4 MB on 256 compute units) live in one static 8 MiB device array
 * per GPU, held until the process ends; a device whose sampling grid would
 * need more is refused with HTRI_E_UNSUPPORTED.  Calls that overlap on one
 * GPU share that array and race: issue them one after another (one stream,
 * or synchronised).  Work is only enqueued on the handle's stream; nothing
 * is synchronised.
 *   dev_est     device double[21]: the estimate (bit-identical to
 *               htri_estimate's est for the same draws).
 *   dev_stderr  NULL or device double[21]: the standard errors.
 * Errors: HTRI_E_INVALID (NULL, num_samples < 1), HTRI_E_STATE (no
 * hyperwedges yet), HTRI_E_UNSUPPORTED, HTRI_E_DEVICE. */
htri_status htri_estimate_uniform_noalloc(htri_graph *g, int64_t num_samples, uint64_t seed, double *dev_est,
                                          double *dev_stderr);

/* Sub-hypergraph for sigma-sampling (Algorithm 6, with sigma in (0, 1]: the
 * hyperedges are subsampled before the hyperwedges are, and the estimate is
 * scaled back; Section 4.2).  Hyperedge x of g (normalised id) gets the
 * 64-bit word number x of Philox-4x32-10 stream 4 under `seed` (counter
 * (x lo, x hi, 4, 0), key (seed lo, seed hi)).
 *   mode 0: x is kept when its word is below floor(sigma * 2^64) (all when
 *           sigma = 1): each hyperedge independently with probability sigma.
 *   mode 1: exactly n = floor(sigma * m + 1/2) hyperedges, those with the n
 *           smallest words (equal words by id): a uniform n-subset.
 * The hypergraph the kept hyperedges induce (same vertex ids, the flags,
 * allocator and stream of g) is loaded as *out; its input order is the kept
 * ids ascending.
 *   kept_ids        NULL or host int32[m]: the kept normalised ids of g,
 *                   ascending (num_kept of them).
 *   num_kept        NULL or the number kept.
 *   triangle_scale  NULL or the inverse of the probability that a given
 *                   hyper-triangle of g keeps all three hyperedges:
 *                   sigma^-3 (mode 0), m(m-1)(m-2) / (n(n-1)(n-2)) (mode 1;
 *                   0 when n < 3).  Counts or estimates on *out times this
 *                   are unbiased for g.
 * Errors: HTRI_E_INVALID (sigma outside (0, 1], unknown mode, NULL out),
 * HTRI_E_OOM, HTRI_E_DEVICE; *out is NULL on error. */
htri_status htri_subgraph(htri_graph *g, double sigma, uint64_t seed, int32_t mode, htri_graph **out,
                          int32_t *kept_ids, int64_t *num_kept, double *triangle_scale);

/* Close an explicit list of wedges (indices into the htri_get_wedges order)
 * and return per-pattern closure counts, int64[n*21] host array (row w:
 * [0] total, [p] pattern p).  The sampling kernels' closure step. */
htri_status htri_close_wedges(htri_graph *g, const int64_t *wedge_idx, int64_t n, int64_t *out);

/* The learned proposal's score of listed hyperwedges (the s_u of
 * htri_estimate): expm1(min(max(f(x_w), 0), 30)) with f the network and x_w
 * the 16 features of hyperwedge w, computed in float32 and returned as
 * float64.  wedge_idx: host int64[n] indices in the htri_get_wedges order,
 * or NULL with n = |wedges| for every hyperwedge; out: host double[n].
 * Errors: HTRI_E_INVALID (index out of range, NULL), HTRI_E_STATE,
 * HTRI_E_OOM, HTRI_E_DEVICE. */
htri_status htri_proposal_scores(htri_graph *g, const htri_model *model, const int64_t *wedge_idx, int64_t n,
                                 double *out);

/* Training target of the learned proposal for every hyperwedge (device
 * float[|wedges|], htri_get_wedges order): log1p(u(w)),
 *   u(w) = sqrt(sum_p (c_p(w) |wedges| / H_p)^2) / n,
 * over the n patterns p with H_p = counts[p] > 0, c_p(w) the forward
 * closure of w in pattern p.  Drawing w in proportion to u(w) minimises
 * sum_p Var(est_p) / H_p^2 (Cauchy-Schwarz), the squared form of the mean
 * per-pattern relative error.  flags HTRI_IMPORTANCE_TOTAL adds the total
 * (counts[0], c_0(w) the whole closure) as one more term, which keeps the
 * variance of the total -- and of the pattern that dominates it -- in the
 * objective.  Errors: HTRI_E_INVALID, HTRI_E_STATE, HTRI_E_OOM,
 * HTRI_E_DEVICE. */
#define HTRI_IMPORTANCE_TOTAL 1u
htri_status htri_wedge_importance(htri_graph *g, const int64_t counts[21], uint32_t flags, float *dev_out);

/* Per-wedge proposal features (16 float32 per wedge, htri_get_wedges order)
 * into a device array float[|wedges|*16]. */
htri_status htri_wedge_features(htri_graph *g, float *dev_features);

/* Proposal network 16 -> 64 -> 64 -> 1 with ReLU, float32 weights.
 * Parameter layout (htri_model_params): W1[64][16], b1[64], W2[64][64],
 * b2[64], w3[64], b3 -- 5313 floats. */
#define HTRI_MODEL_NUM_PARAMS 5313
htri_status htri_model_create(uint64_t seed, void *stream, htri_model **out);
void htri_model_free(htri_model *m);
htri_status htri_model_get_params(const htri_model *m, float *host_params);
htri_status htri_model_set_params(htri_model *m, const float *host_params);
/* Save the parameters as raw float32 (little endian, the layout above,
 * 21,252 bytes) at `path`, and their description as JSON at `path`.json
 * (format "htri-proposal-mlp", layers, dtype, num_params, layout).  Load
 * reads both back: the JSON must name this network and the raw file hold
 * exactly 5313 finite float32 values; the Adam state is reset as by
 * htri_model_set_params.  Errors: HTRI_E_INVALID (NULL, I/O failure,
 * mismatched file; htri_model_last_error says which), HTRI_E_DEVICE. */
htri_status htri_model_save(const htri_model *m, const char *path);
htri_status htri_model_load(htri_model *m, const char *path);
/* Message of the last failure on m. */
const char *htri_model_last_error(const htri_model *m);
/* Forward over n feature rows (device arrays): out[n] = network output. */
htri_status htri_model_forward(const htri_model *m, const float *dev_x, int64_t n, float *dev_out);
/* Mean-squared-error loss 0.5*mean((f(x)-y)^2) and its gradient with
 * respect to every parameter (device arrays x[n*16], y[n]; host grad
 * float[HTRI_MODEL_NUM_PARAMS]); loss written to *loss. */
htri_status htri_model_loss_grad(const htri_model *m, const float *dev_x, const float *dev_y,
                                 int64_t n, double *loss, float *host_grad);
/* Adam training on device rows x[n*16], targets y[n]: `steps` minibatch
 * steps of `batch` rows drawn with a Philox stream from `seed`. *final_loss
 * receives the last minibatch loss. */
htri_status htri_model_train(htri_model *m, const float *dev_x, const float *dev_y, int64_t n,
                             int32_t steps, int32_t batch, float lr, uint64_t seed,
                             double *final_loss);

/* ---------------------------------------------------------------- batching */

typedef struct htri_batch htri_batch;

/* Closure schedule: chunk = entries of N+(r) held in LDS per work item (256
 * or 512), partners = hyperwedges (r, j) per work item (128 or 256), order =
 * 0 (work items in graph order) or 1 (graphs with the most hyperwedges
 * started first). */
typedef struct {
    int32_t chunk;
    int32_t partners;
    int32_t order;
} htri_schedule;

/* Load `count` independent hypergraphs (host CSR arrays, one per graph, as
 * in htri_graph_load), normalise them and build their hyperwedges.  flags:
 * 0 or HTRI_DEDUPE_EDGES.  The batch owns a stream of its own (default
 * priority) and device memory from hipMalloc.  Errors as htri_graph_load,
 * the message (htri_batch_last_error / htri_last_error(NULL)) names the
 * graph. */
htri_status htri_batch_load(int32_t count, const int64_t *const *edge_offsets, const int64_t *num_edges,
                            const int32_t *const *members, const int32_t *num_vertices, uint32_t flags,
                            htri_batch **out);
/* Hyperwedges of every graph, int64[count]. */
htri_status htri_batch_info(const htri_batch *b, int64_t *wedges_per_graph);
/* Exact count of every pattern of every graph in ONE persistent launch of the
 * closure kernel (all graphs' work items in one queue), replayed from a
 * captured HIP graph when use_graph != 0.  counts: int64[count][21] host
 * array ([g][0] total).  time_ms: device time of the launch. */
htri_status htri_batch_count(htri_batch *b, const htri_schedule *sched, int32_t use_graph, int64_t *counts,
                             double *time_ms);
/* Try every schedule (graph-replayed, best of `repeats` runs each) and
 * return the fastest. */
htri_status htri_batch_autotune(htri_batch *b, int32_t repeats, htri_schedule *best, double *best_ms);
/* Baseline: the same counts with one closure launch per graph, issued back
 * to back on the batch's stream; time_ms covers all launches. */
htri_status htri_batch_count_per_graph(htri_batch *b, const htri_schedule *sched, int64_t *counts,
                                       double *time_ms);
/* Schedules per size class.  A graph's class is its hyperwedge count:
 * class 0 below 2^18, class 1 below 2^21, class 2 from 2^21 (written to
 * class_of_graph, int32[count], by htri_batch_size_classes).
 * htri_batch_autotune_classes times every schedule on the graphs of each
 * class (graph-replayed, best of `repeats`) and returns the fastest per
 * class in best[3] (classes without graphs get 512/256/1 and 0 ms);
 * cache_path (NULL: none) names a JSON file: when it holds schedules for
 * this device's architecture and compute-unit count and every populated
 * class, they are returned without timing (*from_cache = 1), else the
 * tuned ones are written to it.  htri_batch_count_classes counts every
 * graph with its class's schedule: one persistent launch per populated
 * class, all captured in one HIP graph when use_graph != 0.
 * Errors: HTRI_E_INVALID (also an unwritable cache), HTRI_E_DEVICE. */
htri_status htri_batch_size_classes(const htri_batch *b, int32_t *class_of_graph);
htri_status htri_batch_autotune_classes(htri_batch *b, int32_t repeats, const char *cache_path, htri_schedule *best,
                                        double *best_ms, int32_t *from_cache);
htri_status htri_batch_count_classes(htri_batch *b, const htri_schedule *sched, int32_t use_graph, int64_t *counts,
                                     double *time_ms);

/* The whole hot path of every graph -- step 1 (hyperwedges), the closure
 * work items and the closure -- in ONE captured HIP graph, replayed: each
 * replay rebuilds every graph's hyperwedges from its loaded hypergraph and
 * counts all of them.  The first call with a schedule records the per-graph
 * host code once (its readbacks and allocation sizes), then captures it
 * with every buffer taken from one device arena the batch keeps (about the
 * step-1 working memory of all graphs together); later calls only replay.
 * counts: int64[count][21]; time_ms: device time of the replay. */
htri_status htri_batch_count_full(htri_batch *b, const htri_schedule *sched, int64_t *counts, double *time_ms);
/* Baseline for the above: step 1, work items and closure issued graph by
 * graph from the host, as a caller without the batch would (one launch
 * sequence per graph, its readbacks included); time_ms is wall time. */
htri_status htri_batch_count_full_per_graph(htri_batch *b, const htri_schedule *sched, int64_t *counts,
                                            double *time_ms);
const char *htri_batch_last_error(const htri_batch *b);
void htri_batch_free(htri_batch *b); /* NULL-safe */

/* ---------------------------------------------------------------- misc */

const char *htri_status_string(htri_status s);
/* Message of the last failure on g (g NULL: the last failed load). */
const char *htri_last_error(const htri_graph *g);
void htri_graph_free(htri_graph *g); /* NULL-safe */

#ifdef __cplusplus
}
#endif
#endif /* HTRI_H */
