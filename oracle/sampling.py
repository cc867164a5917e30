"""Oracle side of hyperwedge sampling -- test infrastructure only.

Philox4x32-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011): a 4x32-bit counter and 2x32-bit key, ten rounds
of two 32x32->64 multiplications by 0xD2511F53 and 0xCD9E8D57 with the key
bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.

The estimators follow Algorithm 6 with sigma = 1 (hyperwedges drawn with
replacement, each closed with the third hyperedges that come after it, the
sum scaled by |wedges| / samples), unbiased by Lemma 4.1, and its
importance-sampling generalisation (each closure divided by the realised
draw probability).
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One block: ctr = 4 uint32 (numpy arrays broadcast), key = 2 uint32."""
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) for k in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = x0 * np.uint64(M0)
        p1 = x2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0) & MASK, lo1, (hi0 ^ x3 ^ k1) & MASK, lo0
    return x0, x1, x2, x3


def draws_u64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """n 64-bit uniform words: counter (t lo, t hi, stream, 0), key = seed."""
    t = np.arange(start, start + n, dtype=np.uint64)
    ctr = (t & np.uint64(MASK), t >> np.uint64(32), np.full(n, stream, np.uint64), np.zeros(n, np.uint64))
    key = (np.uint64(seed & MASK), np.uint64((seed >> 32) & MASK))
    x0, x1, _, _ = philox4x32_10(ctr, key)
    return (x1 << np.uint64(32)) | x0


def uniform_indices(seed: int, stream: int, n: int, N: int) -> np.ndarray:
    """floor(u * N / 2^64) for the 64-bit words u -- exact integer arithmetic."""
    u = draws_u64(seed, stream, n)
    hi = u >> np.uint64(32)
    lo = u & np.uint64(MASK)
    N = np.uint64(N)
    # (u * N) >> 64 with u = hi*2^32 + lo, N < 2^63
    nh = N >> np.uint64(32)
    nl = N & np.uint64(MASK)
    ll = lo * nl
    lh = lo * nh
    hl = hi * nl
    hh = hi * nh
    mid = (ll >> np.uint64(32)) + (lh & np.uint64(MASK)) + (hl & np.uint64(MASK))
    return (hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))).astype(np.int64)


def uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each 64-bit word."""
    return (draws_u64(seed, stream, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def prec_wedge_order(rank: np.ndarray, wi: np.ndarray, wj: np.ndarray):
    """Hyperwedges oriented from the earlier to the later hyperedge in the
    order `rank`, listed by (rank of the earlier, rank of the later)."""
    lo = np.where(rank[wi] < rank[wj], wi, wj)
    hi = np.where(rank[wi] < rank[wj], wj, wi)
    order = np.lexsort((rank[hi], rank[lo]))
    return lo[order], hi[order]


def uniform_estimate(closures: np.ndarray, num_wedges: int):
    """Algorithm 6 with sigma = 1.  closures: int64[n, 21] per drawn wedge.
    Returns (estimate[21], standard error[21])."""
    n = closures.shape[0]
    sums = closures.sum(axis=0)
    est = sums.astype(np.float64) * float(num_wedges) / float(n)
    y = closures.astype(np.float64) * float(num_wedges)
    var = (y ** 2).sum(axis=0) - n * (est ** 2)
    se = np.sqrt(np.maximum(var, 0.0) / (n * max(n - 1, 1)))
    return est, se


def learned_cdf(scores: np.ndarray, lam: float) -> np.ndarray:
    """Mixed proposal CDF over a pool of P candidates: the inclusive float64
    sums S of the scores, C_u = (1 - lam) / S_P * S_u + lam / P * (u + 1)
    (uniform, (u + 1) / P, when every score is 0)."""
    P = scores.shape[0]
    S = np.cumsum(np.asarray(scores, np.float64))
    tot = S[-1]
    if tot > 0:
        return ((1.0 - lam) / tot) * S + (lam / P) * np.arange(1, P + 1, dtype=np.float64)
    return (1.0 / P) * np.arange(1, P + 1, dtype=np.float64)


def learned_estimate(scores: np.ndarray, pool: np.ndarray, num_wedges: int, lam: float, seed: int, n: int,
                     close):
    """Importance-sampling estimate with a learned proposal over a pool
    (Hansen-Hurwitz with replacement, each closure divided by its realised
    draw probability; the pool's uniform estimate scaled by |wedges| / P).

    scores: float64[P] the proposal's scores of the pool members; pool:
    int64[P] their wedge indices; close(idx) -> int64[n, 21] the forward
    closures of the listed wedges.  Draw t is the first u with
    C_u > U_t * C_P, U_t the t-th double of Philox stream 2; its probability
    is q_u = (C_u - C_{u-1}) / C_P.
    Returns (est[21], stderr[21], q float64[P], drawn positions int64[n])."""
    P = scores.shape[0]
    C = learned_cdf(scores, lam)
    CP = C[-1]
    U = uniform01(seed, 2, n) * CP
    u = np.searchsorted(C, U, side="right")
    q = np.diff(np.concatenate([[0.0], C])) / CP
    wgt = (float(num_wedges) / float(P)) / q[u]
    cl = close(pool[u])
    y = cl.astype(np.float64) * wgt[:, None]
    est = y.sum(axis=0) / n
    var = (y ** 2).sum(axis=0) - n * est * est
    se = np.sqrt(np.maximum(var, 0.0) / (n * max(n - 1, 1)))
    return est, se, q, u


# ---------------------------------------------------------------- Appro-adv (Algorithm 7)

ADV_STREAMS = (8, 9, 10, 11)          # TTT, CCC, TTC, TCC draws
CLASS_PATTERNS = {"TTT": range(9, 21), "CCC": (1,), "TTC": (6, 7, 8), "TCC": (2, 3, 4, 5)}


def adv_split(n_inter: int, n_incl: int, alpha: int):
    """Algorithm 7, line 4: alpha1 = |T|^2 a / |W|^2, alpha2 = |C|^2 a / |W|^2,
    alpha3 = alpha4 = |T| |C| a / |W|^2, rounded half up, at least 1 where
    the lists drawn from are non-empty (0 otherwise)."""
    w = float(n_inter + n_incl)

    def share(num, ok):
        if not ok or w <= 0:
            return 0
        return max(int(np.floor(num / (w * w) * alpha + 0.5)), 1)
    a3 = share(float(n_inter) * n_incl, n_inter > 0 and n_incl > 0)
    return [share(float(n_inter) ** 2, n_inter > 0), share(float(n_incl) ** 2, n_incl > 0), a3, a3]


def adv_cross_count(E, rank, x: int, y: int, cpart, cls: str) -> np.ndarray:
    """Mixed-class hyper-triangles attributed to the hyperwedge {x, y}
    (normalised ids; E their vertex sets; cpart[z] the hyperedges joined to z
    by an inclusion hyperwedge).  cls "TTC" (x, y an intersection
    hyperwedge): the triangles with exactly one inclusion hyperwedge, counted
    when {x, y} is the earlier of their two intersection hyperwedges; "TCC"
    (x, y an inclusion hyperwedge): exactly two inclusion hyperwedges,
    counted when {x, y} is the earlier of the two.  Hyperwedges are ordered
    by their (smaller rank, larger rank) pairs.  Patterns by the canonical
    region masks.  Returns int64[21]."""
    from oracle import brute

    def key(a, b):
        return tuple(sorted((int(rank[a]), int(rank[b]))))
    out = np.zeros(21, np.int64)
    me = key(x, y)
    for k in sorted((cpart.get(x, set()) | cpart.get(y, set())) - {x, y}):
        ix, iy = k in cpart.get(x, set()), k in cpart.get(y, set())
        if ix and iy:
            continue                           # three inclusion hyperwedges
        inc_end, other = (x, y) if ix else (y, x)
        if not (E[other] & E[k]):
            continue
        rival = key(other, k) if cls == "TTC" else key(inc_end, k)
        if me < rival:
            p = brute.pattern_of(E[x], E[y], E[k])
            assert p in CLASS_PATTERNS[cls], (cls, p)
            out[p] += 1
            out[0] += 1
    return out


def appro_adv(seed: int, alpha: int, t_pos: np.ndarray, c_pos: np.ndarray, close_fwd, cross):
    """Algorithm 7 with sigma = 1 over the hyperwedge list of some order:
    t_pos / c_pos the positions of the intersection / inclusion hyperwedges
    in it (ascending); close_fwd(positions) -> int64[n, 21] forward closures;
    cross(cls, positions) -> int64[n, 21] mixed-class counts.  Draw t of a
    list is its element floor(u_t * size / 2^64), u_t from Philox streams
    8..11.  Returns (est[21], alphas[4])."""
    nT, nC = int(t_pos.shape[0]), int(c_pos.shape[0])
    alphas = adv_split(nT, nC, alpha)
    est = np.zeros(21)
    jobs = (("TTT", t_pos, alphas[0], ADV_STREAMS[0]), ("CCC", c_pos, alphas[1], ADV_STREAMS[1]),
            ("TTC", t_pos, alphas[2], ADV_STREAMS[2]), ("TCC", c_pos, alphas[3], ADV_STREAMS[3]))
    for cls, lst, a, stream in jobs:
        if a <= 0:
            continue
        pos = lst[uniform_indices(seed, stream, a, lst.shape[0])]
        counts = close_fwd(pos) if cls in ("TTT", "CCC") else cross(cls, pos)
        tot = counts.sum(axis=0)
        for p in CLASS_PATTERNS[cls]:
            est[p] = float(tot[p]) * float(lst.shape[0]) / float(a)
    est[0] = sum(est[1:].tolist())              # pattern order, left to right
    return est, alphas


def relative_error(est: np.ndarray, exact: np.ndarray):
    """Mean of |H - est| / H over the patterns with H > 0 (the error metric of
    Section 6.3, restricted to patterns that occur), and the per-pattern
    relative errors."""
    H = exact[1:].astype(np.float64)
    E = est[1:]
    nz = H > 0
    rel = np.full(20, np.nan)
    rel[nz] = np.abs(H[nz] - E[nz]) / H[nz]
    return float(np.nanmean(rel)) if nz.any() else 0.0, rel


# ---------------------------------------------------------------- sigma-sampling

SUBGRAPH_STREAM = 4


def subgraph_select(m: int, sigma: float, seed: int, fixed_size: bool) -> np.ndarray:
    """Kept hyperedge ids (normalised ids, ascending) of the sub-hypergraph of
    Algorithm 6's sigma-sampling.  Hyperedge x gets the 64-bit word number x
    of stream SUBGRAPH_STREAM.  Independent (fixed_size False): kept when the
    word is below floor(sigma * 2^64), all when sigma = 1.  Fixed size: the
    n = floor(sigma * m + 1/2) hyperedges with the smallest words, equal
    words by id."""
    if m == 0:
        return np.zeros(0, np.int64)
    u = draws_u64(seed, SUBGRAPH_STREAM, m)
    if not fixed_size:
        if sigma >= 1.0:
            return np.arange(m, dtype=np.int64)
        thr = np.uint64(int(sigma * 2.0 ** 64))
        return np.nonzero(u < thr)[0].astype(np.int64)
    n = int(np.floor(sigma * m + 0.5))
    n = min(max(n, 0), m)
    order = np.lexsort((np.arange(m), u))
    return np.sort(order[:n]).astype(np.int64)


def subgraph_scale(m: int, n: int, sigma: float, fixed_size: bool) -> float:
    """Inverse of the probability that a given hyper-triangle keeps its three
    hyperedges: sigma^-3 when each hyperedge is kept independently, the ratio
    m(m-1)(m-2) / (n(n-1)(n-2)) for a uniform n-subset (0 when n < 3)."""
    if not fixed_size:
        return 1.0 / (sigma * sigma * sigma)
    if n < 3:
        return 0.0
    M, N = float(m), float(n)
    return (M * (M - 1.0) * (M - 2.0)) / (N * (N - 1.0) * (N - 2.0))


def induced_csr(offsets: np.ndarray, members: np.ndarray, kept: np.ndarray):
    """CSR of the hyperedges `kept` (in that order) of a CSR."""
    sizes = (offsets[kept + 1] - offsets[kept]).astype(np.int64)
    off = np.zeros(kept.shape[0] + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    mem = np.concatenate([members[offsets[x]:offsets[x + 1]] for x in kept]) if kept.shape[0] else \
        np.zeros(0, np.int32)
    return off, mem.astype(np.int32)
