"""O(m^3) brute force -- test infrastructure only.

A third, independent way to classify hyper-triangles, used to pin the C
oracle on tiny hypergraphs.  Every unordered triple of hyperedges is tested
for pairwise intersection with Python sets; the seven regions of Section 2
(a = i only, b = j only, c = k only, d = i&j-k, e = j&k-i, f = k&i-j,
g = i&j&k) are materialised as explicit sets; the emptiness pattern is
canonicalised by trying all six relabellings of the three hyperedges, and
the canonical form is looked up among one witness region set per pattern.

The witness sets: patterns 1-8 follow from the arithmetic of Algorithm 5
(chain; the third hyperedge equal to / strictly inside the intersection of
two intersecting ones; equal to / strictly containing their union; and the
three inclusion-plus-two-intersection cases), 5 from the e-mail case study
(Fig. 7), 10 and 12 from the co-authorship case study (Fig. 6).  The order
of 9, 11 and 13-20 is a reading (pair regions, then private regions, both
ascending) -- parity unpinned against the paper for those numbers.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np

# region letter -> index in the 7-tuple (a, b, c, d, e, f, g)
_IDX = {ch: n for n, ch in enumerate("abcdefg")}

# One witness per pattern: the non-empty regions.
WITNESS = {
    1: "cfg", 2: "bcg", 3: "bceg", 4: "efg", 5: "cefg", 6: "bcfg", 7: "cdfg", 8: "bcefg",
    9: "abcg", 10: "abcfg", 11: "bcdfg", 12: "abcefg", 13: "defg", 14: "cdefg",
    15: "bcdefg", 16: "abcdefg", 17: "def", 18: "cdef", 19: "bcdef", 20: "abcdef",
}


def _relabel(mask: Tuple[int, ...], perm: Tuple[int, int, int]) -> Tuple[int, ...]:
    """Region flags after renaming hyperedge x (0=i,1=j,2=k) to perm[x]."""
    single = {0: mask[0], 1: mask[1], 2: mask[2]}
    pair = {frozenset((0, 1)): mask[3], frozenset((1, 2)): mask[4], frozenset((2, 0)): mask[5]}
    ns = [0, 0, 0]
    for x in range(3):
        ns[perm[x]] = single[x]
    npair = {}
    for key, val in pair.items():
        x, y = tuple(key)
        npair[frozenset((perm[x], perm[y]))] = val
    return (ns[0], ns[1], ns[2], npair[frozenset((0, 1))], npair[frozenset((1, 2))],
            npair[frozenset((2, 0))], mask[6])


def canonical(mask: Sequence[int]) -> Tuple[int, ...]:
    m = tuple(int(bool(x)) for x in mask)
    return min(_relabel(m, p) for p in itertools.permutations(range(3)))


def _witness_mask(regions: str) -> Tuple[int, ...]:
    m = [0] * 7
    for ch in regions:
        m[_IDX[ch]] = 1
    return tuple(m)


CANON_TO_PATTERN: Dict[Tuple[int, ...], int] = {}
for _p, _r in WITNESS.items():
    _c = canonical(_witness_mask(_r))
    assert _c not in CANON_TO_PATTERN, "two witnesses share a class"
    CANON_TO_PATTERN[_c] = _p


def closed_classes() -> List[Tuple[int, ...]]:
    """Canonical masks of every emptiness pattern whose three hyperedges are
    pairwise intersecting and pairwise distinct (all 2^7 masks enumerated)."""
    out = set()
    for bits in range(128):
        m = tuple((bits >> t) & 1 for t in range(7))
        a, b, c, d, e, f, g = m
        if not ((d or g) and (e or g) and (f or g)):
            continue
        # distinct sets: i != j needs a region in exactly one of them, etc.
        ei = {"a", "d", "f", "g"}
        ej = {"b", "d", "e", "g"}
        ek = {"c", "e", "f", "g"}
        nonempty = {ch for ch, v in zip("abcdefg", m) if v}
        si, sj, sk = ei & nonempty, ej & nonempty, ek & nonempty
        if si == sj or sj == sk or si == sk:
            continue
        out.add(canonical(m))
    return sorted(out)


def regions(ei: set, ej: set, ek: set):
    return (ei - ej - ek, ej - ek - ei, ek - ei - ej, (ei & ej) - ek, (ej & ek) - ei,
            (ek & ei) - ej, ei & ej & ek)


def pattern_of(ei: set, ej: set, ek: set) -> int:
    return CANON_TO_PATTERN[canonical([len(r) > 0 for r in regions(ei, ej, ek)])]


def normalise(edges: Iterable[Iterable[int]]) -> List[frozenset]:
    """Vertex sets, first occurrence kept (Def. 2.1 and distinct hyperedges)."""
    seen = set()
    out = []
    for e in edges:
        s = frozenset(int(v) for v in e)
        if not s:
            raise ValueError("empty hyperedge")
        if s in seen:
            continue
        seen.add(s)
        out.append(s)
    return out


def count(edges: Sequence[Iterable[int]]):
    """(H[21], t[m]) over the normalised hyperedges, by checking every triple."""
    E = normalise(edges)
    m = len(E)
    H = np.zeros(21, np.int64)
    t = np.zeros(m, np.int64)
    adj = [[bool(E[x] & E[y]) for y in range(m)] for x in range(m)]
    for i in range(m):
        for j in range(i + 1, m):
            if not adj[i][j]:
                continue
            for k in range(j + 1, m):
                if adj[i][k] and adj[j][k]:
                    p = pattern_of(E[i], E[j], E[k])
                    H[p] += 1
                    H[0] += 1
                    t[i] += 1
                    t[j] += 1
                    t[k] += 1
    return H, t


def triangles(edges: Sequence[Iterable[int]]):
    """Pattern -> sorted list of hyper-triangles (i, j, k), i < j < k, over the
    normalised ids, by the same triple loop as count()."""
    E = normalise(edges)
    m = len(E)
    out = {p: [] for p in range(1, 21)}
    adj = [[bool(E[x] & E[y]) for y in range(m)] for x in range(m)]
    for i in range(m):
        for j in range(i + 1, m):
            if not adj[i][j]:
                continue
            for k in range(j + 1, m):
                if adj[i][k] and adj[j][k]:
                    out[pattern_of(E[i], E[j], E[k])].append((i, j, k))
    return out


def hyperwedges(edges: Sequence[Iterable[int]]):
    """Sorted list of (i, j, omega_ij, is_inclusion) over normalised ids, i<j."""
    E = normalise(edges)
    out = []
    for i in range(len(E)):
        for j in range(i + 1, len(E)):
            w = len(E[i] & E[j])
            if w:
                out.append((i, j, w, E[i] <= E[j] or E[j] <= E[i]))
    return out
