"""Reference of the proposal's per-wedge features -- test infrastructure only.

For a hyperwedge oriented r -> j (r earlier in the order `rank`):
 0 log1p|e_r|   1 log1p|e_j|   2 log1p omega   3 inclusion type (omega == min size)
 4 log1p d+(r)  5 log1p d+(j)  (later neighbours)
 6 log1p a, a = later neighbours of r that come after j
 7 log1p min(a, d+(j))
 8 log1p deg(r) 9 log1p deg(j)  (all neighbours)
10 omega / min size  11 omega / max size
12-14 log1p of the max, min and mean of |E_v| over the shared vertices v
15 constant 1
"""
from __future__ import annotations

import numpy as np


def features(off, mem, num_vertices, rank, wi, wj, wo, lo, hi):
    """16 features (float64) for the oriented wedges (lo[t] -> hi[t]); wi, wj,
    wo list every hyperwedge with its omega (any orientation)."""
    m = off.shape[0] - 1
    sizes = np.diff(off)
    dv = np.bincount(mem, minlength=num_vertices)
    a = np.where(rank[wi] < rank[wj], wi, wj)
    b = np.where(rank[wi] < rank[wj], wj, wi)
    dplus = np.bincount(a, minlength=m)
    deg = dplus + np.bincount(b, minlength=m)
    om = {}
    for x, y, w in zip(wi.tolist(), wj.tolist(), wo.tolist()):
        om[(x, y)] = w
        om[(y, x)] = w
    fwd = {}
    for x, y in zip(a.tolist(), b.tolist()):
        fwd.setdefault(x, []).append(rank[y])
    for x in fwd:
        fwd[x].sort()
    out = np.zeros((len(lo), 16))
    for t, (r, j) in enumerate(zip(lo.tolist(), hi.tolist())):
        w = om[(r, j)]
        si, sj = int(sizes[r]), int(sizes[j])
        mn, mx = min(si, sj), max(si, sj)
        lst = fwd[r]
        pos = int(np.searchsorted(lst, rank[j]))
        after = len(lst) - pos - 1
        shared = np.intersect1d(mem[off[r]:off[r + 1]], mem[off[j]:off[j + 1]])
        d = dv[shared].astype(np.float64)
        out[t] = [np.log1p(si), np.log1p(sj), np.log1p(w), 1.0 if w == mn else 0.0,
                  np.log1p(dplus[r]), np.log1p(dplus[j]), np.log1p(after), np.log1p(min(after, dplus[j])),
                  np.log1p(deg[r]), np.log1p(deg[j]), w / mn, w / mx,
                  np.log1p(d.max()), np.log1p(d.min()), np.log1p(d.mean()), 1.0]
    return out
