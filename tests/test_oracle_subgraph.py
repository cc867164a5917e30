"""Pins of the sigma-sampling oracle (sub-hypergraph selection and the
triangle scale, Algorithm 6 with sigma < 1): every subset of a tiny
hypergraph counted by brute force."""
import itertools
import math

import numpy as np

from oracle import brute, sampling


def _tiny():
    rng = np.random.default_rng(12)
    edges = []
    while len(edges) < 9:
        e = sorted(rng.choice(7, size=int(rng.integers(2, 5)), replace=False).tolist())
        if e not in edges:
            edges.append(e)
    return edges


def test_fixed_size_scale_averages_to_the_count():
    """Over all n-subsets S, the mean of H(G[S]) times the fixed-size scale is
    H(G) exactly (per pattern), for every n >= 3."""
    edges = _tiny()
    m = len(edges)
    H = brute.count(edges)[0]
    assert H[0] > 0
    for n in range(3, m + 1):
        tot = np.zeros(21, np.int64)
        for S in itertools.combinations(range(m), n):
            tot += brute.count([edges[x] for x in S])[0]
        # sum over subsets = H * C(m-3, n-3); the scale is C(m, n) / C(m-3, n-3)
        assert np.array_equal(tot, H * math.comb(m - 3, n - 3)), n
        scale = sampling.subgraph_scale(m, n, n / m, True)
        assert math.isclose(scale, math.comb(m, n) / math.comb(m - 3, n - 3), rel_tol=1e-14)
        assert np.allclose(tot / math.comb(m, n) * scale, H, rtol=1e-12)
    assert sampling.subgraph_scale(m, 2, 2 / m, True) == 0.0


def test_independent_scale_averages_to_the_count():
    """Weighted by sigma^|S| (1-sigma)^(m-|S|) over all subsets S, H(G[S])
    times sigma^-3 is H(G)."""
    edges = _tiny()
    m = len(edges)
    H = brute.count(edges)[0].astype(np.float64)
    per_subset = {}
    for mask in range(1 << m):
        S = [x for x in range(m) if mask >> x & 1]
        per_subset[mask] = (len(S), brute.count([edges[x] for x in S])[0].astype(np.float64))
    for sigma in (0.25, 0.5, 0.9):
        acc = np.zeros(21)
        for k, h in per_subset.values():
            acc += sigma ** k * (1 - sigma) ** (m - k) * h
        assert np.allclose(acc * sampling.subgraph_scale(m, 0, sigma, False), H, rtol=1e-12), sigma


def test_selection_rules():
    m = 100000
    for sigma in (0.1, 0.5):
        kept = sampling.subgraph_select(m, sigma, 7, False)
        assert (np.diff(kept) > 0).all()
        assert abs(kept.shape[0] / m - sigma) < 5 * math.sqrt(sigma * (1 - sigma) / m)
        fixed = sampling.subgraph_select(m, sigma, 7, True)
        assert fixed.shape[0] == int(math.floor(sigma * m + 0.5)) and (np.diff(fixed) > 0).all()
        # the fixed-size set is the n smallest words
        u = sampling.draws_u64(7, sampling.SUBGRAPH_STREAM, m)
        assert u[fixed].max() < np.delete(u, fixed).min()
    assert np.array_equal(sampling.subgraph_select(50, 1.0, 3, False), np.arange(50))
    assert sampling.subgraph_select(0, 0.5, 3, True).shape == (0,)


def test_induced_csr():
    off = np.array([0, 2, 5, 6], np.int64)
    mem = np.array([0, 1, 1, 2, 3, 4], np.int32)
    o, mm = sampling.induced_csr(off, mem, np.array([0, 2], np.int64))
    assert o.tolist() == [0, 2, 3] and mm.tolist() == [0, 1, 4]
