"""Listing the hyper-triangles of one pattern (the enumeration half of the
problem statement) through the C ABI, against the brute-force listing."""
import numpy as np
import pytest

from oracle import brute, core
from paper_2504_02271_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def htri():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_02271_amd import htri as h
    h.load_library()
    return h


def _edges(g):
    return [g.edge(x).tolist() for x in range(g.num_edges)]


@pytest.mark.parametrize("seed", range(12))
def test_every_pattern_small_universes(htri, seed):
    g = synth.random_small(seed, 50 + 5 * seed, 5 + 3 * seed, 1, 6)
    want = brute.triangles(_edges(g))
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    for p in range(1, 21):
        got, found = G.enumerate(p)
        assert found == len(want[p]), (seed, p)
        assert sorted(map(tuple, got.tolist())) == want[p], (seed, p)


def test_capacity_and_errors(htri):
    g = synth.random_small(5, 120, 20, 1, 6)
    want = brute.triangles(_edges(g))
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    p = max(range(1, 21), key=lambda q: len(want[q]))
    got, found = G.enumerate(p, capacity=3)
    assert found == len(want[p]) and got.shape == (3, 3)
    assert set(map(tuple, got.tolist())) <= set(want[p])
    with pytest.raises(htri.HtriError):
        G.enumerate(21)


def test_rare_patterns_coauthorship(htri):
    """Co-authorship-shaped graph: every listed triple of a rare pattern is a
    hyper-triangle of that pattern (checked on its vertex sets), listed once,
    and there are as many as the exact count."""
    g = synth.generate(synth.config("coauth"))
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    counts, _, _ = G.count_patterns()
    E = brute.normalise(_edges(g))
    for p in range(1, 21):
        if counts[p] == 0 or counts[p] > 20000:
            continue
        got, found = G.enumerate(p)
        assert found == counts[p], p
        trip = [tuple(t) for t in got.tolist()]
        assert len(set(trip)) == len(trip)
        for a, b, c in trip:
            assert a < b < c
            assert E[a] & E[b] and E[a] & E[c] and E[b] & E[c]
            assert brute.pattern_of(E[a], E[b], E[c]) == p
