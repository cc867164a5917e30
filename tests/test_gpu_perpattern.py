"""Per-hyperedge counts of every pattern in one call, and the local
clustering coefficients built on them (Def. 5.1 of Section 5, applied per
hyperedge), against the oracle's per-hyperedge counts restricted to one
pattern at a time."""
import numpy as np
import pytest

from oracle import core
from paper_2504_02271_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def htri():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_02271_amd import htri as h
    h.load_library()
    return h


def _family(name):
    if name.startswith("small"):
        q = int(name[5:])
        return synth.random_small(q, 50 + 5 * q, 5 + 3 * q, 1, 6)
    if name == "clique":
        rng = np.random.default_rng(9)
        edges = [[0] + sorted(rng.choice(np.arange(1, 200), size=2, replace=False).tolist()) for _ in range(900)]
        edges += [[0, 1, 2] + sorted(rng.choice(np.arange(3, 90), size=3, replace=False).tolist())
                  for _ in range(300)]
        edges.append(list(range(50, 250)))
        return synth.from_lists(edges, 260, "clique")
    if name == "nested":
        # chains of nested hyperedges and shared cores: patterns 1-8 and the
        # thick pairs of 10-16 in quantity
        rng = np.random.default_rng(4)
        edges = []
        for c in range(40):
            base = sorted(rng.choice(np.arange(300), size=6, replace=False).tolist())
            edges += [base[:2], base[:3], base[:4], base, base[:2] + [300 + c], base[1:3] + [340 + c]]
        return synth.from_lists(edges, 400, "nested")
    return synth.generate(synth.config(name))


def _oracle_per_pattern(o):
    t = np.zeros((o.m, 21), np.int64)
    for p in range(1, 21):
        t[:, p] = o.count(edge_mask=1 << p).t
    t[:, 0] = o.count().t
    return t


@pytest.mark.parametrize("name", ["small0", "small5", "small9", "small11", "tiny", "clique", "nested"])
def test_per_edge_patterns_exact(htri, name):
    g = _family(name)
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    want = _oracle_per_pattern(o)
    H = o.count(per_edge=False).H
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    counts, t = G.count_per_edge_patterns()
    assert np.array_equal(counts, H), (counts, H)
    assert t.shape == want.shape
    bad = np.argwhere(t != want)
    assert bad.size == 0, (name, bad[:5], t[tuple(bad[0])], want[tuple(bad[0])])
    # each triangle holds three hyperedges
    assert np.array_equal(t.sum(axis=0), 3 * H)
    # a second call on the same handle gives the same result
    counts2, t2 = G.count_per_edge_patterns()
    assert np.array_equal(counts2, counts) and np.array_equal(t2, t)
    G.close()


def test_per_edge_patterns_coauthorship_sampled(htri):
    """500,000 hyperedges: the full per-hyperedge count and the column sums
    against the oracle's count, each pattern's column on 300 sampled
    hyperedges against the oracle's per-hyperedge triangle listing."""
    g = synth.generate(synth.config("coauth"))
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    r = o.count()
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    counts, t = G.count_per_edge_patterns()
    print(f"\n[perpattern] coauth: {G.last_timings()}", flush=True)
    assert np.array_equal(counts, r.H)
    assert np.array_equal(t[:, 0], r.t)
    assert np.array_equal(t[:, 1:].sum(axis=1), r.t)
    assert np.array_equal(t.sum(axis=0), 3 * r.H)
    rng = np.random.default_rng(12)
    xs = np.sort(rng.choice(o.m, size=300, replace=False)).astype(np.int32)
    for p in range(1, 21):
        want = o.edge_triangles(xs, 1 << p)
        assert np.array_equal(t[xs, p], want), (p, np.nonzero(t[xs, p] != want)[0][:5])
    G.close()


@pytest.mark.parametrize("name", ["small9", "tiny", "nested"])
def test_local_clustering(htri, name):
    """cc_x = t_x / C(deg_x, 2) with every weight 1 (in [0, 1]: a triangle
    holding x is fixed by its other two hyperedges, a pair of neighbours of
    x), and sum_p eps_p t[x][p] / C(deg_x, 2) with weights per pattern."""
    g = _family(name)
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    want = _oracle_per_pattern(o)
    deg = o.degrees().astype(np.float64)
    pairs = deg * (deg - 1) / 2
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    cc = G.local_clustering()
    ref = np.where(deg >= 2, want[:, 0] / np.where(pairs > 0, pairs, 1), 0.0)
    assert np.allclose(cc, ref, rtol=1e-15, atol=0)
    assert (cc >= 0).all() and (cc <= 1).all()
    eps = np.random.default_rng(3).random(21)
    eps[0] = 0.0
    ccw = G.local_clustering(eps)
    num = (want[:, 1:] * eps[1:]).sum(axis=1)
    refw = np.where(deg >= 2, num / np.where(pairs > 0, pairs, 1), 0.0)
    # 20 products summed in a different order: a few units in the last place
    assert np.allclose(ccw, refw, rtol=64 * 2.0 ** -53, atol=0)
    with pytest.raises(htri.HtriError) as e:
        bad = eps.copy()
        bad[4] = 1.5
        G.local_clustering(bad)
    assert e.value.code == -1
    G.close()


def test_per_edge_patterns_empty_and_wedgeless(htri):
    g = synth.from_lists([], 5, "empty")
    G = htri.graph_load(g.offsets, g.members, 5)
    G.build_wedges()
    counts, t = G.count_per_edge_patterns()
    assert not counts.any() and t.shape == (0, 21)
    assert G.local_clustering().shape == (0,)
    G.close()
    g = synth.from_lists([[0, 1], [2, 3], [4, 5, 6]], 7, "wedgeless")
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    counts, t = G.count_per_edge_patterns()
    assert not counts.any() and t.shape == (3, 21) and not t.any()
    assert not G.local_clustering().any()
    G.close()
