"""The later ends' side of the forward adjacency at a size that spans several
rank buckets and several chunks per bucket: in-degrees per hyperedge (through
W and the local clustering coefficients) and the in-list of the closure
around the middle for three window starts, against the oracle.

Co-authorship-shaped graph, 149,991 hyperedges and 5.16e6 hyperwedges: 10
buckets of 2^14 ranks for the in-list (the largest 2.16e6 entries, 33
placing chunks) and 5 of 2^15 for the in-degrees."""
import numpy as np
import pytest

from oracle import core
from paper_2504_02271_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def graphs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_02271_amd import htri as h
    h.load_library()
    g = synth.generate(synth.config("coauth", 0.3))
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    r = o.count()
    G = h.graph_load(g.offsets, g.members, g.num_vertices)
    yield h, g, o, r, G
    G.close()


def test_summary_and_degrees(graphs):
    h, g, o, r, G = graphs
    s = G.build_wedges()
    assert G.num_edges == 149991 and s[0] == 5156863
    # W = sum over hyperedges of C(deg, 2): every in-degree enters it
    assert np.array_equal(s, o.summary()), (s, o.summary())
    # cc_x = t_x / C(deg_x, 2) for every hyperedge: each in-degree on its own
    deg = o.degrees().astype(np.float64)
    pairs = deg * (deg - 1) / 2
    want = np.where(deg >= 2, r.t / np.where(pairs > 0, pairs, 1), 0.0)
    cc = G.local_clustering()
    assert np.allclose(cc, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("window", ["off", "always", "auto"])
def test_inlist_for_each_window_start(graphs, window):
    h, g, o, r, G = graphs
    G.build_wedges()
    counts, pe, _ = G.count_patterns(per_edge=True, window=window, probe="middle")
    st = G.closure_stats()
    print(f"\n[transpose] window={window}: rows {st[5]}, in-list {st[13]} of {G.num_wedges}", flush=True)
    if window == "off":
        assert st[5] == 0 and st[13] == G.num_wedges
    if window == "always":
        # the largest window, 131,072 rows: the in-list holds the hyperwedges
        # of the 18,919 owners below it
        assert st[5] == 131072 and 0 < st[13] < G.num_wedges
    assert st[12] == 1 and st[13] == st[8], st
    assert np.array_equal(counts, r.H), (window, counts, r.H)
    assert np.array_equal(pe, r.t), window
