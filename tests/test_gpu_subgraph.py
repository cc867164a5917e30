"""Sub-hypergraphs of sigma-sampling (htri_subgraph) against the oracle: the
kept hyperedges of both selection modes, the triangle scale, exact and
per-hyperedge counts of the induced subgraph, and the scaled counts averaging
to the full count over seeds."""
import math

import numpy as np
import pytest

from oracle import core, sampling
from paper_2504_02271_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def htri():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_02271_amd import htri as h
    h.load_library()
    return h


@pytest.fixture(scope="module")
def base(htri):
    g = synth.generate(synth.config("tiny"))
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    off, mem, _ = o.csr()
    return g, G, o, off, mem


@pytest.mark.parametrize("fixed", [False, True])
@pytest.mark.parametrize("sigma,seed", [(0.3, 1), (0.7, 2), (1.0, 3), (0.05, 4)])
def test_subgraph_matches_oracle(htri, base, fixed, sigma, seed):
    g, G, o, off, mem = base
    m = G.num_edges
    Gs, kept, scale = G.subgraph(sigma, seed, fixed_size=fixed)
    want = sampling.subgraph_select(m, sigma, seed, fixed)
    assert np.array_equal(kept, want), (sigma, seed, fixed)
    assert Gs.num_edges == kept.shape[0] and Gs.removed == 0
    assert scale == sampling.subgraph_scale(m, kept.shape[0], sigma, fixed)
    so, sm = sampling.induced_csr(off, mem, want)
    # the subgraph's normalised CSR is the induced CSR, in the kept order
    go, gm = Gs.csr()
    assert np.array_equal(go, so) and np.array_equal(gm, sm)
    Gs.build_wedges()
    counts, pe, _ = Gs.count_patterns(per_edge=True)
    r = core.OracleGraph(so, sm, g.num_vertices).count()
    assert np.array_equal(counts, r.H)
    assert np.array_equal(pe, r.t)
    print(f"\n[subgraph] sigma {sigma} fixed {fixed}: {kept.shape[0]} of {m} kept, {int(counts[0])} triangles, "
          f"scale {scale:.4g}", flush=True)


def test_scaled_counts_average_to_the_count(htri, base):
    """Over 200 seeds, the exact count of the subgraph times the scale
    averages to the full count (both selection modes; 4 standard errors)."""
    g, G, o, off, mem = base
    G.build_wedges()
    H = G.count_patterns()[0]
    for fixed in (True, False):
        vals = []
        for seed in range(200):
            Gs, kept, scale = G.subgraph(0.5, 1000 + seed, fixed_size=fixed)
            Gs.build_wedges()
            vals.append(float(Gs.count_patterns()[0][0]) * scale)
            Gs.close()
        vals = np.array(vals)
        se = vals.std(ddof=1) / math.sqrt(vals.shape[0])
        print(f"\n[subgraph] fixed {fixed}: mean {vals.mean():.1f} vs {int(H[0])} (se {se:.1f})", flush=True)
        assert abs(vals.mean() - H[0]) < 4 * se, (fixed, vals.mean(), H[0], se)


def test_subgraph_errors(htri, base):
    _, G, _, _, _ = base
    for sigma, mode in ((0.0, False), (1.5, True), (-0.1, False)):
        with pytest.raises(htri.HtriError) as e:
            G.subgraph(sigma, 1, fixed_size=mode)
        assert e.value.code == -1
    # the parent is still usable
    assert G.subgraph(0.5, 1)[0].num_edges > 0
